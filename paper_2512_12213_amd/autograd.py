"""torch.autograd binding of the C ABI's differentiable run.

``WallForceObjective(workload, T, ckpt_every, group, axis, uw_group)`` holds
one lattice; calling it with a per-node body-force field ``a`` (CUDA float32
tensor [3, nz, ny, nx]) and the velocity ``u_w`` ([3] float64) of wall group
``uw_group`` restarts the lattice from the workload's initial state, runs T
steps with checkpoints (lbm_adjoint_forward) and returns J, the raw Eq. (25)
force on wall group ``group`` along ``axis`` during the last step.
``J.backward()`` calls lbm_adjoint_backward, which writes dJ/da straight into
the gradient tensor on the caller's stream.  Argument marshalling only: the
forward and adjoint steps run in the HIP library.
"""
import numpy as np
import torch

from . import lbm as _lbm
from . import workloads as W


class _WallForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, uw, obj):
        lat = obj.lat
        if not (a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()):
            raise TypeError("a must be a contiguous CUDA float32 tensor [3, nz, ny, nx]")
        if tuple(a.shape) != (3, obj.w.nz, obj.w.ny, obj.w.nx):
            raise ValueError("a has shape %s, expected %s" % (tuple(a.shape), (3, obj.w.nz, obj.w.ny, obj.w.nx)))
        lat.set_stream(torch.cuda.current_stream(a.device).cuda_stream)
        lat.set_body_force_field(a.data_ptr())
        lat.set_wall_velocity(obj.uw_group, [float(v) for v in uw.detach().cpu().tolist()])
        lat.init_equilibrium(obj.u0)
        J = lat.adjoint_forward(obj.T, obj.ckpt_every, obj.group, obj.axis)
        ctx.obj = obj
        ctx.a_shape = a.shape
        ctx.a_device = a.device
        ctx.uw_dtype = uw.dtype
        ctx.uw_device = uw.device
        # keep the field alive: the recorded run reads it again in backward
        ctx.save_for_backward(a)
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        obj = ctx.obj
        (a,) = ctx.saved_tensors
        lat = obj.lat
        lat.set_stream(torch.cuda.current_stream(a.device).cuda_stream)
        grad_a = torch.empty(ctx.a_shape, dtype=torch.float32, device=ctx.a_device)
        gu = lat.adjoint_backward(float(gJ), grad_a.data_ptr(), False)
        grad_uw = torch.tensor(gu[obj.uw_group], dtype=ctx.uw_dtype, device=ctx.uw_device)
        return grad_a, grad_uw, None


class WallForceObjective:
    """Differentiable J(a, u_w) on one lattice built from a workload."""

    def __init__(self, w: W.Workload, T, ckpt_every, group, axis, uw_group, storage=None):
        self.w = w
        self.T, self.ckpt_every, self.group, self.axis, self.uw_group = T, ckpt_every, group, axis, uw_group
        self.lat = _lbm.from_workload(w, storage=storage, init=False)
        u0 = W.initial_velocity(w)
        self.u0 = None if u0 is None else np.ascontiguousarray(u0)

    def __call__(self, a, uw):
        return _WallForce.apply(a, uw, self)

    def close(self):
        self.lat.close()
