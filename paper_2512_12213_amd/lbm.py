"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function of the C ABI is exposed under the same name; ``Lattice`` wraps
a context with numpy-shaped inputs and outputs.  The native library must have
been built (``paper_2512_12213_amd.build.build()``); nothing here computes
any part of the method, and there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY names another build of the same library (the host-sanitizer
# build of build.py); by default the in-tree one
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_FORCE_HE, LBM_FORCE_LUO, LBM_FORCE_SHANCHEN, LBM_FORCE_EDM, LBM_FORCE_GUO = range(5)
LBM_F64, LBM_F32, LBM_F16, LBM_BF16 = range(4)
LBM_EQ_NS, LBM_EQ_STOKES = 0, 1
LBM_MHD_EQUILIBRIUM, LBM_MHD_LORENTZ_FORCE = 0, 1
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_ESTATE, LBM_EUNSTABLE = 0, -1, -2, -3, -4, -5
LBM_MAX_GROUPS, LBM_NREC = 16, 24
LBM_SCRATCH_BYTES = 8 << 20

# (name, restype, argtypes)
_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = [
    ("lbm_create", _P, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]),
    ("lbm_destroy", None, [_P]),
    ("lbm_last_error", C.c_char_p, []),
    ("lbm_set_storage", C.c_int, [_P, C.c_int]),
    ("lbm_set_rho0", C.c_int, [_P, C.c_double]),
    ("lbm_add_plane_walls", C.c_int, [_P, C.c_int, C.c_int, C.c_int]),
    ("lbm_add_solid_mask", C.c_int, [_P, C.c_void_p, C.c_int]),
    ("lbm_set_link_fractions", C.c_int, [_P, _D]),
    ("lbm_set_wall_velocity", C.c_int, [_P, C.c_int, C.c_double, C.c_double, C.c_double]),
    ("lbm_set_body_force", C.c_int, [_P, C.c_double, C.c_double, C.c_double]),
    ("lbm_set_body_force_field", C.c_int, [_P, C.c_void_p]),
    ("lbm_set_les", C.c_int, [_P, C.c_double]),
    ("lbm_set_equilibrium", C.c_int, [_P, C.c_int]),
    ("lbm_set_darcy", C.c_int, [_P, C.c_double]),
    ("lbm_set_artefact", C.c_int, [_P, C.c_int]),
    ("lbm_set_step_stress", C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int]),
    ("lbm_set_mhd", C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]),
    ("lbm_set_mhd_coupling", C.c_int, [_P, C.c_int]),
    ("lbm_set_stream", C.c_int, [_P, C.c_void_p]),
    ("lbm_init_equilibrium", C.c_int, [_P, _D]),
    ("lbm_set_state", C.c_int, [_P, _D]),
    ("lbm_get_state", C.c_int, [_P, _D]),
    ("lbm_get_induction", C.c_int, [_P, _D]),
    ("lbm_step", C.c_int, [_P, C.c_int]),
    ("lbm_step_noalloc", C.c_int, [_P, C.c_int]),
    ("lbm_get_macro", C.c_int, [_P, _D, _D]),
    ("lbm_get_field_B", C.c_int, [_P, _D]),
    ("lbm_stress", C.c_int, [_P, _D, _D]),
    ("lbm_halfstep", C.c_int, [_P, _D, _D, _D, _D]),
    ("lbm_halfstep_device", C.c_int, [_P, _P, _P, _P, _P]),
    ("lbm_stress_device", C.c_int, [_P, _P, _P]),
    ("lbm_wall_force", C.c_int, [_P, _D]),
    ("lbm_force_balance", C.c_int, [_P, _D]),
    ("lbm_set_wall_force_history", C.c_int, [_P, C.c_int]),
    ("lbm_wall_force_history", C.c_int, [_P, _D, C.c_int, C.POINTER(C.c_int)]),
    ("lbm_num_groups", C.c_int, [_P]),
    ("lbm_link_count", C.c_long, [_P, C.c_int]),
    ("lbm_steps_taken", C.c_long, [_P]),
    ("lbm_adjoint_forward", C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _D]),
    ("lbm_adjoint_backward", C.c_int, [_P, C.c_double, C.c_void_p, C.c_int, _D]),
    ("lbm_set_adjoint_precision", C.c_int, [_P, C.c_int]),
    ("lbm_set_timing", C.c_int, [_P, C.c_int]),
    ("lbm_step_timings", C.c_int, [_P, _D]),
]
EXPORTED = [s[0] for s in _SIGS]

_lib = None


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


def lib():
    """Load liblbm.so (raises if it has not been built).

    PyTorch for ROCm ships its own HIP runtime.  If the library were loaded
    first, a later ``import torch`` would bring a second HIP runtime into the
    process and torch would find no device; importing torch first (when it is
    installed) makes the library bind to torch's runtime, so that both share
    one runtime, one device context and interoperable streams."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm.so is not built; run paper_2512_12213_amd.build.build() first")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().lbm_last_error().decode()


def _chk(rc):
    if rc < 0:
        raise LBMError(rc, last_error())
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# Thin module-level aliases with the C names.
def __getattr__(name):
    if name in EXPORTED:
        return getattr(lib(), name)
    raise AttributeError(name)


class Lattice:
    """One lattice on the current GPU.  Shapes follow include/lbm.h:
    state [Q, nz, ny, nx]; rho [nz, ny, nx]; v [D, nz, ny, nx];
    stress [ncomp, nz, ny, nx]."""

    def __init__(self, lattice, nx, ny, nz, tau, dx=1.0, dt=1.0, force_model=LBM_FORCE_GUO, storage=LBM_F32):
        L = lib()
        self.L = L
        self.lattice, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.D = 2 if lattice == LBM_D2Q9 else 3
        self.Q = 9 if lattice == LBM_D2Q9 else 19
        self.NC = 3 if self.D == 2 else 6
        self.N = nx * ny * nz
        self.h = L.lbm_create(lattice, nx, ny, nz, tau, dx, dt, force_model)
        if not self.h:
            raise LBMError(LBM_EINVAL, last_error())
        self.mhd = False
        _chk(L.lbm_set_storage(self.h, storage))

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # set-up
    def set_rho0(self, rho0):
        _chk(self.L.lbm_set_rho0(self.h, rho0))

    def add_plane_walls(self, axis, g_lo, g_hi):
        _chk(self.L.lbm_add_plane_walls(self.h, axis, g_lo, g_hi))

    def add_solid_mask(self, mask, group):
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.size == self.N
        _chk(self.L.lbm_add_solid_mask(self.h, m.ctypes.data, group))

    def set_link_fractions(self, q):
        """q [Q, nz, ny, nx]: wall distance / link length of wall links (1/2 halfway), or None."""
        q = _f64(q)
        if q is not None:
            assert q.size == self.Q * self.N
        _chk(self.L.lbm_set_link_fractions(self.h, _dp(q)))

    def set_wall_velocity(self, group, u):
        u = list(u) + [0.0] * (3 - len(u))
        _chk(self.L.lbm_set_wall_velocity(self.h, group, *u[:3]))

    def set_body_force(self, a):
        a = list(a) + [0.0] * (3 - len(a))
        _chk(self.L.lbm_set_body_force(self.h, *a[:3]))

    def set_body_force_field(self, dev_ptr):
        """dev_ptr: int device address of float32 [3, nz, ny, nx], or None."""
        _chk(self.L.lbm_set_body_force_field(self.h, dev_ptr))

    def set_les(self, cs):
        _chk(self.L.lbm_set_les(self.h, cs))

    def set_equilibrium(self, kind):
        _chk(self.L.lbm_set_equilibrium(self.h, kind))

    def set_darcy(self, sigma):
        _chk(self.L.lbm_set_darcy(self.h, sigma))

    def set_artefact(self, on):
        _chk(self.L.lbm_set_artefact(self.h, int(on)))

    def set_step_stress(self, sigma_ptr, strain_ptr, every=1):
        """Device float buffers [ncomp, nz, ny, nx] (int addresses, or None)
        that every `every`-th step fills with the stress and strain rate of
        the state it starts from."""
        _chk(self.L.lbm_set_step_stress(self.h, sigma_ptr, strain_ptr, every))

    def set_mhd(self, B0, mu, tau_m):
        _chk(self.L.lbm_set_mhd(self.h, B0[0], B0[1], B0[2], mu, tau_m))
        self.mhd = True

    def set_mhd_coupling(self, kind):
        """LBM_MHD_EQUILIBRIUM (Eq. 10, default) or LBM_MHD_LORENTZ_FORCE."""
        _chk(self.L.lbm_set_mhd_coupling(self.h, kind))

    def set_stream(self, stream_ptr):
        _chk(self.L.lbm_set_stream(self.h, stream_ptr))

    # state
    def init_equilibrium(self, u0=None):
        u0 = _f64(u0)
        if u0 is not None:
            assert u0.size == self.D * self.N
        _chk(self.L.lbm_init_equilibrium(self.h, _dp(u0)))

    def set_state(self, d):
        d = _f64(d)
        assert d.size == self.Q * self.N
        _chk(self.L.lbm_set_state(self.h, _dp(d)))

    def get_state(self):
        d = np.empty((self.Q, self.nz, self.ny, self.nx))
        _chk(self.L.lbm_get_state(self.h, _dp(d)))
        return d

    def get_induction(self):
        g = np.empty((7, 3, self.nz, self.ny, self.nx) if self.Q == 19 else (5, 2, self.nz, self.ny, self.nx))
        _chk(self.L.lbm_get_induction(self.h, _dp(g)))
        return g

    # hot path and outputs
    def step(self, n=1):
        _chk(self.L.lbm_step(self.h, n))

    def step_noalloc(self, n=1):
        """lbm_step with the step's scratch in the library's fixed device array."""
        _chk(self.L.lbm_step_noalloc(self.h, n))

    def get_macro(self):
        rho = np.empty((self.nz, self.ny, self.nx))
        v = np.empty((self.D, self.nz, self.ny, self.nx))
        _chk(self.L.lbm_get_macro(self.h, _dp(rho), _dp(v)))
        return rho, v

    def get_field_B(self):
        B = np.empty((3, self.nz, self.ny, self.nx))
        _chk(self.L.lbm_get_field_B(self.h, _dp(B)))
        return B

    def stress(self):
        sig = np.empty((self.NC, self.nz, self.ny, self.nx))
        S = np.empty_like(sig)
        _chk(self.L.lbm_stress(self.h, _dp(sig), _dp(S)))
        return sig, S

    def halfstep(self):
        """Half-step distribution of the last step (Eq. 27) and its moments:
        (fbar [Q, ...] deviations, rho_bar, u_bar [D, ...], sigma_bar [ncomp, ...])."""
        sh = (self.nz, self.ny, self.nx)
        fb = np.empty((self.Q,) + sh)
        rb = np.empty(sh)
        ub = np.empty((self.D,) + sh)
        sb = np.empty((self.NC,) + sh)
        _chk(self.L.lbm_halfstep(self.h, _dp(fb), _dp(rb), _dp(ub), _dp(sb)))
        return fb, rb, ub, sb

    def stress_device(self, sigma_ptr, strain_ptr):
        """lbm_stress_device: sigma and S of the current state into caller
        device buffers (pointers; None for one not wanted), enqueued on the
        library's stream."""
        _chk(self.L.lbm_stress_device(self.h, sigma_ptr, strain_ptr))

    def halfstep_device(self, fbar_ptr, rho_ptr, u_ptr, sigma_ptr):
        """lbm_halfstep_device: the same outputs into caller device buffers
        (pointers, e.g. torch tensors' data_ptr(); None for any not wanted),
        enqueued on the library's stream."""
        _chk(self.L.lbm_halfstep_device(self.h, fbar_ptr, rho_ptr, u_ptr, sigma_ptr))

    def num_groups(self):
        return _chk(self.L.lbm_num_groups(self.h))

    def wall_force(self):
        G = self.num_groups()
        out = np.empty((G, 4, 3))
        _chk(self.L.lbm_wall_force(self.h, _dp(out)))
        return out

    def set_wall_force_history(self, on=True):
        _chk(self.L.lbm_set_wall_force_history(self.h, int(on)))

    def wall_force_history(self, max_steps=1 << 20):
        """[n, G, 4, 3]: the wall-force variants of every step of the last call."""
        G = self.num_groups()
        nmax = min(max_steps, int(self.steps_taken()))
        out = np.empty((max(nmax, 1), G, 4, 3))
        n = C.c_int(0)
        _chk(self.L.lbm_wall_force_history(self.h, _dp(out), nmax, C.byref(n)))
        return out[:n.value]

    def force_balance(self):
        out = np.empty(LBM_NREC)
        _chk(self.L.lbm_force_balance(self.h, _dp(out)))
        return out

    def link_count(self, group=-1):
        return _chk(self.L.lbm_link_count(self.h, group))

    def steps_taken(self):
        return self.L.lbm_steps_taken(self.h)

    # differentiation
    def adjoint_forward(self, T, ckpt_every, group, axis):
        """Record T steps (checkpoint every ckpt_every) and return J, the raw
        wall force of `group` along `axis` during the last step."""
        J = np.zeros(1)
        _chk(self.L.lbm_adjoint_forward(self.h, T, ckpt_every, group, axis, _dp(J)))
        return float(J[0])

    def adjoint_backward(self, gJ=1.0, grad_a_ptr=None, grad_f64=False):
        """gJ dJ/du_w as [G, 3]; gJ dJ/da into the device buffer at
        grad_a_ptr ([3, nz, ny, nx], float32 or float64) when given."""
        G = self.num_groups()
        gu = np.zeros((G, 3))
        _chk(self.L.lbm_adjoint_backward(self.h, gJ, grad_a_ptr, int(grad_f64), _dp(gu)))
        return gu

    def set_adjoint_precision(self, precision):
        _chk(self.L.lbm_set_adjoint_precision(self.h, precision))

    def set_timing(self, on=True):
        _chk(self.L.lbm_set_timing(self.h, int(on)))

    def step_timings(self):
        """dict of seconds: even, odd (mean step launches), diag, tail, launches, call"""
        out = np.empty(6)
        _chk(self.L.lbm_step_timings(self.h, _dp(out)))
        return dict(zip(("even", "odd", "diag", "tail", "launches", "call"), out.tolist()))


def from_workload(w, storage=None, u0=None, init=True):
    """Configure a Lattice from a workloads.Workload description."""
    from . import workloads as W
    lat = Lattice(w.lattice, w.nx, w.ny, w.nz, w.tau, w.dx, w.dt, w.model,
                  w.storage if storage is None else storage)
    for axis, glo, ghi in w.walls:
        lat.add_plane_walls(axis, glo, ghi)
    for g, ux, uy, uz in w.wall_velocity:
        lat.set_wall_velocity(g, [ux, uy, uz])
    mask = W.obstacle_mask(w)
    if mask is not None:
        lat.add_solid_mask(mask, w.obstacle[-1])
    qf = W.link_fractions(w)
    if qf is not None:
        lat.set_link_fractions(qf)
    lat.set_body_force(list(w.body_force))
    if w.les_cs:
        lat.set_les(w.les_cs)
    if w.stokes:
        lat.set_equilibrium(LBM_EQ_STOKES)
    if w.darcy:
        lat.set_darcy(w.darcy)
    if w.mhd is not None:
        lat.set_mhd(w.mhd[:3], w.mhd[3], w.mhd[4])
        if w.lorentz:
            lat.set_mhd_coupling(LBM_MHD_LORENTZ_FORCE)
    if init:
        lat.init_equilibrium(W.initial_velocity(w) if u0 is None else u0)
    return lat
