"""Test helpers: configure the oracle (and, in GPU tests, the library) from a
workload description."""
import numpy as np

from paper_2512_12213_amd import workloads as W


def make_oracle(w: W.Workload, complex_step=False, u0=None, init=True):
    import oracle
    o = oracle.Oracle(w.lattice, w.nx, w.ny, w.nz, w.tau, w.dx, w.dt, w.model, complex_step=complex_step)
    for axis, glo, ghi in w.walls:
        o.set_walls(axis, glo, ghi)
    for g, ux, uy, uz in w.wall_velocity:
        o.set_wall_velocity(g, [ux, uy, uz])
    mask = W.obstacle_mask(w)
    if mask is not None:
        o.set_solid(mask, w.obstacle[-1])
    o.set_body_force(list(w.body_force))
    if w.les_cs:
        o.set_les(w.les_cs)
    if w.mhd is not None:
        o.set_mhd(w.mhd[:3], w.mhd[3], w.mhd[4])
    o.groups = max(o.groups, w.groups)
    if init:
        o.init_equilibrium(W.initial_velocity(w) if u0 is None else u0)
    return o


def rel_inf(x, ref):
    """max|x - ref| / max|ref| (0 when both vanish)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.abs(ref).max()
    num = np.abs(x - ref).max()
    if den == 0:
        return float(num)
    return float(num / den)
