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
    qf = W.link_fractions(w)
    if qf is not None:
        o.set_link_fraction(qf)
    if w.les_cs:
        o.set_les(w.les_cs)
    if w.stokes:
        o.set_equilibrium(True)
    if w.darcy:
        o.set_darcy(w.darcy)
    if w.mhd is not None:
        o.set_mhd(w.mhd[:3], w.mhd[3], w.mhd[4])
        if w.lorentz:
            o.set_lorentz_force(True)
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


# ---------------------------------------------------------------------------
# Storage formats of include/lbm.h, applied to oracle states.  They let the
# 16-bit GPU paths be compared element-wise with the oracle's FP64 arithmetic
# carrying the same storage rounding (the "quantized oracle").
# ---------------------------------------------------------------------------
def _weights(Q):
    from closed_forms import lattice
    _, w = lattice("D2Q9" if Q == 9 else "D3Q19")
    return w


def bf16_round(x):
    """Round float64 -> float32 -> bfloat16 (nearest even), back to float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def quantize_state(d, storage):
    """Deviations d [Q, ...] rounded as the library stores them."""
    from paper_2512_12213_amd import workloads as W
    if storage == W.F64:
        return d
    if storage == W.F32:
        return d.astype(np.float32).astype(np.float64)
    w = _weights(d.shape[0]).reshape((-1,) + (1,) * (d.ndim - 1))
    if storage == W.F16:
        s = 1024.0 / w
        return (d * s).astype(np.float32).astype(np.float16).astype(np.float64) / s
    return bf16_round(d / w) * w


def quantized_steps(o, storage, n):
    """Advance the oracle n steps, rounding the state to the storage format
    after each step (the wall-force / balance records of the last step are
    kept by the oracle)."""
    for _ in range(n):
        o.step(1)
        o.set_state(quantize_state(o.get_state(), storage), keep_records=True)


# ---------------------------------------------------------------------------
# Stated accuracy targets and the misses recorded as not met.
# ---------------------------------------------------------------------------
def check_targets(errs, target, misses=None, what=""):
    """Assert each error in `errs` (name -> value) at `target` (a number or a
    name -> number dict), except the names in `misses` (name -> bound): those
    are results recorded as not meeting the target; each must stay within its
    recorded bound (a regression check), and if any of them is above its
    target the test ends as an expected failure that states the measured
    values."""
    import pytest
    misses = misses or {}
    tgt = (lambda k: target[k]) if isinstance(target, dict) else (lambda k: target)
    over = {}
    for k, v in errs.items():
        if k in misses:
            assert v <= misses[k], "%s: %s = %.3e beyond its recorded bound %.1e" % (what, k, v, misses[k])
            if v > tgt(k):
                over[k] = v
        else:
            assert v <= tgt(k), "%s: %s = %.3e above the target %.1e" % (what, k, v, tgt(k))
    if over:
        pytest.xfail("not met (recorded): %s: %s" % (what, ", ".join("%s %.2e > %.0e" % (k, v, tgt(k))
                                                                     for k, v in over.items())))
