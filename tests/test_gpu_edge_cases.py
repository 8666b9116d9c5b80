"""Edge cases of the step on the GPU: calls of zero steps (nothing changes,
the records still refer to the last step taken) and a negative count
(LBM_EINVAL); degenerate lattices against the oracle: one node, periodic in
every direction (every link streams back into the node), and lattices
smaller than one 256-node tile or ending in a partial tile, in both
lattices, FP64 and FP32."""
import sys

import numpy as np
import pytest

from helpers import make_oracle, rel_inf
from paper_2512_12213_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_12213_amd import lbm as L
    L.lib()
    return L


def test_zero_and_negative_step_counts(lbm):
    w = W.duct_sphere(nx=24, ny=16, nz=14, r=3.0)
    say("case zero steps")
    g = lbm.from_workload(w)
    g.step(5)
    s0, f0, b0 = g.get_state(), g.wall_force(), g.force_balance()
    g.step(0)
    assert np.array_equal(g.get_state(), s0)
    assert np.array_equal(g.wall_force(), f0) and np.array_equal(g.force_balance(), b0)
    with pytest.raises(lbm.LBMError) as ei:
        g.step(-1)
    assert ei.value.code == lbm.LBM_EINVAL
    assert np.array_equal(g.get_state(), s0)


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_single_periodic_node(lbm, lattice, storage):
    """One node, periodic everywhere, with a body force and LES: the GPU
    against the oracle after 1, 2 and 7 more steps (both parities)."""
    nz = 1
    w = W.Workload("one_node", lattice, 1, 1, nz, 0.7, dx=0.5, dt=0.2, model=W.GUO, storage=storage,
                   body_force=(0.05, -0.02, 0.03 if lattice == W.D3Q19 else 0.0), les_cs=0.1)
    say("case single node", lattice, storage)
    g = lbm.from_workload(w, init=False)
    o = make_oracle(w, init=False)
    u0 = np.zeros((w.D, 1, 1, 1))
    u0[0] = 0.01
    g.init_equilibrium(u0)
    o.init_equilibrium(u0)
    tol = 1e-12 if storage == W.F64 else 1e-5
    for n in (1, 2, 7):
        g.step(n)
        o.step(n)
        _, vg = g.get_macro()
        _, vo = o.get_macro()
        sg, _ = g.stress()
        so, _ = o.stress()
        e = rel_inf(vg, vo)
        say("  after %d: v %.2e" % (n, e))
        assert e <= tol
        assert np.abs(sg - so).max() <= tol * max(np.abs(so).max(), 1e-30) + 1e-300


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("shape", [(7, 5, 3), (13, 11, 1), (40, 9, 3)])
def test_lattices_smaller_than_a_tile_or_ending_in_a_partial_one(lbm, shape, storage):
    """105, 143 and 1080 nodes (one partial tile; four whole and one partial
    tile) with walls, a moving wall and a seeded state: the GPU against the
    oracle after calls of 3 and 4 steps."""
    nx, ny, nz = shape
    lattice = W.D2Q9 if nz == 1 else W.D3Q19
    walls = ((1, 0, 1),) if nz == 1 else ((1, 0, 1), (2, 2, 3))
    w = W.Workload("ragged", lattice, nx, ny, nz, 0.66, dx=0.5, dt=0.2, model=W.GUO, storage=storage,
                   body_force=(0.05, -0.02, 0.03 if nz > 1 else 0.0), walls=walls,
                   wall_velocity=((1, 0.08, 0.0, 0.03 if nz > 1 else 0.0),), groups=4)
    say("case ragged", shape, storage)
    d0 = W.random_state(w.Q, nx, ny, nz, 2e-3, seed=41)
    g = lbm.from_workload(w, init=False)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_state(d0.astype(np.float32).astype(np.float64) if storage == W.F32 else d0)
    tol = 1e-12 if storage == W.F64 else 1e-5
    for n in (3, 4):
        g.step(n)
        o.step(n)
        e_s = rel_inf(g.get_state(), o.get_state())
        fg = g.wall_force()[:, 0]
        fo = o.wall_force(fg.shape[0])[:, 0]
        e_f = np.linalg.norm(fg - fo) / np.linalg.norm(fo)
        say("  after %d: state %.2e wall %.2e" % (n, e_s, e_f))
        assert e_s <= tol and e_f <= (1e-12 if storage == W.F64 else 1e-4)
