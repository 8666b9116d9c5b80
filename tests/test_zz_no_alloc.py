"""lbm_step_noalloc (the step with its scratch in the library's fixed device
array, for callers that cannot allocate) against lbm_step through the C ABI:
the same kernels and the same deterministic reductions, so the state, the
wall-force record and the balance record must be bit-identical.  Two calls in
a row on the fixed array, the second on a smaller lattice (its contents from
the first call must not matter), and a lattice too large for the array is
refused before any work."""
import sys

import numpy as np
import pytest

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


def records(g):
    return g.get_state(), g.wall_force(), g.force_balance()


def same_as_lbm_step(lbm, w, calls):
    a = lbm.from_workload(w)
    b = lbm.from_workload(w)
    for n in calls:
        a.step(n)
        b.step_noalloc(n)
        ra, rb = records(a), records(b)
        for x, y, name in zip(ra, rb, ("state", "wall force", "balance")):
            assert np.array_equal(x, y), (w.name, n, name, np.abs(x - y).max())
    a.close()
    b.close()


def test_noalloc_matches_lbm_step_on_two_calls_in_a_row(lbm):
    # first call: a 3D duct with a sphere whose walls are not halfway (the
    # interpolated-wall buffers are in the fixed array too) and a moving wall
    w1 = W.duct_sphere(nx=64, ny=32, nz=32, r=5.0, steps=0)
    w1.curved = True
    say("case noalloc duct+sphere 64x32x32 curved, calls of 7 and 4 steps")
    same_as_lbm_step(lbm, w1, (7, 4))
    # second call: a smaller 2D lattice (Couette channel with a cylinder)
    w2 = W.couette_cylinder(nx=96, ny=24, r=4.0, cx=30.0, cy=12.0, steps=0)
    say("case noalloc couette+cylinder 96x24, calls of 5 and 1 steps")
    same_as_lbm_step(lbm, w2, (5, 1))


def test_noalloc_refuses_a_lattice_beyond_the_array(lbm):
    # 256 x 256 x 200 nodes: 51 200 tiles x 184 bytes of partial sums > 8 MiB
    w = W.duct_les(nx=256, ny=256, nz=200, storage=W.F16, steps=0)
    say("case noalloc refusal 256x256x200")
    g = lbm.from_workload(w)
    before = g.steps_taken()
    with pytest.raises(lbm.LBMError) as ei:
        g.step_noalloc(1)
    assert ei.value.code == lbm.LBM_EINVAL
    assert "scratch" in str(ei.value)
    assert g.steps_taken() == before
    g.close()
