"""Outputs the step itself produces beyond lbm_step's records: the shear
stress and strain rate of Eqs. (8)-(9) written by flagged steps
(lbm_set_step_stress), against the oracle's stress of the same state,
element by element, and against lbm_stress of the same GPU state.

Tolerances (max-norm relative): the stored values are FP32, so FP64 storage
is held to 1e-6 (a few FP32 roundings of the output); FP32 storage 1e-5;
FP16 storage 2e-3 against the quantized oracle.
"""
import sys

import numpy as np
import pytest

from helpers import make_oracle, quantize_state, quantized_steps, rel_inf
from paper_2512_12213_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {W.F64: 1e-6, W.F32: 1e-5, W.F16: 2e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2512_12213_amd import lbm as L
    L.lib()
    return L, torch


def case(lattice, model, storage):
    if lattice == W.D2Q9:
        nx, ny, nz = 64, 19, 1
        mask = W.cylinder_mask(nx, ny, 12.3, 9.1, 3.2)
        walls = ((1, 0, 1),)
    else:
        nx, ny, nz = 64, 13, 11
        mask = W.sphere_mask(nx, ny, nz, 9.4, 6.2, 5.1, 2.6)
        walls = ((1, 0, 1), (2, 2, 3))
    w = W.Workload("step_stress", lattice, nx, ny, nz, 0.62, dx=0.5, dt=0.2, model=model, storage=storage,
                   body_force=(0.05, -0.02, 0.03), walls=walls, wall_velocity=((1, 0.08, 0.0, 0.03),),
                   les_cs=0.1, groups=5)
    return w, mask


@pytest.mark.parametrize("storage", [W.F64, W.F32, W.F16])
@pytest.mark.parametrize("model", [0, 2, 4])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_step_stress_matches_oracle(env, lattice, model, storage):
    """Seeded state with walls, a moving wall, a solid body, LES and
    non-unity dx, dt; calls of 1, 1 and 2 steps storing every step (the
    buffers then hold the state each last step started from: step indices
    0, 1 and 3, both A-A parities), the last call with the artefact term;
    then every third step (a 5-step call from index 4 stores at index 6)."""
    L, torch = env
    w, mask = case(lattice, model, storage)
    Q = w.Q
    nc = 3 if lattice == W.D2Q9 else 6
    say("case step stress", lattice, model, storage)
    d0 = W.random_state(Q, w.nx, w.ny, w.nz, 2e-3, seed=27) * (1 - mask[None])
    g = L.from_workload(w, init=False)
    g.add_solid_mask(mask, 4)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_state(quantize_state(d0, storage))
    sig = torch.full((nc, w.nz, w.ny, w.nx), 7.0, dtype=torch.float32, device="cuda")
    S = torch.full_like(sig, 7.0)
    g.set_step_stress(sig.data_ptr(), S.data_ptr(), 1)
    torch.cuda.synchronize()
    assert float(sig.abs().max()) == 0.0 and float(S.abs().max()) == 0.0
    low = storage == W.F16

    def advance_oracle(n):
        if low:
            quantized_steps(o, storage, n)
        else:
            o.step(n)

    def check(what):
        torch.cuda.synchronize()
        so, Sg_o = o.stress()
        e = dict(sigma=rel_inf(sig.cpu().numpy().astype(np.float64), so),
                 S=rel_inf(S.cpu().numpy().astype(np.float64), Sg_o))
        say("  %s: %s" % (what, {k: "%.2e" % v for k, v in e.items()}))
        assert e["sigma"] <= TOL[storage] and e["S"] <= TOL[storage]

    # each check compares the oracle's stress of the state the GPU's last
    # step started from: the oracle is kept one step behind
    g.step(1)
    check("index 0")
    advance_oracle(1)
    g.step(1)
    check("index 1")
    advance_oracle(1)
    g.set_artefact(True)
    o.set_artefact(True)
    g.step(2)
    advance_oracle(1)
    check("index 3, artefact")
    advance_oracle(1)
    # every third step: a 5-step call from index 4 (steps 4 ... 8) stores at 6
    g.set_step_stress(sig.data_ptr(), S.data_ptr(), 3)
    g.step(5)
    advance_oracle(2)
    check("index 6 of every 3")


def test_step_stress_equals_lbm_stress_full_size(env):
    """256x128x128 duct with LES, FP32, in the bench's launch configuration:
    the values a step stores (FP32 arithmetic) against lbm_stress of the
    state it starts from (FP64 arithmetic on the same stored values): after
    6 steps, and at the end of a 9-step call storing every step (the state
    after 15 steps, taken from a second run of the same deterministic
    steps)."""
    L, torch = env
    w = W.duct_les()
    say("case step stress full size")
    g = L.from_workload(w)
    g.step(6)
    s_ref, S_ref = g.stress()
    sig = torch.empty((6, w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
    S = torch.empty_like(sig)
    g.set_step_stress(sig.data_ptr(), S.data_ptr(), 1)
    g.step(1)
    torch.cuda.synchronize()
    e1 = rel_inf(sig.cpu().numpy().astype(np.float64), s_ref)
    e2 = rel_inf(S.cpu().numpy().astype(np.float64), S_ref)
    say("  index 6: sigma %.2e S %.2e" % (e1, e2))
    assert e1 <= 1e-5 and e2 <= 1e-5
    g.step(9)  # indices 7 ... 15: the buffers hold the state after 15 steps
    torch.cuda.synchronize()
    got = sig.cpu().numpy().astype(np.float64)
    g.close()
    h = L.from_workload(w)
    h.step(15)
    s_ref, _ = h.stress()
    h.close()
    e3 = rel_inf(got, s_ref)
    say("  index 15: sigma %.2e" % e3)
    assert e3 <= 1e-5


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_stress_into_device_buffers_equals_host_outputs(env, storage):
    """lbm_stress_device writes the same values (bit for bit) into caller
    device buffers as lbm_stress does into host buffers, for a seeded state
    with walls, a solid body and LES; either output alone."""
    L, torch = env
    w, mask = case(W.D3Q19, 4, storage)
    say("case stress device", storage)
    g = L.from_workload(w, init=False)
    g.add_solid_mask(mask, 4)
    g.set_state(W.random_state(w.Q, w.nx, w.ny, w.nz, 2e-3, seed=29) * (1 - mask[None]))
    g.step(3)
    sh, Sh = g.stress()
    dev = dict(dtype=torch.float64, device="cuda")
    sd = torch.full(sh.shape, 7.0, **dev)
    Sd = torch.full(Sh.shape, 7.0, **dev)
    torch.cuda.synchronize()
    g.stress_device(sd.data_ptr(), Sd.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(sd.cpu().numpy(), sh) and np.array_equal(Sd.cpu().numpy(), Sh)
    sd.fill_(7.0)
    Sd.fill_(7.0)
    torch.cuda.synchronize()
    g.stress_device(None, Sd.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(Sd.cpu().numpy(), Sh) and float(sd.cpu().max()) == 7.0


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_step_stress_with_interpolated_walls(env, storage):
    """The duct with an off-lattice sphere (64 wide: the steps interpolate
    the sphere's links themselves) storing the stress every step: a 5-step
    call leaves the stress of the state its last step started from, against
    the oracle's stress of that state (after 4 steps): FP64 1e-6, FP32 1e-5;
    and the state after the call against the oracle's."""
    L, torch = env
    w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7, storage=storage)
    w.curved = True
    say("case step stress curved", storage)
    g = L.from_workload(w)
    o = make_oracle(w)
    sig = torch.empty((6, w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
    S = torch.empty_like(sig)
    g.set_step_stress(sig.data_ptr(), S.data_ptr(), 1)
    g.step(5)
    o.step(4)
    torch.cuda.synchronize()
    so, So = o.stress()
    e = dict(sigma=rel_inf(sig.cpu().numpy().astype(np.float64), so),
             S=rel_inf(S.cpu().numpy().astype(np.float64), So))
    o.step(1)
    e["state"] = rel_inf(g.get_state(), o.get_state())
    say("  %s" % {k: "%.2e" % v for k, v in e.items()})
    assert e["sigma"] <= TOL[storage] and e["S"] <= TOL[storage]
    assert e["state"] <= (1e-12 if storage == W.F64 else 1e-5)


def test_step_stress_argument_checks(env):
    L, torch = env
    w = W.poiseuille(nx=8, ny=8)
    g = L.from_workload(w)
    sig = torch.zeros((3, 1, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(L.LBMError) as ei:
        g.set_step_stress(sig.data_ptr(), None, 0)
    assert ei.value.code == L.LBM_EINVAL
    g.set_step_stress(None, None, 0)  # off
    g.step(2)
    g.close()


# ---------------------------------------------------------------------------
# Per-step wall-force record (Eq. 25 for every step of a call)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage", [W.F64, W.F32, W.F16, W.BF16])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_wall_force_history_matches_oracle(env, lattice, storage):
    """A 7-step call with the history on, from a seeded state with a wall
    moving along its normal and tangentially (all four variants nonzero or
    exactly zero as in the oracle), a static wall group, a solid body and
    non-unity dx, dt: every step's record against the oracle's record of
    that step; FP64 1e-12, FP32 1e-4, 16-bit 2e-3 against the oracle whose
    state is rounded to the format after every step (2-norm per group and
    variant)."""
    L, torch = env
    if lattice == W.D2Q9:
        nx, ny, nz = 40, 17, 1
        mask = W.cylinder_mask(nx, ny, 14.2, 8.3, 3.1)
        walls = ((1, 0, 1),)
    else:
        nx, ny, nz = 24, 13, 11
        mask = W.sphere_mask(nx, ny, nz, 9.4, 6.2, 5.1, 2.6)
        walls = ((1, 0, 1), (2, 2, 3))
    c = 0.5 / 0.2
    w = W.Workload("history", lattice, nx, ny, nz, 0.66, dx=0.5, dt=0.2, model=W.GUO, storage=storage,
                   body_force=(0.05, -0.02, 0.03), walls=walls,
                   wall_velocity=((1, 0.03 * c, 0.02 * c, 0.01 * c),), groups=5)
    Q = w.Q
    say("case wall-force history", lattice, storage)
    d0 = W.random_state(Q, nx, ny, nz, 2e-3, seed=51) * (1 - mask[None])
    g = L.from_workload(w, init=False)
    g.add_solid_mask(mask, 4)
    g.set_wall_force_history(True)
    g.set_state(d0)
    o = make_oracle(w, init=False)
    o.set_solid(mask, 4)
    o.groups = 5
    o.set_state(quantize_state(d0, storage))
    g.step(7)
    hist = g.wall_force_history()
    assert hist.shape == (7, 5, 4, 3)
    assert np.array_equal(hist[-1], g.wall_force())
    tol = {W.F64: 1e-12, W.F32: 1e-4}.get(storage, 2e-3)
    worst = 0.0
    for s in range(7):
        if storage in (W.F16, W.BF16):
            quantized_steps(o, storage, 1)
        else:
            o.step(1)
        fo = o.wall_force(5)
        for k in range(5):
            for var in range(4):
                ref = np.linalg.norm(fo[k, var])
                if ref > 0:
                    worst = max(worst, np.linalg.norm(hist[s, k, var] - fo[k, var]) / ref)
                else:
                    assert np.abs(hist[s, k, var]).max() == 0.0
    say("  worst relative error over 7 steps: %.2e" % worst)
    assert worst <= tol
    # the normal motion gives a momentum-flux correction
    assert np.abs(hist[:, 1, 1] - hist[:, 1, 0]).max() > 0


def test_wall_force_history_of_a_long_call_equals_one_step_calls(env):
    """A 300-step call (two chunks of the 256-step ring) against 300
    one-step calls of the same deterministic steps: the same states, records
    summed in another order (FP64 sums, 1e-12 relative)."""
    L, torch = env
    w = W.couette_cylinder(nx=128, ny=32, r=5.0, cx=40.0, cy=16.0, steps=0)
    say("case history 300 steps")
    a = L.from_workload(w)
    a.set_wall_force_history(True)
    a.step(300)
    hist = a.wall_force_history()
    assert hist.shape[0] == 300
    b = L.from_workload(w)
    worst = 0.0
    for s in range(300):
        b.step(1)
        fb = b.wall_force()
        worst = max(worst, float(np.abs(hist[s] - fb).max() / np.abs(fb).max()))
    say("  worst %.2e" % worst)
    assert worst <= 1e-12
    assert np.array_equal(a.get_state(), b.get_state())
    # the history also caps at max_steps and refuses lbm_step_noalloc
    assert a.wall_force_history(max_steps=5).shape[0] == 5
    with pytest.raises(L.LBMError) as ei:
        a.step_noalloc(1)
    assert ei.value.code == L.LBM_EINVAL
    a.set_wall_force_history(False)
    a.step_noalloc(1)


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_wall_force_history_with_walls_that_are_not_halfway(env, storage):
    """Duct with a moving curved sphere (links at their wall distance), a
    moving plane wall: a 6-step call with the history on (the interpolation
    runs as a pass after every step), every step's record against the
    oracle's wall force after that step (2-norm per group and variant;
    FP64 1e-12, FP32 1e-4); the last entry equals lbm_wall_force."""
    L, torch = env
    w = W.duct_sphere(nx=64, ny=20, nz=18, r=4.3, uw=0.01, a=1e-4, steps=0)
    w.curved = True
    w.wall_velocity = ((1, 0.01, 0.0, 0.0), (4, 0.004, -0.003, 0.002))
    say("case wall-force history with interpolated walls", storage)
    g = L.from_workload(w, storage=storage)
    with pytest.raises(L.LBMError) as ei:
        g.wall_force_history()
    assert ei.value.code == L.LBM_ESTATE
    g.set_wall_force_history(True)
    g.step(6)
    hist = g.wall_force_history()
    assert hist.shape[0] == 6
    assert np.array_equal(hist[-1], g.wall_force())
    o = make_oracle(w)
    tol = 1e-12 if storage == W.F64 else 1e-4
    worst = 0.0
    G = hist.shape[1]
    for s in range(6):
        o.step(1)
        fo = o.wall_force(G)
        for k in range(G):
            for var in range(4):
                ref = np.linalg.norm(fo[k, var])
                if ref > 0:
                    worst = max(worst, np.linalg.norm(hist[s, k, var] - fo[k, var]) / ref)
    say("  worst relative error over 6 steps: %.2e" % worst)
    assert worst <= tol
    # the interpolated links' share is in every step's record: the sphere's
    # force differs from that of the same call without the record only by rounding
    g2 = L.from_workload(w, storage=storage)
    g2.step(3)
    f3 = g2.wall_force()[4, 0]
    assert np.linalg.norm(hist[2, 4, 0] - f3) <= (1e-12 if storage == W.F64 else 1e-5) * np.linalg.norm(f3)
    g.close()
    g2.close()
