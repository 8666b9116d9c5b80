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
