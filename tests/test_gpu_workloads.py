"""The five synthetic workloads at their full shapes on the GPU, against the
FP64 oracle and the closed forms and balances the paper fixes.

  channel 64x32 FP64, 60 000 steps: steady profile (bounce-back closed form),
      wall shear = momentum exchange = body force (Eq. 33), all force models;
  Couette channel + cylinder 512x128, 20 000 steps, FP32 and FP64: fields and
      every wall-force variant against the oracle;
  square duct with LES 256x128x128, 1 000 steps, every storage format against
      one FP64 oracle run;
  Hartmann channel (192x96x1) to the closed form, and the Hartmann duct
      192x96x96 against the oracle, with the per-step balance (Eq. 32).
Tolerances as in test_gpu_parity (FP64 1e-12, FP32 1e-5 fields / 1e-4 wall
force, 16-bit 2e-3); the 16-bit results that miss 2e-3 against the
unquantized oracle are recorded as not met (expected failures stating the
measured values, each within a recorded bound).
"""
import sys

import numpy as np
import pytest

from closed_forms import hartmann, poiseuille_steady
from helpers import check_targets, make_oracle, rel_inf
from paper_2512_12213_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    import oracle
    from paper_2512_12213_amd import lbm as L
    L.lib()
    oracle.threads(16)
    return L


def errors(g, o, groups):
    rg, vg = g.get_macro()
    ro, vo = o.get_macro()
    sg, Sg = g.stress()
    so, So = o.stress()
    fg = g.wall_force()[:groups]
    fo = o.wall_force(groups)
    ef = max(np.linalg.norm(fg[k, v] - fo[k, v]) / np.linalg.norm(fo[k, v])
             for k in range(groups) for v in range(4) if np.linalg.norm(fo[k, v]) > 0)
    return dict(rho=float(np.abs(rg - ro).max()), v=rel_inf(vg, vo), sigma=rel_inf(sg, so), S=rel_inf(Sg, So),
                wall=ef)


@pytest.mark.parametrize("model", [0, 1, 2, 3, 4])
def test_channel_60000_steps_steady(lbm, model):
    w = W.poiseuille(model=model, steps=60000)
    say("case channel steady model", model)
    g = lbm.from_workload(w)
    g.step(w.steps)
    rho, v = g.get_macro()
    rec = g.force_balance()
    fw = g.wall_force()
    say("model %d: F_wall / sum rho a = %.15f, stress integral / F = %.15f"
        % (model, rec[0] / rec[3], rec[18] / rec[0]))
    # Eq. (33): steady, static walls: total wall force = integral of rho a,
    # and the stress integral at the walls carries the same force
    assert abs(rec[0] / rec[3] - 1) < 1e-10
    assert abs(rec[18] / rec[0] - 1) < 1e-9
    # the two walls share it equally
    assert abs(fw[0, 0, 0] - fw[1, 0, 0]) < 1e-10 * abs(fw[0, 0, 0])
    if model == 4:
        ref = poiseuille_steady(w.ny, w.dx, w.dt, w.tau, w.body_force[0])
        assert rel_inf(v[0, 0, :, 0], ref) < 1e-10
        assert np.abs(v[0] - v[0, :, :, :1]).max() < 1e-15


@pytest.mark.parametrize("storage", [W.F32, W.F64])
def test_couette_cylinder_full_20000_steps(lbm, storage):
    w = W.couette_cylinder()
    say("case couette cylinder 512x128, 20000 steps, storage", storage)
    g = lbm.from_workload(w, storage=storage)
    o = make_oracle(w)
    g.step(w.steps)
    o.step(w.steps)
    e = errors(g, o, 3)
    fw = g.wall_force()
    say("storage %d: %s; cylinder drag %.6e lift %.6e" % (storage, {k: "%.2e" % x for k, x in e.items()},
                                                         fw[2, 0, 0], fw[2, 0, 1]))
    tol = 1e-12 if storage == W.F64 else 1e-5
    assert e["rho"] <= tol and e["v"] <= tol
    # The stress is the non-equilibrium part of the state, a small difference
    # of stored values: FP32 storage alone (the oracle with its state rounded
    # to FP32 after every step) leaves 3e-6 to 1e-5 on it over this run (1e-5
    # at step 9000, 3e-6 at 20 000)
    assert e["sigma"] <= tol and e["S"] <= tol
    assert e["wall"] <= (1e-12 if storage == W.F64 else 1e-4)
    # tangentially moving lid and static walls: no momentum-flux correction
    assert np.abs(fw[:3, 1] - fw[:3, 0]).max() <= 1e-6 * np.abs(fw[:3, 0]).max()
    # Eq. (32) per step.  FP64: relative to the largest of its terms (sums over
    # 64k nodes round at about 1e-12 of them).  FP32: the momentum change is
    # taken from states rounded to FP32, so the residual is bounded by the
    # storage rounding of the momentum, half an FP32 unit of the largest stored
    # value times the 6 (2D: 6 of 9 directions carry x momentum) per node and
    # the fluid nodes (dx = dt = 1); measured 9.9e-6 against that bound of 4e-4
    rec = g.force_balance()
    res = np.abs(rec[9:12]).max()
    if storage == W.F64:
        assert res <= 1e-11 * np.abs(rec[0:9]).max()
    else:
        dmax = np.abs(g.get_state()).max()
        nfluid = int((W.obstacle_mask(w) == 0).sum())
        bound = 0.5 * float(np.spacing(np.float32(dmax))) * 6 * nfluid
        say("balance residual %.2e, FP32 storage-rounding bound %.2e" % (res, bound))
        assert res <= bound


def test_duct_les_full_size_1000_steps_every_format(lbm):
    w = W.duct_les()
    say("case duct 256x128x128 LES, 1000 steps: oracle")
    o = make_oracle(w)
    o.step(w.steps)
    res = {}
    for st in (W.F64, W.F32, W.F16, W.BF16):
        g = lbm.from_workload(w, storage=st)
        g.step(w.steps)
        res[st] = errors(g, o, 4)
        rec = g.force_balance()
        res[st]["balance"] = float(np.abs(rec[9:12]).max() / abs(rec[3]))
        say("storage %d: %s" % (st, {k: "%.2e" % x for k, x in res[st].items()}))
        g.close()
    e = res[W.F64]
    assert max(e["rho"], e["v"], e["sigma"], e["S"], e["wall"]) <= 1e-12
    e = res[W.F32]
    assert max(e["rho"], e["v"], e["sigma"], e["S"]) <= 1e-5 and e["wall"] <= 1e-4
    # 16-bit formats at 2e-3; recorded as not met (format floors; bounds about
    # 1.5 times the largest measured): FP16 stress and strain rate, BF16 all
    errs = {"f16 %s" % k: res[W.F16][k] for k in ("rho", "v", "sigma", "S", "wall")}
    errs.update({"bf16 %s" % k: res[W.BF16][k] for k in ("rho", "v", "sigma", "S", "wall")})
    check_targets(errs, 2e-3, {"f16 sigma": 1.2e-2, "f16 S": 1.2e-2, "bf16 rho": 8e-3, "bf16 v": 1.2e-2,
                               "bf16 sigma": 1e-1, "bf16 S": 1e-1, "bf16 wall": 8e-3}, "duct 1000 steps")


def test_hartmann_channel_full_size_closed_form(lbm):
    """D3Q19 with the MHD equilibrium and the D3Q7 induction lattice, walls
    across y only (192x96x1, periodic x and z), FP32, 20 000 steps: the
    Hartmann profile (Ha = 20) within 2 % (velocity) and 5 % (induced field),
    and the steady balance wall force = body force."""
    w = W.hartmann_duct(nx=192, ny=96, nz=1, steps=20000)
    g = lbm.from_workload(w)
    g.step(w.steps)
    _, v = g.get_macro()
    B = g.get_field_B()
    B0x, B0y, B0z, mu, tau_m = w.mhd
    nu = (w.tau - 0.5) / 3
    eta = 0.25 * (tau_m - 0.5)
    u_ref, b_ref, Ha = hartmann(w.ny, nu, eta, mu, 1.0, w.body_force[0], B0y)
    u = v[0, 0, :, :].mean(axis=1)
    b = B[0, 0, :, :].mean(axis=1)
    eu = np.abs(u - u_ref).max() / u_ref.max()
    eb = np.abs(np.abs(b) - np.abs(b_ref)).max() / np.abs(b_ref).max()
    rec = g.force_balance()
    say("Hartmann channel Ha %.1f: u %.2e, b %.2e, F_wall / sum rho a %.6f" % (Ha, eu, eb, rec[0] / rec[3]))
    assert eu < 0.02 and eb < 0.05
    assert abs(rec[0] / rec[3] - 1) < 1e-4


def test_hartmann_duct_full_size_vs_oracle(lbm):
    """Hartmann duct 192x96x96, FP32, 200 steps from rest against the oracle
    (fields, induced field, wall forces incl. the Maxwell variant), then to
    20 000 steps with the per-step momentum balance (Eq. 32)."""
    w = W.hartmann_duct()
    say("case Hartmann duct 192x96x96: 200 steps vs oracle")
    g = lbm.from_workload(w)
    o = make_oracle(w)
    g.step(200)
    o.step(200)
    e = errors(g, o, 4)
    Bg = g.get_field_B()
    _, _, Bo = o.get_macro(with_B=True)
    b0 = np.array(w.mhd[:3])[:, None, None, None]
    e["b"] = rel_inf(Bg - b0, Bo - b0)
    say("Hartmann duct: %s" % {k: "%.2e" % x for k, x in e.items()})
    assert e["rho"] <= 1e-5 and e["v"] <= 1e-5 and e["sigma"] <= 1e-5 and e["S"] <= 1e-5 and e["wall"] <= 1e-4
    assert e["b"] <= 1e-5
    g.step(w.steps - 200)
    rec = g.force_balance()
    say("after %d steps: residual %.2e, F_wall / sum rho a %.6f, Maxwell total %.2e"
        % (w.steps, np.abs(rec[9:12]).max() / abs(rec[3]), rec[0] / rec[3], np.abs(rec[12:15]).max()))
    assert np.abs(rec[9:12]).max() <= 1e-4 * abs(rec[3])
