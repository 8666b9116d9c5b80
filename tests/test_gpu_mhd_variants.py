"""MHD variants on the GPU against the oracle: two-dimensional MHD (D2Q9 with
the planar induction lattice, Eq. 10 without -c^2 B^2 / 6) and the Lorentz
force through the force term with a hydrodynamic equilibrium (the third
approach of Section 4; balance after Eq. 36), for both lattices.

Tolerances as in the other parity tests: FP64 1e-12, FP32 1e-5 on fields and
1e-4 on wall forces."""
import sys

import numpy as np
import pytest

from closed_forms import hartmann
from helpers import make_oracle, rel_inf
from paper_2512_12213_amd import workloads as W
from test_gpu_parity import TOL_FIELD, TOL_WALL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_12213_amd import lbm as L
    L.lib()
    return L


def mhd_case(lattice, lorentz, storage, model=W.GUO):
    dx, dt, mu = 0.5, 0.25, 1.3
    c = dx / dt
    if lattice == W.D2Q9:
        nx, ny, nz = 24, 16, 1
        walls, groups = ((1, 0, 1),), 3
        obstacle = ("cylinder", 8.3, 7.6, 2.7, 2)
        B0 = (0.05, 0.12, 0.0)
    else:
        nx, ny, nz = 12, 16, 10
        walls, groups = ((1, 0, 1), (2, 2, 3)), 5
        obstacle = ("sphere", 5.2, 7.7, 4.4, 2.1, 4)
        B0 = (0.05, 0.12, -0.04)
    B0 = tuple(b * c * np.sqrt(mu) for b in B0)
    w = W.Workload("mhd_variant", lattice, nx, ny, nz, 0.75, dx=dx, dt=dt, model=model, storage=storage,
                   body_force=(2e-3 * c / dt, -5e-4 * c / dt, 0.0), walls=walls,
                   wall_velocity=((1, 0.02 * c, 0.0, 0.0),), obstacle=obstacle, mhd=B0 + (mu, 0.85),
                   lorentz=lorentz, u0_amp=0.03 * c, u0_seed=17, groups=groups)
    return w


def compare(g, o, w, storage, what):
    tf = TOL_FIELD[storage]
    rg, vg = g.get_macro()
    ro, vo, Bo = o.get_macro(with_B=True)
    Bg = g.get_field_B()
    B0 = np.array(w.mhd[:3])[:, None, None, None]
    fluid = W.obstacle_mask(w)[None] == 0
    e = dict(rho=np.abs(rg - ro).max(), v=rel_inf(vg, vo), B=rel_inf((Bg - B0) * fluid, (Bo - B0) * fluid))
    sg, Sg = g.stress()
    so, So = o.stress()
    e["sigma"] = rel_inf(sg, so)
    e["S"] = rel_inf(Sg, So)
    fg = g.wall_force()[:w.groups]
    fo = o.wall_force(w.groups)
    e["wall"] = max(np.linalg.norm(fg[k, var] - fo[k, var]) / np.linalg.norm(fo[k, var])
                    for k in range(w.groups) for var in range(4) if np.linalg.norm(fo[k, var]) > 0)
    say("%s %s" % (what, {k: "%.2e" % v for k, v in e.items()}))
    assert e["rho"] <= tf and e["v"] <= tf and e["B"] <= tf
    assert e["sigma"] <= tf and e["S"] <= tf
    assert e["wall"] <= TOL_WALL[storage]
    return e


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("lorentz", [False, True])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_mhd_variant_matches_oracle(lbm, lattice, lorentz, storage):
    """A seeded velocity field in a uniform transverse field (induced currents
    from the first step), walls with a moving wall, a solid body, body force,
    non-unity dx and dt; both A-A parities end a call."""
    if lattice == W.D3Q19 and not lorentz:
        pytest.skip("the three-dimensional equilibrium coupling is covered by test_gpu_parity")
    w = mhd_case(lattice, lorentz, storage)
    say("case mhd variant lattice %d lorentz %d storage %d" % (lattice, lorentz, storage))
    g = lbm.from_workload(w)
    o = make_oracle(w)
    for n in (60, 61):
        g.step(n)
        o.step(n)
        compare(g, o, w, storage, "  after %d" % n)
    rg, ro = g.force_balance(), o.force_balance()
    if lorentz:
        # no Maxwell stress in P
        assert np.abs(rg[12:15]).max() == 0.0
    assert np.abs(rg[9:12]).max() <= (1e-12 if storage == W.F64 else 1e-4) * np.abs(rg[0:9]).max()


@pytest.mark.parametrize("model", [0, 2, 4])
def test_lorentz_force_through_every_force_model(lbm, model):
    """The Lorentz force enters the force term: each model's own u^F and C."""
    w = mhd_case(W.D3Q19, True, W.F64, model=model)
    say("case lorentz model %d" % model)
    g = lbm.from_workload(w)
    o = make_oracle(w)
    g.step(31)
    o.step(31)
    compare(g, o, w, W.F64, "  model %d" % model)


@pytest.mark.parametrize("lorentz", [False, True])
def test_halfstep_mhd_variants(lbm, lorentz):
    """Half-step distribution and stress (Eqs. 27-28) under both couplings in
    two dimensions and under the Lorentz coupling in three."""
    for lattice in (W.D2Q9, W.D3Q19):
        if lattice == W.D3Q19 and not lorentz:
            continue
        w = mhd_case(lattice, lorentz, W.F64)
        say("case halfstep lattice %d lorentz %d" % (lattice, lorentz))
        g = lbm.from_workload(w)
        o = make_oracle(w)
        for n in (40, 1):
            g.step(n)
            o.step(n)
            fg, rg, ug, sg = g.halfstep()
            fo, ro, uo, so = o.halfstep()
            e = dict(f=rel_inf(fg, fo), rho=np.abs(rg - ro).max(), u=rel_inf(ug, uo), sigma=rel_inf(sg, so))
            say("  %s" % {k: "%.2e" % v for k, v in e.items()})
            assert e["f"] <= 1e-12 and e["rho"] <= 1e-12 and e["u"] <= 1e-12
            assert e["sigma"] <= 1e-12


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("lorentz", [False, True])
def test_hartmann_channel_2d_on_the_gpu(lbm, lorentz, storage):
    """D2Q9 Hartmann channel (Ha = 20, 96 nodes across, 20 000 steps) on the
    GPU alone: the closed-form profile within 2 % and induced field within
    5 %, the steady wall force balancing the body force; with the Lorentz
    coupling the Maxwell variant equals the raw force and the walls carry the
    external body force (the Lorentz force integrates to ~0 between
    insulating walls, Eq. 36)."""
    w = W.hartmann_channel(nx=4, ny=96, lattice=W.D2Q9, lorentz=lorentz, storage=storage, steps=20000)
    say("case hartmann 2d lorentz %d storage %d" % (lorentz, storage))
    g = lbm.from_workload(w)
    g.step(w.steps)
    rho, v = g.get_macro()
    B = g.get_field_B()
    B0x, B0y, B0z, mu, tau_m = w.mhd
    nu = (w.tau - 0.5) / 3
    eta = 0.25 * (tau_m - 0.5)
    u_ref, b_ref, Ha = hartmann(96, nu, eta, mu, 1.0, w.body_force[0], B0y)
    eu = np.abs(v[0, 0, :, 0] - u_ref).max() / u_ref.max()
    eb = np.abs(np.abs(B[0, 0, :, 0]) - np.abs(b_ref)).max() / np.abs(b_ref).max()
    rec = g.force_balance()
    say("  u %.2e b %.2e F_wall / sum rho a %.6f" % (eu, eb, rec[0] / rec[3]))
    assert eu < 0.02 and eb < 0.05
    assert abs(rec[0] / rec[3] - 1) < 1e-4
    fw = g.wall_force()
    if lorentz:
        assert np.array_equal(fw[:2, 2], fw[:2, 0])
        ext = w.body_force[0] * rho.sum()
        assert abs(rec[3] / ext - 1) < 0.01
    else:
        # the raw force holds -L; the Maxwell variant removes it
        assert np.abs(fw[:2, 2] - fw[:2, 0]).max() > 0


def test_mhd_variant_errors(lbm):
    g = lbm.Lattice(lbm.LBM_D2Q9, 8, 8, 1, 0.8)
    with pytest.raises(lbm.LBMError):
        g.set_mhd([0.01, 0.02, 0.003], 1.0, 0.9)
    with pytest.raises(lbm.LBMError):
        g.set_mhd_coupling(lbm.LBM_MHD_LORENTZ_FORCE)
    g.set_mhd([0.01, 0.02, 0.0], 1.0, 0.9)
    g.set_darcy(0.1)
    with pytest.raises(lbm.LBMError):
        g.set_mhd_coupling(lbm.LBM_MHD_LORENTZ_FORCE)
    g.set_darcy(0.0)
    g.set_mhd_coupling(lbm.LBM_MHD_LORENTZ_FORCE)
    with pytest.raises(lbm.LBMError):
        g.set_darcy(0.1)
    with pytest.raises(lbm.LBMError):
        g.set_mhd_coupling(7)
    g.init_equilibrium()
    assert g.get_induction().shape == (5, 2, 1, 8, 8)
