"""Pins of the oracle's MHD variants: two-dimensional MHD (D2Q9 with the
equilibrium of Eq. 10 less its -c^2 B^2 / 6 term, planar induction lattice)
and the third coupling of Section 4, the Lorentz force through the force term
with a hydrodynamic equilibrium (its balance: the text after Eq. 36).

Fixed independently of the oracle's formulas by:
  * the Hartmann channel's closed form (profile and induced field) for both
    couplings and both dimensions;
  * exact reductions: a planar flow on a one-node D3Q19/D3Q7 slab is the
    two-dimensional computation (the z links fold into the rest direction)
    when the equilibrium is hydrodynamic; a uniform field and uniform flow
    carry no current, so the Lorentz-force run equals the plain hydrodynamic
    run;
  * the balance statements: with the Lorentz force in the force term the
    momentum exchange carries no Maxwell stress, and the per-step balance
    holds with the Lorentz force counted as body force.
"""
import numpy as np
import pytest

import oracle
from closed_forms import hartmann
from helpers import make_oracle, rel_inf
from paper_2512_12213_amd import workloads as W


def test_two_dimensional_mhd_needs_a_planar_field():
    o = oracle.Oracle(oracle.D2Q9, 4, 4, 1, 0.8)
    with pytest.raises(ValueError):
        o.set_mhd([0.01, 0.02, 0.003], 1.0, 0.9)
    o.set_mhd([0.01, 0.02, 0.0], 1.0, 0.9)
    o.init_equilibrium()
    assert o.get_induction().shape == (5, 3, 1, 4, 4)


def test_lorentz_coupling_needs_mhd_and_excludes_darcy():
    o = oracle.Oracle(oracle.D3Q19, 3, 3, 3, 0.8)
    with pytest.raises(ValueError):
        o.set_lorentz_force(True)
    o.set_mhd([0.0, 0.01, 0.0], 1.0, 0.9)
    o.set_darcy(0.1)
    with pytest.raises(ValueError):
        o.set_lorentz_force(True)
    o.set_darcy(0.0)
    o.set_lorentz_force(True)
    with pytest.raises(ValueError):
        o.set_darcy(0.1)


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q19])
def test_uniform_field_and_flow_carry_no_current(lat):
    """u uniform, B uniform: curl B = 0, so the Lorentz force vanishes and the
    flow is the hydrodynamic one (an error in the sign or factor of the
    equilibrium part of the induction moment would leave a spurious current)."""
    nz = 1 if lat == oracle.D2Q9 else 3
    D = 2 if lat == oracle.D2Q9 else 3
    dx, dt = 0.6, 0.2
    c = dx / dt
    u0 = np.zeros((D, nz, 5, 6))
    u0[0] = 0.03 * c
    u0[1] = -0.02 * c
    runs = []
    for mhd in (False, True):
        o = oracle.Oracle(lat, 6, 5, nz, 0.8, dx, dt, oracle.GUO)
        if mhd:
            o.set_mhd([0.02, -0.03, 0.0], 1.3, 0.9)
            o.set_lorentz_force(True)
        o.init_equilibrium(u0)
        o.step(5)
        runs.append(o.get_state())
    assert rel_inf(runs[1], runs[0]) < 1e-13


def _planar_pair(lorentz, steps=120):
    """The same planar channel on D2Q9 + planar induction lattice and on a
    one-node-thick D3Q19 + D3Q7 slab."""
    out = []
    for lat in (oracle.D2Q9, oracle.D3Q19):
        o = oracle.Oracle(lat, 12, 10, 1, 0.75, 0.5, 0.25, oracle.GUO)
        o.set_walls(1, 0, 1)
        o.set_wall_velocity(1, [0.02 * 2.0, 0.0, 0.0])
        o.set_body_force([2e-4 * 8.0, -1e-4 * 8.0, 0.0])
        o.set_mhd([0.03, 0.05, 0.0], 0.7, 0.85)
        if lorentz:
            o.set_lorentz_force(True)
        u = W.random_velocity(2, 1, 10, 12, amp=0.02 * 2.0, seed=5)
        o.init_equilibrium(u if lat == oracle.D2Q9 else np.concatenate([u, np.zeros((1, 1, 10, 12))]))
        o.step(steps)
        out.append(o)
    return out


def test_planar_lorentz_run_equals_the_d3q7_slab():
    """With the equilibrium hydrodynamic (Lorentz force in the force term) a
    planar flow on the slab is the two-dimensional computation exactly: the
    flow lattices coincide (D3Q19 folds onto D2Q9), the two z links of D3Q7
    fold into the planar rest weight 1/4 + 2/8 = 1/2, and they carry no first
    moment, so the current and the force are the same."""
    o2, o3 = _planar_pair(True)
    r2, v2, B2 = o2.get_macro(with_B=True)
    r3, v3, B3 = o3.get_macro(with_B=True)
    assert rel_inf(v2, v3[:2]) < 1e-12
    assert np.abs(r2 - r3).max() < 1e-13
    assert rel_inf(B2, B3) < 1e-12
    # two-dimensional forces are per unit depth; the slab is dx deep
    assert rel_inf(o2.wall_force(2) * 0.5, o3.wall_force(2)) < 1e-11


def test_planar_equilibrium_coupling_differs_from_the_slab_only_through_phi():
    """Under the MHD equilibrium the slab's magnetic term does not fold onto
    the planar one beyond second moments, so the runs differ, but only by
    terms of the magnetic term's size (B^2 / mu)."""
    o2, o3 = _planar_pair(False)
    _, v2, B2 = o2.get_macro(with_B=True)
    _, v3, B3 = o3.get_macro(with_B=True)
    d = rel_inf(v2, v3[:2])
    assert 0 < d < 0.05


@pytest.mark.slow
@pytest.mark.parametrize("lat,lorentz", [(oracle.D2Q9, False), (oracle.D2Q9, True), (oracle.D3Q19, True)])
def test_hartmann_channel_closed_form(lat, lorentz):
    """Both couplings reach the Hartmann profile (Ha = 20) within 2 % and the
    induced field within 5 %, as the three-dimensional equilibrium coupling
    does; the steady wall force balances the body force."""
    w = W.hartmann_channel(nx=1, ny=96, lattice=lat, lorentz=lorentz, steps=20000)
    o = make_oracle(w)
    o.step(w.steps)
    rho, v, B = o.get_macro(with_B=True)
    B0x, B0y, B0z, mu, tau_m = w.mhd
    nu = (w.tau - 0.5) / 3
    eta = 0.25 * (tau_m - 0.5)
    u_ref, b_ref, Ha = hartmann(96, nu, eta, mu, 1.0, w.body_force[0], B0y)
    u = v[0, 0, :, 0]
    eu = np.abs(u - u_ref).max() / u_ref.max()
    b = B[0, 0, :, 0]
    eb = np.abs(np.abs(b) - np.abs(b_ref)).max() / np.abs(b_ref).max()
    print("Hartmann lat %d lorentz %d: u %.2e b %.2e" % (lat, lorentz, eu, eb))
    assert eu < 0.02
    assert eb < 0.05
    rec = o.force_balance()
    assert abs(rec[0] / rec[3] - 1) < 1e-4
    if lorentz:
        # the Lorentz force integrates to ~0 (insulating walls, Eq. 36): the
        # walls carry the external body force alone
        ext = w.body_force[0] * rho.sum()
        assert abs(rec[3] / ext - 1) < 0.01


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q19])
def test_lorentz_coupling_has_no_maxwell_correction_and_balances(lat):
    """Text after Eq. 36: with the Lorentz force in the force term, P holds
    no -L, so the Maxwell variant equals the raw force; the per-step balance
    holds with the Lorentz force counted in the body force."""
    nz = 1 if lat == oracle.D2Q9 else 6
    w = W.Workload("t", lat, 8, 12, nz, 0.8, body_force=(1e-5, 0.0, 0.0), walls=((1, 0, 1),) if nz == 1 else
                   ((1, 0, 1), (2, 2, 3)), mhd=(0.01, 0.04, 0.0, 1.0, 0.9), lorentz=True, groups=2 if nz == 1 else 4)
    o = make_oracle(w)
    o.set_state(W.random_state(w.Q, w.nx, w.ny, w.nz, amp=1e-4, seed=9), keep_records=False)
    o.step(40)
    fw = o.wall_force(w.groups)
    assert np.array_equal(fw[:, 2], fw[:, 0])
    rec = o.force_balance()
    assert np.abs(rec[9:12]).max() < 1e-12 * max(np.abs(rec[0:9]).max(), 1e-30)
    assert np.abs(rec[12:15]).max() == 0.0
