"""Pins of the oracle's half-step distribution (Section 5, Eqs. 27-30).

fbar = (f_rel(x, t) + f(x, t + dt)) / 2 and the stress of Eq. (28),
sigma_bar = -sum e e fbar + Mbar^eq.  Checked against what the paper and the
update rule fix, without retyping the oracle's formulas:
  * density and momentum: relaxation conserves mass and adds rho a dt of
    momentum, so rho_bar = (rho(t) + rho(t + dt)) / 2 and
    rho_bar u_bar = (rho u(t) + rho(t) a dt + rho u(t + dt)) / 2 exactly,
    every node, every force model;
  * steady flows (f(t + dt) = f(t)): sigma_bar = sigma - Theta / 2 +
    rho (v v - u^eq u^eq) exactly, with sigma from Eq. (9) and Theta the
    force term's second moment (the first row of Eq. 30, plus the difference
    of the two equilibria's velocities), so sigma_bar_xy = -rho a y in the
    steady channel and rho nu u_w / H in steady Couette flow.
"""
import numpy as np
import pytest

import oracle
from closed_forms import node_positions
from helpers import make_oracle, rel_inf
from paper_2512_12213_amd import workloads as W

ALL_MODELS = [oracle.HE, oracle.LUO, oracle.SHANCHEN, oracle.EDM, oracle.GUO, oracle.SHANCHEN_ORIG, oracle.EDM_ORIG]


@pytest.mark.parametrize("lat", [oracle.D2Q9, oracle.D3Q19])
@pytest.mark.parametrize("model", ALL_MODELS)
def test_halfstep_density_and_momentum(lat, model):
    dx, dt = 0.7, 0.3
    c = dx / dt
    if lat == oracle.D2Q9:
        w = W.couette_cylinder(nx=24, ny=14, r=3.0, cx=9.0, cy=7.0, uw=0.04 * c, tau=0.7)
    else:
        w = W.duct_sphere(nx=12, ny=10, nz=9, r=2.0, uw=0.04 * c)
    w.model, w.dx, w.dt = model, dx, dt
    D, Q = w.D, w.Q
    o = make_oracle(w, init=False)
    a = W.force_field(w.nx, w.ny, w.nz, base=(2e-3 * c / dt, -1e-3 * c / dt, 5e-4 * c / dt), amp=0.5, seed=3)
    if D == 2:
        a[2] = 0.0
    o.set_body_force_field(a)
    o.set_state(W.random_state(Q, w.nx, w.ny, w.nz, amp=1e-3, seed=4))
    o.step(1)
    rho0, v0 = o.get_macro()
    o.step(1)
    rho1, v1 = o.get_macro()
    fb, rb, ub, sb = o.halfstep()
    fluid = W.obstacle_mask(w)
    fluid = np.ones((w.nz, w.ny, w.nx), bool) if fluid is None else (fluid == 0)
    u0 = v0 - 0.5 * dt * a[:D]
    u1 = v1 - 0.5 * dt * a[:D]
    assert np.abs(rb - 0.5 * (rho0 + rho1))[fluid].max() < 1e-14
    mom = 0.5 * (rho0 * u0 + rho0 * a[:D] * dt + rho1 * u1)
    assert np.abs(rb * ub - mom)[:, fluid].max() < 1e-13 * c
    assert np.abs(fb[:, ~fluid]).max() == 0.0


def _theta(model, tau, rho, v, u, a, dt):
    """Second moment Theta_ij = sum e_i e_j F of each force model for a
    two-dimensional (u, a) pair, from the lattice moments
    sum w e_i e_j = c^2/3 delta, sum w e_i e_j e_k e_l = c^4/9 (dd + dd + dd)."""
    def uf():
        if model in (oracle.LUO,):
            return u
        if model == oracle.SHANCHEN:
            return u + 0.5 * tau * dt * a
        return v
    if model in (oracle.HE, oracle.SHANCHEN_ORIG):
        return np.zeros((2, 2))
    if model == oracle.EDM_ORIG:
        us = u + dt * a
        return rho * (np.outer(us, us) - np.outer(u, u))
    C = 1.0 - 1.0 / (2.0 * tau) if model == oracle.GUO else 1.0
    F = uf()
    # C rho dt [ -(uF.a) I ... ] reduces to C rho dt (uF_i a_j + uF_j a_i)
    return C * rho * dt * (np.outer(F, a) + np.outer(a, F))


@pytest.mark.parametrize("model", ALL_MODELS)
def test_halfstep_stress_in_the_steady_channel(model):
    dx, dt, H, tau = 0.5, 0.1, 12, 0.9
    c = dx / dt
    a = 1e-4 * c / dt
    o = oracle.Oracle(oracle.D2Q9, 1, H, 1, tau, dx, dt, model)
    o.set_walls(1, 0, 1)
    o.set_body_force([a, 0, 0])
    o.init_equilibrium()
    o.step(40000)
    rho, v = o.get_macro()
    sig, _ = o.stress()
    _, rb, ub, sb = o.halfstep()
    y = node_positions(H, dx)
    # xy: Theta_xy = 0 and v_x v_y = 0, so the half-step stress is the exact shear
    assert rel_inf(sb[1, 0, :, 0], -1.0 * a * y) < 1e-9
    assert rel_inf(sb[1, 0, :, 0], sig[1, 0, :, 0]) < 1e-9
    # xx: sigma_bar = sigma - Theta/2 + rho (v v - u^eq u^eq)
    for k in range(H):
        r = rho[0, k, 0]
        vv = np.array([v[0, 0, k, 0], 0.0])
        av = np.array([a, 0.0])
        uu = vv - 0.5 * dt * av
        ueq = {oracle.GUO: vv, oracle.SHANCHEN_ORIG: uu + tau * dt * av}.get(model, uu)
        th = _theta(model, tau, r, vv, uu, av, dt)
        ref = sig[0, 0, k, 0] - 0.5 * th[0, 0] + r * (vv[0] ** 2 - ueq[0] ** 2)
        assert abs(sb[0, 0, k, 0] - ref) < 1e-12 * c * c
    # steady: rho_bar = rho, u_bar = v
    assert np.abs(rb - rho).max() < 1e-14
    assert np.abs(ub[0] - v[0]).max() < 1e-14 * c


def test_halfstep_stress_in_steady_couette():
    """Lid-driven channel at steady state: the half-step shear stress is the
    exact rho nu u_w / H (halfway bounce-back makes the linear profile exact)."""
    uw, tau, H = 0.05, 0.8, 16
    o = oracle.Oracle(oracle.D2Q9, 1, H, 1, tau, 1.0, 1.0, oracle.GUO)
    o.set_walls(1, 0, 1)
    o.set_wall_velocity(1, [uw, 0, 0])
    o.init_equilibrium()
    o.step(30000)
    _, _, _, sb = o.halfstep()
    nu = (tau - 0.5) / 3.0
    assert rel_inf(sb[1, 0, :, 0], np.full(H, nu * uw / H)) < 1e-10


def test_halfstep_stress_in_the_steady_hartmann_channel():
    """Under the MHD equilibrium Mbar^eq carries L(Bbar); at steady state the
    half-step stress equals the Eq. (9) stress (Guo: u^eq = v, Theta_xy = 0)."""
    w = W.hartmann_duct(nx=1, ny=32, nz=1, steps=8000)
    o = make_oracle(w)
    o.step(w.steps)
    sig, _ = o.stress()
    _, _, _, sb = o.halfstep()
    assert rel_inf(sb[3, 0, :, 0], sig[3, 0, :, 0]) < 1e-8


def test_halfstep_before_any_step_is_an_error():
    o = oracle.Oracle(oracle.D2Q9, 4, 4, 1, 0.8)
    o.init_equilibrium()
    with pytest.raises(ValueError):
        o.halfstep()
