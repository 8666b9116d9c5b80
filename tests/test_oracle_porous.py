"""Pins of the oracle's Stokes equilibrium and porous (Brinkman) resistance.

The text after Eq. (11): the equilibrium rho w [1 + 3 e.u^eq / c^2] changes
M^eq to c^2 rho delta / 3 and recovers the Stokes equation; a
velocity-dependent body force then gives the Brinkman equation.  The
resistance is -sigma v with the model-independent velocity v = u + dt a / 2
(Section 2), so the force a node applies is a = (a_ext - sigma u) /
(1 + sigma dt / 2).
"""
import numpy as np
import pytest

import oracle
from closed_forms import brinkman_channel, channel_recurrence, lattice, node_positions
from helpers import rel_inf
from paper_2512_12213_amd import workloads as W

MODELS = [oracle.HE, oracle.LUO, oracle.SHANCHEN, oracle.EDM, oracle.GUO]


@pytest.mark.parametrize("lat,name", [(oracle.D2Q9, "D2Q9"), (oracle.D3Q19, "D3Q19")])
def test_stokes_equilibrium_moments(lat, name):
    dx, dt = 0.6, 0.25
    c = dx / dt
    nx, ny, nz = 3, 4, (1 if lat == oracle.D2Q9 else 2)
    D = 2 if lat == oracle.D2Q9 else 3
    o = oracle.Oracle(lat, nx, ny, nz, 0.9, dx, dt, oracle.GUO)
    rho0 = 1.2
    o.set_rho0(rho0)
    o.set_equilibrium(True)
    u0 = W.direction((D, nz, ny, nx), 8) * 0.05 * c
    o.init_equilibrium(u0)
    e, w = lattice(name)
    Q = len(w)
    f = o.get_state().reshape(Q, -1) + w[:, None] * rho0
    E = c * e.astype(float)
    u = u0.reshape(D, -1)
    np.testing.assert_allclose(f.sum(0), rho0, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("qi,qn->in", E, f)[:D], rho0 * u, atol=1e-14 * c)
    m2 = np.einsum("qi,qj,qn->ijn", E, E, f)
    for i in range(D):
        for j in range(D):
            ref = rho0 * c * c / 3 if i == j else 0.0
            np.testing.assert_allclose(m2[i, j], ref, atol=1e-13 * c * c)


@pytest.mark.parametrize("model", MODELS)
def test_darcy_channel_matches_recurrence(model):
    ny, tau, a, sigma = 16, 0.8, 1e-6, 0.02
    o = oracle.Oracle(oracle.D2Q9, 2, ny, 1, tau, 1.0, 1.0, model)
    o.set_walls(1, 0, 1)
    o.set_body_force([a, 0, 0])
    o.set_darcy(sigma)
    o.init_equilibrium()
    o.step(700)
    _, v = o.get_macro()
    assert rel_inf(v[0, 0, :, 0], channel_recurrence(ny, tau, a, 700, darcy=sigma)) < 1e-12


def test_brinkman_steady_profile_second_order():
    """Steady Brinkman channel against the continuous closed form: the error
    falls by about 4 when the resolution doubles at fixed L / H."""
    errs = []
    for n in (16, 32):
        tau = 0.8
        nu = (tau - 0.5) / 3
        L = n / 4.0
        sigma = nu / L ** 2
        a = 1e-6
        o = oracle.Oracle(oracle.D2Q9, 1, n, 1, tau, 1.0, 1.0, oracle.GUO)
        o.set_walls(1, 0, 1)
        o.set_body_force([a, 0, 0])
        o.set_darcy(sigma)
        o.init_equilibrium()
        o.step(int(40 / sigma))
        _, v = o.get_macro()
        ref = brinkman_channel(n, nu, sigma, a)
        errs.append(rel_inf(v[0, 0, :, 0], ref))
        # steady, static walls: the walls carry the body force net of the resistance
        rec = o.force_balance()
        assert abs(rec[0] - rec[3]) < 1e-9 * abs(rec[3])
    assert errs[1] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_darcy_per_step_momentum_balance():
    """Eq. (32) per step with the resistance inside the body-force term."""
    w = W.duct_sphere(nx=12, ny=10, nz=10, r=2.0, uw=0.02)
    o = oracle.Oracle(w.lattice, w.nx, w.ny, w.nz, w.tau, 1.0, 1.0, oracle.GUO)
    o.set_walls(1, 0, 1)
    o.set_walls(2, 2, 3)
    o.set_wall_velocity(1, [0.02, 0, 0])
    o.set_solid(W.obstacle_mask(w), 4)
    o.set_body_force([1e-4, 2e-5, 0])
    o.set_darcy(0.05)
    o.set_equilibrium(True)
    o.init_equilibrium(W.direction((3, w.nz, w.ny, w.nx), 3) * 1e-3)
    o.step(30)
    rec = o.force_balance()
    assert np.abs(rec[9:12]).max() < 1e-12 * np.abs(rec[0:9]).max()
    # the resistance opposes the flow: sum rho a is below the external force
    assert rec[3] < 1e-4 * (w.nx * w.ny * w.nz - W.obstacle_mask(w).sum()) * 1.0
