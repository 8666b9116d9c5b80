"""Pins of the oracle's reverse-mode gradient (the FP64 CPU adjoint).

The paper does not differentiate its method; the objective here is its
Eq. (25) wall force on one wall group during the last step, differentiated
with respect to the per-node body force a(x) and the wall velocities.  The
adjoint is checked against quantities it does not compute itself:
  * directional derivatives of the complex-step forward run (exact to
    rounding, a different code path: forward-mode through every step);
  * central finite differences of the double build;
  * the closed-form linear channel, whose bottom-wall force is a linear
    function of the per-row force and the lid velocity (class-sum recurrence).
"""
import numpy as np
import pytest

import oracle
from closed_forms import channel_bottom_force_recurrence
from helpers import make_oracle
from paper_2512_12213_amd import workloads as W

H = 1e-30  # complex step


def duct_case(model=oracle.GUO, les=0.0):
    w = W.duct_sphere(nx=16, ny=12, nz=12, r=3.0, uw=0.01, a=1e-4)
    w.model = model
    w.les_cs = les
    a0 = W.force_field(w.nx, w.ny, w.nz, base=w.body_force, amp=0.3, seed=1)
    return w, a0, 8, 4, 0


def couette_case(model):
    w = W.couette_cylinder(nx=48, ny=24, r=4.0, cx=20.0, cy=12.0, uw=0.05, tau=0.6, a=2e-5)
    w.model = model
    a0 = W.force_field(w.nx, w.ny, w.nz, base=w.body_force, amp=0.5, seed=2)
    a0[2] = 0.0
    return w, a0, 20, 2, 0


def adjoint_of(w, a0, T, group, axis):
    o = make_oracle(w, complex_step=True)
    o.set_body_force_field(a0)
    return o.adjoint(T, group, axis)


def jvp(w, a0, T, group, axis, da=None, uw_group=None, duw=None):
    """Complex-step directional derivative of J along (da, duw)."""
    o = make_oracle(w, complex_step=True, init=False)
    o.set_body_force_field(a0, None if da is None else H * da)
    if uw_group is not None:
        base = [0.0, 0.0, 0.0]
        for g, ux, uy, uz in w.wall_velocity:
            if g == uw_group:
                base = [ux, uy, uz]
        o.set_wall_velocity(uw_group, base, H * np.asarray(duw, dtype=float))
    o.init_equilibrium(W.initial_velocity(w))
    o.step(T)
    re, im = o.wall_force(imag=True)
    return re[group, 0, axis], im[group, 0, axis] / H


CASES = [("duct_guo", lambda: duct_case()),
         ("duct_les", lambda: duct_case(les=0.1)),
         ("duct_he", lambda: duct_case(oracle.HE))] + \
        [("couette_m%d" % m, (lambda m=m: couette_case(m))) for m in range(5)]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_adjoint_field_gradient_matches_complex_step(name, make):
    w, a0, T, group, axis = make()
    J, ga, _ = adjoint_of(w, a0, T, group, axis)
    for seed in (5, 6):
        da = W.direction(a0.shape, seed)
        if w.D == 2:
            da[2] = 0.0
        J1, dJ = jvp(w, a0, T, group, axis, da=da)
        assert J == J1
        assert abs(np.sum(ga * da) - dJ) <= 1e-10 * abs(dJ), (name, seed)


def test_adjoint_single_entries_match_complex_step():
    w, a0, T, group, axis = duct_case()
    _, ga, _ = adjoint_of(w, a0, T, group, axis)
    # nodes next to the sphere, next to a wall, and in the bulk
    for (k, z, y, x) in [(0, 5, 5, 4), (1, 6, 3, 8), (2, 0, 6, 7), (0, 11, 11, 15), (1, 2, 9, 1)]:
        da = np.zeros_like(a0)
        da[k, z, y, x] = 1.0
        _, dJ = jvp(w, a0, T, group, axis, da=da)
        assert abs(ga[k, z, y, x] - dJ) <= 1e-10 * max(abs(dJ), 1e-12 * np.abs(ga).max())


@pytest.mark.parametrize("name,make", CASES[:1] + CASES[3:4], ids=["duct_guo", "couette_m0"])
def test_adjoint_wall_velocity_gradient_matches_complex_step(name, make):
    w, a0, T, group, axis = make()
    _, _, gu = adjoint_of(w, a0, T, group, axis)
    moving = w.wall_velocity[0][0]
    for k in range(w.D):
        duw = np.zeros(3)
        duw[k] = 1.0
        _, dJ = jvp(w, a0, T, group, axis, uw_group=moving, duw=duw)
        assert abs(gu[moving, k] - dJ) <= 1e-10 * max(abs(dJ), 1e-8), (k, gu[moving, k], dJ)
    # a static group also gets its (nonzero) sensitivity
    _, dJ0 = jvp(w, a0, T, group, axis, uw_group=0, duw=[1.0, 0.0, 0.0])
    assert abs(gu[0, 0] - dJ0) <= 1e-10 * abs(dJ0)


def test_adjoint_matches_central_differences_of_double_build():
    w, a0, T, group, axis = duct_case()
    J, ga, gu = adjoint_of(w, a0, T, group, axis)
    da = W.direction(a0.shape, 9)
    h = 1e-3 * np.abs(a0).max()

    def Jd(field, uw=None):
        o = make_oracle(w, init=False)
        o.set_body_force_field(field)
        if uw is not None:
            o.set_wall_velocity(1, uw)
        o.init_equilibrium(W.initial_velocity(w))
        o.step(T)
        return o.wall_force()[group, 0, axis]

    assert abs(Jd(a0) - J) <= 1e-14 * abs(J)
    fd = (Jd(a0 + h * da) - Jd(a0 - h * da)) / (2 * h)
    assert abs(np.sum(ga * da) - fd) <= 1e-6 * abs(fd)
    hu = 1e-3
    fdu = (Jd(a0, [0.01 + hu, 0, 0]) - Jd(a0, [0.01 - hu, 0, 0])) / (2 * hu)
    assert abs(gu[1, 0] - fdu) <= 1e-6 * abs(fdu)


def test_adjoint_sum_equals_uniform_force_derivative():
    w, _, T, group, axis = duct_case()
    a_uni = np.array(w.body_force, dtype=float)
    o = make_oracle(w, complex_step=True)
    J, ga, _ = o.adjoint(T, group, axis)
    for k in range(3):
        im = np.zeros(3)
        im[k] = H
        o2 = make_oracle(w, complex_step=True, init=False)
        o2.set_body_force(a_uni, im)
        o2.init_equilibrium(W.initial_velocity(w))
        o2.step(T)
        re, imv = o2.wall_force(imag=True)
        dJ = imv[group, 0, axis] / H
        assert re[group, 0, axis] == J
        # components with a vanishing total (symmetry) are held to the scale of the terms summed
        assert abs(ga[k].sum() - dJ) <= 1e-10 * max(abs(dJ), np.abs(ga[k]).sum())


def test_adjoint_linear_channel_closed_form():
    """Force-driven D2Q9 channel with a moving lid: the bottom-wall force is
    linear in the per-row body force a_x(y) and in the lid velocity, so its
    gradient is the recurrence's response to unit impulses."""
    nx, ny, tau, T, uw = 4, 16, 0.8, 60, 0.01
    a_rows = np.random.default_rng(3).uniform(0.5, 1.5, ny) * 1e-5
    o = oracle.Oracle(oracle.D2Q9, nx, ny, 1, tau, 1.0, 1.0, oracle.GUO, complex_step=True)
    o.set_walls(1, 0, 1)
    o.set_wall_velocity(1, [uw, 0.0, 0.0])
    field = np.zeros((3, 1, ny, nx))
    field[0] = a_rows[None, :, None]
    o.set_body_force_field(field)
    o.init_equilibrium()
    J, ga, gu = o.adjoint(T, 0, 0)
    J_ref = nx * channel_bottom_force_recurrence(ny, tau, a_rows, T, uw)
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
    imp = np.array([channel_bottom_force_recurrence(ny, tau, np.eye(ny)[y], T) for y in range(ny)])
    assert np.abs(ga[0, 0] - imp[:, None]).max() <= 1e-12 * np.abs(imp).max()
    dJ_duw = nx * channel_bottom_force_recurrence(ny, tau, 0.0, T, 1.0)
    assert abs(gu[1, 0] - dJ_duw) <= 1e-12 * abs(dJ_duw)


def test_adjoint_needs_complex_build_and_rejects_mhd():
    o = oracle.Oracle(oracle.D2Q9, 4, 4, 1, 0.8)
    with pytest.raises(ValueError):
        o.adjoint(2, 0, 0)
    m = oracle.Oracle(oracle.D3Q19, 4, 4, 4, 0.8, complex_step=True)
    m.set_walls(1, 0, 1)
    m.set_mhd([0.0, 0.01, 0.0], 1.0, 0.9)
    m.init_equilibrium()
    with pytest.raises(ValueError):
        m.adjoint(2, 0, 0)
