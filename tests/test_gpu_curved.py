"""Walls that are not halfway between nodes on the GPU: linearly interpolated
bounce-back (Bouzidi, Firdaouss and Lallemand 2001), inside the steps before
the last of a call (row-uniform lattices, widths that are multiples of 64)
or in a pass after each step (other widths), against the oracle element by
element, and the Section 5 statement that
the momentum exchange of Eq. (25) then gives the stress at the half-grid point
x_f + e dt / 2, checked on the GPU alone in steady flows.

Tolerances are those of the halfway parity tests: FP64 1e-12, FP32 1e-5 on
fields and 1e-4 on wall forces."""
import sys

import numpy as np
import pytest

from helpers import make_oracle, quantize_state, quantized_steps, rel_inf
from paper_2512_12213_amd import workloads as W
from test_gpu_parity import compare_all

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_12213_amd import lbm as L
    L.lib()
    return L


def offset_channel(nx, n, qb, qt, tau=0.8, a=1e-6, uw=0.0, storage=W.F64):
    w = W.Workload("offset_channel_d2q9_%dx%d" % (nx, n), W.D2Q9, nx, n, 1, tau, storage=storage,
                   body_force=(a, 0.0, 0.0), walls=((1, 0, 1),),
                   wall_velocity=((1, uw, 0.0, 0.0),) if uw else (), groups=2)
    q = np.full((9, 1, n, nx), 0.5)
    q[:, 0, 0, :] = qb
    q[:, 0, n - 1, :] = qt
    return w, q


def pair(lbm, w, q, storage=None):
    g = lbm.from_workload(w, storage=storage, init=False)
    o = make_oracle(w, init=False)
    if q is not None:
        g.set_link_fractions(q)
        o.set_link_fraction(q)
    u0 = W.initial_velocity(w)
    g.init_equilibrium(u0)
    o.init_equilibrium(u0)
    return g, o


@pytest.mark.parametrize("nx", [8, 64])
@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("steps", [300, 301])
def test_offset_channel_matches_oracle(lbm, storage, steps, nx):
    """Force-driven channel with walls at q = 0.25 below and 0.8 above the
    end nodes; both A-A parities end the call."""
    w, q = offset_channel(nx, 16, 0.25, 0.8, a=2e-5)
    say("case offset channel", storage, steps, nx)
    g, o = pair(lbm, w, q, storage)
    g.step(steps)
    o.step(steps)
    compare_all(g, o, storage, 2, "offset channel")


@pytest.mark.parametrize("nx", [8, 64])
@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_offset_couette_matches_oracle(lbm, storage, nx):
    """Moving top wall with fractions 0.9 (bottom) and 0.3 (top): the
    moving-wall term enters both interpolation branches."""
    w, q = offset_channel(nx, 12, 0.9, 0.3, a=0.0, uw=0.03)
    say("case offset couette", storage, nx)
    g, o = pair(lbm, w, q, storage)
    for _ in range(3):
        g.step(67)
        o.step(67)
    compare_all(g, o, storage, 2, "offset couette")


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_curved_cylinder_matches_oracle(lbm, storage):
    """Couette channel with a cylinder whose links carry the exact circle's
    fractions (both interpolation branches, the halfway fallback where the
    upstream node is solid), moving top wall, body force."""
    w = W.couette_cylinder(nx=64, ny=32, r=5.3, cx=20.4, cy=15.7, uw=0.03, tau=0.7, a=2e-5, storage=storage)
    w.curved = True
    q = W.link_fractions(w)
    assert (q < 0.5).any() and (q > 0.5).any()
    say("case curved cylinder", storage)
    g, o = pair(lbm, w, None, storage)
    for n in (150, 151):
        g.step(n)
        o.step(n)
        compare_all(g, o, storage, 3, "curved cylinder")
    bg = g.force_balance()
    assert np.abs(bg[9:12]).max() <= (1e-12 if storage == W.F64 else 1e-4) * np.abs(bg[0:9]).max()


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_curved_sphere_matches_oracle(lbm, storage):
    """D3Q19 duct with an off-lattice sphere (fractions of the exact sphere)
    and a moving top wall; 64 wide, so that the steps before the last of a
    call interpolate inside the step."""
    w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7, storage=storage)
    w.curved = True
    say("case curved sphere", storage)
    g, o = pair(lbm, w, None, storage)
    for n in (60, 61):
        g.step(n)
        o.step(n)
        compare_all(g, o, storage, 5, "curved sphere")


def mhd_sphere(storage, lorentz, curved):
    w = W.hartmann_duct(nx=32, ny=16, nz=14, storage=storage, steps=0)
    w.obstacle = ("sphere", 15.3, 7.6, 6.4, 3.7, 4)
    w.curved = curved
    w.groups = 5
    w.lorentz = lorentz
    return w


@pytest.mark.parametrize("lorentz", [False, True])
@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_mhd_with_interpolated_walls_matches_oracle(lbm, storage, lorentz):
    """Hartmann duct (32x16x14, B0 = 0.25) with an off-lattice sphere whose
    links carry the exact fractions, under the MHD equilibrium or the
    Lorentz-force coupling: the pass after every step interpolates the flow
    distributions, the induction distributions keep halfway
    anti-bounce-back, and every wall link keeps its Maxwell correction.
    Calls of 200 and 201 steps against the oracle: fields, stresses, wall
    forces, the induced field and the half-step output (FP64 1e-12, FP32
    1e-5 on fields and 1e-4 on wall forces)."""
    w = mhd_sphere(storage, lorentz, True)
    q = W.link_fractions(w)
    assert (q < 0.5).any() and (q > 0.5).any()
    say("case mhd curved", storage, lorentz)
    g, o = pair(lbm, w, None, storage)
    b0 = np.array(w.mhd[:3])[:, None, None, None]
    tol = 1e-12 if storage == W.F64 else 1e-5
    for n in (200, 201):
        g.step(n)
        o.step(n)
        compare_all(g, o, storage, 5, "mhd curved")
        Bg = g.get_field_B()
        _, _, Bo = o.get_macro(with_B=True)
        e_b = rel_inf(Bg - b0, Bo - b0)
        say("  induced field B %.2e" % e_b)
        assert e_b <= tol
    fg, rg, ug, sg = g.halfstep()
    fo, ro, uo, so = o.halfstep()
    e = dict(f=rel_inf(fg, fo), u=rel_inf(ug, uo), sigma=rel_inf(sg, so))
    say("  half-step: %s" % {k: "%.2e" % v for k, v in e.items()})
    assert max(e.values()) <= tol


@pytest.mark.parametrize("storage", [W.F16, W.BF16])
def test_curved_sphere_16bit_matches_quantized_oracle(lbm, storage):
    """The sphere duct in 16-bit storage (interpolated links in the steps,
    their q < 1/2 parts stored in the format between steps) against the
    oracle whose state is rounded to the format after every step: the
    tolerances of the 16-bit parity tests (2e-3; BF16's recorded bounds)."""
    w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7, storage=storage)
    w.curved = True
    say("case curved sphere 16-bit", storage)
    g, o = pair(lbm, w, None, storage)
    d0 = o.get_state()
    g.set_state(d0)
    o.set_state(quantize_state(d0, storage))
    for n in (20, 21):
        g.step(n)
        quantized_steps(o, storage, n)
        compare_all(g, o, storage, 5, "curved sphere %d" % storage)


@pytest.mark.parametrize("storage", [W.F64, W.F32])
def test_interpolation_in_the_step_equals_the_pass(lbm, storage):
    """Steps before the last of a call interpolate inside the step (q < 1/2
    links completed when the next step reads the node); a call's last step
    leaves it to the pass after it.  A 40-step call against 40 one-step
    calls (every step then ends a call): the same states and wall forces up
    to the rounding order (FP64 1e-13, FP32 1e-5 relative).  64 wide (the
    row-uniform form, which has the in-step variant)."""
    w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7, storage=storage)
    w.curved = True
    say("case in-step interpolation", storage)
    a = lbm.from_workload(w)
    b = lbm.from_workload(w)
    a.step(40)
    for _ in range(40):
        b.step(1)
    tol = 1e-13 if storage == W.F64 else 1e-5
    es = rel_inf(a.get_state(), b.get_state())
    ef = rel_inf(a.wall_force(), b.wall_force())
    say("  state %.2e wall force %.2e" % (es, ef))
    assert es <= tol and ef <= 10 * tol
    assert es > 0  # the two forms round differently: the in-step one ran


@pytest.mark.parametrize("qv", [0.25, 0.7, 1.0])
def test_gpu_momentum_exchange_is_the_half_grid_stress(lbm, qv):
    """Steady offset channel on the GPU alone: the bottom wall carries half
    the body force on the n fluid nodes of a column (the enveloped domain of
    Section 6), rho a n / 2, equal to the Eq. (9) stress extrapolated to
    y_i = -dx/2 and not to the wall at y_w = -q dx (Section 5)."""
    n, a = 16, 1e-6
    w, q = offset_channel(4, n, qv, qv, a=a)
    say("case half-grid stress", qv)
    g = lbm.from_workload(w, init=False)
    g.set_link_fractions(q)
    g.init_equilibrium()
    g.step(60000)
    fw = g.wall_force()
    sig, _ = g.stress()
    s = sig[1, 0, :, 0]
    slope = s[1] - s[0]
    s_i = s[0] - 0.5 * slope
    s_w = s[0] - qv * slope
    P = fw[0, 0, 0] / w.nx  # per node width
    assert abs(P - a * n / 2) < 1e-12 * a * n
    assert abs(s_i - P) < 1e-9 * P
    assert abs((s_w - P) - a * (qv - 0.5)) < 1e-9 * P


@pytest.mark.parametrize("nx", [4, 64])
def test_gpu_offset_couette_is_exact(lbm, nx):
    """Linear interpolation makes the linear profile between the true walls
    exact: u(y) = U (y + q_b) / H with H = n - 1 + q_b + q_t, and both walls
    carry rho nu U / H.  4 wide: the pass after each step; 64 wide: inside
    the steps."""
    n, tau, U = 16, 0.8, 0.02
    for qb, qt in ((0.25, 0.8), (0.9, 0.3)):
        w, q = offset_channel(nx, n, qb, qt, tau=tau, a=0.0, uw=U)
        say("case exact couette", nx, qb, qt)
        g = lbm.from_workload(w, init=False)
        g.set_link_fractions(q)
        g.init_equilibrium()
        g.step(40000)
        _, v = g.get_macro()
        H = n - 1 + qb + qt
        y = np.arange(n, dtype=float)
        assert np.abs(v[0, 0, :, 0] - U * (y + qb) / H).max() < 1e-12 * U
        fw = g.wall_force() / w.nx
        nu = (tau - 0.5) / 3
        assert abs(fw[0, 0, 0] - nu * U / H) < 1e-10 * nu * U / H
        assert abs(fw[1, 0, 0] + nu * U / H) < 1e-10 * nu * U / H
        # the half-step stress (Eq. 28) is the exact shear stress at every
        # node, the ones next to the interpolated walls included
        _, rb, _, sb = g.halfstep()
        assert np.abs(sb[1, 0, :, 0] - rb[0, :, 0] * nu * U / H).max() < 1e-10 * nu * U / H


@pytest.mark.parametrize("storage", [W.F64, W.F32])
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_halfstep_with_interpolated_walls_matches_oracle(lbm, lattice, storage):
    """Half-step distribution and its moments (Eqs. 27-28) after calls of 5
    and 4 steps (both A-A parities end a call) in a channel with a cylinder
    (D2Q9) or a duct with a sphere (D3Q19) whose links carry the exact
    fractions (both interpolation branches), a moving wall and a body force:
    FP64 1e-12, FP32 1e-5 on f_bar, rho_bar, u_bar and 1e-5 on sigma_bar."""
    if lattice == W.D2Q9:
        w = W.couette_cylinder(nx=64, ny=24, r=4.3, cx=16.4, cy=11.7, uw=0.03, tau=0.7, a=2e-5, storage=storage)
    else:
        w = W.duct_sphere(nx=64, ny=16, nz=14, r=3.7, storage=storage)
    w.curved = True
    q = W.link_fractions(w)
    assert (q < 0.5).any() and (q > 0.5).any()
    say("case halfstep curved", lattice, storage)
    g, o = pair(lbm, w, None, storage)
    tol = 1e-12 if storage == W.F64 else 1e-5
    for n in (5, 4):
        g.step(n)
        o.step(n)
        fg, rg, ug, sg = g.halfstep()
        fo, ro, uo, so = o.halfstep()
        e = dict(f=rel_inf(fg, fo), rho=np.abs(rg - ro).max(), u=rel_inf(ug, uo), sigma=rel_inf(sg, so))
        say("  after %d steps: %s" % (n, {k: "%.2e" % v for k, v in e.items()}))
        assert max(e.values()) <= tol


def test_halfway_fractions_change_nothing(lbm):
    w = W.couette_cylinder(nx=40, ny=20, r=3.0, cx=12.0, cy=10.0, storage=W.F64)
    g1 = lbm.from_workload(w)
    g2 = lbm.from_workload(w, init=False)
    g2.set_link_fractions(np.full((9, 1, w.ny, w.nx), 0.5))
    g2.init_equilibrium(W.initial_velocity(w))
    g1.step(50)
    g2.step(50)
    assert np.array_equal(g1.get_state(), g2.get_state())
    assert np.array_equal(g1.wall_force(), g2.wall_force())


def test_link_fraction_errors(lbm):
    w, q = offset_channel(4, 8, 0.3, 0.3)
    g = lbm.from_workload(w, init=False)
    with pytest.raises(lbm.LBMError):
        g.set_link_fractions(np.zeros((9, 1, 8, 4)))
    g.set_link_fractions(q)
    g.init_equilibrium()
    g.step(2)
    with pytest.raises(lbm.LBMError):
        g.set_link_fractions(q)  # set-up only

