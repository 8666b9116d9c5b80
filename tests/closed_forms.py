"""Closed forms and independent reference models used to pin the oracle.

Nothing here calls the oracle or the GPU library.  Each function states the
mathematics it encodes; the derivations are summarised in the docstrings.
"""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lattice(name):
    """Velocity set (integer unit vectors) and weights from the golden table."""
    es, ws = [], []
    with open(os.path.join(GOLDEN, "lattices.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] != name:
                continue
            es.append([int(parts[2]), int(parts[3]), int(parts[4])])
            ws.append(float(Fraction(parts[5])))
    return np.array(es), np.array(ws)


def channel_recurrence(ny, tau, a, steps, uw=0.0, darcy=0.0):
    """Exact evolution of a body-force-driven D2Q9 channel (lattice units,
    halfway bounce-back walls across y, periodic x, start from rest).

    For a flow that is uniform along x with rho = 1, only the class sums
    m_s = sum_{e_y = s} e_x f (s = +1, 0, -1) matter; u = m_+ + m_0 + m_-.
    The body force may include a porous resistance -darcy v with
    v = u + a/2, which gives a = (a_ext - darcy u) / (1 + darcy / 2).
    BGK collision with any of the five force models gives, written in v,
        m*_(+-1) = (1 - 1/tau) m_(+-1) + v / (6 tau) + C a / 6,
        m*_0     = (1 - 1/tau) m_0     + 2 v / (3 tau) + 2 C a / 3,
    with C = 1 - 1/(2 tau) (equilibrium odd moments of D2Q9 plus the force
    term's first moment).  Streaming moves m_+ up and m_- down one row;
    bounce-back gives m_+(0) = -m*_-(0) and, at a lid moving with u_w (Ladd
    term 6 w rho e.u_w), m_-(top) = -m*_+(top) + u_w / 3.
    Returns v(y) at the final step."""
    mp = np.zeros(ny)
    m0 = np.zeros(ny)
    mm = np.zeros(ny)
    C = 1.0 - 1.0 / (2.0 * tau)
    for _ in range(steps):
        u = mp + m0 + mm
        ae = (a - darcy * u) / (1.0 + 0.5 * darcy)
        v = u + 0.5 * ae
        sp = (1 - 1 / tau) * mp + v / (6 * tau) + C * ae / 6
        s0 = (1 - 1 / tau) * m0 + 2 * v / (3 * tau) + 2 * C * ae / 3
        sm = (1 - 1 / tau) * mm + v / (6 * tau) + C * ae / 6
        mp2 = np.empty(ny)
        mm2 = np.empty(ny)
        mp2[1:] = sp[:-1]
        mm2[:-1] = sm[1:]
        mp2[0] = -sm[0]
        mm2[-1] = -sp[-1] + uw / 3.0
        mp, m0, mm = mp2, s0, mm2
    u = mp + m0 + mm
    ae = (a - darcy * u) / (1.0 + 0.5 * darcy)
    return u + 0.5 * ae


def node_positions(n, dx):
    """Centre-relative coordinates of n nodes between halfway walls."""
    return (np.arange(n) + 0.5) * dx - 0.5 * n * dx


def poiseuille_steady(n, dx, dt, tau, a):
    """Steady velocity of the bounce-back channel with BGK and halfway walls:
    v(y) = (a / 2 nu) [y_w^2 - y^2 + dx^2 (16 tau^2 - 16 tau + 1) / 12],
    nu = dt c^2 (tau - 1/2) / 3.  The extra constant is the exact discrete
    slip of halfway bounce-back (it follows from the class-sum recurrence at
    steady state); the plain parabola misses it."""
    c = dx / dt
    nu = dt * c * c * (tau - 0.5) / 3.0
    y = node_positions(n, dx)
    yw = 0.5 * n * dx
    return a / (2 * nu) * (yw ** 2 - y ** 2 + dx ** 2 * (16 * tau ** 2 - 16 * tau + 1) / 12.0)


def couette_force_steady(n, dx, dt, tau, a, uw):
    """Steady Couette flow with a body force: lid at the top moving with u_w,
    v = u_w (y - y_b) / H + (a / 2 nu) [(y - y_b)(y_t - y) + dx^2 (16 tau^2 - 16 tau + 1) / 12]."""
    c = dx / dt
    nu = dt * c * c * (tau - 0.5) / 3.0
    yb = 0.0
    H = n * dx
    y = (np.arange(n) + 0.5) * dx
    return uw * (y - yb) / H + a / (2 * nu) * ((y - yb) * (H - y) + dx ** 2 * (16 * tau ** 2 - 16 * tau + 1) / 12.0)


def hartmann(n, nu, eta, mu, rho, a_x, B0):
    """Hartmann channel between insulating walls at y = +-a (a = n/2, lattice
    units): u = U [1 - cosh(Ha y/a) / cosh Ha], U = a_x a^2 / (nu Ha tanh Ha),
    Ha = B0 a / sqrt(mu rho nu eta); induced field
    b_x = (rho a_x a mu / B0) [sinh(Ha y/a) / sinh Ha - y/a]."""
    half = 0.5 * n
    Ha = B0 * half / np.sqrt(mu * rho * nu * eta)
    y = node_positions(n, 1.0)
    U = a_x * half ** 2 / (nu * Ha * np.tanh(Ha))
    u = U * (1 - np.cosh(Ha * y / half) / np.cosh(Ha))
    b = rho * a_x * half * mu / B0 * (np.sinh(Ha * y / half) / np.sinh(Ha) - y / half)
    return u, b, Ha


def channel_bottom_force_recurrence(ny, tau, a_rows, steps, uw=0.0):
    """x-force per column on the bottom wall during the last step of the
    channel of `channel_recurrence`, with a body force that may vary by row
    (a_rows: scalar or [ny]).  Momentum exchange at a static halfway wall
    (Eq. 25): each link leaving row 0 downwards carries e_x (2 f_rel); the
    rest-state parts of the two diagonal links cancel, so the force is
    2 m*_-(0).  The map (a_rows, u_w) -> force is linear."""
    a = np.broadcast_to(np.asarray(a_rows, dtype=float), (ny,)).copy()
    mp = np.zeros(ny)
    m0 = np.zeros(ny)
    mm = np.zeros(ny)
    C = 1.0 - 1.0 / (2.0 * tau)
    F = 0.0
    for _ in range(steps):
        v = mp + m0 + mm + 0.5 * a
        sp = (1 - 1 / tau) * mp + v / (6 * tau) + C * a / 6
        s0 = (1 - 1 / tau) * m0 + 2 * v / (3 * tau) + 2 * C * a / 3
        sm = (1 - 1 / tau) * mm + v / (6 * tau) + C * a / 6
        F = 2.0 * sm[0]
        mp2 = np.empty(ny)
        mm2 = np.empty(ny)
        mp2[1:] = sp[:-1]
        mm2[:-1] = sm[1:]
        mp2[0] = -sm[0]
        mm2[-1] = -sp[-1] + uw / 3.0
        mp, m0, mm = mp2, s0, mm2
    return F


def brinkman_channel(n, nu, sigma, a):
    """Steady channel of width n (lattice units) with walls at y = +-n/2 and a
    uniform porous resistance sigma: nu u'' - sigma u + a = 0, u(+-n/2) = 0,
    u = (a / sigma) [1 - cosh(y / L) / cosh(n / (2 L))], L = sqrt(nu / sigma)."""
    y = node_positions(n, 1.0)
    L = np.sqrt(nu / sigma)
    return a / sigma * (1.0 - np.cosh(y / L) / np.cosh(0.5 * n / L))


def channel_stress_recurrence(ny, tau0, a, steps, model=4, stokes=False, cs=0.0):
    """Non-equilibrium second moments of the force-driven D2Q9 channel of
    `channel_recurrence` (lattice units, rho = 1, static halfway walls),
    with either equilibrium (Eq. 1, or the Stokes form of the text after
    Eq. 11) and, for cs > 0, a Smagorinsky relaxation time per node.

    Classes by e_y = s in {+1, 0, -1}: x momentum m_s = sum_{e_y = s} e_x f
    (as in `channel_recurrence`) and xx energy n_s = sum_{e_y = s} e_x^2 f.
    For u = (u, 0) and a = (a, 0) the collision acts on them as
      m*_s = (1 - 1/tau) m_s + k_s (u^eq / tau + C a)        k = 1/6, 2/3, 1/6
      n*_s = (1 - 1/tau) n_s + c_s (1 + 3 q u^eq^2) / tau + k'_s C u^F a
                                                             c = 1/18, 2/9, 1/18
                                                             k' = 1/3, 4/3, 1/3
    (q = 1 for Eq. 1, 0 for the Stokes form; the force classes follow from
    Eq. 3 summed over e_x = +-1; He's force term [a] has no xx part), then
    the s = +-1 classes stream along y and a static wall returns them with
    e_x kept (m changes sign, n does not).  n is carried less its rest value
    c_s (the c_s / tau parts cancel), which keeps the small non-equilibrium
    part free of the rounding of 1/3.  Pi^neq_xx = sum_s n_s - 1/3 -
    q u^eq^2, Pi^neq_xy = m_+1 - m_-1 (Pi^neq_yy = 0: the e_y classes of the
    density stay at equilibrium).  The Smagorinsky tau is the positive root of
    tau^2 - tau0 tau - 9 sqrt(2) cs^2 |Pi| / 2 = 0, |Pi|^2 = Pi_xx^2 +
    2 Pi_xy^2, from the pre-step state.

    Returns, for the state after `steps` steps, per row: Pi_xx, Pi_xy, tau,
    u, v, u^eq, u^F, C (the last four as the force model defines them)."""
    q = 0.0 if stokes else 1.0
    kmo = np.array([1 / 6, 2 / 3, 1 / 6])
    cen = np.array([1 / 18, 2 / 9, 1 / 18])
    ken = np.array([1 / 3, 4 / 3, 1 / 3])
    m = np.zeros((3, ny))                  # classes s = +1, 0, -1
    n = np.zeros((3, ny))                  # xx classes less their rest values c_s
    out = None
    for it in range(steps + 1):
        u = m.sum(0)                       # rho = 1: u = sum e_x f
        pxy = m[0] - m[2]
        # Pi_xx needs u^eq, which needs tau ([c] does not enter u^eq)
        ueq = u + 0.5 * a if model == 4 else u
        pxx = n.sum(0) - q * ueq ** 2       # sum_s c_s = 1/3
        if cs > 0:
            Qn = np.sqrt(pxx ** 2 + 2 * pxy ** 2)
            tau = 0.5 * (tau0 + np.sqrt(tau0 ** 2 + 18 * np.sqrt(2) * cs ** 2 * Qn))
        else:
            tau = np.full(ny, tau0)
        C = 1 - 1 / (2 * tau) if model == 4 else np.ones(ny)
        v = u + 0.5 * a
        uF = {0: 0 * u, 1: u, 2: u + 0.5 * tau * a, 3: v, 4: v}[model]
        if it == steps:
            out = dict(pxx=pxx, pxy=pxy, tau=tau, u=u, v=v, ueq=ueq, uF=uF, C=C)
            break
        ms = (1 - 1 / tau) * m + kmo[:, None] * (ueq / tau + C * a)
        ns = (1 - 1 / tau) * n + cen[:, None] * 3 * q * ueq ** 2 / tau
        if model != 0:
            ns = ns + ken[:, None] * C * uF * a
        m2 = np.empty_like(m)
        n2 = np.empty_like(n)
        m2[1], n2[1] = ms[1], ns[1]
        m2[0, 1:], n2[0, 1:] = ms[0, :-1], ns[0, :-1]
        m2[2, :-1], n2[2, :-1] = ms[2, 1:], ns[2, 1:]
        m2[0, 0], n2[0, 0] = -ms[2, 0], ns[2, 0]
        m2[2, -1], n2[2, -1] = -ms[0, -1], ns[0, -1]
        m, n = m2, n2
    return out
