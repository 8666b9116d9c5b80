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
