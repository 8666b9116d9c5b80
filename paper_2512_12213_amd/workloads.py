"""Synthetic workloads: sizes, parameters and seeded input generators.

This module holds no lattice Boltzmann arithmetic.  It only produces inputs
(geometry masks, initial velocities, random distribution states, body-force
fields) that the GPU library and the CPU reference both consume, so that both
start from bit-identical host arrays.

The five configurations are the synthetic stand-ins for the flows the paper
analyses (it reports no numerical experiments of its own): a force-driven
channel, a Couette channel with a cylinder, a turbulent square duct with
Smagorinsky closure, a Hartmann duct with the MHD equilibrium of Eq. (10), and
a duct with a sphere for the adjoint.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

D2Q9, D3Q19 = 0, 1
HE, LUO, SHANCHEN, EDM, GUO = range(5)
F64, F32, F16, BF16 = range(4)


@dataclass
class Workload:
    name: str
    lattice: int
    nx: int
    ny: int
    nz: int
    tau: float
    dx: float = 1.0
    dt: float = 1.0
    model: int = GUO
    storage: int = F32
    body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    walls: Tuple = ()                   # tuples (axis, group_lo, group_hi)
    wall_velocity: Tuple = ()           # tuples (group, ux, uy, uz)
    les_cs: float = 0.0
    stokes: bool = False                # Stokes form of the equilibrium
    darcy: float = 0.0                  # porous resistance sigma (1/time)
    mhd: Optional[Tuple] = None         # (B0x, B0y, B0z, mu, tau_m)
    lorentz: bool = False               # MHD: Lorentz force through the force term, equilibrium hydrodynamic
    obstacle: Optional[Tuple] = None    # ("cylinder", cx, cy, r, group) or ("sphere", cx, cy, cz, r, group)
    curved: bool = False                # obstacle walls at their exact distance (link fractions), not halfway
    u0_amp: float = 0.0
    u0_seed: int = 2512
    steps: int = 0
    groups: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def D(self):
        return 2 if self.lattice == D2Q9 else 3

    @property
    def Q(self):
        return 9 if self.lattice == D2Q9 else 19


def poiseuille(nx=64, ny=32, storage=F64, model=GUO, tau=0.8, a=1e-6, steps=5000):
    """Force-driven channel: halfway walls across y, periodic x, rest start."""
    return Workload("poiseuille_d2q9_%dx%d" % (nx, ny), D2Q9, nx, ny, 1, tau, model=model, storage=storage,
                    body_force=(a, 0.0, 0.0), walls=((1, 0, 1),), steps=steps, groups=2)


def couette_cylinder(nx=512, ny=128, storage=F32, r=12.0, cx=128.0, cy=64.0, uw=0.05, tau=0.6, a=5e-7,
                     steps=20000):
    """Couette channel (moving top wall) with body force and a fixed cylinder."""
    return Workload("couette_cylinder_d2q9_%dx%d" % (nx, ny), D2Q9, nx, ny, 1, tau, storage=storage,
                    body_force=(a, 0.0, 0.0), walls=((1, 0, 1),), wall_velocity=((1, uw, 0.0, 0.0),),
                    obstacle=("cylinder", cx, cy, r, 2), steps=steps, groups=3)


def duct_les(nx=256, ny=128, nz=128, storage=F32, tau=0.52, cs=0.1, a=1e-5, amp=1e-3, seed=2512, steps=1000):
    """Square duct, periodic x, halfway walls on y and z, Smagorinsky closure,
    initial velocity with seeded uniform +-amp perturbations."""
    return Workload("duct_les_d3q19_%dx%dx%d" % (nx, ny, nz), D3Q19, nx, ny, nz, tau, storage=storage,
                    body_force=(a, 0.0, 0.0), walls=((1, 0, 1), (2, 2, 3)), les_cs=cs, u0_amp=amp, u0_seed=seed,
                    steps=steps, groups=4)


def hartmann_duct(nx=192, ny=96, nz=96, storage=F32, Ha=20.0, tau=0.8, tau_m=0.9, mu=1.0, a=1e-5, steps=20000):
    """Hartmann duct: uniform transverse field B0 along y, insulating walls,
    MHD equilibrium, D3Q7 induction.  B0 is set from the Hartmann number on
    the half-width along B: Ha = B0 (ny/2) / sqrt(mu rho nu eta)."""
    nu = (tau - 0.5) / 3.0
    eta = 0.25 * (tau_m - 0.5)
    B0 = Ha * np.sqrt(mu * 1.0 * nu * eta) / (0.5 * ny)
    walls = ((1, 0, 1),) if nz == 1 else ((1, 0, 1), (2, 2, 3))
    return Workload("hartmann_duct_d3q19_%dx%dx%d" % (nx, ny, nz), D3Q19, nx, ny, nz, tau, storage=storage,
                    body_force=(a, 0.0, 0.0), walls=walls, mhd=(0.0, float(B0), 0.0, mu, tau_m), steps=steps,
                    groups=2 if nz == 1 else 4)


def hartmann_channel(nx=1, ny=96, lattice=D2Q9, storage=F64, Ha=20.0, tau=0.8, tau_m=0.9, mu=1.0, a=1e-5,
                     lorentz=False, steps=20000):
    """Hartmann channel between insulating walls across y, periodic x (and z):
    D2Q9 with the planar induction lattice, or a one-node-thick D3Q19 slab.
    B0 along y from the Hartmann number on the half-width, as for the duct."""
    nu = (tau - 0.5) / 3.0
    eta = 0.25 * (tau_m - 0.5)
    B0 = Ha * np.sqrt(mu * 1.0 * nu * eta) / (0.5 * ny)
    d = "d2q9" if lattice == D2Q9 else "d3q19"
    return Workload("hartmann_channel_%s_%dx%d%s" % (d, nx, ny, "_lorentz" if lorentz else ""), lattice, nx, ny, 1,
                    tau, storage=storage, body_force=(a, 0.0, 0.0), walls=((1, 0, 1),),
                    mhd=(0.0, float(B0), 0.0, mu, tau_m), lorentz=lorentz, steps=steps, groups=2)


def duct_sphere(nx=128, ny=64, nz=64, storage=F32, r=8.0, tau=0.55, a=1e-5, uw=0.01, steps=400):
    """Duct with a sphere at the centre; the top (y) wall moves with u_w along x."""
    c = (0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1))
    return Workload("duct_sphere_d3q19_%dx%dx%d" % (nx, ny, nz), D3Q19, nx, ny, nz, tau, storage=storage,
                    body_force=(a, 0.0, 0.0), walls=((1, 0, 1), (2, 2, 3)), wall_velocity=((1, uw, 0.0, 0.0),),
                    obstacle=("sphere", c[0], c[1], c[2], r, 4), steps=steps, groups=5)


# ---------------------------------------------------------------------------
# seeded generators
# ---------------------------------------------------------------------------
def cylinder_mask(nx, ny, cx, cy, r):
    """[1, ny, nx] uint8: node solid iff (x - cx)^2 + (y - cy)^2 <= r^2."""
    y, x = np.mgrid[0:ny, 0:nx]
    return ((x - cx) ** 2 + (y - cy) ** 2 <= r * r).astype(np.uint8)[None]


def sphere_mask(nx, ny, nz, cx, cy, cz, r):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    return ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r).astype(np.uint8)


def link_fractions_sphere(Q, nx, ny, nz, cx, cy, cz, r):
    """[Q, nz, ny, nx] wall distance / link length for links from fluid nodes
    into the solid ball (x - c)^2 <= r^2 (1/2 elsewhere): the smallest t in
    (0, 1] with |x + t e - c| = r.  Two-dimensional lattices use nz = 1 and
    the circle in the plane."""
    if Q == 9:
        e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [1, 1, 0], [-1, -1, 0],
                      [1, -1, 0], [-1, 1, 0]], float)
    else:
        e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                      [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
                      [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], float)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    p = np.stack([x - cx, y - cy, (z - cz) if Q == 19 else 0.0 * z])
    inside = (p ** 2).sum(0) <= r * r
    q = np.full((Q, nz, ny, nx), 0.5)
    for a in range(1, Q):
        ea = e[a].reshape(3, 1, 1, 1)
        # |p + t e|^2 = r^2: (e.e) t^2 + 2 (p.e) t + (p.p - r^2) = 0, smallest root
        A = float((e[a] ** 2).sum())
        B = 2.0 * (p * ea).sum(0)
        Cc = (p ** 2).sum(0) - r * r
        disc = np.maximum(B * B - 4 * A * Cc, 0.0)
        t = (-B - np.sqrt(disc)) / (2 * A)
        tgt = np.roll(inside, shift=(-int(e[a, 2]), -int(e[a, 1]), -int(e[a, 0])), axis=(0, 1, 2)) if Q == 19 else \
            np.roll(inside, shift=(-int(e[a, 1]), -int(e[a, 0])), axis=(1, 2))
        hit = (~inside) & tgt
        q[a][hit] = np.clip(t[hit], 1e-6, 1.0)
    return q


def link_fractions(w: Workload):
    """[Q, nz, ny, nx] link fractions of the workload's obstacle surface when
    it is curved, else None (halfway walls everywhere)."""
    if not w.curved or w.obstacle is None:
        return None
    if w.obstacle[0] == "cylinder":
        _, cx, cy, r, _g = w.obstacle
        return link_fractions_sphere(9, w.nx, w.ny, 1, cx, cy, 0.0, r)
    _, cx, cy, cz, r, _g = w.obstacle
    return link_fractions_sphere(19, w.nx, w.ny, w.nz, cx, cy, cz, r)


def obstacle_mask(w: Workload):
    if w.obstacle is None:
        return None
    if w.obstacle[0] == "cylinder":
        _, cx, cy, r, _g = w.obstacle
        return cylinder_mask(w.nx, w.ny, cx, cy, r)
    _, cx, cy, cz, r, _g = w.obstacle
    return sphere_mask(w.nx, w.ny, w.nz, cx, cy, cz, r)


def initial_velocity(w: Workload):
    """[D, nz, ny, nx] float64 i.i.d. uniform(-amp, amp), or None at rest."""
    if w.u0_amp == 0.0:
        return None
    rng = np.random.default_rng(w.u0_seed)
    return rng.uniform(-w.u0_amp, w.u0_amp, size=(w.D, w.nz, w.ny, w.nx))


def random_velocity(D, nz, ny, nx, amp=1e-3, seed=0):
    """[D, nz, ny, nx] float64 i.i.d. uniform(-amp, amp)."""
    return np.random.default_rng(seed).uniform(-amp, amp, size=(D, nz, ny, nx))


def random_state(Q, nx, ny, nz, amp=1e-3, seed=0):
    """[Q, nz, ny, nx] float64 i.i.d. uniform(-amp, amp): an arbitrary
    distribution-deviation state, used to exercise every term of a step."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(Q, nz, ny, nx))


def force_field(nx, ny, nz, base=(1e-5, 0.0, 0.0), amp=0.0, seed=0):
    """[3, nz, ny, nx] float64: base + i.i.d. uniform(-amp, amp) * max|base|."""
    f = np.empty((3, nz, ny, nx))
    for k in range(3):
        f[k] = base[k]
    if amp:
        rng = np.random.default_rng(seed)
        f += amp * max(abs(b) for b in base) * rng.uniform(-1.0, 1.0, size=f.shape)
    return f


def direction(shape, seed):
    """Seeded direction for directional-derivative checks, entries U[-1, 1]."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)
