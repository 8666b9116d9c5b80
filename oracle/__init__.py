"""ctypes front end of the CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product package.

``Oracle`` mirrors the GPU library's calls (same argument meanings and array
layouts) on an independent FP64 implementation.  ``complex_step=True`` loads
the double-complex build: inputs may then carry imaginary parts and outputs
return them, so that ``imag(out) / h`` is the exact derivative of ``out``
along the perturbation ``i*h*delta`` put on the inputs.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the sanitizer builds of oracle/build.py are loaded from another folder
LIBDIR = os.environ.get("ORACLE_LIB_DIR", HERE)

D2Q9, D3Q19 = 0, 1
HE, LUO, SHANCHEN, EDM, GUO, SHANCHEN_ORIG, EDM_ORIG = range(7)

_libs = {}


def _lib(complex_step: bool):
    name = "liboracle_cs.so" if complex_step else "liboracle.so"
    if name not in _libs:
        path = os.path.join(LIBDIR, name)
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = C.CDLL(path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int]
        lib.orc_destroy.argtypes = [P]
        lib.orc_threads.argtypes = [C.c_int]
        lib.orc_set_rho0.argtypes = [P, C.c_double]
        lib.orc_set_walls.argtypes = [P, C.c_int, C.c_int, C.c_int]
        lib.orc_set_solid.argtypes = [P, C.c_void_p, C.c_int]
        lib.orc_set_wall_velocity.argtypes = [P, C.c_int, dp, dp]
        lib.orc_set_body_force.argtypes = [P, dp, dp]
        lib.orc_set_body_force_field.argtypes = [P, dp, dp]
        lib.orc_set_les.argtypes = [P, C.c_double]
        lib.orc_set_equilibrium.argtypes = [P, C.c_int]
        lib.orc_set_darcy.argtypes = [P, C.c_double]
        lib.orc_set_link_fraction.argtypes = [P, dp]
        lib.orc_set_artefact.argtypes = [P, C.c_int]
        lib.orc_set_mhd.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        lib.orc_set_lorentz_force.argtypes = [P, C.c_int]
        lib.orc_init_equilibrium.argtypes = [P, dp]
        lib.orc_set_state.argtypes = [P, dp, dp]
        lib.orc_get_state.argtypes = [P, dp, dp]
        lib.orc_replace_state.argtypes = [P, dp]
        lib.orc_get_induction.argtypes = [P, dp]
        lib.orc_step.argtypes = [P, C.c_int]
        lib.orc_get_macro.argtypes = [P, dp, dp, dp]
        lib.orc_stress.argtypes = [P, dp, dp]
        lib.orc_wall_force.argtypes = [P, dp, dp, C.c_int]
        lib.orc_force_balance.argtypes = [P, dp]
        lib.orc_link_count.restype = C.c_long
        lib.orc_link_count.argtypes = [P, C.c_int]
        lib.orc_adjoint.argtypes = [P, C.c_int, C.c_int, C.c_int, dp, dp, dp]
        lib.orc_halfstep.argtypes = [P, dp, dp, dp, dp]
        _libs[name] = lib
    return _libs[name]


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64)


def threads(n: int = 0, complex_step: bool = False) -> int:
    return _lib(complex_step).orc_threads(n)


class Oracle:
    """One lattice on the CPU.  Shapes: state [Q, nz, ny, nx]; macro rho
    [nz, ny, nx], v [D, nz, ny, nx]; stress [ncomp, nz, ny, nx]."""

    def __init__(self, lattice, nx, ny, nz, tau, dx=1.0, dt=1.0, model=GUO, complex_step=False):
        self.cs = complex_step
        self.lib = _lib(complex_step)
        self.lattice, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.D = 2 if lattice == D2Q9 else 3
        self.Q = 9 if lattice == D2Q9 else 19
        self.N = nx * ny * nz
        self.h = self.lib.orc_create(lattice, nx, ny, nz, tau, dx, dt, model)
        if not self.h:
            raise ValueError("oracle rejected the lattice parameters")
        self.groups = 1
        self.mhd = False

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _chk(self, rc):
        if rc != 0:
            raise ValueError("oracle call failed")

    # -- set-up ------------------------------------------------------------
    def set_rho0(self, rho0):
        self._chk(self.lib.orc_set_rho0(self.h, rho0))

    def set_walls(self, axis, g_lo, g_hi):
        self._chk(self.lib.orc_set_walls(self.h, axis, g_lo, g_hi))
        self.groups = max(self.groups, g_lo + 1, g_hi + 1)

    def set_solid(self, mask, group):
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        self._chk(self.lib.orc_set_solid(self.h, m.ctypes.data, group))
        self.groups = max(self.groups, group + 1)

    def set_wall_velocity(self, group, u, u_im=None):
        self._chk(self.lib.orc_set_wall_velocity(self.h, group, _dp(_f64(u)), _dp(_f64(u_im))))
        self.groups = max(self.groups, group + 1)

    def set_body_force(self, a, a_im=None):
        self._chk(self.lib.orc_set_body_force(self.h, _dp(_f64(a)), _dp(_f64(a_im))))

    def set_body_force_field(self, a, a_im=None):
        a = _f64(a)
        a_im = _f64(a_im)
        self._keep = (a, a_im)
        self._chk(self.lib.orc_set_body_force_field(self.h, _dp(a), _dp(a_im)))

    def set_les(self, cs):
        self._chk(self.lib.orc_set_les(self.h, cs))

    def set_equilibrium(self, stokes):
        self._chk(self.lib.orc_set_equilibrium(self.h, int(stokes)))

    def set_darcy(self, sigma):
        self._chk(self.lib.orc_set_darcy(self.h, sigma))

    def set_link_fraction(self, q):
        """q [Q, nz, ny, nx]: wall distance / link length of wall links (1/2 halfway), or None."""
        q = _f64(q)
        self._chk(self.lib.orc_set_link_fraction(self.h, _dp(q)))

    def set_artefact(self, on):
        self._chk(self.lib.orc_set_artefact(self.h, int(on)))

    def set_mhd(self, B0, mu, tau_m):
        self._chk(self.lib.orc_set_mhd(self.h, B0[0], B0[1], B0[2], mu, tau_m))
        self.mhd = True

    def set_lorentz_force(self, on):
        """MHD coupling: True = Lorentz force through the force term (equilibrium
        hydrodynamic), False = magnetic stress in the equilibrium (Eq. 10)."""
        self._chk(self.lib.orc_set_lorentz_force(self.h, int(on)))

    def init_equilibrium(self, u0=None):
        self._chk(self.lib.orc_init_equilibrium(self.h, _dp(_f64(u0))))

    def set_state(self, d, d_im=None, keep_records=False):
        d = _f64(d)
        assert d.size == self.Q * self.N
        if keep_records:
            self._chk(self.lib.orc_replace_state(self.h, _dp(d)))
        else:
            self._chk(self.lib.orc_set_state(self.h, _dp(d), _dp(_f64(d_im))))

    def get_state(self, imag=False):
        d = np.empty((self.Q, self.nz, self.ny, self.nx))
        di = np.empty_like(d) if imag else None
        self._chk(self.lib.orc_get_state(self.h, _dp(d), _dp(di)))
        return (d, di) if imag else d

    def get_induction(self):
        g = np.empty((7 if self.D == 3 else 5, 3, self.nz, self.ny, self.nx))
        self._chk(self.lib.orc_get_induction(self.h, _dp(g)))
        return g

    # -- stepping and outputs ---------------------------------------------
    def step(self, n=1):
        self._chk(self.lib.orc_step(self.h, n))

    def get_macro(self, with_B=False):
        rho = np.empty((self.nz, self.ny, self.nx))
        v = np.empty((self.D, self.nz, self.ny, self.nx))
        B = np.empty((3, self.nz, self.ny, self.nx)) if with_B else None
        self._chk(self.lib.orc_get_macro(self.h, _dp(rho), _dp(v), _dp(B)))
        return (rho, v, B) if with_B else (rho, v)

    def stress(self):
        nc = 3 if self.D == 2 else 6
        sig = np.empty((nc, self.nz, self.ny, self.nx))
        S = np.empty_like(sig)
        self._chk(self.lib.orc_stress(self.h, _dp(sig), _dp(S)))
        return sig, S

    def wall_force(self, groups=None, imag=False):
        G = groups or self.groups
        out = np.empty((G, 4, 3))
        oi = np.empty_like(out) if imag else None
        self._chk(self.lib.orc_wall_force(self.h, _dp(out), _dp(oi), G))
        return (out, oi) if imag else out

    def force_balance(self):
        out = np.empty(24)
        self._chk(self.lib.orc_force_balance(self.h, _dp(out)))
        return out

    def link_count(self, group=-1):
        return self.lib.orc_link_count(self.h, group)

    def halfstep(self):
        """Half-step distribution of the last step (Eq. 27) and its moments:
        (fbar [Q, ...] deviations, rho_bar, u_bar [D, ...], sigma_bar [ncomp, ...])."""
        nc = 3 if self.D == 2 else 6
        sh = (self.nz, self.ny, self.nx)
        fb = np.empty((self.Q,) + sh)
        rb = np.empty(sh)
        ub = np.empty((self.D,) + sh)
        sb = np.empty((nc,) + sh)
        self._chk(self.lib.orc_halfstep(self.h, _dp(fb), _dp(rb), _dp(ub), _dp(sb)))
        return fb, rb, ub, sb

    def adjoint(self, T, group, axis):
        """Reverse-mode gradient of J = component `axis` of the raw wall force
        on `group` during the last of T steps from the current state (complex
        build only).  Returns (J, grad_a [3, nz, ny, nx], grad_uw [G, 3]) in
        physical units; the state is left at step T."""
        if not self.cs:
            raise ValueError("the adjoint needs the complex-step build")
        J = np.zeros(1)
        ga = np.zeros((3, self.nz, self.ny, self.nx))
        gu = np.zeros((max(self.groups, 1), 3))
        self._chk(self.lib.orc_adjoint(self.h, T, group, axis, _dp(J), _dp(ga), _dp(gu)))
        return float(J[0]), ga, gu
