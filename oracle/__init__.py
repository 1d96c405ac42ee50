"""FP64 CPU oracle for the MEMD lattice update with a spatially varying
permittivity (Fahrenberger & Holm, arXiv:1309.7859).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library and never calls it.

The arithmetic lives in ``memd_oracle.c`` (plain C, FP64); this module loads it
with ctypes and strings the calls together in the order the paper gives:
charge assignment, permittivity mapping, the initial recursion plus
relaxation, then per step the leapfrog halves, the current deposit, and the
observables (forces with self-energy and dipole corrections, energies, Gauss
residual, dipole moment); and the ions' own dynamics driven by those forces
(velocity Verlet, ``System.md_step``).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    i, d = C.c_int, C.c_double
    sig = {
        "orc_version": (i, []),
        "orc_threads": (i, []),
        "orc_set_threads": (None, [i]),
        "orc_spread": (None, [i, d, i, _P, _P, _P]),
        "orc_eps_site_to_link": (i, [i, _P, d, _P]),
        "orc_eps_derived": (None, [i, _P, _P, _P, _P]),
        "orc_salt_eps": (None, [i, d, i, _P, d, d, d, _P]),
        "orc_curl": (None, [i, d, _P, _P]),
        "orc_curl_adj": (None, [i, d, _P, _P]),
        "orc_div": (None, [i, d, _P, _P]),
        "orc_recursion": (None, [i, d, _P, _P]),
        "orc_mean_shift": (None, [i, d, _P, _P]),
        "orc_relax": (i, [i, d, _P, _P, d, i, C.POINTER(i), _P]),
        "orc_curl_measure": (d, [i, d, _P, _P]),
        "orc_faraday": (None, [i, d, d, _P, _P, _P]),
        "orc_ampere": (None, [i, d, d, d, _P, _P]),
        "orc_deposit": (None, [i, d, i, _P, _P, _P, _P]),
        "orc_step": (None, [i, d, d, d, _P, i, _P, _P, _P, _P, _P]),
        "orc_gauss_residual": (None, [i, d, _P, _P, _P, _P]),
        "orc_dipole": (None, [i, _P, _P, _P]),
        "orc_greens": (None, [i, _P]),
        "orc_self_sum": (None, [_P, _P, _P, _P]),
        "orc_forces": (None, [i, d, i, _P, _P, _P, _P, _P, _P, _P, _P, i, _P, _P]),
        "orc_energy": (None, [i, d, d, d, _P, _P, _P, d, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    U = C.POINTER(C.c_uint)
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox4x32_10.argtypes = [U, U, U]
    lib.orc_seeded_displacements.restype = None
    lib.orc_seeded_displacements.argtypes = [C.c_ulonglong, i, i, d, _P]
    _lib = lib
    return lib


def _ptr(x: np.ndarray):
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(_P)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ----------------------------------------------------------------- primitives

def spread(L: int, a: float, q, r) -> np.ndarray:
    q, r = _f64(q), _f64(r).reshape(-1)
    rho = np.zeros(L ** 3)
    _load().orc_spread(L, a, len(q), _ptr(q), _ptr(r), _ptr(rho))
    return rho


def eps_site_to_link(L: int, eps_site, r_thr: float = 4.0):
    e = _f64(eps_site).reshape(-1)
    out = np.zeros(3 * L ** 3)
    nif = _load().orc_eps_site_to_link(L, _ptr(e), r_thr, _ptr(out))
    return out, nif


def eps_derived(L: int, eps_link):
    e = _f64(eps_link).reshape(-1)
    eta = np.zeros(3 * L ** 3)
    eh = np.zeros(3)
    ec = np.zeros(L ** 3)
    _load().orc_eps_derived(L, _ptr(e), _ptr(eta), _ptr(eh), _ptr(ec))
    return eta, eh, ec


def salt_eps(L: int, a: float, r, eps_w=80.0, slope=15.0, eps_floor=1.0) -> np.ndarray:
    r = _f64(r).reshape(-1)
    out = np.zeros(3 * L ** 3)
    _load().orc_salt_eps(L, a, len(r) // 3, _ptr(r), eps_w, slope, eps_floor, _ptr(out))
    return out


def curl(L, a, X):
    X = _f64(X).reshape(-1)
    Y = np.zeros_like(X)
    _load().orc_curl(L, a, _ptr(X), _ptr(Y))
    return Y


def curl_adj(L, a, Y):
    Y = _f64(Y).reshape(-1)
    X = np.zeros_like(Y)
    _load().orc_curl_adj(L, a, _ptr(Y), _ptr(X))
    return X


def div(L, a, X):
    X = _f64(X).reshape(-1)
    out = np.zeros(L ** 3)
    _load().orc_div(L, a, _ptr(X), _ptr(out))
    return out


def recursion(L, a, rho):
    rho = _f64(rho)
    D = np.zeros(3 * L ** 3)
    _load().orc_recursion(L, a, _ptr(rho), _ptr(D))
    return D


def greens(L: int) -> np.ndarray:
    G = np.zeros(4)
    _load().orc_greens(L, _ptr(G))
    return G


def self_sum(G, f):
    G, f = _f64(G), _f64(f)
    S = np.zeros(1)
    dS = np.zeros(3)
    _load().orc_self_sum(_ptr(G), _ptr(f), _ptr(S), _ptr(dS))
    return float(S[0]), dS


def dipole(q, r) -> np.ndarray:
    q, r = _f64(q), _f64(r).reshape(-1)
    P = np.zeros(3)
    _load().orc_dipole(len(q), _ptr(q), _ptr(r), _ptr(P))
    return P


def philox4x32_10(ctr, key):
    c = (C.c_uint * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint * 4)()
    _load().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def seeded_displacements(seed: int, step: int, n: int, sigma: float) -> np.ndarray:
    out = np.zeros(3 * n)
    _load().orc_seeded_displacements(int(seed), int(step), int(n), float(sigma), _ptr(out))
    return out.reshape(n, 3)


def threads() -> int:
    return _load().orc_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n > 0)."""
    _load().orc_set_threads(int(n))


def default_c(a: float, dt: float, eps_min: float, nu: float = 0.25) -> float:
    """Speed of light for a Courant number nu = c dt sqrt(3) / (a sqrt(eps_min))."""
    return nu * (a / dt) * math.sqrt(eps_min / 3.0)


# ------------------------------------------------------------------- a system

class System:
    """One MEMD system advanced step by step in FP64 on the CPU."""

    def __init__(self, L: int, a: float, dt: float, c: float, q, r0):
        self.lib = _load()
        self.L, self.a, self.dt, self.c = int(L), float(a), float(dt), float(c)
        self.Ns = self.L ** 3
        self.q = _f64(q).copy()
        self.n = len(self.q)
        self.r = _f64(r0).reshape(-1).copy()
        assert self.r.size == 3 * self.n
        self.V = (self.L * self.a) ** 3
        self.D = np.zeros(3 * self.Ns)
        self.B = np.zeros(3 * self.Ns)
        self.G = greens(self.L)
        self.set_eps_uniform(1.0)
        # section "Periodicity": with the correction, the force of the uniform
        # mode of D on each ion, -q_i P/(V eps_h), is removed (metallic
        # boundaries at infinity) and U_dip leaves the energy; without it, the
        # plain lattice algorithm holds the dipole moment in a harmonic well
        self.dipole_correction = True
        # section "Self energy interaction": "green" subtracts the lattice
        # Green's-function self force with the cell's harmonic-mean eps,
        # "direct" the field of the ion's own assigned charges on each of
        # its cell's links, divided by that link's eps
        self.self_scheme = "green"

    # -- permittivity
    def set_eps_link(self, eps_link):
        self.eps_link = _f64(eps_link).reshape(-1).copy()
        self.eta, self.eps_h, self.eps_cell = eps_derived(self.L, self.eps_link)

    def set_eps_uniform(self, eps: float):
        self.set_eps_link(np.full(3 * self.Ns, float(eps)))

    def set_eps_site(self, eps_site, r_thr: float = 4.0) -> int:
        link, nif = eps_site_to_link(self.L, eps_site, r_thr)
        self.set_eps_link(link)
        return nif

    def set_eps_zsite(self, eps_z, r_thr: float = 4.0) -> int:
        """Site permittivity that depends on the z plane only (eps_z[L])."""
        ez = _f64(eps_z)
        site = np.repeat(ez, self.L * self.L)  # k slowest
        return self.set_eps_site(site, r_thr)

    def set_eps_salt(self, eps_w=80.0, slope=15.0, eps_floor=1.0):
        self.set_eps_link(salt_eps(self.L, self.a, self.r, eps_w, slope, eps_floor))

    # -- initial solution
    def initial_solve(self, tol: float = 1e-13, max_iter: int = 200000):
        rho = spread(self.L, self.a, self.q, self.r)
        self.D = recursion(self.L, self.a, rho)
        P = self.dipole()
        self.lib.orc_mean_shift(self.L, self.a, _ptr(P), _ptr(self.D))
        it = C.c_int(0)
        res = C.c_double(0.0)
        rc = self.lib.orc_relax(self.L, self.a, _ptr(self.eta), _ptr(self.D), tol, max_iter,
                                C.byref(it), C.byref(res))
        self.B[:] = 0.0
        return rc, it.value, res.value

    def recursion_only(self):
        rho = spread(self.L, self.a, self.q, self.r)
        self.D = recursion(self.L, self.a, rho)
        P = self.dipole()
        self.lib.orc_mean_shift(self.L, self.a, _ptr(P), _ptr(self.D))
        self.B[:] = 0.0

    def curl_measure(self) -> float:
        return self.lib.orc_curl_measure(self.L, self.a, _ptr(self.eta), _ptr(self.D))

    # -- dynamics
    def step(self, disp):
        d = _f64(disp).reshape(-1)
        assert d.size == 3 * self.n
        self.lib.orc_step(self.L, self.a, self.dt, self.c, _ptr(self.eta), self.n,
                          _ptr(self.q), _ptr(self.r), _ptr(d), _ptr(self.D), _ptr(self.B))

    def md_step(self, v, m):
        """One step of the ions' own dynamics (velocity Verlet), the fields
        following: the ions obey Newton's equation with the MEMD force (the
        kinetic term of the section "Extension of the algorithm" Lagrangian,
        and eq. force without the magnetic part, as the paper's implementation
        omits it), so the move of the step is dt times the half-kicked
        velocity, and that move is the current of the leapfrog step:
          v <- v + dt F(state n) / (2 m);  step(dt v);  v <- v + dt F(state n+1) / (2 m).
        v [n, 3] is updated in place and returned; m [n] are the masses."""
        v = np.asarray(v)
        m = _f64(m).reshape(-1, 1)
        F, _ = self.forces()
        v += 0.5 * self.dt * F / m
        self.step(self.dt * v)
        F, _ = self.forces()
        v += 0.5 * self.dt * F / m
        return v

    def faraday(self):
        self.lib.orc_faraday(self.L, self.a, self.dt, _ptr(self.eta), _ptr(self.D), _ptr(self.B))

    def ampere(self):
        self.lib.orc_ampere(self.L, self.a, self.dt, self.c, _ptr(self.B), _ptr(self.D))

    def deposit(self, disp):
        d = _f64(disp).reshape(-1)
        self.lib.orc_deposit(self.L, self.a, self.n, _ptr(self.q), _ptr(self.r), _ptr(d),
                             _ptr(self.D))

    # -- observables
    def dipole(self) -> np.ndarray:
        return dipole(self.q, self.r)

    def rho(self) -> np.ndarray:
        return spread(self.L, self.a, self.q, self.r)

    def gauss_residual(self):
        rho = self.rho()
        m = C.c_double(0.0)
        s = C.c_double(0.0)
        self.lib.orc_gauss_residual(self.L, self.a, _ptr(self.D), _ptr(rho), C.byref(m), C.byref(s))
        return m.value, s.value

    def _P_for_correction(self) -> np.ndarray:
        return self.dipole() if self.dipole_correction else np.zeros(3)

    def forces(self, with_self: bool = True):
        F = np.zeros(3 * self.n)
        U = np.zeros(self.n)
        P = self._P_for_correction()
        self.lib.orc_forces(self.L, self.a, self.n, _ptr(self.q), _ptr(self.r), _ptr(self.D),
                            _ptr(self.eta), _ptr(self.eps_cell), _ptr(self.eps_h), _ptr(self.G),
                            _ptr(P), 1 if self.self_scheme == "direct" else 0, _ptr(F), _ptr(U))
        self._uself = U
        return F.reshape(self.n, 3), U

    def energy(self) -> dict:
        _, U = self.forces()
        out = np.zeros(5)
        P = self._P_for_correction()
        self.lib.orc_energy(self.L, self.a, self.dt, self.c, _ptr(self.eta), _ptr(self.D),
                            _ptr(self.B), float(U.sum()), _ptr(P), _ptr(self.eps_h), _ptr(out))
        return dict(W_E=out[0], W_B=out[1], U_self=out[2], U_dip=out[3], E_corrected=out[4])

    def state(self):
        return self.D.copy(), self.B.copy(), self.r.copy()

    def set_state(self, D, B, r):
        self.D = _f64(D).reshape(-1).copy()
        self.B = _f64(B).reshape(-1).copy()
        self.r = _f64(r).reshape(-1).copy()


# -------------------------------------------- dielectric walls (section "Validation")

def wall_image_force_z(charges, z0: float, z_lo: float, z_hi: float, eps_in: float, eps_out: float,
                       period: float = 0.0, lateral: int = 0, n_images: int = 60) -> float:
    """z force on the first of `charges` (a list of (q, x, y), all at height
    z0 inside a slab z_lo < z < z_hi of permittivity eps_in between two
    half-spaces of eps_out: the two infinite dielectric walls of the
    thermodynamic check, Fig. 6), from the images the walls induce.

    Textbook construction by repeated reflection: with Delta = (eps_in -
    eps_out)/(eps_in + eps_out), d = z_hi - z_lo and s = z0 - z_lo, a charge q
    has images Delta^|2m-1| q at z_lo - s + 2 m d (every integer m) and
    Delta^(2|n|) q at z_lo + s + 2 n d (n != 0), the potential inside the slab
    being the charges' and their images' Coulomb potentials q/(4 pi eps_in r).
    The charges themselves, all at height z0, exert no z force on each other.
    With period > 0 every charge repeats at (x + i period, y + j period) for
    |i|, |j| <= lateral (a laterally periodic box); the sum runs over those
    copies of every charge's images (for a neutral set the sheet terms of the
    copies cancel between charges)."""
    Delta = (eps_in - eps_out) / (eps_in + eps_out)
    d = z_hi - z_lo
    s = z0 - z_lo
    q1, x1, y1 = charges[0]
    F = 0.0
    for (qj, xj, yj) in charges:
        # lateral offsets of the copies of charge j seen from charge 1
        offs = []
        for i in range(-lateral, lateral + 1):
            for j in range(-lateral, lateral + 1):
                dx = xj + i * period - x1 if period > 0 else xj - x1
                dy = yj + j * period - y1 if period > 0 else yj - y1
                offs.append(dx * dx + dy * dy)
                if period <= 0:
                    break
            if period <= 0:
                break
        offs = np.array(offs)
        for m in range(-n_images, n_images + 1):
            # the reflected images m and 1 - m (mirror pairs about the slab's
            # centre) are kept or dropped together
            images = [(-s + 2 * m * d, Delta ** abs(2 * m - 1))] if m > -n_images else []
            if m != 0:
                images.append((s + 2 * m * d, Delta ** (2 * abs(m))))
            for zi, strength in images:
                h = s - zi
                F += q1 * qj * strength * h * float(np.sum((offs + h * h) ** -1.5))
    return F / (4.0 * math.pi * eps_in)
