"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle: these are textbook routes to the same
quantities (an FFT lattice Green's function and Poisson solver, a brute-force
lattice pair sum with analytic derivatives of the linear weights, an Ewald sum
for a periodic Coulomb pair, Watson's closed form of the cubic-lattice
integral).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, gamma


def lattice_symbol(L: int) -> np.ndarray:
    """sum_d 4 sin^2(k_d/2) on the L^3 grid of k = 2 pi m / L (index order [z, y, x])."""
    s = 4.0 * np.sin(np.pi * np.arange(L) / L) ** 2
    return s[:, None, None] + s[None, :, None] + s[None, None, :]


def green_table(L: int) -> np.ndarray:
    """Periodic lattice Green's function with the k = 0 mode removed, G[z, y, x], by FFT."""
    sym = lattice_symbol(L)
    ghat = np.zeros_like(sym)
    nz = sym > 0
    ghat[nz] = 1.0 / sym[nz]
    return np.real(np.fft.ifftn(ghat))


def watson_half() -> float:
    """Half of Watson's simple-cubic lattice integral (Watson 1939, closed form
    via Gamma functions); the L -> infinity limit of G(0)."""
    # (1/pi^3) int dk / (1 - (cos kx + cos ky + cos kz)/3) in closed form (Glasser & Zucker)
    W3 = math.sqrt(6.0) / (32.0 * math.pi ** 3) * gamma(1 / 24) * gamma(5 / 24) * gamma(7 / 24) * gamma(11 / 24)
    W = W3 / 3.0  # (1/pi^3) int dk / (3 - sum cos) = 0.50546...
    return W / 2.0


def to_zyx(field_flat: np.ndarray, L: int) -> np.ndarray:
    """Flat site array (x fastest) -> [z, y, x]."""
    return field_flat.reshape(L, L, L)


def fft_poisson_field(L: int, a: float, eps: float, rho_flat: np.ndarray, meanD: np.ndarray):
    """Link field E = -grad phi + meanD/eps of the lattice Poisson solution for
    vertex charges rho (uniform eps).  Returns a flat link array (3*L^3)."""
    rho = to_zyx(rho_flat, L)
    sym = lattice_symbol(L)
    ghat = np.zeros_like(sym)
    ghat[sym > 0] = 1.0 / sym[sym > 0]
    phi = np.real(np.fft.ifftn(np.fft.fftn(rho) * ghat)) / (eps * a)
    out = []
    for d, axis in ((0, 2), (1, 1), (2, 0)):
        grad = (np.roll(phi, -1, axis=axis) - phi) / a
        out.append((-grad + meanD[d] / eps).reshape(-1))
    return np.concatenate(out)


def cic_corners(r: np.ndarray, a: float, L: int):
    """Cell index, fractions, and the 8 corner weights and weight gradients."""
    t = r / a
    k = np.floor(t)
    f = t - k
    c = (k.astype(np.int64)) % L
    corners = []
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                o = np.array([ox, oy, oz])
                w1 = np.where(o == 1, f, 1.0 - f)
                dw1 = np.where(o == 1, 1.0, -1.0) / a
                w = np.prod(w1)
                grad = np.array([dw1[0] * w1[1] * w1[2], w1[0] * dw1[1] * w1[2], w1[0] * w1[1] * dw1[2]])
                corners.append(((c + o) % L, w, grad))
    return corners


def pair_sum_forces(L: int, a: float, eps: float, q: np.ndarray, r: np.ndarray) -> np.ndarray:
    """F_i = -d/dr_i sum_{j != i} q_i q_j/(eps a) sum_{v,v'} w_v(r_i) G(v - v') w_v'(r_j)
    by brute force with analytic derivatives of the linear weights."""
    G = green_table(L)
    n = len(q)
    corners = [cic_corners(r[i], a, L) for i in range(n)]
    F = np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            acc = np.zeros(3)
            for (vi, wi, gi) in corners[i]:
                for (vj, wj, gj) in corners[j]:
                    dz, dy, dx = (vi[2] - vj[2]) % L, (vi[1] - vj[1]) % L, (vi[0] - vj[0]) % L
                    acc += gi * wj * G[dz, dy, dx]
            F[i] -= q[i] * q[j] / (eps * a) * acc
    return F


def ewald_pair_force(box: float, q1: float, q2: float, r1, r2, eps: float = 1.0,
                     alpha: float | None = None, tol: float = 1e-14) -> np.ndarray:
    """Force on charge 1 from charge 2 and all periodic images of both, metallic
    boundary at infinity, Coulomb prefactor 1/(4 pi eps).  Cutoffs are raised
    until the result changes by less than tol."""
    if alpha is None:
        alpha = 5.0 / box
    dr = np.asarray(r1, float) - np.asarray(r2, float)
    V = box ** 3

    def real_part(nmax):
        s = np.zeros(3)
        rng = range(-nmax, nmax + 1)
        for nx in rng:
            for ny in rng:
                for nz in rng:
                    rv = dr + box * np.array([nx, ny, nz])
                    d = np.linalg.norm(rv)
                    s += (erfc(alpha * d) / d ** 2 + 2 * alpha / math.sqrt(math.pi) * math.exp(-(alpha * d) ** 2) / d) * rv / d
        return s

    def recip_part(mmax):
        s = np.zeros(3)
        rng = range(-mmax, mmax + 1)
        for mx in rng:
            for my in rng:
                for mz in rng:
                    if mx == 0 and my == 0 and mz == 0:
                        continue
                    k = 2 * math.pi / box * np.array([mx, my, mz])
                    k2 = k @ k
                    s += k / k2 * math.exp(-k2 / (4 * alpha ** 2)) * math.sin(k @ dr)
        return 4 * math.pi / V * s

    prev = None
    nmax = 1
    while True:
        tot = real_part(nmax) + recip_part(nmax + 2)
        if prev is not None and np.max(np.abs(tot - prev)) < tol * max(1.0, np.max(np.abs(tot))):
            break
        prev = tot
        nmax += 1
        if nmax > 8:
            break
    return q1 * q2 / (4 * math.pi * eps) * tot


def slab_self_force_k_integral(q: float, s: float, d: float, eps_in: float, eps_out: float) -> float:
    """z force on a charge q at distance s above the lower of two parallel
    interfaces a distance d apart (eps_in between them, eps_out outside), from
    the Fourier-Bessel form of its reflected potential: with
    D = (eps_in - eps_out)/(eps_in + eps_out), the self energy is
    W(s) = q^2/(8 pi eps_in) int_0^inf dk [D e^{-2ks} + D e^{-2k(d-s)} + 2 D^2 e^{-2kd}]
           / (1 - D^2 e^{-2kd}),
    and F = -dW/ds is integrated numerically (scipy quad), independently of any
    image sum."""
    from scipy.integrate import quad
    D = (eps_in - eps_out) / (eps_in + eps_out)

    def integrand(k):
        den = 1.0 - D * D * math.exp(-2.0 * k * d)
        return (-2.0 * k * D * math.exp(-2.0 * k * s) + 2.0 * k * D * math.exp(-2.0 * k * (d - s))) / den

    val, _ = quad(integrand, 0.0, math.inf, epsabs=1e-15, epsrel=1e-12, limit=400)
    return -q * q / (8.0 * math.pi * eps_in) * val
