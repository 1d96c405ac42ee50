// ion_ops.hpp -- per-ion device operations shared by the single-system and
// the batched replica kernels: the current deposit of one ion's move and the
// corrected force on one ion.
#pragma once

#include "device_util.hpp"
#include "memd_internal.hpp"

namespace memd {

// Permittivity seen by the ion kernels: one value, a per-plane profile, or
// one value per link.
template <typename T>
struct EtaView {
    int mode;
    double uni;
    const T *prof;  // [3L]
    const T *link;  // [3Ns]
    __device__ __forceinline__ double at(int d, int k, size_t off, int L, size_t Ns) const {
        if (mode == ETA_UNIFORM) return uni;
        if (mode == ETA_ZPROF) return (double)prof[d * L + k];
        return (double)link[(size_t)d * Ns + off];
    }
};

// A displacement component that is not finite or longer than (L + 1024) a is
// not a move the method can take in one step: it is replaced by 0 and counted
// in *bad (when given), which bounds every face-crossing loop.
__device__ __forceinline__ void sanitize_move(double (&du)[3], double a, int L, unsigned int *bad) {
    const double lim = ((double)L + 1024.0) * a;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (!(fabs(du[d]) <= lim)) {
            du[d] = 0.0;
            if (bad) atomicAdd(bad, 1u);
        }
}

// Current assignment that keeps Gauss's law (eq. constraint): the ion moves by
// du axis by axis (x, y, z), the others held at their current values.  Along
// the moving axis the path is cut at cell faces; the piece [ua, ub] inside
// cell kc carries the current q (ub - ua)/a onto the 4 links of that cell
// along d with the transverse linear weights:
//   D_d(kc, c1 + o1, c2 + o2) -= q (ub - ua)/a * w(o1; f1) w(o2; f2) / a^2.
// u is updated in place.  Accumulation uses hardware float/double atomics.
template <typename T>
__device__ __forceinline__ void deposit_ion(int L, size_t Ns, double a, double qi, double (&u)[3],
                                            const double (&du)[3], T *__restrict__ D) {
    const double a2 = a * a;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
        int c1, c2;
        double f1, f2;
        fold(u[d1], a, L, c1, f1);
        fold(u[d2], a, L, c2, f2);
        const double u0 = u[d];
        const double u1 = u0 + du[d];
        if (u1 != u0) {
            const double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
            const double sgn = u1 > u0 ? 1.0 : -1.0;
            const double klo = floor(div_a(lo, a)), khi = floor(div_a(hi, a));
            const int c1p = c1 + 1 == L ? 0 : c1 + 1, c2p = c2 + 1 == L ? 0 : c2 + 1;
            for (double kc = klo; kc <= khi; kc += 1.0) {
                const double s0 = kc * a, s1 = (kc + 1.0) * a;
                const double sa = lo > s0 ? lo : s0;
                const double sb = hi < s1 ? hi : s1;
                const double len = sb - sa;
                if (!(len > 0.0)) continue;
                const double amount = div_a(qi * sgn * div_a(len, a), a2);
                const int km = mod_cell(kc, L);
                int x[3];
                x[d] = (int)km;
#pragma unroll
                for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 2; ++o1) {
                        x[d1] = o1 ? c1p : c1;
                        x[d2] = o2 ? c2p : c2;
                        const double val = amount * lin_w(o1, f1) * lin_w(o2, f2);
                        unsafeAtomicAdd(&D[(size_t)d * Ns + site_index(x[0], x[1], x[2], L)], (T)(-val));
                    }
            }
        }
        u[d] = u1;
    }
}

// One lane's share of deposit_ion: the same dimension-split walk, but only the
// links of axis `dm` with transverse corner (o1, o2) = (corner & 1, corner >> 1)
// are updated.  Sixteen lanes per ion (dm = 0..2, corner = 0..3; dm = 3 idle)
// together make every update of deposit_ion, with u advanced identically in
// all of them.
template <typename T>
__device__ __forceinline__ void deposit_ion_part(int L, size_t Ns, double a, double qi, double (&u)[3],
                                                 const double (&du)[3], T *__restrict__ D, int dm,
                                                 int corner) {
    const double a2 = a * a;
    const int o1 = corner & 1, o2 = corner >> 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u0 = u[d];
        const double u1 = u0 + du[d];
        if (d == dm && u1 != u0) {
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
            int c1, c2;
            double f1, f2;
            fold(u[d1], a, L, c1, f1);
            fold(u[d2], a, L, c2, f2);
            const int x1 = o1 ? (c1 + 1 == L ? 0 : c1 + 1) : c1;
            const int x2 = o2 ? (c2 + 1 == L ? 0 : c2 + 1) : c2;
            const double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
            const double sgn = u1 > u0 ? 1.0 : -1.0;
            const double klo = floor(div_a(lo, a)), khi = floor(div_a(hi, a));
            for (double kc = klo; kc <= khi; kc += 1.0) {
                const double s0 = kc * a, s1 = (kc + 1.0) * a;
                const double sa = lo > s0 ? lo : s0;
                const double sb = hi < s1 ? hi : s1;
                const double len = sb - sa;
                if (!(len > 0.0)) continue;
                const double amount = div_a(qi * sgn * div_a(len, a), a2);
                const int km = mod_cell(kc, L);
                int x[3];
                x[d] = (int)km;
                x[d1] = x1;
                x[d2] = x2;
                const double val = amount * lin_w(o1, f1) * lin_w(o2, f2);
                unsafeAtomicAdd(&D[(size_t)d * Ns + site_index(x[0], x[1], x[2], L)], (T)(-val));
            }
        }
        u[d] = u1;
    }
}

// Linear assignment of charge qi at u to the 8 corners of its cell (FP64 atomics).
__device__ __forceinline__ void spread_ion(int L, double a, double qi, const double (&u)[3],
                                           double *__restrict__ dst) {
    int cc[3];
    double ff[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fold(u[d], a, L, cc[d], ff[d]);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        const double w = lin_w(ox, ff[0]) * lin_w(oy, ff[1]) * lin_w(oz, ff[2]);
        const int xi = ox ? (cc[0] + 1 == L ? 0 : cc[0] + 1) : cc[0];
        const int yi = oy ? (cc[1] + 1 == L ? 0 : cc[1] + 1) : cc[1];
        const int zi = oz ? (cc[2] + 1 == L ? 0 : cc[2] + 1) : cc[2];
        unsafeAtomicAdd(&dst[site_index(xi, yi, zi, L)], qi * w);
    }
}

// The current of one ion's move (deposit_ion's arithmetic, every axis and
// transverse corner) restricted to the links whose site lies in the box
// org + [0, ext), which does not wrap, added into acc[d][z][y][x] (relative
// to org) with LDS atomics.  u is moved in place.
template <typename T, int NZ, int NY>
__device__ __forceinline__ void deposit_ion_box(int L, double a, double qi, double (&u)[3], const double (&du)[3],
                                                const int (&org)[3], const int (&ext)[3], T (*acc)[NZ][NY][64]) {
    const double a2 = a * a;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u0 = u[d];
        const double u1 = u0 + du[d];
        if (u1 != u0) {
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
            int c1, c2;
            double f1, f2;
            fold(u[d1], a, L, c1, f1);
            fold(u[d2], a, L, c2, f2);
            const double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
            const double sgn = u1 > u0 ? 1.0 : -1.0;
            const double klo = floor(div_a(lo, a)), khi = floor(div_a(hi, a));
#pragma unroll
            for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                for (int o1 = 0; o1 < 2; ++o1) {
                    const int x1 = o1 ? (c1 + 1 == L ? 0 : c1 + 1) : c1;
                    const int x2 = o2 ? (c2 + 1 == L ? 0 : c2 + 1) : c2;
                    const int l1 = x1 - org[d1], l2 = x2 - org[d2];
                    if ((unsigned)l1 >= (unsigned)ext[d1] || (unsigned)l2 >= (unsigned)ext[d2]) continue;
                    for (double kc = klo; kc <= khi; kc += 1.0) {
                        const int ld = mod_cell(kc, L) - org[d];
                        if ((unsigned)ld >= (unsigned)ext[d]) continue;
                        const double s0 = kc * a, s1 = (kc + 1.0) * a;
                        const double sa = lo > s0 ? lo : s0;
                        const double sb = hi < s1 ? hi : s1;
                        const double len = sb - sa;
                        if (!(len > 0.0)) continue;
                        const double amount = div_a(qi * sgn * div_a(len, a), a2);
                        const double val = amount * lin_w(o1, f1) * lin_w(o2, f2);
                        int l[3];
                        l[d] = ld;
                        l[d1] = l1;
                        l[d2] = l2;
                        atomicAdd(&acc[d][l[2]][l[1]][l[0]], (T)(-val));
                    }
                }
        }
        u[d] = u1;
    }
}

// Cell self-energy sum S(f) = sum_{o,o'} w_o w_o' G(o - o') and its gradient:
// per axis, equal corners weigh alpha = 1 - beta, different corners
// beta = 2 f (1 - f); G depends on the number of differing axes.
__device__ __forceinline__ void self_sum(const double *G, const double f[3], double &S, double dS[3]) {
    double be[3], al[3], db[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        be[d] = 2.0 * f[d] * (1.0 - f[d]);
        al[d] = 1.0 - be[d];
        db[d] = 2.0 - 4.0 * f[d];
    }
    S = 0.0;
    dS[0] = dS[1] = dS[2] = 0.0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int m0 = m & 1, m1 = (m >> 1) & 1, m2 = m >> 2;
        const double g = G[m0 + m1 + m2];
        const double f0 = m0 ? be[0] : al[0], f1 = m1 ? be[1] : al[1], f2 = m2 ? be[2] : al[2];
        const double g0 = m0 ? db[0] : -db[0], g1 = m1 ? db[1] : -db[1], g2 = m2 ? db[2] : -db[2];
        S += g * f0 * f1 * f2;
        dS[0] += g * g0 * f1 * f2;
        dS[1] += g * f0 * g1 * f2;
        dS[2] += g * f0 * f1 * g2;
    }
}

// Corrected force on one ion (eq. force without v x B; F = +q E):
//   q sum_{4 d-links of the cell} w w eta_d D_d
//   - F_self: the lattice Green's-function self force with eps_cell = the
//     harmonic mean of the cell's 12 edges, or, with direct, the direct
//     subtraction (section "Self energy interaction"): the ion's own
//     assigned charges produce on the cell's d-link with transverse corner
//     offsets (o1, o2) the homogeneous-lattice field
//       D_self = -(q/a^2) (1 - 2 f_d) X,  X = sum_{k1,k2} p1(k1) p2(k2) (G[k1+k2+1] - G[k1+k2])
//     (p(0) = w(o; f), the charge on the link's own side of the transverse
//     axis; p(1) = 1 - w(o; f)), and F_self_d = q sum w w eta_link D_self
//   + q P_d / (V eps_h_d)   (dipole correction, section "Periodicity").
// Returns the ion's self energy (the Green's-function form in both cases).
template <typename T>
__device__ __forceinline__ double force_ion(int L, size_t Ns, double a, double V, double qi,
                                            const double (&u)[3], const T *__restrict__ D,
                                            const EtaView<T> &eta, const double *G, const double *P,
                                            const double *epsh, double (&F)[3], bool direct = false) {
    int c[3];
    double f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fold(u[d], a, L, c[d], f[d]);
    const int cp[3] = {c[0] + 1 == L ? 0 : c[0] + 1, c[1] + 1 == L ? 0 : c[1] + 1, c[2] + 1 == L ? 0 : c[2] + 1};
    double Flat[3], Fdir[3];
    double etasum = 0.0;
    const double dG0 = G[1] - G[0], dG1 = G[2] - G[1], dG2 = G[3] - G[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
        double s = 0.0, sd = 0.0;
#pragma unroll
        for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
            for (int o1 = 0; o1 < 2; ++o1) {
                int x[3] = {c[0], c[1], c[2]};
                x[d1] = o1 ? cp[d1] : c[d1];
                x[d2] = o2 ? cp[d2] : c[d2];
                const size_t off = site_index(x[0], x[1], x[2], L);
                const double e = eta.at(d, x[2], off, L, Ns);
                etasum += e;
                const double w1 = lin_w(o1, f[d1]), w2 = lin_w(o2, f[d2]);
                s += w1 * w2 * (e * (double)D[(size_t)d * Ns + off]);
                if (direct) {
                    const double X = w1 * w2 * dG0 + (w1 * (1.0 - w2) + (1.0 - w1) * w2) * dG1 +
                                     (1.0 - w1) * (1.0 - w2) * dG2;
                    sd += w1 * w2 * e * X;
                }
            }
        Flat[d] = qi * s;
        Fdir[d] = -div_a(div_a(qi * qi * (1.0 - 2.0 * f[d]) * sd, a), a);
    }
    const double eps_cell = 12.0 / etasum;
    double S, dS[3];
    self_sum(G, f, S, dS);
    const double pref = qi * qi / (2.0 * eps_cell * a);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double Fself = direct ? Fdir[d] : div_a(-pref * dS[d], a);
        F[d] = Flat[d] - Fself + qi * P[d] / (V * epsh[d]);
    }
    return pref * S;
}

// Self energies U_i = q_i^2 S(f_i) / (2 eps_cell a) (section "Self energy
// interaction"), eps_cell = 12 / (sum of eta over the cell's 12 edges), with
// the arithmetic of force_ion but no field read: the partial of block b of
// nb (256 threads; the ions of the block as k_forces groups them, so the sum
// is deterministic) into partials[b].
struct SelfEnergyArgs {
    int n, nb;
    double a;
    const double *q, *r, *G;
    double *partials;
};

template <typename T>
__device__ __forceinline__ void self_energy_block(int b, const SelfEnergyArgs &U, int L, size_t Ns,
                                                  const EtaView<T> &eta) {
    const int i = xcd_logical(b, U.nb) * blockDim.x + threadIdx.x;
    double us = 0.0;
    if (i < U.n) {
        const double u[3] = {U.r[3 * i], U.r[3 * i + 1], U.r[3 * i + 2]};
        const double qi = U.q[i];
        int c[3];
        double f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) fold(u[d], U.a, L, c[d], f[d]);
        const int cp[3] = {c[0] + 1 == L ? 0 : c[0] + 1, c[1] + 1 == L ? 0 : c[1] + 1, c[2] + 1 == L ? 0 : c[2] + 1};
        double etasum = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
#pragma unroll
            for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                for (int o1 = 0; o1 < 2; ++o1) {
                    int x[3] = {c[0], c[1], c[2]};
                    x[d1] = o1 ? cp[d1] : c[d1];
                    x[d2] = o2 ? cp[d2] : c[d2];
                    etasum += eta.at(d, x[2], site_index(x[0], x[1], x[2], L), L, Ns);
                }
        }
        const double eps_cell = 12.0 / etasum;
        double S, dS[3];
        self_sum(U.G, f, S, dS);
        us = qi * qi / (2.0 * eps_cell * U.a) * S;
    }
    double v[1] = {us};
    block_sum<1>(v);
    if (threadIdx.x == 0) U.partials[b] = v[0];
}

}  // namespace memd
