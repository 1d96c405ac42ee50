// kernels_ions.hip -- per-ion kernels for gfx950: current deposition, charge
// assignment, dipole moment, corrected forces; deterministic finalisers of
// the per-block partial sums; the lattice Green's function table.
#include "device_util.hpp"
#include "memd_internal.hpp"

namespace memd {

// ----------------------------------------------------------- deposition

// Current assignment that keeps Gauss's law (eq. constraint): each ion moves
// by its displacement axis by axis (x, y, z), the others held at their
// current values.  Along the moving axis the path is cut at cell faces; the
// piece [ua, ub] inside cell kc carries the current q (ub - ua)/a onto the 4
// links of that cell along d with the transverse linear weights:
//   D_d(kc, c1 + o1, c2 + o2) -= q (ub - ua)/a * w(o1; f1) w(o2; f2) / a^2.
// Accumulation into D uses hardware float/double atomics (the lattice is
// sparse in ions, so contention is rare).  The block sums of q r^{n+1} (dipole)
// are written to partials[3*block].  When spread_rho is set the new charge
// assignment q w_v(r^{n+1}) is added to rho (FP64) for the Gauss audit.
template <typename T>
__global__ __launch_bounds__(256) void k_deposit(int n, int L, size_t Ns, double a,
                                                 const double *__restrict__ q, double *__restrict__ r,
                                                 const double *__restrict__ disp, T *__restrict__ D,
                                                 int spread_rho, double *__restrict__ rho,
                                                 double *__restrict__ partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double P[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const double qi = q[i];
        const double a2 = a * a;
        double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
            int c1, c2;
            double f1, f2;
            fold(u[d1], a, L, c1, f1);
            fold(u[d2], a, L, c2, f2);
            const double u0 = u[d];
            const double u1 = u0 + disp[3 * i + d];
            if (u1 != u0) {
                const double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
                const double sgn = u1 > u0 ? 1.0 : -1.0;
                const long long klo = (long long)floor(lo / a), khi = (long long)floor(hi / a);
                const int c1p = c1 + 1 == L ? 0 : c1 + 1, c2p = c2 + 1 == L ? 0 : c2 + 1;
                for (long long kc = klo; kc <= khi; ++kc) {
                    const double s0 = (double)kc * a, s1 = (double)(kc + 1) * a;
                    const double sa = lo > s0 ? lo : s0;
                    const double sb = hi < s1 ? hi : s1;
                    const double len = sb - sa;
                    if (!(len > 0.0)) continue;
                    const double amount = qi * sgn * (len / a) / a2;
                    long long km = kc % (long long)L;
                    if (km < 0) km += L;
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
        r[3 * i] = u[0];
        r[3 * i + 1] = u[1];
        r[3 * i + 2] = u[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) P[d] = qi * u[d];
        if (spread_rho) {
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
                unsafeAtomicAdd(&rho[site_index(xi, yi, zi, L)], qi * w);
            }
        }
    }
    block_sum<3>(P);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = P[0];
        partials[3 * blockIdx.x + 1] = P[1];
        partials[3 * blockIdx.x + 2] = P[2];
    }
}

static int ion_blocks(int n) { return n > 0 ? (n + kThreads - 1) / kThreads : 1; }

hipError_t launch_deposit(memd_ctx *c, void *D, const double *disp, bool spread_rho,
                          double *partials, int *nblk) {
    const int nb = ion_blocks(c->n);
    *nblk = nb;
    if (c->fp32)
        hipLaunchKernelGGL(k_deposit<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (float *)D, spread_rho ? 1 : 0, c->rho, partials);
    else
        hipLaunchKernelGGL(k_deposit<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (double *)D, spread_rho ? 1 : 0, c->rho, partials);
    return hipGetLastError();
}

// ------------------------------------------------------- charge assignment

// Linear assignment of each ion's charge (or of 1 when q is null) to the 8
// corners of its cell, added into dst (FP64 atomics).
__global__ __launch_bounds__(256) void k_spread(int n, int L, double a, const double *__restrict__ q,
                                                const double *__restrict__ r, double *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double qi = q ? q[i] : 1.0;
    int cc[3];
    double ff[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fold(r[3 * i + d], a, L, cc[d], ff[d]);
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

hipError_t launch_spread(memd_ctx *c, const double *charges_or_null, double *dst) {
    if (c->n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spread, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                       charges_or_null ? c->q : nullptr, c->r, dst);
    return hipGetLastError();
}

// ------------------------------------------------------------------ dipole

__global__ __launch_bounds__(256) void k_dipole(int n, const double *__restrict__ q,
                                                const double *__restrict__ r, double *partials) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double P[3] = {0.0, 0.0, 0.0};
    if (i < n) {
#pragma unroll
        for (int d = 0; d < 3; ++d) P[d] = q[i] * r[3 * i + d];
    }
    block_sum<3>(P);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = P[0];
        partials[3 * blockIdx.x + 1] = P[1];
        partials[3 * blockIdx.x + 2] = P[2];
    }
}

hipError_t launch_dipole(memd_ctx *c, double *partials, int *nblk) {
    const int nb = ion_blocks(c->n);
    *nblk = nb;
    hipLaunchKernelGGL(k_dipole, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->q, c->r, partials);
    return hipGetLastError();
}

// ------------------------------------------------------------------ forces

template <typename T>
struct ForceArgs {
    int n, L;
    size_t Ns;
    double a, V;
    const double *q, *r;
    const T *D, *eta_link, *eta_prof;
    double eta_uni;
    int mode;
    const double *scal;  // P, eps_h, G
    double *F;
    double *uself_partials;  // optional: per-block sums of the self energy
};

template <typename T>
__device__ __forceinline__ double eta_f(const ForceArgs<T> &A, int d, int k, size_t off) {
    if (A.mode == ETA_UNIFORM) return A.eta_uni;
    if (A.mode == ETA_ZPROF) return (double)A.eta_prof[d * A.L + k];
    return (double)A.eta_link[(size_t)d * A.Ns + off];
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

// F_i = q_i sum_{4 d-links of the cell} w w E_d  (eq. force without v x B; F = +qE)
//       - F_self (lattice Green's-function self force, eps_cell = harmonic mean
//         of the cell's 12 edges)
//       + q_i P_d / (V eps_h_d)  (dipole correction, section "Periodicity").
template <typename T>
__global__ __launch_bounds__(256) void k_forces(ForceArgs<T> A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double us = 0.0;
    if (i < A.n) {
        const int L = A.L;
        int c[3];
        double f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) fold(A.r[3 * i + d], A.a, L, c[d], f[d]);
        const int cp[3] = {c[0] + 1 == L ? 0 : c[0] + 1, c[1] + 1 == L ? 0 : c[1] + 1,
                           c[2] + 1 == L ? 0 : c[2] + 1};
        const double qi = A.q[i];
        double Flat[3];
        double etasum = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
            double s = 0.0;
#pragma unroll
            for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                for (int o1 = 0; o1 < 2; ++o1) {
                    int x[3] = {c[0], c[1], c[2]};
                    x[d1] = o1 ? cp[d1] : c[d1];
                    x[d2] = o2 ? cp[d2] : c[d2];
                    const size_t off = site_index(x[0], x[1], x[2], L);
                    const double e = eta_f(A, d, x[2], off);
                    etasum += e;
                    s += lin_w(o1, f[d1]) * lin_w(o2, f[d2]) * (e * (double)A.D[(size_t)d * A.Ns + off]);
                }
            Flat[d] = qi * s;
        }
        const double eps_cell = 12.0 / etasum;
        double S, dS[3];
        self_sum(A.scal + S_G, f, S, dS);
        const double pref = qi * qi / (2.0 * eps_cell * A.a);
        us = pref * S;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double Fself = -pref * dS[d] / A.a;
            A.F[3 * i + d] = Flat[d] - Fself + qi * A.scal[S_P + d] / (A.V * A.scal[S_EPSH + d]);
        }
    }
    if (A.uself_partials) {
        double s[1] = {us};
        block_sum<1>(s);
        if (threadIdx.x == 0) A.uself_partials[blockIdx.x] = s[0];
    }
}

template <typename T>
static ForceArgs<T> force_args(memd_ctx *c, const void *D) {
    ForceArgs<T> A;
    A.n = c->n;
    A.L = c->L;
    A.Ns = c->Ns;
    A.a = c->a;
    A.V = c->V;
    A.q = c->q;
    A.r = c->r;
    A.D = (const T *)D;
    A.eta_link = (const T *)c->eta_link;
    A.eta_prof = (const T *)c->eta_prof;
    A.eta_uni = c->eta_uni;
    A.mode = c->eta_mode;
    A.scal = c->scal;
    A.F = c->F;
    A.uself_partials = nullptr;
    return A;
}

hipError_t launch_forces(memd_ctx *c, const void *D) {
    if (c->n == 0) return hipSuccess;
    const int nb = ion_blocks(c->n);
    if (c->fp32)
        hipLaunchKernelGGL(k_forces<float>, dim3(nb), dim3(kThreads), 0, c->stream, force_args<float>(c, D));
    else
        hipLaunchKernelGGL(k_forces<double>, dim3(nb), dim3(kThreads), 0, c->stream, force_args<double>(c, D));
    return hipGetLastError();
}

// Self energies (through the force kernel, writing the same forces again).
hipError_t launch_uself(memd_ctx *c, double *partials, int *nblk) {
    const int nb = ion_blocks(c->n);
    *nblk = nb;
    const void *D = c->D[c->cur];
    if (c->fp32) {
        auto A = force_args<float>(c, D);
        A.uself_partials = partials;
        hipLaunchKernelGGL(k_forces<float>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    } else {
        auto A = force_args<double>(c, D);
        A.uself_partials = partials;
        hipLaunchKernelGGL(k_forces<double>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- finalisers

// One block of 256 threads sums `width` values per partial block; thread t
// takes blocks t, t+256, ... in order, then the block tree reduces: the
// order is fixed, so results repeat bit for bit.
template <int W>
__device__ void fin_sum(const double *partials, int nblk, double (&out)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) out[w] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] += partials[W * b + w];
    block_sum<W>(out);
}

__global__ void k_fin_dipole(const double *partials, int nblk, double *P) {
    double s[3];
    fin_sum<3>(partials, nblk, s);
    if (threadIdx.x == 0) {
        P[0] = s[0];
        P[1] = s[1];
        P[2] = s[2];
    }
}

hipError_t launch_finalize_dipole(hipStream_t s, const double *partials, int nblk, double *P) {
    hipLaunchKernelGGL(k_fin_dipole, dim3(1), dim3(kThreads), 0, s, partials, nblk, P);
    return hipGetLastError();
}

__global__ void k_fin_sum(const double *partials, int nblk, int width, double *dst) {
    for (int w = 0; w < width; ++w) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partials[width * b + w];
        double v[1] = {s};
        block_sum<1>(v);
        if (threadIdx.x == 0) dst[w] = v[0];
    }
}

hipError_t launch_finalize_sum(hipStream_t s, const double *partials, int nblk, int width, double *dst) {
    hipLaunchKernelGGL(k_fin_sum, dim3(1), dim3(kThreads), 0, s, partials, nblk, width, dst);
    return hipGetLastError();
}

__global__ void k_fin_audit(const double *partials, int nblk, double Ns, double *dst, double *hist) {
    double mx = 0.0, ss = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        mx = fmax(mx, partials[2 * b]);
        ss += partials[2 * b + 1];
    }
    double v[1] = {ss};
    block_sum<1>(v);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        dst[0] = m;
        dst[1] = sqrt(v[0] / Ns);
        if (hist) {
            hist[0] = m;
            hist[1] = dst[1];
        }
    }
}

hipError_t launch_finalize_audit(hipStream_t s, const double *partials, int nblk, double Ns, double *dst,
                                 double *hist) {
    hipLaunchKernelGGL(k_fin_audit, dim3(1), dim3(kThreads), 0, s, partials, nblk, Ns, dst, hist);
    return hipGetLastError();
}

__global__ void k_fin_energy(const double *fpart, int fblk, const double *ipart, int iblk, double a3,
                             double c2, double V, const double *scal, double *dst, double *hist) {
    double s[2];
    fin_sum<2>(fpart, fblk, s);
    double u[1];
    fin_sum<1>(ipart, iblk, u);
    if (threadIdx.x == 0) {
        const double we = 0.5 * a3 * s[0];
        const double wb = 0.5 * c2 * a3 * s[1];
        double ud = 0.0;
        for (int d = 0; d < 3; ++d) ud += scal[S_P + d] * scal[S_P + d] / (2.0 * V * scal[S_EPSH + d]);
        const double e[5] = {we, wb, u[0], ud, we + wb - u[0] - ud};
        for (int t = 0; t < 5; ++t) {
            dst[t] = e[t];
            if (hist) hist[t] = e[t];
        }
    }
}

hipError_t launch_finalize_energy(memd_ctx *c, const double *fpart, int fblk, const double *ipart, int iblk,
                                  double *dst, double *hist) {
    const double a3 = c->a * c->a * c->a;
    hipLaunchKernelGGL(k_fin_energy, dim3(1), dim3(kThreads), 0, c->stream, fpart, fblk, ipart, iblk, a3,
                       c->c * c->c, c->V, c->scal, dst, hist);
    return hipGetLastError();
}

__global__ void k_fin_epsh4(const double *partials, int nblk, double Ns, double *epsh, double *etamax) {
    double s[3] = {0.0, 0.0, 0.0};
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        s[0] += partials[4 * b];
        s[1] += partials[4 * b + 1];
        s[2] += partials[4 * b + 2];
        mx = fmax(mx, partials[4 * b + 3]);
    }
    block_sum<3>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        epsh[0] = Ns / s[0];
        epsh[1] = Ns / s[1];
        epsh[2] = Ns / s[2];
        *etamax = m;
    }
}

hipError_t launch_finalize_epsh(hipStream_t s, const double *partials, int nblk, double Ns, double *epsh,
                                double *etamax) {
    hipLaunchKernelGGL(k_fin_epsh4, dim3(1), dim3(kThreads), 0, s, partials, nblk, Ns, epsh, etamax);
    return hipGetLastError();
}

}  // namespace memd
