// kernels_solve.hip -- the initial solution of Gauss's law on the GPU, FP64:
// plane -> line -> vertex recursion (Fig. 1), the uniform mode set to -P/V
// (section "Periodicity"), and the relaxation to curl E = 0 by minimising the
// field energy over D + C^T theta (conjugate gradients on C eta C^T theta =
// -C eta D; D is updated in place of theta), preconditioned by the inverse
// lattice Laplacian through 3-D FFTs when L is a power of two up to 1024,
// else by the diagonal.
// For a uniform or planar permittivity the same minimiser is computed
// directly (a 2-D DFT and one tridiagonal solve per mode).  Also the
// periodic lattice Green's function used by the self-energy correction
// (eq. greens and the Brillouin-zone sum that follows it).
#include "device_util.hpp"
#include "memd_internal.hpp"

#include <algorithm>
#include <cmath>

namespace memd {

// ----------------------------------------------------------- recursion

// Q[k] = sum over plane k of rho (one block per plane).
__global__ __launch_bounds__(256) void k_plane_sum(const double *__restrict__ rho, int L, double *Q) {
    const int k = blockIdx.x;
    const size_t LL = (size_t)L * L;
    double s[1] = {0.0};
    for (size_t t = threadIdx.x; t < LL; t += blockDim.x) s[0] += rho[(size_t)k * LL + t];
    block_sum<1>(s);
    if (threadIdx.x == 0) Q[k] = s[0];
}

// qbar_k = Q_k / L^2; Dz_k = (sum_{k' <= k} qbar_k') / a^2 (one thread).
__global__ void k_zprefix(const double *Q, int L, double a2, double *qbar, double *dz) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double run = 0.0;
    for (int k = 0; k < L; ++k) {
        const double qp = Q[k] / ((double)L * L);
        qbar[k] = qp;
        run += qp;
        dz[k] = run / a2;
    }
}

// qline[j,k] = sum_i (rho - qbar_k) / L   (one thread per line).
__global__ void k_line_sum(const double *__restrict__ rho, const double *__restrict__ qbar, int L,
                           double *qline) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L * L) return;
    const int k = t / L;
    const double qb = qbar[k];
    const size_t base = (size_t)t * L;
    double s = 0.0;
    for (int i = 0; i < L; ++i) s += rho[base + i] - qb;
    qline[t] = s / (double)L;
}

// Dy[j,k] = (sum_{j' <= j} qline[j',k]) / a^2   (one thread per plane).
__global__ void k_yprefix(const double *__restrict__ qline, int L, double a2, double *dy) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L) return;
    double run = 0.0;
    for (int j = 0; j < L; ++j) {
        run += qline[(size_t)k * L + j];
        dy[(size_t)k * L + j] = run / a2;
    }
}

// Per line (j,k): D_z, D_y from the prefixes; D_x from the running sum over i
// of the remaining vertex charge rho - qbar_k - qline_jk.
__global__ void k_row_fill(const double *__restrict__ rho, const double *__restrict__ qbar,
                           const double *__restrict__ qline, const double *__restrict__ dz,
                           const double *__restrict__ dy, int L, double a2, double *D) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L * L) return;
    const size_t Ns = (size_t)L * L * L;
    const int k = t / L;
    const double qb = qbar[k], ql = qline[t], vz = dz[k], vy = dy[t];
    const size_t base = (size_t)t * L;
    double run = 0.0;
    for (int i = 0; i < L; ++i) {
        const double rem = (rho[base + i] - qb) - ql;
        run += rem;
        D[base + i] = run / a2;
        D[Ns + base + i] = vy;
        D[2 * Ns + base + i] = vz;
    }
}

hipError_t solve_recursion(memd_ctx *c, double *D) {
    hipError_t e;
    const int L = c->L;
    const double a2 = c->a * c->a;
    // rho <- charge assignment of the ions
    if ((e = launch_spread_dense(c, true, c->rho)) != hipSuccess) return e;
    double *w = nullptr;
    const size_t LL = (size_t)L * L;
    if ((e = hipMallocAsync((void **)&w, (3 * L + 2 * LL) * sizeof(double), c->stream)) != hipSuccess) return e;
    double *Q = w, *qbar = w + L, *dz = w + 2 * L, *qline = w + 3 * L, *dy = w + 3 * L + LL;
    hipLaunchKernelGGL(k_plane_sum, dim3(L), dim3(kThreads), 0, c->stream, c->rho, L, Q);
    hipLaunchKernelGGL(k_zprefix, dim3(1), dim3(64), 0, c->stream, Q, L, a2, qbar, dz);
    const int nl = (int)((LL + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_line_sum, dim3(nl), dim3(kThreads), 0, c->stream, c->rho, qbar, L, qline);
    hipLaunchKernelGGL(k_yprefix, dim3((L + 63) / 64), dim3(64), 0, c->stream, qline, L, a2, dy);
    hipLaunchKernelGGL(k_row_fill, dim3(nl), dim3(kThreads), 0, c->stream, c->rho, qbar, qline, dz, dy, L,
                       a2, D);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipFreeAsync(w, c->stream);
}

// ----------------------------------------------------------- mean shift

__global__ __launch_bounds__(256) void k_dsum(const double *__restrict__ D, size_t Ns, double *partials) {
    double s[3] = {0.0, 0.0, 0.0};
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
        s[0] += D[v];
        s[1] += D[Ns + v];
        s[2] += D[2 * Ns + v];
    }
    block_sum<3>(s);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = s[0];
        partials[3 * blockIdx.x + 1] = s[1];
        partials[3 * blockIdx.x + 2] = s[2];
    }
}

// D_d += -P_d / V - sum_d / Ns
__global__ void k_shift(double *D, size_t Ns, const double *sums, const double *P, double V) {
    __shared__ double sh[3];
    if (threadIdx.x < 3) sh[threadIdx.x] = -P[threadIdx.x] / V - sums[threadIdx.x] / (double)Ns;
    __syncthreads();
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < 3 * Ns;
         t += (size_t)gridDim.x * blockDim.x)
        D[t] += sh[t / Ns];
}

static int red_blocks(size_t Ns) {
    size_t b = (Ns + kThreads - 1) / kThreads;
    return (int)(b < (size_t)kRedBlocks ? b : (size_t)kRedBlocks);
}

hipError_t solve_mean_shift(memd_ctx *c, double *D) {
    hipError_t e;
    int nb = 0;
    if ((e = launch_dipole(c, c->partials, &nb)) != hipSuccess) return e;
    if ((e = launch_finalize_dipole(c->stream, c->partials, nb, c->scal + S_P)) != hipSuccess) return e;
    const int nr = red_blocks(c->Ns);
    hipLaunchKernelGGL(k_dsum, dim3(nr), dim3(kThreads), 0, c->stream, D, c->Ns, c->partials);
    if ((e = launch_finalize_sum(c->stream, c->partials, nr, 3, c->scal + S_MEAN)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_shift, dim3(red_blocks(3 * c->Ns)), dim3(kThreads), 0, c->stream, D, c->Ns,
                       c->scal + S_MEAN, c->scal + S_P, c->V);
    return hipGetLastError();
}

// ------------------------------------------------------------ relaxation

struct CgArgs {
    int L;
    size_t Ns;
    double inv_a;
    const double *eta;  // FP64 eta [3Ns] (expanded for the solve)
};

__device__ __forceinline__ void site_ijk(size_t v, int L, int &i, int &j, int &k) {
    i = (int)(v % L);
    j = (int)((v / L) % L);
    k = (int)(v / ((size_t)L * L));
}

// out = sgn * C(eta * X) (plaquettes); optional partials: max|out| and max|eta X|,
// or the dot <p, out>.
template <bool WITH_MAX, bool WITH_DOT>
__global__ __launch_bounds__(256) void k_curl_eta(CgArgs A, const double *__restrict__ X, double sgn,
                                                  double *__restrict__ out, const double *__restrict__ p,
                                                  double *partials, const int *stop) {
    if (stop && *stop) return;
    const int L = A.L;
    const size_t Ns = A.Ns;
    double m1 = 0.0, m2 = 0.0, dot = 0.0;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
        int i, j, k;
        site_ijk(v, L, i, j, k);
        const size_t vx = site_index(i + 1 == L ? 0 : i + 1, j, k, L);
        const size_t vy = site_index(i, j + 1 == L ? 0 : j + 1, k, L);
        const size_t vz = site_index(i, j, k + 1 == L ? 0 : k + 1, L);
        auto Xe = [&](int d, size_t s) { return A.eta[(size_t)d * Ns + s] * X[(size_t)d * Ns + s]; };
        const double x0 = Xe(0, v), x1 = Xe(1, v), x2 = Xe(2, v);
        const double cx = (Xe(2, vy) - x2 - Xe(1, vz) + x1) * A.inv_a;
        const double cy = (Xe(0, vz) - x0 - Xe(2, vx) + x2) * A.inv_a;
        const double cz = (Xe(1, vx) - x1 - Xe(0, vy) + x0) * A.inv_a;
        const double o0 = sgn * cx, o1 = sgn * cy, o2 = sgn * cz;
        out[v] = o0;
        out[Ns + v] = o1;
        out[2 * Ns + v] = o2;
        if (WITH_MAX) {
            m1 = fmax(m1, fmax(fabs(o0), fmax(fabs(o1), fabs(o2))));
            m2 = fmax(m2, fmax(fabs(x0), fmax(fabs(x1), fabs(x2))));
        }
        if (WITH_DOT) dot += p[v] * o0 + p[Ns + v] * o1 + p[2 * Ns + v] * o2;
    }
    if (WITH_MAX) {
        const double a1 = block_max(m1);
        const double a2 = block_max(m2);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = a1;
            partials[2 * blockIdx.x + 1] = a2;
        }
    }
    if (WITH_DOT) {
        double s[1] = {dot};
        block_sum<1>(s);
        if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
    }
}

// w = C^T p (links)
__global__ __launch_bounds__(256) void k_curl_adj(CgArgs A, const double *__restrict__ p,
                                                  double *__restrict__ w, const int *stop) {
    if (stop && *stop) return;
    const int L = A.L;
    const size_t Ns = A.Ns;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
        int i, j, k;
        site_ijk(v, L, i, j, k);
        const size_t vx = site_index(i == 0 ? L - 1 : i - 1, j, k, L);
        const size_t vy = site_index(i, j == 0 ? L - 1 : j - 1, k, L);
        const size_t vz = site_index(i, j, k == 0 ? L - 1 : k - 1, L);
        const double p0 = p[v], p1 = p[Ns + v], p2 = p[2 * Ns + v];
        w[v] = (p2 - p[2 * Ns + vy] - p1 + p[Ns + vz]) * A.inv_a;
        w[Ns + v] = (p0 - p[vz] - p2 + p[2 * Ns + vx]) * A.inv_a;
        w[2 * Ns + v] = (p1 - p[Ns + vx] - p0 + p[vy]) * A.inv_a;
    }
}

// dinv = a^2 / (sum of eta on the 4 links of each plaquette)
__global__ void k_dinv(CgArgs A, double a2, double *dinv) {
    const int L = A.L;
    const size_t Ns = A.Ns;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
        int i, j, k;
        site_ijk(v, L, i, j, k);
        const size_t vx = site_index(i + 1 == L ? 0 : i + 1, j, k, L);
        const size_t vy = site_index(i, j + 1 == L ? 0 : j + 1, k, L);
        const size_t vz = site_index(i, j, k + 1 == L ? 0 : k + 1, L);
        const double *e = A.eta;
        dinv[v] = a2 / (e[2 * Ns + vy] + e[2 * Ns + v] + e[Ns + vz] + e[Ns + v]);
        dinv[Ns + v] = a2 / (e[vz] + e[v] + e[2 * Ns + vx] + e[2 * Ns + v]);
        dinv[2 * Ns + v] = a2 / (e[Ns + vx] + e[Ns + v] + e[vy] + e[v]);
    }
}

// z = dinv * r; partial <r, z>
__global__ __launch_bounds__(256) void k_precond(const double *__restrict__ dinv, const double *__restrict__ r,
                                                 double *__restrict__ z, size_t M, double *partials) {
    double s[1] = {0.0};
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < M; t += (size_t)gridDim.x * blockDim.x) {
        const double zz = dinv[t] * r[t];
        z[t] = zz;
        s[0] += r[t] * zz;
    }
    block_sum<1>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

// ---------------------------------------------- spectral preconditioner
//
// On plaquette fields in the range of C (the only ones the iteration sees:
// the right-hand side and every C eta w are curls), C C^T is the lattice
// Laplacian -Delta acting on each component alike: in Fourier space its
// symbol is |kappa|^2 = sum_d 4 sin^2(pi m_d / L) / a^2.  z = (-Delta)^{-1} r
// is therefore the exact inverse of C eta C^T for a uniform eta (up to the
// scale, which conjugate gradients do not see), and for a varying eta the
// preconditioned operator's condition number is at most max eta / min eta.
// The three components go through two complex transforms: r_x + i r_y
// (the symbol is real and even, so real and imaginary parts stay apart) and
// r_z.

// z (complex, batch of two L^3 arrays) = (r_x + i r_y, r_z + 0 i)
__global__ __launch_bounds__(256) void k_spec_pack(const double *__restrict__ r, size_t Ns,
                                                   double2 *__restrict__ Z, const int *stop) {
    if (stop && *stop) return;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns; v += (size_t)gridDim.x * blockDim.x) {
        Z[v] = make_double2(r[v], r[Ns + v]);
        Z[Ns + v] = make_double2(r[2 * Ns + v], 0.0);
    }
}

// In-place radix-2 FFT of lines along `axis` of `batch` complex L^3 arrays
// (L = 2^lg <= 1024), exp(sign 2 pi i m n / L), unnormalised.  A workgroup
// takes G = min(L, 2048 / L) lines that are neighbours along the fastest
// other axis (so that its loads along y and z are coalesced across lines):
// bit-reversed into LDS, lg butterfly stages, stored back.
__global__ __launch_bounds__(256) void k_fft_lines(double2 *__restrict__ data, int L, int lg, int axis, double sign,
                                                   const int *stop) {
    if (stop && *stop) return;
    extern __shared__ double2 fsh[];
    const int G = min(L, 2048 / L);
    double2 *tw = fsh + (size_t)G * L;
    const size_t LL = (size_t)L * L, Ns = LL * L;
    const int groups = L / G;
    const int a0 = (int)(blockIdx.x % groups) * G;
    const size_t rest = blockIdx.x / groups;
    const int b = (int)(rest % L);
    double2 *base = data + (rest / L) * Ns;
    for (int k = threadIdx.x; k < L / 2; k += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / L, &sn, &cs);
        tw[k] = make_double2(cs, sign * sn);
    }
    auto addr = [&](int g, int j) -> size_t {
        const int a = a0 + g;
        if (axis == 0) return (size_t)j + (size_t)L * a + LL * b;
        if (axis == 1) return (size_t)a + (size_t)L * j + LL * b;
        return (size_t)a + (size_t)L * b + LL * j;
    };
    for (int t = threadIdx.x; t < G * L; t += blockDim.x) {
        const int g = axis == 0 ? t / L : t % G, j = axis == 0 ? t % L : t / G;
        fsh[g * L + (int)(__brev((unsigned)j) >> (32 - lg))] = base[addr(g, j)];
    }
    for (int h = 1; h < L; h *= 2) {
        __syncthreads();
        const int stride = L / (2 * h);
        for (int bt = threadIdx.x; bt < G * L / 2; bt += blockDim.x) {
            const int g = bt / (L / 2), bb = bt % (L / 2);
            const int j = (bb / h) * 2 * h + bb % h;
            const double2 w = tw[(bb % h) * stride];
            const double2 u = fsh[g * L + j], x = fsh[g * L + j + h];
            const double2 v = make_double2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
            fsh[g * L + j] = make_double2(u.x + v.x, u.y + v.y);
            fsh[g * L + j + h] = make_double2(u.x - v.x, u.y - v.y);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < G * L; t += blockDim.x) {
        const int g = axis == 0 ? t / L : t % G, j = axis == 0 ? t % L : t / G;
        base[addr(g, j)] = fsh[g * L + j];
    }
}

// Z(m) *= 1 / sum_d 4 sin^2(pi m_d / L) (the mean, m = 0, to zero), batch of two.
__global__ __launch_bounds__(256) void k_spec_scale(double2 *__restrict__ Z, int L, size_t Ns, const int *stop) {
    if (stop && *stop) return;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < 2 * Ns; t += (size_t)gridDim.x * blockDim.x) {
        const size_t v = t % Ns;
        int i, j, k;
        site_ijk(v, L, i, j, k);
        const double si = sinpi((double)i / L), sj = sinpi((double)j / L), sk = sinpi((double)k / L);
        const double lam = 4.0 * (si * si + sj * sj + sk * sk);
        const double f = v == 0 ? 0.0 : 1.0 / lam;
        Z[t] = make_double2(Z[t].x * f, Z[t].y * f);
    }
}

// z = (Re Z0, Im Z0, Re Z1) / Ns; partial <r, z> of this block into
// partials[stride * block].
__global__ __launch_bounds__(256) void k_spec_unpack(const double2 *__restrict__ Z, const double *__restrict__ r,
                                                     double *__restrict__ z, size_t Ns, double *partials, int stride,
                                                     const int *stop) {
    if (stop && *stop) return;
    const double inv = 1.0 / (double)Ns;
    double s[1] = {0.0};
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns; v += (size_t)gridDim.x * blockDim.x) {
        const double2 a = Z[v], c = Z[Ns + v];
        const double z0 = a.x * inv, z1 = a.y * inv, z2 = c.x * inv;
        z[v] = z0;
        z[Ns + v] = z1;
        z[2 * Ns + v] = z2;
        s[0] += r[v] * z0 + r[Ns + v] * z1 + r[2 * Ns + v] * z2;
    }
    block_sum<1>(s);
    if (threadIdx.x == 0) partials[(size_t)stride * blockIdx.x] = s[0];
}

static bool spectral_ok(int L) { return L >= 2 && L <= 1024 && (L & (L - 1)) == 0; }

// z = (-Delta)^{-1} r on the three components, partial <r, z> per block of
// `blocks` into partials[stride * b]; Z holds 2 L^3 complex values.
static void launch_spectral(hipStream_t s, int L, const double *r, double *z, double2 *Z, int blocks,
                            double *partials, int stride, const int *stop) {
    const size_t Ns = (size_t)L * L * L;
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    const int G = std::min(L, 2048 / L);
    const int wgs = 2 * (L / G) * L;
    const size_t lds = ((size_t)G * L + L / 2) * sizeof(double2);
    hipLaunchKernelGGL(k_spec_pack, dim3(blocks), dim3(kThreads), 0, s, r, Ns, Z, stop);
    for (int ax = 0; ax < 3; ++ax)
        hipLaunchKernelGGL(k_fft_lines, dim3(wgs), dim3(kThreads), lds, s, Z, L, lg, ax, -1.0, stop);
    hipLaunchKernelGGL(k_spec_scale, dim3(blocks), dim3(kThreads), 0, s, Z, L, Ns, stop);
    for (int ax = 0; ax < 3; ++ax)
        hipLaunchKernelGGL(k_fft_lines, dim3(wgs), dim3(kThreads), lds, s, Z, L, lg, ax, 1.0, stop);
    hipLaunchKernelGGL(k_spec_unpack, dim3(blocks), dim3(kThreads), 0, s, Z, r, z, Ns, partials, stride, stop);
}

// CG scalar slots (relative to S_CG)
enum { CG_RZ = 0, CG_ALPHA = 1, CG_BETA = 2, CG_RMAX = 3, CG_DEN = 4, CG_TOL = 5, CG_AINV = 6 };

// alpha = rz / <p, q>; a non-positive curvature stops the sweep (flag 2).
__global__ void k_cg_alpha(const double *partials, int nblk, double *cg, int *flags) {
    if (flags[0]) return;
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s[0] += partials[b];
    block_sum<1>(s);
    if (threadIdx.x == 0) {
        if (!(s[0] > 0.0)) {
            flags[0] = 2;
        } else {
            cg[CG_ALPHA] = cg[CG_RZ] / s[0];
        }
    }
}

// D += alpha w; r -= alpha q; z = dinv r; partials: <r,z>, max|r| (with
// dinv null, z and <r,z> are left to the spectral preconditioner, which
// writes partials[2 b] after this kernel)
__global__ __launch_bounds__(256) void k_cg_update(double *__restrict__ D, double *__restrict__ r,
                                                   double *__restrict__ z, const double *__restrict__ w,
                                                   const double *__restrict__ q,
                                                   const double *__restrict__ dinv, size_t M, const double *cg,
                                                   double *partials, const int *flags) {
    if (flags[0]) return;
    const double alpha = cg[CG_ALPHA];
    double s[1] = {0.0};
    double mx = 0.0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < M; t += (size_t)gridDim.x * blockDim.x) {
        D[t] += alpha * w[t];
        const double rr = r[t] - alpha * q[t];
        r[t] = rr;
        if (dinv) {
            const double zz = dinv[t] * rr;
            z[t] = zz;
            s[0] += rr * zz;
        }
        mx = fmax(mx, fabs(rr));
    }
    block_sum<1>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        if (dinv) partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = m;
    }
}

// beta = rz_new / rz; when the recursive residual passes the test, flag 1.
__global__ void k_cg_beta(const double *partials, int nblk, double a, double *cg, int *flags, int *iters) {
    if (flags[0]) return;
    double s[1] = {0.0};
    double mx = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        s[0] += partials[2 * b];
        mx = fmax(mx, partials[2 * b + 1]);
    }
    block_sum<1>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        cg[CG_BETA] = s[0] / cg[CG_RZ];
        cg[CG_RZ] = s[0];
        cg[CG_RMAX] = m;
        iters[0] += 1;
        if (a * m <= cg[CG_TOL] * cg[CG_DEN]) flags[0] = 1;
    }
}

// p = z + beta p, only for the iteration whose beta was just formed (the
// iteration counter equals `expected`): this also runs in the iteration where
// the recursive test passed, so a rejected test continues consistently.
__global__ void k_cg_p(double *__restrict__ p, const double *__restrict__ z, size_t M, const double *cg,
                       const int *flags, int expected) {
    if (flags[0] == 2 || flags[1] != expected) return;
    const double beta = cg[CG_BETA];
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < M; t += (size_t)gridDim.x * blockDim.x)
        p[t] = z[t] + beta * p[t];
}

template <typename T>
__global__ void k_eta_expand(const T *eta_link, const T *eta_prof, double eta_uni, int mode, int L, size_t Ns,
                             double *out) {
    const size_t LL = (size_t)L * L;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < 3 * Ns;
         t += (size_t)gridDim.x * blockDim.x) {
        const int d = (int)(t / Ns);
        const size_t v = t % Ns;
        double e;
        if (mode == ETA_UNIFORM) e = eta_uni;
        else if (mode == ETA_ZPROF) e = (double)eta_prof[d * L + (int)(v / LL)];
        else e = (double)eta_link[t];
        out[t] = e;
    }
}

__global__ void k_cg_set(double *cg, double den, double tol, int *flags) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cg[CG_DEN] = den;
        cg[CG_TOL] = tol;
        flags[0] = 0;
    }
}

__global__ void k_copy(const double *__restrict__ s, double *__restrict__ d, size_t M) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < M; t += (size_t)gridDim.x * blockDim.x)
        d[t] = s[t];
}

static int grid_m(size_t M) {
    size_t b = (M + kThreads - 1) / kThreads;
    if (b > (size_t)kRedBlocks) b = kRedBlocks;
    return (int)(b ? b : 1);
}

memd_status solve_relax(memd_ctx *c, double *D, double tol, int max_iter, int *iters_out, double *res_out) {
    const size_t Ns = c->Ns, M = 3 * Ns;
    hipStream_t s = c->stream;
    const bool spectral = spectral_ok(c->L);
    double *buf = nullptr;
    // eta, dinv (the spectral preconditioner's complex work array in its
    // place, 4 Ns doubles), r, z, p, w, q, Dbest
    if (hipMallocAsync((void **)&buf, (8 * M + (spectral ? Ns : 0)) * sizeof(double), s) != hipSuccess)
        return MEMD_ENOMEM;
    double *eta = buf, *dinv = buf + M, *r = buf + 2 * M + (spectral ? Ns : 0);
    double *z = r + M, *p = r + 2 * M, *w = r + 3 * M, *q = r + 4 * M, *Dbest = r + 5 * M;
    double2 *Z = reinterpret_cast<double2 *>(dinv);
    int *flags = nullptr;
    if (hipMallocAsync((void **)&flags, 4 * sizeof(int), s) != hipSuccess) {
        hipFreeAsync(buf, s);
        return MEMD_ENOMEM;
    }
    hipMemsetAsync(flags, 0, 4 * sizeof(int), s);
    const int g = grid_m(Ns), gm = grid_m(M);
    if (c->fp32)
        hipLaunchKernelGGL(k_eta_expand<float>, dim3(gm), dim3(kThreads), 0, s, (const float *)c->eta_link,
                           (const float *)c->eta_prof, c->eta_uni, c->eta_mode, c->L, Ns, eta);
    else
        hipLaunchKernelGGL(k_eta_expand<double>, dim3(gm), dim3(kThreads), 0, s, (const double *)c->eta_link,
                           (const double *)c->eta_prof, c->eta_uni, c->eta_mode, c->L, Ns, eta);
    CgArgs A{c->L, Ns, 1.0 / c->a, eta};
    if (!spectral) hipLaunchKernelGGL(k_dinv, dim3(g), dim3(kThreads), 0, s, A, c->a * c->a, dinv);
    double *cg = c->scal + S_CG;
    double *part = c->partials;

    memd_status st = MEMD_OK;
    int it_total = 0, stalls = 0;
    double best = HUGE_VAL, res = HUGE_VAL;
    bool first = true, converged = false;
    const int chunk = 10;
    for (;;) {
        // residual replacement: r = -C(eta D) from D; test on the true residual
        hipLaunchKernelGGL((k_curl_eta<true, false>), dim3(g), dim3(kThreads), 0, s, A, D, -1.0, r, nullptr,
                           part, nullptr);
        double h[2 * kRedBlocks];
        hipMemcpyAsync(h, part, 2 * g * sizeof(double), hipMemcpyDeviceToHost, s);
        int hf[2] = {0, 0};
        hipMemcpyAsync(hf, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess) {
            st = MEMD_EDEVICE;
            break;
        }
        double rmax = 0.0, den = 0.0;
        for (int b = 0; b < g; ++b) {
            rmax = fmax(rmax, h[2 * b]);
            den = fmax(den, h[2 * b + 1]);
        }
        it_total = hf[1];
        res = den > 0.0 ? c->a * rmax / den : 0.0;
        if (hf[0] == 1) ++stalls;  // the recursive residual had passed the test
        if (res <= tol) {
            converged = true;
            break;
        }
        if (res < best) {
            best = res;
            hipLaunchKernelGGL(k_copy, dim3(gm), dim3(kThreads), 0, s, D, Dbest, M);
        }
        if (it_total >= max_iter || stalls >= 3 || res > 1e3 * best) {
            hipLaunchKernelGGL(k_copy, dim3(gm), dim3(kThreads), 0, s, Dbest, D, M);
            res = best;
            break;
        }
        if (spectral)
            launch_spectral(s, c->L, r, z, Z, gm, part, 1, nullptr);
        else
            hipLaunchKernelGGL(k_precond, dim3(gm), dim3(kThreads), 0, s, dinv, r, z, M, part);
        launch_finalize_sum(s, part, gm, 1, cg + CG_RZ);
        if (first || hf[0] == 2) {
            hipLaunchKernelGGL(k_copy, dim3(gm), dim3(kThreads), 0, s, z, p, M);
            first = false;
        }
        hipLaunchKernelGGL(k_cg_set, dim3(1), dim3(64), 0, s, cg, den, tol, flags);
        for (int t = 0; t < chunk; ++t) {
            hipLaunchKernelGGL(k_curl_adj, dim3(g), dim3(kThreads), 0, s, A, p, w, flags);
            hipLaunchKernelGGL((k_curl_eta<false, true>), dim3(g), dim3(kThreads), 0, s, A, w, 1.0, q, p, part,
                               flags);
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, part, g, cg, flags);
            hipLaunchKernelGGL(k_cg_update, dim3(gm), dim3(kThreads), 0, s, D, r, z, w, q,
                               spectral ? nullptr : dinv, M, cg, part, flags);
            if (spectral) launch_spectral(s, c->L, r, z, Z, gm, part, 2, flags);
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kThreads), 0, s, part, gm, c->a, cg, flags, flags + 1);
            hipLaunchKernelGGL(k_cg_p, dim3(gm), dim3(kThreads), 0, s, p, z, M, cg, flags, it_total + t + 1);
        }
        if (hipGetLastError() != hipSuccess) {
            st = MEMD_EDEVICE;
            break;
        }
    }
    hipFreeAsync(flags, s);
    hipFreeAsync(buf, s);
    if (hipStreamSynchronize(s) != hipSuccess) st = MEMD_EDEVICE;
    if (iters_out) *iters_out = it_total;
    if (res_out) *res_out = res;
    if (st == MEMD_OK && !converged) st = MEMD_ENOCONV;
    return st;
}

// ------------------------------------------------ direct planar solution
//
// When eta is uniform or depends only on the plane (eta_d(k)), the field the
// relaxation converges to is reached directly.  Its non-uniform part is
// E = -grad phi with phi periodic: Gauss's law, with D_d = -eps_d (phi(v+e_d)
// - phi(v)) / a, reads
//   a sum_d [eps_d(v) (phi(v+e_d) - phi(v)) - eps_d(v-e_d) (phi(v) - phi(v-e_d))] = -q_v,
// which a 2-D DFT over (x, y) turns into one cyclic tridiagonal system along
// z per mode (mx, my) != (0, 0):
//   eps_z(k-1) phi_{k-1} + [eps_x(k) lx + eps_y(k) ly - eps_z(k) - eps_z(k-1)] phi_k
//   + eps_z(k) phi_{k+1} = -q_k / a,   l = 2 cos(2 pi m / L) - 2.
// The plane means (mode (0, 0)) are fixed by the constraints the relaxation
// keeps: mean D = -P/V (section "Periodicity") and no circulation on any
// plaquette, so E_x and E_y are one constant across planes (D_x(k) =
// eps_x(k) E0_x), and D_z(k) follows the plane charges by Gauss's law up to
// the constant that sets its mean.  Everything is FP64.

// eps_d(k) = 1 / eta_d(k) of the stored permittivity (uniform or per plane)
template <typename T>
__global__ void k_planar_eps(int mode, double eta_uni, const T *__restrict__ prof, int L, double *__restrict__ eps) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * L) return;
    eps[t] = 1.0 / (mode == ETA_UNIFORM ? eta_uni : (double)prof[t]);
}

__global__ void k_to_complex(const double *__restrict__ x, size_t n, double2 *__restrict__ out) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = make_double2(x[t], 0.0);
}

// One DFT of length L (<= 256) along x (axis 0) or y (axis 1) per workgroup:
// out[m] = sum_n in[n] exp(sign 2 pi i m n / L), the twiddles from a table
// of the L angles 2 pi t / L (t = m n mod L).
__global__ __launch_bounds__(256) void k_dft_line(const double2 *__restrict__ in, double2 *__restrict__ out, int L,
                                                  int axis, double sign) {
    __shared__ double2 line[256];
    __shared__ double2 tw[256];
    const int b = blockIdx.x;  // line: (j, k) along x, (i, k) along y
    const size_t LL = (size_t)L * L;
    const size_t base = axis == 0 ? (size_t)b * L : (size_t)(b % L) + (size_t)(b / L) * LL;
    const size_t stride = axis == 0 ? 1 : (size_t)L;
    const int t = threadIdx.x;
    if (t < L) {
        line[t] = in[base + t * stride];
        double sn, cs;
        sincospi(2.0 * t / L, &sn, &cs);
        tw[t] = make_double2(cs, sign * sn);
    }
    __syncthreads();
    if (t < L) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int n = 0; n < L; ++n) {
            const double2 x = line[n], w = tw[idx];
            re += x.x * w.x - x.y * w.y;
            im += x.x * w.y + x.y * w.x;
            idx += t;
            idx -= idx >= L ? L : 0;
        }
        out[base + t * stride] = make_double2(re, im);
    }
}

// Plane means: from the plane charges q_k (the (0,0) coefficients of the
// forward transform), D_z(k) - D_z(k-1) = q_k / (a^2 L^2) shifted to mean
// -P_z/V, and E0_{x,y} = -P_{x,y} / (V mean_k eps_{x,y}(k)).  One thread.
__global__ void k_planar_means(const double2 *__restrict__ A, const double *__restrict__ eps, int L, double a,
                               double V, const double *__restrict__ P, double *__restrict__ dz, double *__restrict__ e0) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const size_t LL = (size_t)L * L;
    const double scale = 1.0 / (a * a * (double)LL);
    double run = 0.0, sum = 0.0;
    for (int k = 0; k < L; ++k) {
        run += A[(size_t)k * LL].x * scale;
        dz[k] = run;
        sum += run;
    }
    const double shift = -P[2] / V - sum / L;
    for (int k = 0; k < L; ++k) dz[k] += shift;
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < L; ++k) {
        mx += eps[k];
        my += eps[L + k];
    }
    e0[0] = -P[0] / (V * (mx / L));
    e0[1] = -P[1] / (V * (my / L));
}

// The cyclic tridiagonal system of each mode (mx, my) != (0, 0), in place on
// A (right-hand side -q_k / a in, phi_k out), by the Sherman-Morrison form of
// the Thomas algorithm; w holds 4 L doubles per mode.
__global__ void k_planar_tridiag(double2 *__restrict__ A, const double *__restrict__ eps, int L, double a,
                                 double *__restrict__ w) {
    const int mode = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t LL = (size_t)L * L;
    if (mode >= (int)LL) return;
    double2 *x = A + mode;  // element k at x[k LL]
    if (mode == 0) {
        for (int k = 0; k < L; ++k) x[(size_t)k * LL] = make_double2(0.0, 0.0);
        return;
    }
    const int mx = mode % L, my = mode / L;
    const double lx = 2.0 * cospi(2.0 * mx / L) - 2.0, ly = 2.0 * cospi(2.0 * my / L) - 2.0;
    const double *ex = eps, *ey = eps + L, *ez = eps + 2 * L;
    double *cp = w + (size_t)mode * 4 * L, *yr = cp + L, *yi = cp + 2 * L, *zz = cp + 3 * L;
    auto diag = [&](int k) { return ex[k] * lx + ey[k] * ly - ez[k] - ez[k == 0 ? L - 1 : k - 1]; };
    const double a0 = ez[L - 1];   // row 0, column L-1
    const double cl = ez[L - 1];   // row L-1, column 0
    const double gam = -diag(0);
    // forward elimination of T (corners removed, b_0 - gam, b_{L-1} - a0 cl / gam) for the
    // right-hand sides d (real, imaginary) and u = (gam, 0, ..., 0, cl)
    double bp = diag(0) - gam;
    double2 d0 = x[0];
    cp[0] = ez[0] / bp;
    yr[0] = (-d0.x / a) / bp;
    yi[0] = (-d0.y / a) / bp;
    zz[0] = gam / bp;
    for (int k = 1; k < L; ++k) {
        const double lo = ez[k - 1];
        double bk = diag(k);
        if (k == L - 1) bk -= a0 * cl / gam;
        const double m = bk - lo * cp[k - 1];
        const double2 dk = x[(size_t)k * LL];
        cp[k] = ez[k] / m;
        yr[k] = (-dk.x / a - lo * yr[k - 1]) / m;
        yi[k] = (-dk.y / a - lo * yi[k - 1]) / m;
        zz[k] = ((k == L - 1 ? cl : 0.0) - lo * zz[k - 1]) / m;
    }
    for (int k = L - 2; k >= 0; --k) {
        yr[k] -= cp[k] * yr[k + 1];
        yi[k] -= cp[k] * yi[k + 1];
        zz[k] -= cp[k] * zz[k + 1];
    }
    const double vf = a0 / gam;
    const double den = 1.0 + zz[0] + vf * zz[L - 1];
    const double fr = (yr[0] + vf * yr[L - 1]) / den, fi = (yi[0] + vf * yi[L - 1]) / den;
    for (int k = 0; k < L; ++k) x[(size_t)k * LL] = make_double2(yr[k] - zz[k] * fr, yi[k] - zz[k] * fi);
}

// D from phi (the inverse transform, not yet divided by L^2) and the plane
// means.
__global__ void k_planar_field(const double2 *__restrict__ A, const double *__restrict__ eps,
                               const double *__restrict__ dz, const double *__restrict__ e0, int L, double a,
                               double *__restrict__ D) {
    const size_t Ns = (size_t)L * L * L, LL = (size_t)L * L;
    const double inv = 1.0 / ((double)LL * a);
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns; v += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(v % L), j = (int)((v / L) % L), k = (int)(v / LL);
        const size_t row = v - (size_t)i, plane = v - (size_t)j * L - (size_t)i;
        const size_t vx = row + (i + 1 == L ? 0 : i + 1);
        const size_t vy = plane + (size_t)(j + 1 == L ? 0 : j + 1) * L + i;
        const size_t vz = (size_t)(k + 1 == L ? 0 : k + 1) * LL + (size_t)j * L + i;
        const double ph = A[v].x;
        D[v] = -eps[k] * (A[vx].x - ph) * inv + eps[k] * e0[0];
        D[Ns + v] = -eps[L + k] * (A[vy].x - ph) * inv + eps[L + k] * e0[1];
        D[2 * Ns + v] = -eps[2 * L + k] * (A[vz].x - ph) * inv + dz[k];
    }
}

bool planar_solve_ok(const memd_ctx *c) {
    return (c->eta_mode == ETA_UNIFORM || c->eta_mode == ETA_ZPROF) && c->L >= 4 && c->L <= 128;
}

hipError_t solve_planar(memd_ctx *c, double *D) {
    hipError_t e;
    const int L = c->L;
    const size_t Ns = c->Ns, LL = (size_t)L * L;
    hipStream_t s = c->stream;
    // the dipole of the ions (their mean field) and their charge assignment
    int nb = 0;
    if ((e = launch_dipole(c, c->partials, &nb)) != hipSuccess) return e;
    if ((e = launch_finalize_dipole(s, c->partials, nb, c->scal + S_P)) != hipSuccess) return e;
    if ((e = launch_spread_dense(c, true, c->rho)) != hipSuccess) return e;
    double *buf = nullptr;
    const size_t nbytes = 2 * Ns * sizeof(double2) + (4 * LL * L + 6 * L + 2) * sizeof(double);
    if ((e = hipMallocAsync((void **)&buf, nbytes, s)) != hipSuccess) return e;
    double2 *A = (double2 *)buf, *Bt = A + Ns;
    double *w = (double *)(Bt + Ns), *eps = w + 4 * LL * L, *dz = eps + 3 * L, *e0 = dz + L;
    if (c->fp32)
        hipLaunchKernelGGL(k_planar_eps<float>, dim3((3 * L + 255) / 256), dim3(256), 0, s, c->eta_mode, c->eta_uni,
                           (const float *)c->eta_prof, L, eps);
    else
        hipLaunchKernelGGL(k_planar_eps<double>, dim3((3 * L + 255) / 256), dim3(256), 0, s, c->eta_mode,
                           c->eta_uni, (const double *)c->eta_prof, L, eps);
    const int gs = grid_m(Ns);
    hipLaunchKernelGGL(k_to_complex, dim3(gs), dim3(kThreads), 0, s, c->rho, Ns, A);
    const int lines = (int)LL;  // L^2 lines along each axis
    hipLaunchKernelGGL(k_dft_line, dim3(lines), dim3(256), 0, s, A, Bt, L, 0, -1.0);
    hipLaunchKernelGGL(k_dft_line, dim3(lines), dim3(256), 0, s, Bt, A, L, 1, -1.0);
    hipLaunchKernelGGL(k_planar_means, dim3(1), dim3(64), 0, s, A, eps, L, c->a, c->V, c->scal + S_P, dz, e0);
    hipLaunchKernelGGL(k_planar_tridiag, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, s, A, eps, L, c->a, w);
    hipLaunchKernelGGL(k_dft_line, dim3(lines), dim3(256), 0, s, A, Bt, L, 1, 1.0);
    hipLaunchKernelGGL(k_dft_line, dim3(lines), dim3(256), 0, s, Bt, A, L, 0, 1.0);
    hipLaunchKernelGGL(k_planar_field, dim3(gs), dim3(kThreads), 0, s, A, eps, dz, e0, L, c->a, D);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipFreeAsync(buf, s);
}

// ------------------------------------------------------- Green's function

// G(n) = (1/Ns) sum_{k != 0} cos(k.n) / sum_d 4 sin^2(k_d/2), k = 2 pi m / L,
// at n = (0,0,0), (1,0,0), (1,1,0), (1,1,1).
__global__ __launch_bounds__(256) void k_greens(int L, double *partials) {
    const size_t Ns = (size_t)L * L * L;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const double pi = 3.14159265358979323846;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < Ns; t += (size_t)gridDim.x * blockDim.x) {
        if (t == 0) continue;
        const int mx = (int)(t % L), my = (int)((t / L) % L), mz = (int)(t / ((size_t)L * L));
        const double hx = sin(pi * mx / L), hy = sin(pi * my / L), hz = sin(pi * mz / L);
        const double inv = 1.0 / (4.0 * hx * hx + 4.0 * hy * hy + 4.0 * hz * hz);
        const double cx = cos(2.0 * pi * mx / L), cy = cos(2.0 * pi * my / L), cz = cos(2.0 * pi * mz / L);
        s[0] += inv;
        s[1] += cx * inv;
        s[2] += cx * cy * inv;
        s[3] += cx * cy * cz * inv;
    }
    block_sum<4>(s);
    if (threadIdx.x == 0)
        for (int w = 0; w < 4; ++w) partials[4 * blockIdx.x + w] = s[w];
}

__global__ void k_greens_fin(const double *partials, int nblk, double Ns, double *G) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int w = 0; w < 4; ++w) s[w] += partials[4 * b + w];
    block_sum<4>(s);
    if (threadIdx.x == 0)
        for (int w = 0; w < 4; ++w) G[w] = s[w] / Ns;
}

hipError_t launch_greens(memd_ctx *c, double *G) {
    const int g = grid_m(c->Ns);
    hipLaunchKernelGGL(k_greens, dim3(g), dim3(kThreads), 0, c->stream, c->L, c->partials);
    hipLaunchKernelGGL(k_greens_fin, dim3(1), dim3(kThreads), 0, c->stream, c->partials, g, (double)c->Ns, G);
    return hipGetLastError();
}

}  // namespace memd
