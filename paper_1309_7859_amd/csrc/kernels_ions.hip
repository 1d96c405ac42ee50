// kernels_ions.hip -- per-ion kernels for gfx950: current deposition, charge
// assignment, dipole moment, corrected forces; deterministic finalisers of
// the per-block partial sums; the lattice Green's function table.
#include "device_util.hpp"
#include "ion_ops.hpp"
#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"
#include "philox.hpp"

namespace memd {

// ----------------------------------------------------------- deposition

// The deposit kernel: sixteen lanes per ion (one per axis and transverse
// corner, deposit_ion_part), ions taken in the order of `order` (binned by
// lattice row, so that neighbouring lanes update neighbouring links).  Lane 0
// of each ion writes the new position and, when spread_rho is set, adds the
// new charge assignment to rho (FP64) for the Gauss audit.  Block sums of
// q r^{n+1} go to partials (summed in block order by k_fin_dipole).
template <typename T>
__global__ __launch_bounds__(256) void k_deposit(int n, int L, size_t Ns, double a,
                                                 const double *__restrict__ q, double *__restrict__ r,
                                                 const double *__restrict__ disp, T *__restrict__ D,
                                                 int spread_rho, double *__restrict__ rho,
                                                 const int *__restrict__ order,
                                                 double *__restrict__ partials, unsigned int *bad,
                                                 uint64_t seed, uint32_t t, double sigma) {
    const int lane = threadIdx.x & 15;
    // consecutive (spatially sorted) ions stay on one XCD and share its L2
    const int slot = xcd_logical(blockIdx.x, gridDim.x) * (blockDim.x >> 4) + (threadIdx.x >> 4);
    double P[3] = {0.0, 0.0, 0.0};
    if (slot < n) {
        const int i = order ? order[slot] : slot;
        const double qi = q[i];
        double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
        double du[3];
        if (disp) {
            du[0] = disp[3 * i];
            du[1] = disp[3 * i + 1];
            du[2] = disp[3 * i + 2];
        } else {
            if (lane == 0) philox_displacement(seed, t, (uint32_t)i, sigma, du);
#pragma unroll
            for (int d = 0; d < 3; ++d) du[d] = __shfl(du[d], 0, 16);
        }
        sanitize_move(du, a, L, lane == 0 ? bad : nullptr);
        deposit_ion_part<T>(L, Ns, a, qi, u, du, D, lane >> 2, lane & 3);
        if (lane == 0) {
            r[3 * i] = u[0];
            r[3 * i + 1] = u[1];
            r[3 * i + 2] = u[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) P[d] = qi * u[d];
            if (spread_rho) spread_ion(L, a, qi, u, rho);
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
// grid of the sorted-order ion kernels (lanes_per_ion lanes per ion): a
// multiple of the 8 XCDs
static int ion_blocks_x8(int n, int lanes_per_ion = 1) {
    const long long t = (long long)(n > 0 ? n : 1) * lanes_per_ion;
    const int b = (int)((t + kThreads - 1) / kThreads);
    return (b + 7) / 8 * 8;
}

hipError_t launch_deposit(memd_ctx *c, void *D, const double *disp, bool spread_rho,
                          double *partials, int *nblk, uint64_t seed, uint32_t t, double sigma) {
    const int nb = ion_blocks_x8(c->n, 16);
    *nblk = nb;
    if (c->fp32)
        hipLaunchKernelGGL(k_deposit<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (float *)D, spread_rho ? 1 : 0, c->rho, c->order, partials,
                           c->bad_moves, seed, t, sigma);
    else
        hipLaunchKernelGGL(k_deposit<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (double *)D, spread_rho ? 1 : 0, c->rho, c->order, partials,
                           c->bad_moves, seed, t, sigma);
    return hipGetLastError();
}

// Records of the ions in bin order for the fused deposit (leapfrog_tile.hpp,
// DepCon): ions are read in index order (coalesced), one lane per ion, and
// ion i's record goes to its slot slot_of[i].  The axes of the
// dimension-split move are taken in turn with the arithmetic of deposit_ion
// (bit for bit); for each the box corner and the values -q (ub - ua)/a w w /
// a^2 (in the field type) are stored.  An irregular ion gets the head -1.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_ions(int n, int L, double a, const double *__restrict__ q,
                                                   const double *__restrict__ r, const double *__restrict__ disp,
                                                   const int *__restrict__ slot_of, const int *__restrict__ binrow,
                                                   int4 *__restrict__ head, DepCon<T> *__restrict__ con,
                                                   uint64_t seed, uint32_t t, double sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = slot_of[i];
    double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    double du[3];
    if (disp) {
        du[0] = disp[3 * i];
        du[1] = disp[3 * i + 1];
        du[2] = disp[3 * i + 2];
    } else {
        philox_displacement(seed, t, (uint32_t)i, sigma, du);
    }
    sanitize_move(du, a, L, nullptr);
    int c0[3];
    {
        double f;
#pragma unroll
        for (int d = 0; d < 3; ++d) fold(u[d], a, L, c0[d], f);
    }
    if (!ion_regular(a, L, u, du, binrow[i])) {
        head[s] = make_int4(-1, 0, 0, 0);
        return;
    }
    const double qi = q[i], a2 = a * a;
    DepCon<T> &o = con[s];
    unsigned int g[3] = {0u, 0u, 0u};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
        const double u0 = u[d], u1 = u0 + du[d];
        if (u1 != u0) {
            int c1, c2;
            double f1, f2;
            fold(u[d1], a, L, c1, f1);
            fold(u[d2], a, L, c2, f2);
            const double lo = u0 < u1 ? u0 : u1, hi = u0 < u1 ? u1 : u0;
            const double sgn = u1 > u0 ? 1.0 : -1.0;
            const double klo = floor(div_a(lo, a)), khi = floor(div_a(hi, a));
            int corner[3];
            corner[d] = mod_cell(klo, L);
            corner[d1] = c1;
            corner[d2] = c2;
            g[d] = (unsigned)pack_cell(corner[0], corner[1], corner[2]) | kGroupOn | (khi > klo ? kGroupTwo : 0u);
            // a regular move spans at most two cells along the axis
#pragma unroll
            for (int cell = 0; cell < 2; ++cell) {
                const double kc = cell ? khi : klo;
                const double s0 = kc * a, s1 = (kc + 1.0) * a;
                const double sa = lo > s0 ? lo : s0;
                const double sb = hi < s1 ? hi : s1;
                const double len = sb - sa;
                const double amount =
                    (cell == 0 || khi > klo) && len > 0.0 ? div_a(qi * sgn * div_a(len, a), a2) : 0.0;
#pragma unroll
                for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 2; ++o1)
                        o.val[kConPerAxis * d + 4 * cell + 2 * o2 + o1] =
                            (T)(-(amount * lin_w(o1, f1) * lin_w(o2, f2)));
            }
        }
        u[d] = u1;
    }
    head[s] = make_int4(pack_cell(c0[0], c0[1], c0[2]), (int)g[0], (int)g[1], (int)g[2]);
}

hipError_t launch_pack_ions(memd_ctx *c, const double *disp, uint64_t seed, uint32_t t, double sigma) {
    if (c->n == 0) return hipSuccess;
    const int nb = ion_blocks(c->n);
    if (c->fp32)
        hipLaunchKernelGGL(k_pack_ions<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L,
                           c->a, c->q, c->r, disp, c->slot, c->binrow, (int4 *)c->ionrec,
                           (DepCon<float> *)((int4 *)c->ionrec + c->n), seed, t, sigma);
    else
        hipLaunchKernelGGL(k_pack_ions<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L,
                           c->a, c->q, c->r, disp, c->slot, c->binrow, (int4 *)c->ionrec,
                           (DepCon<double> *)((int4 *)c->ionrec + c->n), seed, t, sigma);
    return hipGetLastError();
}

// Ion update after the leapfrog with the fused deposit: ions in index order
// (so the dipole's block sums are in a fixed order), the regularity test of
// the fused deposit repeated on the same bits; irregular ions deposit their
// whole move here with global atomics, every ion is moved, and block sums of
// q r^{n+1} go to partials (plus rho for the audit when spread_rho is set).
template <typename T>
__global__ __launch_bounds__(256) void k_ion_update(int n, int L, size_t Ns, double a,
                                                    const double *__restrict__ q, double *__restrict__ r,
                                                    const double *__restrict__ disp, T *__restrict__ D,
                                                    const int *__restrict__ binrow, int spread_rho,
                                                    double *__restrict__ rho, double *__restrict__ partials,
                                                    unsigned int *bad, uint64_t seed, uint32_t t, double sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double P[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
        double du[3];
        if (disp) {
            du[0] = disp[3 * i];
            du[1] = disp[3 * i + 1];
            du[2] = disp[3 * i + 2];
        } else {
            philox_displacement(seed, t, (uint32_t)i, sigma, du);
        }
        sanitize_move(du, a, L, bad);
        const double qi = q[i];
        if (ion_regular(a, L, u, du, binrow[i])) {
#pragma unroll
            for (int d = 0; d < 3; ++d) u[d] = u[d] + du[d];
        } else {
            deposit_ion<T>(L, Ns, a, qi, u, du, D);
        }
        r[3 * i] = u[0];
        r[3 * i + 1] = u[1];
        r[3 * i + 2] = u[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) P[d] = qi * u[d];
        if (spread_rho) spread_ion(L, a, qi, u, rho);
    }
    block_sum<3>(P);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = P[0];
        partials[3 * blockIdx.x + 1] = P[1];
        partials[3 * blockIdx.x + 2] = P[2];
    }
}

hipError_t launch_ion_update(memd_ctx *c, void *D, const double *disp, bool spread_rho, double *partials,
                             int *nblk, uint64_t seed, uint32_t t, double sigma) {
    const int nb = ion_blocks(c->n);
    *nblk = nb;
    if (c->fp32)
        hipLaunchKernelGGL(k_ion_update<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (float *)D, c->binrow, spread_rho ? 1 : 0, c->rho, partials,
                           c->bad_moves, seed, t, sigma);
    else
        hipLaunchKernelGGL(k_ion_update<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (double *)D, c->binrow, spread_rho ? 1 : 0, c->rho, partials,
                           c->bad_moves, seed, t, sigma);
    return hipGetLastError();
}

// ------------------------------------------------------- charge assignment

// Linear assignment of each ion's charge (or of 1 when q is null) to the 8
// corners of its cell, added into dst (FP64 atomics).
__global__ __launch_bounds__(256) void k_spread(int n, int L, double a, const double *__restrict__ q,
                                                const double *__restrict__ r, double *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    spread_ion(L, a, q ? q[i] : 1.0, u, dst);
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
    double *scal;        // P, eps_h, G
    double *F;
    double *uself_partials;  // optional: per-block sums of the self energy
    const int *order;        // optional: ion order (binned by lattice row)
    const double *dip_partials;  // optional: deposit's per-block q r sums -> P
    int dip_nblk;
};

// Forces on every ion, one lane per ion following `order` (force_ion: the
// lattice part from the 12 links of the cell, self force, dipole
// correction).  With dip_partials set, wavefront 0 of every block sums the
// deposit's per-block q r partials into P (in a fixed order; block 0 also
// stores it) while the other lanes' loads are in flight.
template <typename T>
__global__ __launch_bounds__(256) void k_forces(ForceArgs<T> A) {
    __shared__ double Psh[3];
    const int slot = xcd_logical(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool live = slot < A.n;
    const int i = live ? (A.order ? A.order[slot] : slot) : 0;
    double u[3] = {0.0, 0.0, 0.0}, qi = 0.0;
    if (live) {
        u[0] = A.r[3 * i];
        u[1] = A.r[3 * i + 1];
        u[2] = A.r[3 * i + 2];
        qi = A.q[i];
    }
    // lattice part and self force first (their gathers overlap the dipole
    // sum); the dipole term is added once P is known: x + 0 + y rounds as x + y
    double us = 0.0, F[3] = {0.0, 0.0, 0.0};
    if (live) {
        const EtaView<T> ev{A.mode, A.eta_uni, A.eta_prof, A.eta_link};
        const double zero[3] = {0.0, 0.0, 0.0};
        us = force_ion<T>(A.L, A.Ns, A.a, A.V, qi, u, A.D, ev, A.scal + S_G, zero, A.scal + S_EPSH, F);
    }
    if (threadIdx.x < 64) {
        if (A.dip_partials) {
            double s[3] = {0.0, 0.0, 0.0};
            for (int b = threadIdx.x; b < A.dip_nblk; b += 64)
#pragma unroll
                for (int d = 0; d < 3; ++d) s[d] += A.dip_partials[3 * b + d];
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] = wave_sum(s[d]);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    Psh[d] = s[d];
                    if (blockIdx.x == 0) A.scal[S_P + d] = s[d];
                }
            }
        } else if (threadIdx.x < 3) {
            Psh[threadIdx.x] = A.scal[S_P + threadIdx.x];
        }
    }
    __syncthreads();
    if (live) {
#pragma unroll
        for (int d = 0; d < 3; ++d) A.F[3 * i + d] = F[d] + qi * Psh[d] / (A.V * A.scal[S_EPSH + d]);
    }
    if (A.uself_partials) {
        double v[1] = {us};
        block_sum<1>(v);
        if (threadIdx.x == 0) A.uself_partials[blockIdx.x] = v[0];
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
    A.order = c->order;
    A.dip_partials = nullptr;
    A.dip_nblk = 0;
    return A;
}

hipError_t launch_forces(memd_ctx *c, const void *D, const double *dip_partials, int dip_nblk) {
    if (c->n == 0) return hipSuccess;
    const int nb = ion_blocks_x8(c->n, 1);
    if (c->fp32) {
        auto A = force_args<float>(c, D);
        A.dip_partials = dip_partials;
        A.dip_nblk = dip_nblk;
        hipLaunchKernelGGL(k_forces<float>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    } else {
        auto A = force_args<double>(c, D);
        A.dip_partials = dip_partials;
        A.dip_nblk = dip_nblk;
        hipLaunchKernelGGL(k_forces<double>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- ion binning

// Counting sort of the ions by lattice row (y, z cell of the position): the
// deposit and force kernels then visit neighbouring ions together.
__global__ void k_bin_count(int n, int L, double a, const double *__restrict__ r, int *__restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cy, cz;
    double f;
    fold(r[3 * i + 1], a, L, cy, f);
    fold(r[3 * i + 2], a, L, cz, f);
    atomicAdd(&count[cy + L * cz], 1);
}

// Exclusive scan of count[0..nb) into start and cursor (one block of 1024).
// The bins are taken in super-tiles of 16384: every thread loads its four
// runs of four bins (bins base + 4096 j + 4t .. +3) at once, then the four
// tiles of 4096 are scanned in turn (sums of four, wavefront prefix sums,
// the 16 wavefront totals in LDS) with a running carry.
__global__ __launch_bounds__(1024) void k_bin_scan(const int *__restrict__ count, int nb, int *__restrict__ start,
                                                   int *__restrict__ cursor) {
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    int carry = 0;
    for (int base = 0; base < nb; base += 16384) {
        int v[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + 4096 * j + 4 * t;
            if (idx + 3 < nb && (nb & 3) == 0) {
                const int4 w = *reinterpret_cast<const int4 *>(count + idx);
                v[j][0] = w.x;
                v[j][1] = w.y;
                v[j][2] = w.z;
                v[j][3] = w.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[j][e] = idx + e < nb ? count[idx + e] : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + 4096 * j + 4 * t;
            const int s4 = v[j][0] + v[j][1] + v[j][2] + v[j][3];
            int x = s4;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) wsum[wid] = x;
            __syncthreads();
            int before = carry, total = 0;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const int ws = wsum[w];
                if (w < wid) before += ws;
                total += ws;
            }
            int run = before + x - s4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (idx + e < nb) {
                    start[idx + e] = run;
                    cursor[idx + e] = run;
                }
                run += v[j][e];
            }
            carry += total;
            __syncthreads();
        }
    }
}

__global__ void k_bin_scatter(int n, int L, double a, const double *__restrict__ r, int *__restrict__ cursor,
                              int *__restrict__ order, int *__restrict__ slot_of, int *__restrict__ binrow) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cy, cz;
    double f;
    fold(r[3 * i + 1], a, L, cy, f);
    fold(r[3 * i + 2], a, L, cz, f);
    const int row = cy + L * cz;
    const int slot = atomicAdd(&cursor[row], 1);
    order[slot] = i;
    slot_of[i] = slot;
    binrow[i] = row;
}

__global__ void k_fill_int(int *dst, int v, size_t count) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        dst[t] = v;
}

hipError_t launch_bin_ions(memd_ctx *c) {
    if (c->n == 0 || !c->order) return hipSuccess;
    const int nb = c->L * c->L;
    const int g = (int)((nb + kThreads - 1) / kThreads) < 4096 ? (nb + kThreads - 1) / kThreads : 4096;
    int *count = c->bins, *start = c->bins + nb, *cursor = c->bins + 2 * (size_t)nb;
    hipLaunchKernelGGL(k_fill_int, dim3(g), dim3(kThreads), 0, c->stream, count, 0, (size_t)nb);
    hipLaunchKernelGGL(k_bin_count, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a, c->r,
                       count);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, c->stream, count, nb, start, cursor);
    hipLaunchKernelGGL(k_bin_scatter, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                       c->r, cursor, c->order, c->slot, c->binrow);
    return hipGetLastError();
}

// Self energies (through the force kernel, writing the same forces again).
hipError_t launch_uself(memd_ctx *c, double *partials, int *nblk) {
    const int nb = ion_blocks_x8(c->n, 1);
    *nblk = nb;
    const void *D = c->D[c->cur];
    if (c->fp32) {
        auto A = force_args<float>(c, D);
        A.uself_partials = partials;
        A.order = nullptr;  // index order: the self-energy sum is then deterministic
        hipLaunchKernelGGL(k_forces<float>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    } else {
        auto A = force_args<double>(c, D);
        A.uself_partials = partials;
        A.order = nullptr;
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
