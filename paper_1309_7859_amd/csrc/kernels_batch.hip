// kernels_batch.hip -- one global step of many independent MEMD replicas
// (different L, ion counts, permittivity profiles) in four launches with
// fixed grids.  The replica table lives in device memory and may change
// between launches (replicas join and leave) without re-capturing the graph
// that holds the launches: every workgroup walks the work items (leapfrog
// tiles, ion blocks) of all listed replicas with a grid stride, finds the
// owner replica by binary search over the item offsets, and skips replicas
// that have finished.  Fields are FP32; positions, dipole and the ion
// arithmetic are FP64; displacements come from the replica's Philox stream.
#include "device_util.hpp"
#include "ion_ops.hpp"
#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"
#include "philox.hpp"
#include "serve_internal.hpp"

namespace memd {

// The owner of a work item: the last entry whose first item is at most the
// item, by binary search over the entries' offsets, staged in LDS (dynamic,
// max_slots ints) from the header's compact copy once per workgroup.
extern __shared__ int s_off[];

__device__ __forceinline__ int stage_index(const int *__restrict__ hdr, int range) {
    const int count = hdr[0], max_slots = hdr[3];
    const int *src = hdr + kHdrInts + range * max_slots;
    for (int t = threadIdx.x; t < count; t += blockDim.x) s_off[t] = src[t];
    __syncthreads();
    return count;
}

__device__ __forceinline__ int find_rep(int count, int item) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


__global__ __launch_bounds__(256) void k_batch_leapfrog(const RepDesc *__restrict__ tab,
                                                        const int *__restrict__ hdr) {
    __shared__ LfSmem<float, 1> U;
    const int total = hdr[1];
    const int count = stage_index(hdr, RANGE_TILES);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int ri = find_rep(count, item);
        const RepDesc &R = tab[ri];
        const int step = *R.step;
        if (step >= R.nsteps) continue;
        const int local = item - R.tile_off;
        const int tile_x = local % R.ntx;
        const int rest = local / R.ntx;
        const int cur = step & 1;
        LfArgs<float> A;
        A.Din = R.D[cur];
        A.Bin = R.B[cur];
        A.Dout = R.D[cur ^ 1];
        A.Bout = R.B[cur ^ 1];
        A.eta_link = nullptr;
        A.eta_prof = R.eta_prof;
        A.eta_uni = R.eta_uni;
        A.kB = R.kB;
        A.kD = R.kD;
        A.L = R.L;
        A.Ns = (size_t)R.L * R.L * R.L;
        A.ntx = R.ntx;
        A.nty = R.nty;
        A.tz = R.tz;
        __syncthreads();  // the previous item's LDS use is over
        if (R.eta_mode == ETA_UNIFORM)
            leapfrog_tile<float, ETA_UNIFORM, 1>(A, tile_x, rest % R.nty, rest / R.nty, U);
        else
            leapfrog_tile<float, ETA_ZPROF, 1>(A, tile_x, rest % R.nty, rest / R.nty, U);
    }
}

// Deposit of every ion's move (its Philox displacement of this step) with
// global atomics: an item is 16 ions, 16 lanes per ion (deposit_ion_part: one
// axis and transverse corner each), so that a replica's ions spread over many
// workgroups; lanes 0-2 of each ion draw the displacement's components, lane
// 0 writes r^{n+1}.
// One partial of q r^{n+1} per item.
__global__ __launch_bounds__(256) void k_batch_deposit(const RepDesc *__restrict__ tab,
                                                       const int *__restrict__ hdr) {
    const int total = hdr[4];
    const int count = stage_index(hdr, RANGE_DEP);
    const int lane = threadIdx.x & 15;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int ri = find_rep(count, item);
        const RepDesc &R = tab[ri];
        const int step = *R.step;
        if (step >= R.nsteps) continue;
        const int b = item - R.dep_off;
        const int i = b * kDepIons + (int)(threadIdx.x >> 4);
        double P[3] = {0.0, 0.0, 0.0};
        if (i < R.n) {
            const size_t Ns = (size_t)R.L * R.L * R.L;
            double u[3] = {R.r[3 * i], R.r[3 * i + 1], R.r[3 * i + 2]};
            // lanes 0-2 draw one component each
            const double dc = lane < 3 ? philox_displacement_component(R.seed, (uint32_t)step, (uint32_t)i, R.sigma,
                                                                       lane)
                                       : 0.0;
            double du[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) du[d] = __shfl(dc, d, 16);
            sanitize_move(du, R.a, R.L, nullptr);
            const double qi = R.q[i];
            deposit_ion_part<float>(R.L, Ns, R.a, qi, u, du, R.D[(step & 1) ^ 1], lane >> 2, lane & 3);
            if (lane == 0) {
                R.r[3 * i] = u[0];
                R.r[3 * i + 1] = u[1];
                R.r[3 * i + 2] = u[2];
#pragma unroll
                for (int d = 0; d < 3; ++d) P[d] = qi * u[d];
            }
        }
        block_sum<3>(P);
        if (threadIdx.x == 0) {
            R.dip[3 * b] = P[0];
            R.dip[3 * b + 1] = P[1];
            R.dip[3 * b + 2] = P[2];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_batch_forces(const RepDesc *__restrict__ tab,
                                                      const int *__restrict__ hdr) {
    __shared__ double Psh[3];
    const int total = hdr[2];
    const int count = stage_index(hdr, RANGE_IONS);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int ri = find_rep(count, item);
        const RepDesc &R = tab[ri];
        const int step = *R.step;
        if (step >= R.nsteps) continue;
        const int b = item - R.ion_off;
        double s[3] = {0.0, 0.0, 0.0};
        for (int k = threadIdx.x; k < R.dblocks; k += blockDim.x)
#pragma unroll
            for (int d = 0; d < 3; ++d) s[d] += R.dip[3 * k + d];
        block_sum<3>(s);
        if (threadIdx.x == 0) {
            const double w = R.scal[S_DIPW];  // 1, or 0 without the dipole correction
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Psh[d] = w * s[d];
                if (b == 0) R.scal[S_P + d] = s[d];
            }
        }
        __syncthreads();
        const int i = b * blockDim.x + threadIdx.x;
        if (i < R.n) {
            const size_t Ns = (size_t)R.L * R.L * R.L;
            const double u[3] = {R.r[3 * i], R.r[3 * i + 1], R.r[3 * i + 2]};
            EtaView<float> ev{R.eta_mode, (double)R.eta_uni, R.eta_prof, nullptr};
            double F[3];
            force_ion<float>(R.L, Ns, R.a, R.V, R.q[i], u, R.D[(step & 1) ^ 1], ev, R.scal + S_G, Psh,
                             R.scal + S_EPSH, F);
            R.F[3 * i] = F[0];
            R.F[3 * i + 1] = F[1];
            R.F[3 * i + 2] = F[2];
        }
        __syncthreads();
    }
}

__global__ void k_batch_advance(const RepDesc *__restrict__ tab, const int *__restrict__ hdr) {
    const int count = hdr[0];
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < count; r += gridDim.x * blockDim.x) {
        int *st = tab[r].step;
        if (*st < tab[r].nsteps) *st += 1;
    }
}

hipError_t launch_batch_step(hipStream_t s, const RepDesc *tab, const int *hdr, int max_slots, int lf_grid,
                             int ion_grid, int dep_grid) {
    const size_t lds = (size_t)max_slots * sizeof(int);
    hipLaunchKernelGGL(k_batch_leapfrog, dim3(lf_grid), dim3(256), lds, s, tab, hdr);
    hipLaunchKernelGGL(k_batch_deposit, dim3(dep_grid), dim3(256), lds, s, tab, hdr);
    hipLaunchKernelGGL(k_batch_forces, dim3(ion_grid), dim3(256), lds, s, tab, hdr);
    hipLaunchKernelGGL(k_batch_advance, dim3(4), dim3(256), 0, s, tab, hdr);
    return hipGetLastError();
}

// Displacements of a seeded stream (the single-system seeded step and tests).
__global__ void k_philox_disp(uint64_t seed, uint32_t t, int n, double sigma, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double du[3];
    philox_displacement(seed, t, (uint32_t)i, sigma, du);
    out[3 * i] = du[0];
    out[3 * i + 1] = du[1];
    out[3 * i + 2] = du[2];
}

hipError_t launch_philox_disp(hipStream_t s, uint64_t seed, uint32_t t, int n, double sigma, double *out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_disp, dim3((n + 255) / 256), dim3(256), 0, s, seed, t, n, sigma, out);
    return hipGetLastError();
}

}  // namespace memd
