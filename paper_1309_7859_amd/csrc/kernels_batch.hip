// kernels_batch.hip -- one global step of many independent MEMD replicas
// (different L, ion counts, permittivity profiles) in two launches with
// fixed grids.  The replica table lives in device memory and may change
// between launches (replicas join and leave) without re-capturing the graph
// that holds the launches: every workgroup walks the work items (leapfrog
// tiles, ion blocks) of all listed replicas with a grid stride, finds the
// owner replica by binary search over the item offsets, and skips replicas
// that have finished.  Fields are FP32; positions, dipole and the ion
// arithmetic are FP64; displacements come from the replica's Philox stream.
//
// Step counters (two ints per replica, no launch of their own): the deposit
// launch writes done = s + 1 after the step s it deposits; the leapfrog
// launch reads done and copies it to seen, which the deposit launch reads
// (it cannot read the counter it writes: its workgroups run in any order).
// The forces and energy of a replica's final state are computed when it
// leaves the batch, on its own context's stream.
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
    const int count = hdr[0], max_slots = hdr[2];
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

// LDS of a leapfrog work item: a 64-site row tile, or whole rows of a narrow
// lattice (RepDesc::xrows)
union BatchSmem {
    LfSmem<float, 1> tile;
    RowSmem<float> rows;
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_batch_leapfrog(const RepDesc *__restrict__ tab,
                                                        const int *__restrict__ hdr) {
    __shared__ BatchSmem U;
    const int total = hdr[1];
    const int count = stage_index(hdr, RANGE_TILES);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int ri = find_rep(count, item);
        const RepDesc &R = tab[ri];
        const int step = R.steps[1];
        if (threadIdx.x == 0) R.steps[0] = step;  // every item of the replica stores the same value
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
        if (R.xrows > 0) {
            if (R.eta_mode == ETA_UNIFORM)
                leapfrog_rows<float, ETA_UNIFORM>(A, R.xrows, rest % R.nty, rest / R.nty, U.rows);
            else
                leapfrog_rows<float, ETA_ZPROF>(A, R.xrows, rest % R.nty, rest / R.nty, U.rows);
        } else if (R.eta_mode == ETA_UNIFORM) {
            leapfrog_tile<float, ETA_UNIFORM, 1>(A, tile_x, rest % R.nty, rest / R.nty, U.tile);
        } else {
            leapfrog_tile<float, ETA_ZPROF, 1>(A, tile_x, rest % R.nty, rest / R.nty, U.tile);
        }
    }
}

// Deposit of every ion's move (its Philox displacement of this step) with
// global atomics: an item is 16 ions, 16 lanes per ion (deposit_ion_part: one
// axis and transverse corner each), so that a replica's ions spread over many
// workgroups; lanes 0-2 of each ion draw the displacement's components, lane
// 0 writes r^{n+1}.  Every item of a replica then stores the replica's new
// step count.
__global__ __launch_bounds__(256) void k_batch_deposit(const RepDesc *__restrict__ tab,
                                                       const int *__restrict__ hdr) {
    const int total = hdr[3];
    const int count = stage_index(hdr, RANGE_DEP);
    const int lane = threadIdx.x & 15;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int ri = find_rep(count, item);
        const RepDesc &R = tab[ri];
        const int step = R.steps[0];
        if (step >= R.nsteps) continue;
        const int i = (item - R.dep_off) * kDepIons + (int)(threadIdx.x >> 4);
        if (i < R.n) {
            const size_t Ns = (size_t)R.L * R.L * R.L;
            double u[3] = {R.r[3 * i], R.r[3 * i + 1], R.r[3 * i + 2]};
            // lanes 0-2 draw one component each
            const double dc =
                lane < 3 ? philox_displacement_component(R.seed, (uint32_t)step, (uint32_t)i, R.sigma, lane) : 0.0;
            double du[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) du[d] = __shfl(dc, d, 16);
            sanitize_move(du, R.a, R.L, nullptr);
            deposit_ion_part<float>(R.L, Ns, R.a, R.q[i], u, du, R.D[(step & 1) ^ 1], lane >> 2, lane & 3);
            if (lane == 0) {
                R.r[3 * i] = u[0];
                R.r[3 * i + 1] = u[1];
                R.r[3 * i + 2] = u[2];
            }
        }
        if (threadIdx.x == 0) R.steps[1] = step + 1;
    }
}

hipError_t launch_batch_leapfrog(hipStream_t s, const RepDesc *tab, const int *hdr, int max_slots, int grid) {
    hipLaunchKernelGGL(k_batch_leapfrog, dim3(grid), dim3(256), (size_t)max_slots * sizeof(int), s, tab, hdr);
    return hipGetLastError();
}

hipError_t launch_batch_step(hipStream_t s, const RepDesc *tab, const int *hdr, int max_slots, int lf_grid,
                             int dep_grid) {
    const size_t lds = (size_t)max_slots * sizeof(int);
    hipLaunchKernelGGL(k_batch_leapfrog, dim3(lf_grid), dim3(256), lds, s, tab, hdr);
    hipLaunchKernelGGL(k_batch_deposit, dim3(dep_grid), dim3(256), lds, s, tab, hdr);
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
