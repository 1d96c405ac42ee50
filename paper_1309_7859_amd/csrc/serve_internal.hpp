// serve_internal.hpp -- the device-resident replica table read by the batched
// kernels (one entry per resident replica, ordered by item offsets).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace memd {

struct RepDesc {
    // geometry and tiling
    int L, n;
    int rows, tz;          // leapfrog tile: 64 x (4 rows) sites, tz planes per chunk
    int xrows;             // > 0 (L < 64): tiles of xrows whole rows of L sites instead
    int ntx, nty, nzc;
    int tiles;             // leapfrog work items
    int dblocks;           // deposit work items: 16 ions each, 16 lanes per ion
    int tile_off, dep_off; // first item of this replica in the global item ranges
    int eta_mode;          // ETA_UNIFORM or ETA_ZPROF
    int nsteps;
    float eta_uni, kB, kD; // 1/eps, dt/a, dt c^2/a
    double a, V, sigma;
    uint64_t seed;
    // buffers (owned by the replica's context)
    float *D[2];
    float *B[2];
    const float *eta_prof;
    const double *q;
    double *r;
    int *steps;    // [2] device counters: steps[0] the count the leapfrog launch saw (read by
                   // the deposit launch), steps[1] steps done
};

// table header on the device: {count, total leapfrog tiles, max_slots, total
// deposit items}, then the entries' tile_off[max_slots] and dep_off[max_slots]
// (the offsets again, compact, for the kernels' owner search)
constexpr int kHdrInts = 4;
__host__ __device__ inline int hdr_ints(int max_slots) { return kHdrInts + 2 * max_slots; }
constexpr int kDepIons = 16;  // ions per deposit item (16 lanes each)
// the item ranges of the header
enum ItemRange : int { RANGE_TILES = 0, RANGE_DEP = 1 };

hipError_t launch_batch_step(hipStream_t s, const RepDesc *tab, const int *hdr, int max_slots, int lf_grid,
                             int dep_grid);
hipError_t launch_batch_leapfrog(hipStream_t s, const RepDesc *tab, const int *hdr, int max_slots, int grid);
hipError_t launch_philox_disp(hipStream_t s, uint64_t seed, uint32_t t, int n, double sigma, double *out);

}  // namespace memd
