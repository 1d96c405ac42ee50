// kernels_ions.hip -- per-ion kernels for gfx950: current deposition, charge
// assignment, dipole moment, corrected forces; deterministic finalisers of
// the per-block partial sums; the lattice Green's function table.
#include <utility>

#include "device_util.hpp"
#include "ion_ops.hpp"
#include "ion_records.hpp"
#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"
#include "philox.hpp"

namespace memd {

// ----------------------------------------------------------- deposition

// The deposit kernel: sixteen lanes per ion (one per axis and transverse
// corner, deposit_ion_part), ions taken in the order of `order` (binned by
// lattice row, so that neighbouring lanes update neighbouring links).  Lane 0
// of each ion writes the new position.  Block sums of q r^{n+1} go to
// partials (summed in block order by k_fin_dipole).
template <typename T>
__global__ __launch_bounds__(256) void k_deposit(int n, int L, size_t Ns, double a,
                                                 const double *__restrict__ q, double *__restrict__ r,
                                                 const double *__restrict__ disp, T *__restrict__ D,
                                                 const int *__restrict__ order, const int *__restrict__ perm,
                                                 double *__restrict__ partials, unsigned int *bad,
                                                 uint64_t seed, uint32_t t, double sigma) {
    const int lane = threadIdx.x & 15;
    // consecutive (spatially sorted) ions stay on one XCD and share its L2
    const int slot = xcd_logical(blockIdx.x, gridDim.x) * (blockDim.x >> 4) + (threadIdx.x >> 4);
    double P[3] = {0.0, 0.0, 0.0};
    if (slot < n) {
        const int i = order ? order[slot] : slot;
        const int ci = perm ? perm[i] : i;  // the caller's index of the ion
        const double qi = q[i];
        double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
        double du[3];
        if (disp) {
            du[0] = disp[3 * ci];
            du[1] = disp[3 * ci + 1];
            du[2] = disp[3 * ci + 2];
        } else {
            if (lane == 0) philox_displacement(seed, t, (uint32_t)ci, sigma, du);
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

hipError_t launch_deposit(memd_ctx *c, void *D, const double *disp, double *partials, int *nblk, uint64_t seed,
                          uint32_t t, double sigma) {
    const int nb = ion_blocks_x8(c->n, 16);
    *nblk = nb;
    if (c->fp32)
        hipLaunchKernelGGL(k_deposit<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (float *)D, c->order, c->perm, partials,
                           c->bad_moves, seed, t, sigma);
    else
        hipLaunchKernelGGL(k_deposit<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->Ns, c->a,
                           c->q, c->r, disp, (double *)D, c->order, c->perm, partials,
                           c->bad_moves, seed, t, sigma);
    return hipGetLastError();
}

__global__ void k_fill_int(int *dst, int v, size_t count);

// Records for the step about to run, ions read in storage order
// (coalesced), one lane per ion, ion i's record going to its slot
// slot_of[i]; displacements are indexed by the caller's index perm[i], and
// rejected components are counted here (the movers and the finisher read
// the sanitised displacement back from the record's slot).
template <typename T>
__global__ __launch_bounds__(256) void k_pack_ions(int n, int L, double a, const double *__restrict__ q,
                                                   const double *__restrict__ r, const double *__restrict__ disp,
                                                   const int *__restrict__ slot_of, const int *__restrict__ perm,
                                                   int *__restrict__ dep_atomic, DepOut<T> O, unsigned int *bad,
                                                   uint64_t seed, uint32_t t, double sigma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    double du[3];
    step_displacement(i, L, a, disp, perm, bad, seed, t, sigma, du);
    const int s = slot_of[i];
    dep_atomic[s] = write_record<T>(L, a, q[i], u, du, s, O) ? 1 : 0;
}

// Tile lists, built at a re-binning for the current tile shape: storage
// index j (slot slot_of[j]) records its cell c_b and joins the list of every
// tile that owns a link with origin in [c_b - 2, c_b + 3] along each axis.
// Lanes of a wavefront that join the same tile in the same round reserve
// their entries with one atomic (sorted ions share tiles).  An ion that
// would need more than 4 tiles along an axis or finds a list full is
// marked list_fail: its record head is then -1 at every step, so tiles that
// do list it skip it, and it is deposited with atomics.
struct TileLists {
    int *list, *count;
    int cap, TY, TZ, ntx, nty;
};

// What the list builder needs to write the records too (the pack right
// after a re-binning).
template <typename T>
struct PackArgs {
    const double *q, *disp;
    const int *perm;
    int *dep_atomic;
    DepOut<T> O;
    unsigned int *bad;
    uint64_t seed;
    uint32_t t;
    double sigma;
    // non-null: the position each move ends at (by storage index) and one
    // partial of q r per block (the ions' own dynamics, whose leapfrog then
    // runs no movers)
    double *r_next;
    double *pos_dip;
};

// Lists of the fused deposit, one lane per ion in storage order: the ion's
// cell c goes to cbin, and its slot to every tile owning a link with origin
// in [c - 2, c + 3] along each axis.  A wavefront reserves list places in
// rounds (one per tile of each lane's box), with one atomic per distinct
// tile and round; eight rounds' atomics are issued before their places are
// written.  An ion that would need more than four tiles along an axis, or
// finds a list full, is marked in list_fail.  With PACK the lane then writes
// the ion's record for the step about to run (as k_pack_ions).
template <typename T, bool PACK>
__global__ __launch_bounds__(256) void k_build_lists(int n, int L, double a, const double *__restrict__ r,
                                                     const int *__restrict__ slot_of, int *__restrict__ cbin,
                                                     int *__restrict__ list_fail, TileLists TL, PackArgs<T> PA) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    int nres = 0, s = 0, cb = 0;
    int tid[3][4], nt[3] = {0, 0, 0};
    bool fail = false;
    if (j < n) {
        s = slot_of[j];
        int c[3];
        double f;
#pragma unroll
        for (int e = 0; e < 3; ++e) fold(r[3 * j + e], a, L, c[e], f);
        cb = pack_cell(c[0], c[1], c[2]);
        cbin[s] = cb;
        const int ext[3] = {64, TL.TY, TL.TZ};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            for (int off = -2; off <= 3; ++off) {
                int cell = c[e] + off;
                cell += cell < 0 ? L : (cell >= L ? -L : 0);
                const int tt = cell / ext[e];
                bool seen = false;
                for (int k = 0; k < nt[e]; ++k) seen = seen || tid[e][k] == tt;
                if (seen) continue;
                if (nt[e] == 4) {
                    fail = true;
                    break;
                }
                tid[e][nt[e]++] = tt;
            }
        }
        nres = fail ? 0 : nt[0] * nt[1] * nt[2];
    }
    // every lane of the wavefront takes part in the reservation rounds
    constexpr int kBatch = 8;
    bool ok = !fail;
    for (int k0 = 0; __ballot(k0 < nres) != 0ull; k0 += kBatch) {
        int my[kBatch], lead[kBatch], rank[kBatch], base[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int k = k0 + u;
            my[u] = -1;
            if (k < nres) {
                const int kx = k % nt[0], ky = (k / nt[0]) % nt[1], kz = k / (nt[0] * nt[1]);
                my[u] = tid[0][kx] + TL.ntx * (tid[1][ky] + TL.nty * tid[2][kz]);
            }
            unsigned long long rem = __ballot(my[u] >= 0);
            lead[u] = lane;
            rank[u] = 0;
            int take = 0;
            while (rem) {
                const int l = __ffsll((long long)rem) - 1;
                const int idl = __builtin_amdgcn_readlane(my[u], l);
                const unsigned long long same = __ballot(my[u] == idl);
                if (my[u] == idl) {
                    lead[u] = l;
                    rank[u] = __popcll(same & below);
                }
                if (lane == l) take = __popcll(same);
                rem &= ~same;
            }
            base[u] = 0;
            if (take > 0) base[u] = atomicAdd(&TL.count[(size_t)my[u] * kCountStride], take);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int b = __shfl(base[u], lead[u], 64);
            if (my[u] >= 0) {
                const int pos = b + rank[u];
                if (pos >= TL.cap) ok = false;
                else TL.list[(size_t)my[u] * TL.cap + pos] = s;
            }
        }
    }
    double pn[3] = {0.0, 0.0, 0.0};
    if (j < n) {
        list_fail[s] = ok ? 0 : 1;
        if constexpr (PACK) {
            const double u[3] = {r[3 * j], r[3 * j + 1], r[3 * j + 2]};
            double du[3];
            step_displacement(j, L, a, PA.disp, PA.perm, PA.bad, PA.seed, PA.t, PA.sigma, du);
            PA.dep_atomic[s] = write_record_at<T>(L, a, PA.q[j], u, du, s, PA.O, ok ? 0 : 1, cb) ? 1 : 0;
            if (PA.r_next) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double un = u[d] + du[d];  // the movers' arithmetic
                    PA.r_next[3 * j + d] = un;
                    pn[d] = PA.q[j] * un;
                }
            }
        }
    }
    if constexpr (PACK) {
        if (PA.r_next) {
            block_sum<3>(pn);
            if (threadIdx.x < 3) PA.pos_dip[3 * blockIdx.x + threadIdx.x] = pn[threadIdx.x];
        }
    }
}

// Builds the lists for the current tile shape; with pack, also the records
// for the step about to run.  The counts start from zero: cleared by the
// re-binning's scan for this shape (list_zero_key), else here.
hipError_t launch_build_lists(memd_ctx *c, bool pack, const double *disp, uint64_t seed, uint32_t t,
                              double sigma) {
    if (c->n == 0 || !c->list) return hipSuccess;
    TileLists TL;
    TL.list = c->list;
    TL.count = c->list_count;
    TL.TY = 4 * c->lf_rows;
    TL.TZ = c->lf_tz;
    TL.ntx = (c->L + 63) / 64;
    TL.nty = (c->L + TL.TY - 1) / TL.TY;
    TL.cap = list_cap(c);
    const int key = c->lf_rows * 4096 + c->lf_tz;
    if (c->list_zero_key != key) {
        const size_t nc = (size_t)list_tiles(c) * kCountStride;
        hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((nc + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           c->stream, c->list_count, 0, nc);
    }
    c->list_zero_key = -1;  // the counts are in use from here on
    if (pack && c->tile_irregular && c->irr_zeroed != c->step_index) launch_clear_irregular(c);
    c->irr_zeroed = -1;
    const int nb = ion_blocks(c->n);
    // the ions' own dynamics without movers: the end positions of the moves
    // packed here and their dipole partials come from this kernel too
    double *rn = pack && c->md_pos ? c->r_alt : nullptr;
    double *pd = rn ? c->dip[c->step_index & 1] : nullptr;
    if (rn) c->pos_nb = nb;
    if (pack && c->fp32) {
        PackArgs<float> PA{c->q,  disp, c->perm, c->dep_atomic, dep_out<float>(c), c->bad_moves, seed, t, sigma,
                           rn,    pd};
        hipLaunchKernelGGL((k_build_lists<float, true>), dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                           c->r, c->slot, c->cbin, c->list_fail, TL, PA);
    } else if (pack) {
        PackArgs<double> PA{c->q,  disp, c->perm, c->dep_atomic, dep_out<double>(c), c->bad_moves, seed, t, sigma,
                            rn,    pd};
        hipLaunchKernelGGL((k_build_lists<double, true>), dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                           c->r, c->slot, c->cbin, c->list_fail, TL, PA);
    } else {
        PackArgs<float> PA{};
        hipLaunchKernelGGL((k_build_lists<float, false>), dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                           c->r, c->slot, c->cbin, c->list_fail, TL, PA);
    }
    c->lists_key = key;
    return hipGetLastError();
}

// The count of the atomic-path ions of the step whose records are about to
// be written whole, cleared first (a fill kernel, so that a captured stream
// records no memset).
hipError_t launch_clear_irregular(memd_ctx *c) {
    if (int *cnt = irr_count(c, c->step_index))
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, cnt, 0, (size_t)1);
    return hipGetLastError();
}

hipError_t launch_pack_ions(memd_ctx *c, const double *disp, uint64_t seed, uint32_t t, double sigma) {
    if (c->n == 0) return hipSuccess;
    if (c->tile_irregular && c->irr_zeroed != c->step_index) launch_clear_irregular(c);
    c->irr_zeroed = -1;
    const int nb = ion_blocks(c->n);
    if (c->fp32)
        hipLaunchKernelGGL(k_pack_ions<float>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->a, c->q,
                           c->r, disp, c->slot, c->perm, c->dep_atomic, dep_out<float>(c), c->bad_moves, seed, t,
                           sigma);
    else
        hipLaunchKernelGGL(k_pack_ions<double>, dim3(nb), dim3(kThreads), 0, c->stream, c->n, c->L, c->a, c->q,
                           c->r, disp, c->slot, c->perm, c->dep_atomic, dep_out<double>(c), c->bad_moves, seed, t,
                           sigma);
    return hipGetLastError();
}

// The ion side of one step after the fused leapfrog and its movers, one
// ion per thread in bin order:
//   - the forces of the state the step started from: the lattice part and
//     self force from the leapfrog tile that owns the ion's start cell
//     (stamped with that launch's tag), or gathered here (force_ion on D^n,
//     which the leapfrog left intact) for an ion no tile took; plus the
//     dipole term with P^n, which the leapfrog summed from the previous
//     step's partials into the scalars;
//   - the whole move of each irregular ion of the current records deposited
//     into D^{n+1} with global atomics, from r^n (the movers wrote r^{n+1}
//     elsewhere) and the record's displacement.
template <typename T>
struct IonFinishArgs {
    int n, L;
    size_t Ns;
    double a, V;
    const double *q, *r;
    const int *order;  // null: the identity (ions stored in bin order)
    const T *Dcur;
    T *Dnext;
    int eta_mode;
    double eta_uni;
    const T *eta_prof, *eta_link;
    const double *scal;
    double *F;
    const double *Ft;           // [3n] by slot: lattice part + self force from the leapfrog tiles
    const unsigned int *fdone;  // [n] by slot: == tag when the tiles computed Ft
    unsigned int tag;
    const int *dep_atomic;  // [n] by slot: the ion is left to the atomic path this step
    const double *du;       // [3n] by slot: this step's displacements
    int self_direct;        // 1: direct self subtraction; the tiles' results (Green's function) are not used
    int no_forces;          // 1: only the irregular deposits (the ions' own dynamics gathers the forces after)
    int tiles_deposit;      // 1: the leapfrog tiles deposited the atomic-path ions (none here)
};

template <typename T>
__global__ __launch_bounds__(256) void k_ion_finish(IonFinishArgs<T> A) {
    const int s = xcd_logical(blockIdx.x, gridDim.x) * kThreads + (int)threadIdx.x;
    if (s >= A.n) return;
    const int i = A.order ? A.order[s] : s;
    const double qi = A.q[i];
    if (A.no_forces) {
        if (A.dep_atomic[s] != 0 && !A.tiles_deposit) {
            double w[3] = {A.r[3 * i], A.r[3 * i + 1], A.r[3 * i + 2]};
            const double du[3] = {A.du[3 * s], A.du[3 * s + 1], A.du[3 * s + 2]};
            deposit_ion<T>(A.L, A.Ns, A.a, qi, w, du, A.Dnext);
        }
        return;
    }
    // the tile result is read with its stamp, not after it
    const double ft[3] = {A.Ft[3 * s], A.Ft[3 * s + 1], A.Ft[3 * s + 2]};
    const bool tiled = !A.self_direct && A.fdone[s] == A.tag;
    const bool atomic_path = A.dep_atomic[s] != 0;
    double F[3] = {ft[0], ft[1], ft[2]};
    if (!tiled || atomic_path) {
        const double u[3] = {A.r[3 * i], A.r[3 * i + 1], A.r[3 * i + 2]};
        const EtaView<T> ev{A.eta_mode, A.eta_uni, A.eta_prof, A.eta_link};
        if (!tiled) {
            // the dipole term is added below (x + 0 + y rounds as x + y)
            const double zero[3] = {0.0, 0.0, 0.0};
            force_ion<T>(A.L, A.Ns, A.a, A.V, qi, u, A.Dcur, ev, A.scal + S_G, zero, A.scal + S_EPSH, F,
                         A.self_direct != 0);
        }
        if (atomic_path && !A.tiles_deposit) {
            double w[3] = {u[0], u[1], u[2]};
            const double du[3] = {A.du[3 * s], A.du[3 * s + 1], A.du[3 * s + 2]};
            deposit_ion<T>(A.L, A.Ns, A.a, qi, w, du, A.Dnext);
        }
    }
    const double w = A.scal[S_DIPW];  // 1, or 0 without the dipole correction
#pragma unroll
    for (int d = 0; d < 3; ++d) A.F[3 * i + d] = F[d] + qi * (w * A.scal[S_P + d]) / (A.V * A.scal[S_EPSH + d]);
}

hipError_t launch_ion_finish(memd_ctx *c, const void *Dcur, void *Dnext, bool forces) {
    const int nb = ion_blocks_x8(c->n);
    auto fill = [&](auto &A) {
        A.n = c->n;
        A.L = c->L;
        A.Ns = c->Ns;
        A.a = c->a;
        A.V = c->V;
        A.q = c->q;
        A.r = c->r;
        A.order = c->sorted ? nullptr : c->order;
        A.eta_mode = c->eta_mode;
        A.eta_uni = c->eta_uni;
        A.scal = c->scal;
        A.F = c->F;
        A.Ft = c->Ft;
        A.fdone = c->fdone;
        A.tag = c->force_tag;
        A.dep_atomic = c->dep_atomic;
        A.du = c->du_slot;
        A.self_direct = c->self_scheme == MEMD_SELF_DIRECT;
        A.no_forces = forces ? 0 : 1;
        A.tiles_deposit = c->tile_irregular ? 1 : 0;
    };
    if (c->fp32) {
        IonFinishArgs<float> A;
        fill(A);
        A.Dcur = (const float *)Dcur;
        A.Dnext = (float *)Dnext;
        A.eta_prof = (const float *)c->eta_prof;
        A.eta_link = (const float *)c->eta_link;
        hipLaunchKernelGGL(k_ion_finish<float>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    } else {
        IonFinishArgs<double> A;
        fill(A);
        A.Dcur = (const double *)Dcur;
        A.Dnext = (double *)Dnext;
        A.eta_prof = (const double *)c->eta_prof;
        A.eta_link = (const double *)c->eta_link;
        hipLaunchKernelGGL(k_ion_finish<double>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    }
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

hipError_t launch_spread_raw(hipStream_t s, int n, int L, double a, const double *q, const double *r,
                             double *dst) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spread, dim3(ion_blocks(n)), dim3(kThreads), 0, s, n, L, a, q, r, dst);
    return hipGetLastError();
}

hipError_t launch_spread(memd_ctx *c, const double *charges_or_null, double *dst) {
    return launch_spread_raw(c->stream, c->n, c->L, c->a, charges_or_null ? c->q : nullptr, c->r, dst);
}

// The same assignment without global atomics, for ions stored in bin order
// (the storage indices start[row] .. start[row + 1] of bin row row = y + L z
// are the ions whose cell lay in that lattice row at the last re-binning).
// A workgroup owns a tile of 64 x 4 x 8 vertices.  Its vertices draw from
// cells one below them along each axis, so it reads the ions of the bin
// rows y0 - 2 .. y0 + 4 and z0 - 2 .. z0 + 8 (every x), keeps those whose
// cell is still within one row of their bin row along y and z, adds their
// weights on its vertices in LDS, and stores every vertex of the tile.  The
// workgroup with x0 = 0 whose rows contain an ion's bin row marks, in
// drifted, whether that ion moved further (k_spread_drifted adds those).
constexpr int kSpTY = 4, kSpTZ = 8;
constexpr int kSpRows = (kSpTY + 3) * (kSpTZ + 3);

// With TWO, the same pass also assigns unit weights into dst2 (the ion
// counts of the salt permittivity beside the charge density of the audit).
template <bool TWO>
__global__ __launch_bounds__(256) void k_spread_tile(int n, int L, double a, const double *__restrict__ q,
                                                     const double *__restrict__ r, const int *__restrict__ start,
                                                     int *__restrict__ drifted, double *__restrict__ dst,
                                                     double *__restrict__ dst2) {
    __shared__ double acc[kSpTZ][kSpTY][64];
    __shared__ double acc2[TWO ? kSpTZ : 1][TWO ? kSpTY : 1][TWO ? 64 : 1];
    __shared__ int row_beg[kSpRows], row_off[kSpRows + 1];
    const int ntx = (L + 63) >> 6, nty = (L + kSpTY - 1) / kSpTY;
    const int tile = blockIdx.x;
    const int x0 = (tile % ntx) * 64, y0 = ((tile / ntx) % nty) * kSpTY, z0 = (tile / (ntx * nty)) * kSpTZ;
    double *accf = &acc[0][0][0];
    for (int t = threadIdx.x; t < kSpTZ * kSpTY * 64; t += blockDim.x) {
        accf[t] = 0.0;
        if constexpr (TWO) (&acc2[0][0][0])[t] = 0.0;
    }
    if (threadIdx.x < kSpRows) {
        const int iy = threadIdx.x % (kSpTY + 3), iz = threadIdx.x / (kSpTY + 3);
        const int row = wrapc(y0 - 2 + iy, L) + L * wrapc(z0 - 2 + iz, L);
        const int b = start[row], e = row + 1 < L * L ? start[row + 1] : n;
        row_beg[threadIdx.x] = b;
        row_off[threadIdx.x + 1] = e - b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        row_off[0] = 0;
        for (int k = 0; k < kSpRows; ++k) row_off[k + 1] += row_off[k];
    }
    __syncthreads();
    const int total = row_off[kSpRows];
    const int own_ny = min(kSpTY, L - y0), own_nz = min(kSpTZ, L - z0);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        int lo = 0, hi = kSpRows - 1;  // the candidate row holding entry e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (row_off[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int i = row_beg[lo] + (e - row_off[lo]);
        const int iy = lo % (kSpTY + 3), iz = lo / (kSpTY + 3);
        const double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
        int cc[3];
        double ff[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) fold(u[d], a, L, cc[d], ff[d]);
        // cell rows relative to the bin row, periodic, in 0 .. L-1
        int dy = cc[1] - wrapc(y0 - 2 + iy, L), dz = cc[2] - wrapc(z0 - 2 + iz, L);
        dy += dy < 0 ? L : 0;
        dz += dz < 0 ? L : 0;
        const bool near = (dy <= 1 || dy >= L - 1) && (dz <= 1 || dz >= L - 1);
        if (x0 == 0 && (unsigned)(iy - 2) < (unsigned)own_ny && (unsigned)(iz - 2) < (unsigned)own_nz)
            drifted[i] = near ? 0 : 1;
        if (!near) continue;
        const double qi = q ? q[i] : 1.0;
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
            const int lx = (ox ? (cc[0] + 1 == L ? 0 : cc[0] + 1) : cc[0]) - x0;
            const int ly = (oy ? (cc[1] + 1 == L ? 0 : cc[1] + 1) : cc[1]) - y0;
            const int lz = (oz ? (cc[2] + 1 == L ? 0 : cc[2] + 1) : cc[2]) - z0;
            if ((unsigned)lx < 64u && (unsigned)ly < (unsigned)kSpTY && (unsigned)lz < (unsigned)kSpTZ) {
                const double w = lin_w(ox, ff[0]) * lin_w(oy, ff[1]) * lin_w(oz, ff[2]);
                atomicAdd(&acc[lz][ly][lx], qi * w);
                if constexpr (TWO) atomicAdd(&acc2[lz][ly][lx], w);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSpTZ * kSpTY * 64; t += blockDim.x) {
        const int lx = t & 63, ly = (t >> 6) % kSpTY, lz = t / (64 * kSpTY);
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (x < L && y < L && z < L) {
            dst[((size_t)z * L + y) * L + x] = acc[lz][ly][lx];
            if constexpr (TWO) dst2[((size_t)z * L + y) * L + x] = acc2[lz][ly][lx];
        }
    }
}

__global__ __launch_bounds__(256) void k_spread_drifted(int n, int L, double a, const double *__restrict__ q,
                                                        const double *__restrict__ r,
                                                        const int *__restrict__ drifted, double *__restrict__ dst,
                                                        double *__restrict__ dst2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !drifted[i]) return;
    const double u[3] = {r[3 * i], r[3 * i + 1], r[3 * i + 2]};
    spread_ion(L, a, q ? q[i] : 1.0, u, dst);
    if (dst2) spread_ion(L, a, 1.0, u, dst2);
}

// dst <- linear assignment of the ions (charges q, or 1 each without
// `weighted`) onto the vertices; every vertex is written.  With dst2 (and
// `weighted`), the same pass also writes the unit-weight assignment (ion
// counts) into dst2.
hipError_t launch_spread_dense(memd_ctx *c, bool weighted, double *dst, double *dst2) {
    const double *q = weighted ? c->q : nullptr;
    if (c->n > 0 && c->sorted && c->L >= 16) {
        const int L = c->L, nb = L * L;
        const int tiles = ((L + 63) / 64) * ((L + kSpTY - 1) / kSpTY) * ((L + kSpTZ - 1) / kSpTZ);
        if (dst2)
            hipLaunchKernelGGL(k_spread_tile<true>, dim3(tiles), dim3(kThreads), 0, c->stream, c->n, L, c->a, q,
                               c->r, c->bins + nb, c->drift, dst, dst2);
        else
            hipLaunchKernelGGL(k_spread_tile<false>, dim3(tiles), dim3(kThreads), 0, c->stream, c->n, L, c->a, q,
                               c->r, c->bins + nb, c->drift, dst, nullptr);
        hipLaunchKernelGGL(k_spread_drifted, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, L, c->a,
                           q, c->r, c->drift, dst, dst2);
        return hipGetLastError();
    }
    hipError_t e = launch_fill(c->stream, dst, 0.0, c->Ns);
    if (e != hipSuccess) return e;
    if ((e = launch_spread(c, q, dst)) != hipSuccess) return e;
    if (!dst2) return hipSuccess;
    if ((e = launch_fill(c->stream, dst2, 0.0, c->Ns)) != hipSuccess) return e;
    return launch_spread(c, nullptr, dst2);
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
    int self_direct;  // 1: direct self subtraction
    int *zero;        // optional: cleared (the next call's atomic-path count)
};

// Forces on every ion, one lane per ion following `order` (force_ion: the
// lattice part from the 12 links of the cell, self force, dipole
// correction).  With dip_partials set, every block sums the per-workgroup
// q r partials of the last step's movers into P (in the dipole finaliser's order;
// block 0 also stores it) while its force gathers are in flight.
template <typename T>
__global__ __launch_bounds__(256) void k_forces(ForceArgs<T> A) {
    __shared__ double Psh[3];
    if (A.zero && blockIdx.x == 0 && threadIdx.x == 0) *A.zero = 0;
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
        us = force_ion<T>(A.L, A.Ns, A.a, A.V, qi, u, A.D, ev, A.scal + S_G, zero, A.scal + S_EPSH, F,
                          A.self_direct != 0);
    }
    if (A.dip_partials) {
        // P summed as the dipole finaliser sums it (fin_sum)
        double s[3];
        strided_sum<3>(A.dip_partials, A.dip_nblk, threadIdx.x, blockDim.x, s);
        block_sum<3>(s);
        if (threadIdx.x < 3) {
            Psh[threadIdx.x] = s[threadIdx.x];
            if (blockIdx.x == 0) A.scal[S_P + threadIdx.x] = s[threadIdx.x];
        }
    } else if (threadIdx.x < 3) {
        Psh[threadIdx.x] = A.scal[S_P + threadIdx.x];
    }
    __syncthreads();
    if (live) {
        const double w = A.scal[S_DIPW];  // 1, or 0 without the dipole correction
#pragma unroll
        for (int d = 0; d < 3; ++d) A.F[3 * i + d] = F[d] + qi * (w * Psh[d]) / (A.V * A.scal[S_EPSH + d]);
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
    A.order = c->sorted ? nullptr : c->order;  // identity once the ions are stored in bin order
    A.dip_partials = nullptr;
    A.dip_nblk = 0;
    A.self_direct = c->self_scheme == MEMD_SELF_DIRECT;
    A.zero = nullptr;
    return A;
}

hipError_t launch_forces(memd_ctx *c, const void *D, const double *dip_partials, int dip_nblk, bool zero_irr) {
    if (c->n == 0) return hipSuccess;
    const int nb = ion_blocks_x8(c->n, 1);
    // the count of the next step's atomic-path ions, cleared here for the
    // pack that starts the next call (nothing appends to it in between)
    int *zero = zero_irr && c->tile_irregular ? irr_count(c, c->step_index) : nullptr;
    if (c->fp32) {
        auto A = force_args<float>(c, D);
        A.dip_partials = dip_partials;
        A.dip_nblk = dip_nblk;
        A.zero = zero;
        hipLaunchKernelGGL(k_forces<float>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    } else {
        auto A = force_args<double>(c, D);
        A.dip_partials = dip_partials;
        A.dip_nblk = dip_nblk;
        A.zero = zero;
        hipLaunchKernelGGL(k_forces<double>, dim3(nb), dim3(kThreads), 0, c->stream, A);
    }
    if (zero) c->irr_zeroed = c->step_index;
    return hipGetLastError();
}

// The ion side of one step of the ions' own dynamics, after the leapfrog
// (and the finisher's irregular deposits) produced the new state: one thread
// per ion in storage order (in bin order once binned, so the gathers of
// neighbouring lanes share lines), caller index ci = perm[i]:
//   - with gather, the forces of the new state (force_ion on D: lattice part,
//     self force, dipole term with P summed, as k_forces does, from the
//     movers' per-workgroup partials), into F; else F as it stands.  When
//     the leapfrog tiles captured E = eta D on the 12 links of the ion's cell
//     (ecap, by slot: every ion but those stamped with cap_tag in ecap_bad),
//     the lattice part comes from those values and the self force from the
//     cell's 12 / sum(eta) (ecell), the arithmetic of force_ion without its
//     gather;
//   - `kicks` half kicks v <- v + (dt/2) F/m (the closing kick of the step and
//     the opening one of the next use the same forces);
//   - with pack, the move of the next step, dt v, into disp (caller order:
//     the plain path's deposit and a re-binning's list builder read it), and
//     with records also, sanitised, into the ion's record of the current
//     record set (as k_pack_ions writes it).
template <typename T>
struct MdIonArgs {
    ForceArgs<T> fa;  // D, permittivity, scalars, F, order, dipole partials, scheme
    int gather;
    const int *perm;
    const int *slot_of;
    const double *mass;
    double *v;
    int kicks;
    double half_dt, dt;
    double *disp;
    int pack;
    int records;
    int *dep_atomic;
    DepOut<T> O;
    unsigned int *bad;
    const T *ecap;  // null: gather
    const unsigned int *ecap_bad;
    unsigned int cap_tag;
    const T *ecell;
    // non-null (with records): the position the next move ends at (by
    // storage index) and one partial of q r of those per block, for the
    // leapfrog of the next step, which then runs no movers
    double *r_next;
    double *pos_dip;
};

// force_ion's lattice part and Green's-function self force from the field
// already interpolated to the cell's 12 links (E[4 d + 2 o2 + o1]) and the
// cell's 12 / sum(eta); the dipole term is added by the caller.
template <typename T>
__device__ __forceinline__ void force_from_links(int L, double a, double qi, const double (&u)[3], const T (&e)[12],
                                                 const T *ecell, const double *G, double (&F)[3]) {
    int c[3];
    double f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fold(u[d], a, L, c[d], f[d]);
    const double eps_cell = (double)ecell[site_index(c[0], c[1], c[2], L)];
    double Flat[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
        double s = 0.0;
#pragma unroll
        for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
            for (int o1 = 0; o1 < 2; ++o1) s += lin_w(o1, f[d1]) * lin_w(o2, f[d2]) * (double)e[4 * d + 2 * o2 + o1];
        Flat[d] = qi * s;
    }
    double S, dS[3];
    self_sum(G, f, S, dS);
    const double pref = qi * qi / (2.0 * eps_cell * a);
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = Flat[d] - div_a(-pref * dS[d], a);
}

template <typename T>
__global__ __launch_bounds__(256) void k_md_ions(MdIonArgs<T> M) {
    const ForceArgs<T> &A = M.fa;
    __shared__ double Psh[3];
    const int slot = xcd_logical(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool live = slot < A.n;
    const int i = live ? (A.order ? A.order[slot] : slot) : 0;
    // Every load that needs only the slot is issued first (position, charge,
    // caller index, record slot, the captured field and its stamp, the
    // dipole partials), then those that depend on them.
    double u[3] = {0.0, 0.0, 0.0}, qi = 0.0;
    int ci = 0, rs = 0;
    if (live) {
        u[0] = A.r[3 * i];
        u[1] = A.r[3 * i + 1];
        u[2] = A.r[3 * i + 2];
        qi = A.q[i];
        ci = M.perm[i];
        if (M.records) rs = M.slot_of[i];
    }
    const bool cap = M.gather && M.ecap != nullptr;
    unsigned int bad = 0u;
    union {
        T v[12];
        uint4 w[kCellWords<T>];
    } E;
    if (cap && live) {
        bad = M.ecap_bad[slot];
        const uint4 *src = reinterpret_cast<const uint4 *>(M.ecap + 12 * (size_t)slot);
#pragma unroll
        for (int q = 0; q < kCellWords<T>; ++q) E.w[q] = src[q];
    }
    const bool psum = M.gather && A.dip_partials != nullptr;
    double Ps[3] = {0.0, 0.0, 0.0};
    if (psum) strided_sum<3>(A.dip_partials, A.dip_nblk, threadIdx.x, blockDim.x, Ps);
    double m = 1.0, vv[3] = {0.0, 0.0, 0.0};
    int lfail = 0, lcell = 0;
    if (live) {
        m = M.mass[ci];
#pragma unroll
        for (int d = 0; d < 3; ++d) vv[d] = M.v[3 * ci + d];
        if (M.records) {
            lfail = M.O.list_fail[rs];
            lcell = M.O.cbin[rs];
        }
    }
    double F[3] = {0.0, 0.0, 0.0};
    if (M.gather) {
        if (live) {
            if (cap && bad != M.cap_tag) {
                force_from_links<T>(A.L, A.a, qi, u, E.v, M.ecell, A.scal + S_G, F);
            } else {
                const EtaView<T> ev{A.mode, A.eta_uni, A.eta_prof, A.eta_link};
                const double zero[3] = {0.0, 0.0, 0.0};
                force_ion<T>(A.L, A.Ns, A.a, A.V, qi, u, A.D, ev, A.scal + S_G, zero, A.scal + S_EPSH, F,
                             A.self_direct != 0);
            }
        }
        // the dipole field w P_d / (V eps_h_d), once per block
        if (psum) block_sum<3>(Ps);
        if (threadIdx.x < 3) {
            const int d = threadIdx.x;
            double Pd = d == 0 ? Ps[0] : (d == 1 ? Ps[1] : Ps[2]);
            if (!psum) Pd = A.scal[S_P + d];
            else if (blockIdx.x == 0) A.scal[S_P + d] = Pd;
            Psh[d] = (A.scal[S_DIPW] * Pd) / (A.V * A.scal[S_EPSH + d]);
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                F[d] = F[d] + qi * Psh[d];
                A.F[3 * i + d] = F[d];
            }
        }
    } else if (live) {
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = A.F[3 * i + d];
    }
    double pn[3] = {0.0, 0.0, 0.0};
    if (live) {
        double du[3];
        const double hm = M.half_dt / m;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double kick = hm * F[d];
            double w = vv[d] + kick;
            if (M.kicks == 2) w = w + kick;
            M.v[3 * ci + d] = w;
            du[d] = M.dt * w;
        }
        if (M.pack) {
#pragma unroll
            for (int d = 0; d < 3; ++d) M.disp[3 * ci + d] = du[d];
        }
        if (M.records) {
            sanitize_move(du, A.a, A.L, M.bad);
            M.dep_atomic[rs] = write_record_at<T, true>(A.L, A.a, qi, u, du, rs, M.O, lfail, lcell) ? 1 : 0;
            if (M.r_next) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double un = u[d] + du[d];  // the movers' arithmetic
                    M.r_next[3 * i + d] = un;
                    pn[d] = qi * un;
                }
            }
        }
    }
    if (M.r_next) {
        block_sum<3>(pn);
        if (threadIdx.x < 3) M.pos_dip[3 * blockIdx.x + threadIdx.x] = pn[threadIdx.x];
    }
}

hipError_t launch_md_ions(memd_ctx *c, const void *D, const double *dip_partials, int dip_nblk, bool gather,
                          const double *mass, double *v, int kicks, double *disp, bool pack, bool records,
                          bool positions) {
    if (c->n == 0) return hipSuccess;
    const int nb = ion_blocks_x8(c->n, 1);
    double *rn = records && positions ? c->r_alt : nullptr;
    if (rn) c->pos_nb = nb;
    auto fill = [&](auto &M) {
        M.gather = gather ? 1 : 0;
        M.fa.dip_partials = dip_partials;
        M.fa.dip_nblk = dip_nblk;
        M.perm = c->perm;
        M.slot_of = c->slot;
        M.mass = mass;
        M.v = v;
        M.kicks = kicks;
        M.half_dt = 0.5 * c->dt;
        M.dt = c->dt;
        M.disp = disp;
        M.pack = pack ? 1 : 0;
        M.records = records ? 1 : 0;
        M.dep_atomic = c->dep_atomic;
        M.bad = c->bad_moves;
        // the field the leapfrog tiles captured for the state just made
        const bool cap = gather && c->ecap_tag != 0u;
        M.ecap_bad = cap ? c->ecap_bad : nullptr;
        M.cap_tag = c->ecap_tag;
        M.r_next = rn;
        M.pos_dip = rn ? c->dip[c->step_index & 1] : nullptr;
    };
    if (c->fp32) {
        MdIonArgs<float> M;
        M.fa = force_args<float>(c, D);
        fill(M);
        M.ecap = M.ecap_bad ? (const float *)c->ecap : nullptr;
        M.ecell = (const float *)c->ecell;
        M.O = dep_out<float>(c);
        hipLaunchKernelGGL(k_md_ions<float>, dim3(nb), dim3(kThreads), 0, c->stream, M);
    } else {
        MdIonArgs<double> M;
        M.fa = force_args<double>(c, D);
        fill(M);
        M.ecap = M.ecap_bad ? (const double *)c->ecap : nullptr;
        M.ecell = (const double *)c->ecell;
        M.O = dep_out<double>(c);
        hipLaunchKernelGGL(k_md_ions<double>, dim3(nb), dim3(kThreads), 0, c->stream, M);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- ion binning

// Counting sort of the ions by lattice row (y, z cell of the position): the
// deposit and force kernels then visit neighbouring ions together.
// Wavefront-aggregated add of 1 to ctr[key] per active lane (key < 0: none):
// one atomic per distinct key, every lane gets its own position (the
// returned value plus its rank among the lanes with its key, in lane order)
// when `ret` is set.  Ions in (nearly) bin order share keys within a wavefront.
__device__ __forceinline__ int wave_add_one(int *ctr, int key, bool ret) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long rem = __ballot(key >= 0);
    int lead = lane, rank = 0, take = 0;
    while (rem) {
        const int l = __ffsll((long long)rem) - 1;
        const int kl = __builtin_amdgcn_readlane(key, l);
        const unsigned long long same = __ballot(key == kl);
        if (key == kl) {
            lead = l;
            rank = __popcll(same & below);
        }
        if (lane == l) take = __popcll(same);
        rem &= ~same;
    }
    // the leaders' atomics all go out together
    int base = 0;
    if (take > 0) {
        if (ret) base = atomicAdd(&ctr[key], take);
        else atomicAdd(&ctr[key], take);
    }
    if (ret) base = __shfl(base, lead, 64);
    return base + rank;
}

// Row counts of the ions (count all zero on entry); also clears the nlc list
// counts lc (the lists are rebuilt after every binning).
__global__ void k_bin_count(int n, int L, double a, const double *__restrict__ r, int *__restrict__ count,
                            int *__restrict__ lc, int nlc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = i; k < nlc; k += gridDim.x * blockDim.x) lc[k] = 0;
    int row = -1;
    if (i < n) {
        int cy, cz;
        double f;
        fold(r[3 * i + 1], a, L, cy, f);
        fold(r[3 * i + 2], a, L, cz, f);
        row = cy + L * cz;
    }
    wave_add_one(count, row, false);
}

// Exclusive scan of count[0..nb) into start and cursor (one block of 1024),
// leaving count all zero for the next binning.  Per pass of 16384 bins each
// thread holds 16 consecutive ones (four 16-byte words): a sequential sum,
// a wavefront prefix sum of the thread totals, the 16 wavefront totals in
// LDS, then the thread's 16 starts written back as 16-byte words.
__global__ __launch_bounds__(1024) void k_bin_scan(int *__restrict__ count, int nb, int *__restrict__ start,
                                                   int *__restrict__ cursor, int *__restrict__ zero) {
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    if (zero && t == 0) *zero = 0;
    const bool vec = (nb & 3) == 0;
    int carry = 0;
    for (int base = 0; base < nb; base += 16384) {
        const int b0 = base + 16 * t;
        int v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = b0 + 4 * q;
            if (vec && idx + 3 < nb) {
                const int4 w = *reinterpret_cast<const int4 *>(count + idx);
                v[4 * q] = w.x;
                v[4 * q + 1] = w.y;
                v[4 * q + 2] = w.z;
                v[4 * q + 3] = w.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[4 * q + e] = idx + e < nb ? count[idx + e] : 0;
            }
        }
        int tot = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) tot += v[e];
        int x = tot;
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
        int run = before + x - tot;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = b0 + 4 * q;
            int st[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                st[e] = run;
                run += v[4 * q + e];
            }
            if (vec && idx + 3 < nb) {
                const int4 w = make_int4(st[0], st[1], st[2], st[3]);
                *reinterpret_cast<int4 *>(start + idx) = w;
                *reinterpret_cast<int4 *>(cursor + idx) = w;
                *reinterpret_cast<int4 *>(count + idx) = make_int4(0, 0, 0, 0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (idx + e < nb) {
                        start[idx + e] = st[e];
                        cursor[idx + e] = st[e];
                        count[idx + e] = 0;
                    }
            }
        }
        carry += total;
        __syncthreads();
    }
}

__global__ void k_bin_scatter(int n, int L, double a, const double *__restrict__ r, int *__restrict__ cursor,
                              int *__restrict__ order, int *__restrict__ slot_of) {
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
}

// Binning with the ion arrays moved into bin order: storage index j goes to
// its slot (r, q, F and the caller index perm), after which order and
// slot_of are the identity and neighbouring storage indices are
// neighbouring ions.
__global__ void k_bin_reorder(int n, int L, double a, const double *__restrict__ r, const double *__restrict__ q,
                              const double *__restrict__ F, const int *__restrict__ perm, int *__restrict__ cursor,
                              double *__restrict__ r2, double *__restrict__ q2, double *__restrict__ F2,
                              int *__restrict__ perm2, int *__restrict__ order, int *__restrict__ slot_of) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    int row = -1;
    if (j < n) {
        int cy, cz;
        double f;
        fold(r[3 * j + 1], a, L, cy, f);
        fold(r[3 * j + 2], a, L, cz, f);
        row = cy + L * cz;
    }
    const int s = wave_add_one(cursor, row, true);
    if (j >= n) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r2[3 * s + d] = r[3 * j + d];
        F2[3 * s + d] = F[3 * j + d];
    }
    q2[s] = q[j];
    perm2[s] = perm[j];
    order[s] = s;
    slot_of[s] = s;
}

__global__ void k_iota(int *dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = i;
}

// out[perm[s] * w + k] = in[s * w + k]: storage order back to the caller's.
__global__ void k_unpermute(int n, int w, const int *__restrict__ perm, const double *__restrict__ in,
                            double *__restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int ci = perm[s];
    for (int k = 0; k < w; ++k) out[(size_t)ci * w + k] = in[(size_t)s * w + k];
}

hipError_t launch_iota(hipStream_t st, int *dst, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, dst, n);
    return hipGetLastError();
}

hipError_t launch_unpermute(memd_ctx *c, int w, const double *in, double *out) {
    if (c->n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, w, c->perm, in,
                       out);
    return hipGetLastError();
}

__global__ void k_fill_int(int *dst, int v, size_t count) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
        dst[t] = v;
}

hipError_t launch_bin_ions(memd_ctx *c, bool reorder, bool zero_irr) {
    if (c->n == 0 || !c->order) return hipSuccess;
    c->lists_key = -1;  // slots and cells change: the fused deposit's lists are rebuilt before use
    const int nb = c->L * c->L;
    // count is all zero here (cleared at allocation and by every scan)
    int *count = c->bins, *start = c->bins + nb, *cursor = c->bins + 2 * (size_t)nb;
    const int nlc = c->list ? list_tiles(c) * kCountStride : 0;
    hipLaunchKernelGGL(k_bin_count, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a, c->r,
                       count, c->list_count, nlc);
    int *zero = zero_irr && c->tile_irregular ? irr_count(c, c->step_index) : nullptr;
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, c->stream, count, nb, start, cursor, zero);
    c->irr_zeroed = zero ? c->step_index : -1;
    c->list_zero_key = c->list ? c->lf_rows * 4096 + c->lf_tz : -1;
    if (reorder) {
        hipLaunchKernelGGL(k_bin_reorder, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                           c->r, c->q, c->F, c->perm, cursor, c->r_alt, c->q_alt, c->F_alt, c->perm_alt, c->order,
                           c->slot);
        std::swap(c->r, c->r_alt);
        std::swap(c->q, c->q_alt);
        std::swap(c->F, c->F_alt);
        std::swap(c->perm, c->perm_alt);
        ++c->perm_version;
        c->sorted = true;
    } else {
        hipLaunchKernelGGL(k_bin_scatter, dim3(ion_blocks(c->n)), dim3(kThreads), 0, c->stream, c->n, c->L, c->a,
                           c->r, cursor, c->order, c->slot);
    }
    return hipGetLastError();
}

// -------------------------------------------------------------- finalisers

// One block of 256 threads sums `width` values per partial block; thread t
// takes blocks t, t+256, ... in order, then the block tree reduces: the
// order is fixed, so results repeat bit for bit.
template <int W>
__device__ void fin_sum(const double *partials, int nblk, double (&out)[W]) {
    strided_sum<W>(partials, nblk, threadIdx.x, blockDim.x, out);
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
        for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * blockDim.x) {
            double v8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u * (int)blockDim.x;
                v8[u] = b < nblk ? partials[width * b + w] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b0 + u * (int)blockDim.x < nblk) s += v8[u];
        }
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
    double f[2];
    strided_fold<2>(partials, nblk, threadIdx.x, blockDim.x, 1u, f);  // max |R|, sum R^2
    double v[1] = {f[1]};
    block_sum<1>(v);
    const double m = block_max(f[0]);
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

// Finaliser of the observables (one block): from the field pass's partials
// (we, wb, max|R|, sum R^2 per block), the self-energy partials and, when
// given, the movers' dipole partials (P is then stored too): the audit
// (max, rms) and the five energies, each into the scalars and its history
// slot when asked for.  The sums run in a fixed order (that of k_fin_audit
// for the audit), so results repeat bit for bit.
__global__ void k_fin_obs(const double *fpart, int fblk, const double *ipart, int iblk, const double *dip, int dipn,
                          int audit, int energy, double Ns, double a3, double c2, double V, double *scal,
                          double *audit_hist, double *energy_hist) {
    double f[4];
    strided_fold<4>(fpart, fblk, threadIdx.x, blockDim.x, 4u, f);  // sums, max of column 2
    double s[3] = {f[0], f[1], f[3]};
    block_sum<3>(s);
    const double m = block_max(f[2]);
    double u[1] = {0.0}, P[3] = {0.0, 0.0, 0.0};
    if (energy) {
        fin_sum<1>(ipart, iblk, u);
        if (dip) fin_sum<3>(dip, dipn, P);
    }
    if (threadIdx.x != 0) return;
    if (audit) {
        scal[S_AUDIT] = m;
        scal[S_AUDIT + 1] = sqrt(s[2] / Ns);
        if (audit_hist) {
            audit_hist[0] = m;
            audit_hist[1] = scal[S_AUDIT + 1];
        }
    }
    if (energy) {
        if (dip) {
            scal[S_P] = P[0];
            scal[S_P + 1] = P[1];
            scal[S_P + 2] = P[2];
        } else {
            P[0] = scal[S_P];
            P[1] = scal[S_P + 1];
            P[2] = scal[S_P + 2];
        }
        const double we = 0.5 * a3 * s[0];
        const double wb = 0.5 * c2 * a3 * s[1];
        double ud = 0.0;  // U_dip, removed from the energy only with the dipole correction
        for (int d = 0; d < 3; ++d) ud += P[d] * P[d] / (2.0 * V * scal[S_EPSH + d]);
        ud *= scal[S_DIPW];
        const double e[5] = {we, wb, u[0], ud, we + wb - u[0] - ud};
        for (int t = 0; t < 5; ++t) {
            scal[S_ENERGY + t] = e[t];
            if (energy_hist) energy_hist[t] = e[t];
        }
    }
}

hipError_t launch_finalize_obs(memd_ctx *c, const double *fpart, int fblk, const double *ipart, int iblk,
                               const double *dip, int dipn, bool audit, bool energy, double *audit_hist,
                               double *energy_hist) {
    const double a3 = c->a * c->a * c->a;
    hipLaunchKernelGGL(k_fin_obs, dim3(1), dim3(kThreads), 0, c->stream, fpart, fblk, ipart, iblk, dip, dipn,
                       audit ? 1 : 0, energy ? 1 : 0, (double)c->Ns, a3, c->c * c->c, c->V, c->scal, audit_hist,
                       energy_hist);
    return hipGetLastError();
}

__global__ void k_fin_epsh4(const double *partials, int nblk, double Ns, double *epsh, double *etamax) {
    double f[4];
    strided_fold<4>(partials, nblk, threadIdx.x, blockDim.x, 8u, f);  // sums of eta_d, max eta
    double s[3] = {f[0], f[1], f[2]};
    block_sum<3>(s);
    const double m = block_max(f[3]);
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
