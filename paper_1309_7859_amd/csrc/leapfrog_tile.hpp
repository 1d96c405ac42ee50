// leapfrog_tile.hpp -- the fused leapfrog (Faraday + Ampere) on one tile of
// the lattice, shared by the single-system kernel and the batched replica
// kernel.
//
//   B^{n+1/2} = B^{n-1/2} - dt C(eta D^n)       (eqs. faraday/bfield, E = D/eps)
//   D*        = D^n + dt c^2 C^T B^{n+1/2}      (eqs. ampere/dfield, no current)
//   (C X)_d(v)   = [X_d2(v+e_d1) - X_d2(v) - X_d1(v+e_d2) + X_d1(v)] / a
//   (C^T Y)_d(v) = [Y_d2(v) - Y_d2(v-e_d1) - Y_d1(v) + Y_d1(v-e_d2)] / a
//
// The workgroup owns a 64 x (4 R) column of sites and marches through a chunk
// of z planes, staging eta*D of the current and next plane (one-site halo) and
// the new B of the current plane (-1 halo) in LDS; the new B of the plane below
// stays in registers.  Input and output are separate buffers (ping-pong).
#pragma once

#include "device_util.hpp"
#include "ion_ops.hpp"
#include "memd_internal.hpp"
#include "philox.hpp"

#include <type_traits>

namespace memd {

template <typename T>
struct LfArgs {
    const T *__restrict__ Din;
    const T *__restrict__ Bin;
    T *__restrict__ Dout;
    T *__restrict__ Bout;
    const T *__restrict__ eta_link;
    const T *__restrict__ eta_prof;
    T eta_uni;
    T kB;  // dt / a
    T kD;  // dt c^2 / a
    int L;
    size_t Ns;
    int ntx, nty, tz;
};

template <typename T, int EM>
__device__ __forceinline__ T eta_at(const LfArgs<T> &A, int d, int gz, size_t off) {
    if constexpr (EM == ETA_UNIFORM) {
        return A.eta_uni;
    } else if constexpr (EM == ETA_ZPROF) {
        return A.eta_prof[d * A.L + gz];
    } else {
        return A.eta_link[(size_t)d * A.Ns + off];
    }
}

// Ions for the deposit fused into the leapfrog.  At every re-binning each
// leapfrog tile gets the list of the ions whose cell c_b at that time lies
// within two cells of a link it owns along each axis ([c_b - 2, c_b + 3]).
// At each step an ion is "regular" when every displacement component is
// shorter than a (so each axis of its dimension-split move spans at most
// two cells) and its start cell c is within one cell of c_b along each axis:
// then all its links have origins in [c - 1, c + 2], inside the boxes the
// lists were built from, and the tiles listing it deposit it.  Other ions
// (irregular ones, drifted ones, and any that did not fit a list) take the
// atomic path: every tile deposits the part of their moves on its own links
// from the step's list of them (irr_cnt), or, without that list, the ion
// finisher deposits them after the leapfrog with global atomics.
//
// A record (one per ion, in slot order): the head, with the start cell
// packed as x | y << 10 | z << 20 (-1: nothing for the tiles), then one word
// per axis d of the move: the corner of the 2 x 2 x 2 box of links it
// touches (the first cell along d, the perpendicular cells c_d1, c_d2 of
// the position it moves from), packed the same way, bit 30 set when the
// move crosses into a second cell along d, bit 31 set when there is a move.
// The values, one array per cell along d: v[4d + 2 o2 + o1] of slot s in
// the first (second) array is what is added to D_d at the first (second)
// cell along d and c_d1 + o1, c_d2 + o2 (each wrapped).  Lattices up to
// 1024 per side.
constexpr unsigned kGroupTwo = 1u << 30, kGroupOn = 1u << 31;

__device__ __forceinline__ int pack_cell(int x, int y, int z) { return x | (y << 10) | (z << 20); }

// Values of one cell of a record, read with 16-byte loads (48 bytes in FP32,
// 96 in FP64).  The first cells of consecutive slots are contiguous; the
// second cells sit in an array of their own, read only when a move crosses
// into one (bit 30 of an axis word).
template <typename T>
struct DepCell {
    T v[12];
};
template <typename T>
constexpr int kCellWords = (int)(12 * sizeof(T) / 16);

// The tile lists: tile b (b = tile_x + ntx (tile_y + nty chunk)) lists
// the slots list[b cap, b cap + min(count[b kCountStride], cap)) (-1: an
// entry to skip).  Each count sits in a 128-byte line of its own (the list
// builder adds to them with atomics).
constexpr int kCountStride = 32;

// Per slot: the fractional position of the ion in its start cell and its
// charge, for the forces the tiles compute (field type).
template <typename T>
struct IonFQ {
    T f[3];
    T q;
};

struct DepArgs {
    const int4 *head;  // [n] by slot
    const void *con0;  // [n] DepCell<T> by slot: first cells
    const void *con1;  // [n] DepCell<T> by slot: second cells
    const int *list;   // [tiles * cap]
    const int *count;  // [tiles * kCountStride]
    int cap;
    // forces of the state the step starts from, for the regular ions whose
    // start cell the tile owns: lattice part and self force into Ft[slot],
    // fdone[slot] = tag (the dipole term is added by the ion finisher, or
    // by the movers of the next launch)
    int own_forces;     // 0: the tiles compute no forces (the ions' own dynamics gathers them)
    const void *fq;     // [n] IonFQ<T> by slot
    const void *ecell;  // [Ns] T: 12 / (sum of eta over the cell's 12 edges)
    double *Ft;         // [3n] by slot
    unsigned int *fdone;
    unsigned int tag;
    const double *G;    // lattice Green's-function table G(0..3)
    double a;
    // the previous step's dipole partials (nparts x 3; null: none), summed by
    // workgroup dip_block (a tile) into P (the scalars) in the dipole
    // finaliser's order
    const double *dip_prev;
    int dip_nparts;
    int dip_block;
    double *P;
    // the ions the atomic path holds this step (irr_count; null: the
    // finisher deposits them): each tile deposits their moves on the links
    // it owns, from r, the record's displacement and q; tile 0 clears the
    // count of the step after next
    const int *irr_cnt;
    int *irr_zero;
    const double *irr_r, *irr_du, *irr_q;
    const int *irr_order;
    // non-null: every ion whose start cell the tile owns gets its force here
    // (the atomic-path ones too, from the list above); the owned ions beyond
    // the LDS list are marked (ovf_mark[slot] = tag) and gathered from D^n
    // after the march, with the permittivity of the launch, V and eps_h
    unsigned int *ovf_mark;
    double V, eta_uni;
    const double *epsh;
    // the ions' own dynamics (the capturing kernel): E = eta D^{n+1} on the
    // 12 links of the cell each move ends in (endc[slot], packed) is written
    // to ecap[12 slot + 4 d + 2 o2 + o1] (field type) by the tile owning the
    // link's site; an ion a tile had no room to list gets ecap_bad[slot] = tag
    const int *endc;
    void *ecap;
    unsigned int *ecap_bad;
};

// Planes per z-chunk when the deposit is fused: up to 4, or up to 8 for the
// tile of 64 x 4 sites (the accumulator is 3 x TZ x TY x 64 values).
constexpr int kDepTZ = 4;
constexpr int kDepTZWide = 8;

// A regular ion moves less than a along every axis, so each axis of its
// dimension-split move spans at most two cells (checked on the cell indices
// too, so that rounding cannot make it three).
__device__ __forceinline__ bool ion_regular(double a, const double (&u)[3], const double (&du)[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (!(fabs(du[d]) < a)) return false;
        const double u1 = u[d] + du[d];
        const double lo = u[d] < u1 ? u[d] : u1, hi = u[d] < u1 ? u1 : u[d];
        if (floor(div_a(hi, a)) - floor(div_a(lo, a)) > 1.0) return false;
    }
    return true;
}

// Tile LDS of the fused deposit: the accumulator, and the ions whose start
// cell the tile owns (slot, and the cell packed as lx | ly << 8 | lz << 16),
// one per thread at most (ions past 256 are gathered after the march, or get
// their forces in the ion finisher).
constexpr int kOwnCap = 256;

template <typename T, int R, int TZ = kDepTZ>
struct DepSmem {
    alignas(16) T acc[3][TZ][4 * R][64];
    double psum[3][4];  // block 0: wavefront sums of the dipole partials
    int own_n;
    int2 own[kOwnCap];
};

// LDS of one tile: eta*D of two planes with a one-site halo, new B of one
// plane with a -1 halo.
template <typename T, int R>
struct LfSmem {
    T sX[2][3][4 * R + 2][66];
    T sB[3][4 * R + 1][65];
};


// One workgroup (256 threads) advances the tile (tile_x, tile_y) over the z
// planes of `chunk`.  Every load wraps periodically; stores are masked to the
// lattice, so any L >= 2 works with any tile shape.  With CAP (the ions' own
// dynamics: the tiles compute no forces) the tile instead captures the new
// field on the links of the cells the moves end in.
template <typename T, int EM, int R, bool DEP = false, int DTZ = kDepTZ, bool CAP = false>
__device__ __forceinline__ void leapfrog_tile(const LfArgs<T> &A, int tile_x, int tile_y, int chunk,
                                              LfSmem<T, R> &S, const DepArgs *dep = nullptr,
                                              DepSmem<T, R, DTZ> *DS = nullptr) {
    static_assert(!CAP || DEP, "the capture rides on the fused deposit");
    constexpr int TX = 64, TY = 4 * R;
    auto &sX = S.sX;
    auto &sB = S.sB;

    const int L = A.L;
    const size_t Ns = A.Ns, LL = (size_t)L * L;
    const int x0 = tile_x * TX, y0 = tile_y * TY, z0 = chunk * A.tz;
    const int z1 = min(z0 + A.tz, L);
    const int lx = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int xx = lx + 1;
    const int gx = wrapc(x0 + lx, L);
    const bool xact = (x0 + lx) < L;
    const T kB = A.kB, kD = A.kD;

    int gyo[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        gyo[r] = wrapc(y0 + wy + 4 * r, L);
        act[r] = xact && (y0 + wy + 4 * r) < L;
    }

    // A plane of eta*D in flight: the own sites' D and eta, and the one halo
    // site this thread stages (rows y0-1 and y0+TY on waves 0-1, columns
    // x0-1 and x0+64 on waves 2-3).  Fetching only issues the loads;
    // storing waits for them and writes eta*D into sX[buf].
    struct PlaneRegs {
        T d[R][3], e[R][3], hd[3], he[3];
    };
    auto fetch_plane = [&](int gz, PlaneRegs &p) {
        const size_t zoff = (size_t)gz * LL;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t off = zoff + (size_t)gyo[r] * L + gx;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                p.d[r][d] = A.Din[(size_t)d * Ns + off];
                p.e[r][d] = eta_at<T, EM>(A, d, gz, off);
            }
        }
        size_t off = 0;
        bool halo = true;
        if (wy < 2) {
            off = zoff + (size_t)wrapc(y0 - 1 + (wy ? TY + 1 : 0), L) * L + gx;
        } else if (lx < TY + 2) {
            off = zoff + (size_t)wrapc(y0 - 1 + lx, L) * L + wrapc(x0 - 1 + ((wy == 2) ? 0 : TX + 1), L);
        } else {
            halo = false;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            p.hd[d] = halo ? A.Din[(size_t)d * Ns + off] : (T)0;
            p.he[d] = halo ? eta_at<T, EM>(A, d, gz, off) : (T)0;
        }
    };
    auto store_plane = [&](int buf, const PlaneRegs &p) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = wy + 4 * r + 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) sX[buf][d][yy][xx] = p.e[r][d] * p.d[r][d];
        }
        if (wy < 2) {
            const int yy = wy ? TY + 1 : 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) sX[buf][d][yy][xx] = p.he[d] * p.hd[d];
        } else if (lx < TY + 2) {
            const int xc = (wy == 2) ? 0 : TX + 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) sX[buf][d][lx][xc] = p.he[d] * p.hd[d];
        }
    };

    // Deposit of the regular ions on the links this tile owns (x in
    // [x0, x0+64), y in [y0, y0+TY), z in [z0, z1)), accumulated in LDS from
    // the records of the ions on the tile's list.  The list entries are read
    // first, then the records' heads, both under the prologue's plane loads.
    // The heads decide which ions the tile owns (their forces) and which
    // records have a link on the tile; only those records' values are read,
    // and they are decoded in the first plane's step, while the next plane is
    // in flight, before its Ampere update reads the accumulator.
    constexpr int kWords = kCellWords<T>;
    static_assert(12 * sizeof(T) % 16 == 0, "values of a cell in whole 16-byte words");
    constexpr int kPF = sizeof(T) == 4 ? 2 : 1;  // entries per thread prefetched
    union RecRegs {
        uint4 raw[kWords];
        T v[12];
    };
    int pf_slot[kPF];
    bool pf_dec[kPF];
    int4 pf_head[kPF];
    int pf_endc[kPF];
    RecRegs pf_con[kPF];
    int dep_cnt = 0;
    size_t dep_base = 0;
    const int org[3] = {x0, y0, z0};
    const int ext[3] = {TX, min(y0 + TY, L) - y0, z1 - z0};
    if constexpr (DEP) {
        const int tile = tile_x + A.ntx * (tile_y + A.nty * chunk);
        dep_base = (size_t)tile * dep->cap;
        dep_cnt = min(dep->count[(size_t)tile * kCountStride], dep->cap);
        // (the kernel runs 256 threads per tile)
        constexpr int kAccWords = 3 * DTZ * TY * 64 * (int)sizeof(T) / 16;
        static_assert(kAccWords % 256 == 0, "accumulator in whole 16-byte words per thread");
        uint4 *accw = reinterpret_cast<uint4 *>(&DS->acc[0][0][0][0]);
#pragma unroll
        for (int t = 0; t < kAccWords / 256; ++t) accw[threadIdx.x + 256 * t] = make_uint4(0u, 0u, 0u, 0u);
        if (threadIdx.x == 0) {
            DS->own_n = 0;
            if (dep->irr_zero && tile == 0) *dep->irr_zero = 0;
        }
        // list entries e < cap belong to this tile: read before the count is known
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            const int e = (int)threadIdx.x + j * (int)blockDim.x;
            pf_slot[j] = e < dep->cap ? dep->list[dep_base + e] : -1;
        }
        if (dep->dip_prev && (int)blockIdx.x == dep->dip_block) {
            // wavefront sums of the dipole partials now, their sum after the
            // prologue's first barrier (the order of the dipole finaliser)
            double ps[3];
            strided_sum<3>(dep->dip_prev, dep->dip_nparts, threadIdx.x, blockDim.x, ps);
#pragma unroll
            for (int d = 0; d < 3; ++d) ps[d] = wave_sum(ps[d]);
            if ((threadIdx.x & 63) == 0)
#pragma unroll
                for (int d = 0; d < 3; ++d) DS->psum[d][threadIdx.x >> 6] = ps[d];
        }
    }
    // An ion whose start cell lies in the tile gets its force here.
    auto own_rec = [&](const int4 &h, int slot) {
        if (!dep->own_forces) return;
        const int lxo = (h.x & 1023) - x0, lyo = ((h.x >> 10) & 1023) - y0, lzo = ((h.x >> 20) & 1023) - z0;
        if (lxo >= 0 && lxo < TX && lyo >= 0 && lyo < ext[1] && lzo >= 0 && lzo < ext[2]) {
            const int pos = atomicAdd(&DS->own_n, 1);
            if (pos < kOwnCap) DS->own[pos] = make_int2(slot, lxo | (lyo << 8) | (lzo << 16));
            else if (dep->ovf_mark) dep->ovf_mark[slot] = dep->tag;
        }
    };
    // With CAP: an ion whose end cell has a link with its site on the tile
    // (cell or cell + 1 along every axis within the tile's real sites) joins
    // the tile's capture list (the LDS list of owned ions, unused then).
    const int exc0 = min(TX, L - x0);
    auto cap_rec = [&](int ec, int slot) {
        const int exr[3] = {exc0, ext[1], ext[2]};
        bool in = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const int v0 = (ec >> (10 * ax)) & 1023;
            const int v1 = v0 + 1 == L ? 0 : v0 + 1;
            in = in && ((unsigned)(v0 - org[ax]) < (unsigned)exr[ax] || (unsigned)(v1 - org[ax]) < (unsigned)exr[ax]);
        }
        if (!in) return;
        const int pos = atomicAdd(&DS->own_n, 1);
        if (pos < kOwnCap) DS->own[pos] = make_int2(slot, ec);
        else dep->ecap_bad[slot] = dep->tag;
    };
    // Whether one of the record's links lies on the tile: per axis group,
    // the box of links is the group's corner and the next cell along each
    // perpendicular axis, and along d the next cell only when the move
    // crosses into it.
    auto meets_tile = [&](const int4 &h) -> bool {
        const unsigned gw[3] = {(unsigned)h.y, (unsigned)h.z, (unsigned)h.w};
        bool any = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const unsigned g = gw[d];
            bool all = (g & kGroupOn) != 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int v0 = (int)((g >> (10 * ax)) & 1023u);
                const int v1 = v0 + 1 == L ? 0 : v0 + 1;
                const bool span = ax != d || (g & kGroupTwo);
                all = all && ((unsigned)(v0 - org[ax]) < (unsigned)ext[ax] ||
                              (span && (unsigned)(v1 - org[ax]) < (unsigned)ext[ax]));
            }
            any = any || all;
        }
        return any;
    };
    // Adds a record's values that fall on this tile's links to the
    // accumulator.  Per axis group the two candidate coordinates along each
    // axis are tested once; each of the (up to) eight links then needs only
    // those flags.
    // The second cell's values are loaded here when a move crosses a face.
    auto deposit_rec = [&](const int4 &h, const RecRegs &c0v, int slot) {
        const bool two = ((unsigned)h.y | (unsigned)h.z | (unsigned)h.w) & kGroupTwo;
        RecRegs c1v;
        if (two) {
            const uint4 *src = reinterpret_cast<const uint4 *>(&((const DepCell<T> *)dep->con1)[slot].v[0]);
#pragma unroll
            for (int q = 0; q < kWords; ++q) c1v.raw[q] = src[q];
        }
        const unsigned gw[3] = {(unsigned)h.y, (unsigned)h.z, (unsigned)h.w};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const unsigned g = gw[d];
            if (!(g & kGroupOn)) continue;
            const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
            int l0[3], l1[3];
            bool i0[3], i1[3];
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int v0 = (int)((g >> (10 * ax)) & 1023u);
                const int v1 = v0 + 1 == L ? 0 : v0 + 1;
                l0[ax] = v0 - org[ax];
                l1[ax] = v1 - org[ax];
                i0[ax] = (unsigned)l0[ax] < (unsigned)ext[ax];
                i1[ax] = (unsigned)l1[ax] < (unsigned)ext[ax];
            }
            const int ncell = (g & kGroupTwo) ? 2 : 1;
#pragma unroll
            for (int cell = 0; cell < 2; ++cell) {
                if (cell >= ncell) break;
#pragma unroll
                for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 2; ++o1) {
                        int sel[3];
                        sel[d] = cell;
                        sel[d1] = o1;
                        sel[d2] = o2;
                        const bool in = (sel[0] ? i1[0] : i0[0]) && (sel[1] ? i1[1] : i0[1]) &&
                                        (sel[2] ? i1[2] : i0[2]);
                        if (!in) continue;
                        const int lxx = sel[0] ? l1[0] : l0[0], lyy = sel[1] ? l1[1] : l0[1],
                                  lzz = sel[2] ? l1[2] : l0[2];
                        atomicAdd(&DS->acc[d][lzz][lyy][lxx], (cell ? c1v.v : c0v.v)[4 * d + 2 * o2 + o1]);
                    }
            }
        }
    };

    T Dc[R][3], prevB[R][2];
    T Ec[CAP ? R : 1][3];  // with CAP: eta of the own sites of the plane being updated

    // Prologue: new B_x, B_y of the plane below the chunk, for the own sites.
    {
        const int gzp = wrapc(z0 - 1, L);
        {
            PlaneRegs p0;
            fetch_plane(gzp, p0);
            store_plane(0, p0);
        }
        if constexpr (DEP) {
            // the list entries have arrived with the plane: issue the heads
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                const int e = (int)threadIdx.x + j * (int)blockDim.x;
                if (e >= dep_cnt || pf_slot[j] < 0) {
                    pf_slot[j] = -1;
                    continue;
                }
                pf_head[j] = dep->head[pf_slot[j]];
                if constexpr (CAP) pf_endc[j] = dep->endc[pf_slot[j]];
            }
        }
        PlaneRegs p1;
        fetch_plane(z0, p1);
        T bo[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t off = (size_t)gzp * LL + (size_t)gyo[r] * L + gx;
            bo[r][0] = A.Bin[off];
            bo[r][1] = A.Bin[Ns + off];
        }
        if constexpr (DEP) {
            // the heads: read the values of the records with a link on the tile
            const DepCell<T> *con = (const DepCell<T> *)dep->con0;
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                if (pf_slot[j] >= 0 && pf_head[j].x < 0) pf_slot[j] = -1;
                pf_dec[j] = pf_slot[j] >= 0 && meets_tile(pf_head[j]);
                if (!pf_dec[j]) continue;
                const uint4 *src = reinterpret_cast<const uint4 *>(&con[pf_slot[j]].v[0]);
#pragma unroll
                for (int q = 0; q < kWords; ++q) pf_con[j].raw[q] = src[q];
            }
        }
        store_plane(1, p1);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int d = 0; d < 3; ++d) Dc[r][d] = p1.d[r][d];
        if constexpr (CAP)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int d = 0; d < 3; ++d) Ec[r][d] = p1.e[r][d];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = wy + 4 * r + 1;
            prevB[r][0] = bo[r][0] - kB * (sX[0][2][yy + 1][xx] - sX[0][2][yy][xx] -
                                           sX[1][1][yy][xx] + sX[0][1][yy][xx]);
            prevB[r][1] = bo[r][1] - kB * (sX[1][0][yy][xx] - sX[0][0][yy][xx] -
                                           sX[0][2][yy][xx + 1] + sX[0][2][yy][xx]);
        }
        if constexpr (DEP) {
            if (dep->dip_prev && (int)blockIdx.x == dep->dip_block && threadIdx.x < 3) {
                double p = 0.0;
#pragma unroll
                for (int w = 0; w < 4; ++w) p += DS->psum[threadIdx.x][w];
                dep->P[threadIdx.x] = p;
            }
            // (the accumulator and the owned count were cleared before the
            // barrier above)
#pragma unroll
            for (int j = 0; j < kPF; ++j) {
                if (pf_slot[j] < 0) continue;
                if constexpr (CAP) cap_rec(pf_endc[j], pf_slot[j]);
                else own_rec(pf_head[j], pf_slot[j]);
            }
            // entries beyond the prefetched ones, if any
            const DepCell<T> *con = (const DepCell<T> *)dep->con0;
            for (int e = (int)threadIdx.x + kPF * (int)blockDim.x; e < dep_cnt; e += blockDim.x) {
                const int slot = dep->list[dep_base + e];
                if (slot < 0) continue;
                const int4 h = dep->head[slot];
                if (h.x < 0) continue;
                if constexpr (CAP) cap_rec(dep->endc[slot], slot);
                else own_rec(h, slot);
                if (!meets_tile(h)) continue;
                RecRegs cn;
                const uint4 *src = reinterpret_cast<const uint4 *>(&con[slot].v[0]);
#pragma unroll
                for (int q = 0; q < kWords; ++q) cn.raw[q] = src[q];
                deposit_rec(h, cn, slot);
            }
            // the atomic-path ions' moves, on this tile's links
            if (dep->irr_cnt) {
                const int ni = *dep->irr_cnt;
                const int *il = dep->irr_cnt + kIrrHead;
                const int ex[3] = {min(TX, L - x0), ext[1], ext[2]};
                for (int e = (int)threadIdx.x; e < ni; e += blockDim.x) {
                    const int s = il[e];
                    const int i = dep->irr_order ? dep->irr_order[s] : s;
                    double u[3] = {dep->irr_r[3 * i], dep->irr_r[3 * i + 1], dep->irr_r[3 * i + 2]};
                    const double du[3] = {dep->irr_du[3 * s], dep->irr_du[3 * s + 1], dep->irr_du[3 * s + 2]};
                    if (dep->ovf_mark) {
                        int cc[3];
                        double ff;
#pragma unroll
                        for (int d = 0; d < 3; ++d) fold(u[d], dep->a, L, cc[d], ff);
                        own_rec(make_int4(pack_cell(cc[0], cc[1], cc[2]), 0, 0, 0), s);
                    }
                    deposit_ion_box<T, DTZ, TY>(L, dep->a, dep->irr_q[i], u, du, org, ex, DS->acc);
                    if constexpr (CAP) {
                        // u has moved to where the move ends
                        int ce[3];
                        double ff;
#pragma unroll
                        for (int d = 0; d < 3; ++d) fold(u[d], dep->a, L, ce[d], ff);
                        cap_rec(pack_cell(ce[0], ce[1], ce[2]), s);
                    }
                }
            }
        }
        __syncthreads();
    }

    // The force of the owned ion this thread takes (loaded now, computed when
    // the march has the planes of its cell in LDS).
    int own_slot = -1, own_cell = 0, own_lz = -1;
    IonFQ<T> own_fq{};
    T own_ec = (T)1;
    T own_X[12];
    if constexpr (DEP && !CAP) {
        if ((int)threadIdx.x < min(DS->own_n, kOwnCap)) {
            const int2 o = DS->own[threadIdx.x];
            own_slot = o.x;
            own_cell = o.y;
            own_lz = o.y >> 16;
            own_fq = ((const IonFQ<T> *)dep->fq)[own_slot];
            const size_t site = (size_t)(x0 + (o.y & 255)) +
                                (size_t)L * ((size_t)(y0 + ((o.y >> 8) & 255)) + (size_t)L * (z0 + own_lz));
            own_ec = ((const T *)dep->ecell)[site];
        }
    }

    // With CAP, after the march: the links of the listed end cells whose
    // site lies on the tile, from E of the tile's planes (the Ampere update
    // leaves E = eta D^{n+1} of each site in its accumulator entry, which is
    // not read again), to the capture array: all 12 LDS reads first, then the
    // values, with three 16-byte stores (FP32; six in FP64) when the tile
    // owns every link of the cell.
    auto cap_links = [&]() {
        if constexpr (CAP) {
            const int ncap = min(DS->own_n, kOwnCap);
            for (int e = (int)threadIdx.x; e < ncap; e += blockDim.x) {
                const int2 o = DS->own[e];
                int c0[3], c1[3];
#pragma unroll
                for (int ax = 0; ax < 3; ++ax) {
                    c0[ax] = (o.y >> (10 * ax)) & 1023;
                    c1[ax] = c0[ax] + 1 == L ? 0 : c0[ax] + 1;
                }
                union {
                    T v[12];
                    uint4 w[kCellWords<T>];
                } E;
                unsigned own = 0u;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
#pragma unroll
                    for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                        for (int o1 = 0; o1 < 2; ++o1) {
                            int x[3] = {c0[0], c0[1], c0[2]};
                            x[d1] = o1 ? c1[d1] : c0[d1];
                            x[d2] = o2 ? c1[d2] : c0[d2];
                            const int lxx = x[0] - x0, lyy = x[1] - y0, lzz = x[2] - z0;
                            const bool in = (unsigned)lxx < (unsigned)exc0 && (unsigned)lyy < (unsigned)ext[1] &&
                                            (unsigned)lzz < (unsigned)ext[2];
                            const int t = 4 * d + 2 * o2 + o1;
                            own |= in ? 1u << t : 0u;
                            E.v[t] = DS->acc[d][in ? lzz : 0][in ? lyy : 0][in ? lxx : 0];
                        }
                }
                T *dst = (T *)dep->ecap + 12 * (size_t)o.x;
                if (own == 0xFFFu) {
                    uint4 *dw = reinterpret_cast<uint4 *>(dst);
#pragma unroll
                    for (int q = 0; q < kCellWords<T>; ++q) dw[q] = E.w[q];
                } else {
#pragma unroll
                    for (int t = 0; t < 12; ++t)
                        if (own & (1u << t)) dst[t] = E.v[t];
                }
            }
        }
    };

    // One plane k of the march.  The first one also decodes the prefetched
    // records, between issuing the next plane's loads and storing it.
    int cur = 1;
    auto march = [&](int k, auto first) {
        const int nxt = cur ^ 1;
        const int gzn = wrapc(k + 1, L);
        const size_t zoff = (size_t)k * LL;
        PlaneRegs pn;
        fetch_plane(gzn, pn);

        T Bo[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t off = zoff + (size_t)gyo[r] * L + gx;
#pragma unroll
            for (int d = 0; d < 3; ++d) Bo[r][d] = A.Bin[(size_t)d * Ns + off];
        }
        // halo B^{n-1/2}: row y0-1 (B_x, B_z) on wave 0, column x0-1 (B_y, B_z) on wave 1
        T hb0 = 0, hb1 = 0;
        if (wy == 0) {
            const size_t off = zoff + (size_t)wrapc(y0 - 1, L) * L + gx;
            hb0 = A.Bin[off];
            hb1 = A.Bin[2 * Ns + off];
        } else if (wy == 1 && lx < TY) {
            const size_t off = zoff + (size_t)wrapc(y0 + lx, L) * L + wrapc(x0 - 1, L);
            hb0 = A.Bin[Ns + off];
            hb1 = A.Bin[2 * Ns + off];
        }
        if constexpr (DEP && decltype(first)::value) {
#pragma unroll
            for (int j = 0; j < kPF; ++j)
                if (pf_dec[j]) deposit_rec(pf_head[j], pf_con[j], pf_slot[j]);
        }
        store_plane(nxt, pn);
        __syncthreads();

        // Faraday: new B on the own sites
        T Bn[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = wy + 4 * r + 1;
            Bn[r][0] = Bo[r][0] - kB * (sX[cur][2][yy + 1][xx] - sX[cur][2][yy][xx] -
                                        sX[nxt][1][yy][xx] + sX[cur][1][yy][xx]);
            Bn[r][1] = Bo[r][1] - kB * (sX[nxt][0][yy][xx] - sX[cur][0][yy][xx] -
                                        sX[cur][2][yy][xx + 1] + sX[cur][2][yy][xx]);
            Bn[r][2] = Bo[r][2] - kB * (sX[cur][1][yy][xx + 1] - sX[cur][1][yy][xx] -
                                        sX[cur][0][yy + 1][xx] + sX[cur][0][yy][xx]);
#pragma unroll
            for (int d = 0; d < 3; ++d) sB[d][yy][xx] = Bn[r][d];
            if (act[r]) {
                const size_t off = zoff + (size_t)gyo[r] * L + gx;
#pragma unroll
                for (int d = 0; d < 3; ++d) A.Bout[(size_t)d * Ns + off] = Bn[r][d];
            }
        }
        // Faraday on the -1 halo
        if (wy == 0) {
            sB[0][0][xx] = hb0 - kB * (sX[cur][2][1][xx] - sX[cur][2][0][xx] -
                                       sX[nxt][1][0][xx] + sX[cur][1][0][xx]);
            sB[2][0][xx] = hb1 - kB * (sX[cur][1][0][xx + 1] - sX[cur][1][0][xx] -
                                       sX[cur][0][1][xx] + sX[cur][0][0][xx]);
        } else if (wy == 1 && lx < TY) {
            const int yy = lx + 1;
            sB[1][yy][0] = hb0 - kB * (sX[nxt][0][yy][0] - sX[cur][0][yy][0] -
                                       sX[cur][2][yy][1] + sX[cur][2][yy][0]);
            sB[2][yy][0] = hb1 - kB * (sX[cur][1][yy][1] - sX[cur][1][yy][0] -
                                       sX[cur][0][yy + 1][0] + sX[cur][0][yy][0]);
        }
        if constexpr (DEP && !CAP) {
            // The owned ion in plane k: capture E = eta D on its cell's 12
            // links (planes k and k+1, rows and columns with the +1 halo, in
            // force_ion's order); its force is computed after the march.
            if (own_lz == k - z0) {
                const int rr = ((own_cell >> 8) & 255) + 1, cc = (own_cell & 255) + 1;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
#pragma unroll
                    for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                        for (int o1 = 0; o1 < 2; ++o1) {
                            int ox[3] = {0, 0, 0};
                            ox[d1] = o1;
                            ox[d2] = o2;
                            own_X[4 * d + 2 * o2 + o1] = sX[ox[2] ? nxt : cur][d][rr + ox[1]][cc + ox[0]];
                        }
                }
            }
        }
        __syncthreads();

        // Ampere: new D on the own sites
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int yy = wy + 4 * r + 1;
            const T dx = Dc[r][0] + kD * (Bn[r][2] - sB[2][yy - 1][xx] - Bn[r][1] + prevB[r][1]);
            const T dy = Dc[r][1] + kD * (Bn[r][0] - prevB[r][0] - Bn[r][2] + sB[2][yy][xx - 1]);
            const T dz = Dc[r][2] + kD * (Bn[r][1] - sB[1][yy][xx - 1] - Bn[r][0] + sB[0][yy - 1][xx]);
            if constexpr (CAP) {
                const int kz = k - z0, ky = wy + 4 * r;
                const T n3[3] = {dx + DS->acc[0][kz][ky][lx], dy + DS->acc[1][kz][ky][lx],
                                 dz + DS->acc[2][kz][ky][lx]};
                // (this thread's own entry: nothing reads it again in the march)
#pragma unroll
                for (int d = 0; d < 3; ++d) DS->acc[d][kz][ky][lx] = Ec[r][d] * n3[d];
                if (act[r]) {
                    const size_t off = zoff + (size_t)gyo[r] * L + gx;
                    A.Dout[off] = n3[0];
                    A.Dout[Ns + off] = n3[1];
                    A.Dout[2 * Ns + off] = n3[2];
                }
            } else if (act[r]) {
                const size_t off = zoff + (size_t)gyo[r] * L + gx;
                if constexpr (DEP) {
                    const int kz = k - z0, ky = wy + 4 * r;
                    A.Dout[off] = dx + DS->acc[0][kz][ky][lx];
                    A.Dout[Ns + off] = dy + DS->acc[1][kz][ky][lx];
                    A.Dout[2 * Ns + off] = dz + DS->acc[2][kz][ky][lx];
                } else {
                    A.Dout[off] = dx;
                    A.Dout[Ns + off] = dy;
                    A.Dout[2 * Ns + off] = dz;
                }
            }
            prevB[r][0] = Bn[r][0];
            prevB[r][1] = Bn[r][1];
#pragma unroll
            for (int d = 0; d < 3; ++d) Dc[r][d] = pn.d[r][d];
            if constexpr (CAP)
#pragma unroll
                for (int d = 0; d < 3; ++d) Ec[r][d] = pn.e[r][d];
        }
        cur = nxt;
    };
    march(z0, std::true_type{});
    for (int k = z0 + 1; k < z1; ++k) march(k, std::false_type{});

    if constexpr (CAP) {
        __syncthreads();
        cap_links();
    }
    if constexpr (DEP && !CAP) {
        // Force of the owned ion: lattice part from the captured E, as
        // force_ion sums it, then the self force (the dipole term is added by
        // the ion finisher, or by the movers of the next launch).
        if (own_slot >= 0) {
            const double f[3] = {(double)own_fq.f[0], (double)own_fq.f[1], (double)own_fq.f[2]};
            const double q = (double)own_fq.q;
            double Fl[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
                double sum = 0.0;
#pragma unroll
                for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 2; ++o1)
                        sum += lin_w(o1, f[d1]) * lin_w(o2, f[d2]) * (double)own_X[4 * d + 2 * o2 + o1];
                Fl[d] = q * sum;
            }
            double S, dS[3];
            self_sum(dep->G, f, S, dS);
            const double pref = q * q / (2.0 * (double)own_ec * dep->a);
#pragma unroll
            for (int d = 0; d < 3; ++d) dep->Ft[3 * (size_t)own_slot + d] = Fl[d] - div_a(-pref * dS[d], dep->a);
            dep->fdone[own_slot] = dep->tag;
        }
        // owned ions beyond the LDS list (marked by own_rec): gathered from
        // D^n, which this launch only reads, as the finisher would
        if (dep->ovf_mark && dep->own_forces && DS->own_n > kOwnCap) {
            const int ni = dep->irr_cnt ? *dep->irr_cnt : 0;
            const EtaView<T> ev{EM, dep->eta_uni, A.eta_prof, A.eta_link};
            const double zero[3] = {0.0, 0.0, 0.0};
            for (int e = (int)threadIdx.x; e < dep_cnt + ni; e += blockDim.x) {
                const int slot = e < dep_cnt ? dep->list[dep_base + e] : dep->irr_cnt[kIrrHead + e - dep_cnt];
                if (slot < 0 || dep->ovf_mark[slot] != dep->tag) continue;
                const int i = dep->irr_order ? dep->irr_order[slot] : slot;
                const double u[3] = {dep->irr_r[3 * i], dep->irr_r[3 * i + 1], dep->irr_r[3 * i + 2]};
                int cc[3];
                double ff;
#pragma unroll
                for (int d = 0; d < 3; ++d) fold(u[d], dep->a, L, cc[d], ff);
                if ((unsigned)(cc[0] - x0) >= (unsigned)TX || (unsigned)(cc[1] - y0) >= (unsigned)ext[1] ||
                    (unsigned)(cc[2] - z0) >= (unsigned)ext[2])
                    continue;  // another tile's
                double F[3];
                force_ion<T>(L, Ns, dep->a, dep->V, dep->irr_q[i], u, A.Din, ev, dep->G, zero, dep->epsh, F);
#pragma unroll
                for (int d = 0; d < 3; ++d) dep->Ft[3 * (size_t)slot + d] = F[d];
                dep->fdone[slot] = dep->tag;
            }
        }
    }
}


// Lattices narrower than a wavefront (L < 64), where a 64-site row tile
// would leave 64 - L lanes of every wavefront idle: a workgroup holds whole
// rows of L sites, thread t on site x = t mod L of row t / L, xrows = 256 / L
// rows (threads past xrows L idle), and marches through a z-chunk as
// leapfrog_tile does, with the same arithmetic.  Along x the tile is the
// whole lattice, so the stencil's x neighbours wrap inside it: no x halo.
// (kRowSites: memd_internal.hpp)

template <typename T>
struct RowSmem {
    T sX[2][3][kRowSites + 128];  // eta*D of two planes, rows y0 - 1 .. y0 + xrows: (xrows + 2) L values
    T sB[3][kRowSites + 64];      // new B of the plane, rows y0 - 1 .. y0 + xrows - 1
};

template <typename T, int EM>
__device__ __forceinline__ void leapfrog_rows(const LfArgs<T> &A, int xrows, int tile_y, int chunk,
                                              RowSmem<T> &S) {
    auto &sX = S.sX;
    auto &sB = S.sB;
    const int L = A.L;
    const size_t Ns = A.Ns, LL = (size_t)L * L;
    const int y0 = tile_y * xrows, z0 = chunk * A.tz;
    const int z1 = min(z0 + A.tz, L);
    const int t = (int)threadIdx.x;
    const int r = t / L, x = t - r * L;
    const bool live = r < xrows;           // the thread holds a site of the tile
    const bool act = live && y0 + r < L;   // and stores it (rows past L wrap, as in leapfrog_tile)
    const int gy = wrapc(y0 + r, L);
    const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
    const int yy = r + 1;
    const T kB = A.kB, kD = A.kD;
    // the halo row this thread stages: y0 - 1 (row 0) for r == 0, y0 + xrows
    // (row xrows + 1) for r == 1
    const bool halo = live && r < 2;
    const int hrow = r == 0 ? 0 : xrows + 1;
    const int hy = wrapc(r == 0 ? y0 - 1 : y0 + xrows, L);

    struct PlaneRegs {
        T d[3], e[3], hd[3], he[3];
    };
    auto fetch_plane = [&](int gz, PlaneRegs &p) {
        if (!live) return;
        const size_t off = (size_t)gz * LL + (size_t)gy * L + x;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            p.d[d] = A.Din[(size_t)d * Ns + off];
            p.e[d] = eta_at<T, EM>(A, d, gz, off);
        }
        const size_t ho = (size_t)gz * LL + (size_t)hy * L + x;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            p.hd[d] = halo ? A.Din[(size_t)d * Ns + ho] : (T)0;
            p.he[d] = halo ? eta_at<T, EM>(A, d, gz, ho) : (T)0;
        }
    };
    auto store_plane = [&](int buf, const PlaneRegs &p) {
        if (!live) return;
#pragma unroll
        for (int d = 0; d < 3; ++d) sX[buf][d][yy * L + x] = p.e[d] * p.d[d];
        if (halo)
#pragma unroll
            for (int d = 0; d < 3; ++d) sX[buf][d][hrow * L + x] = p.he[d] * p.hd[d];
    };

    T Dc[3] = {(T)0, (T)0, (T)0}, prevB[2] = {(T)0, (T)0};
    const int c0 = yy * L + x;  // the thread's own site in the LDS rows
    // Prologue: new B_x, B_y of the plane below the chunk, for the own sites.
    {
        const int gzp = wrapc(z0 - 1, L);
        {
            PlaneRegs p0;
            fetch_plane(gzp, p0);
            store_plane(0, p0);
        }
        PlaneRegs p1;
        fetch_plane(z0, p1);
        T bo[2] = {(T)0, (T)0};
        if (live) {
            const size_t off = (size_t)gzp * LL + (size_t)gy * L + x;
            bo[0] = A.Bin[off];
            bo[1] = A.Bin[Ns + off];
        }
        store_plane(1, p1);
        if (live)
#pragma unroll
            for (int d = 0; d < 3; ++d) Dc[d] = p1.d[d];
        __syncthreads();
        if (live) {
            prevB[0] = bo[0] - kB * (sX[0][2][c0 + L] - sX[0][2][c0] - sX[1][1][c0] + sX[0][1][c0]);
            prevB[1] = bo[1] - kB * (sX[1][0][c0] - sX[0][0][c0] - sX[0][2][yy * L + xp] + sX[0][2][c0]);
        }
        __syncthreads();
    }

    int cur = 1;
    for (int k = z0; k < z1; ++k) {
        const int nxt = cur ^ 1;
        const size_t zoff = (size_t)k * LL;
        PlaneRegs pn;
        fetch_plane(wrapc(k + 1, L), pn);
        T Bo[3] = {(T)0, (T)0, (T)0};
        T hb0 = 0, hb1 = 0;
        if (live) {
            const size_t off = zoff + (size_t)gy * L + x;
#pragma unroll
            for (int d = 0; d < 3; ++d) Bo[d] = A.Bin[(size_t)d * Ns + off];
            if (r == 0) {
                // halo B^{n-1/2} of row y0 - 1: B_x, B_z
                const size_t ho = zoff + (size_t)hy * L + x;
                hb0 = A.Bin[ho];
                hb1 = A.Bin[2 * Ns + ho];
            }
        }
        store_plane(nxt, pn);
        __syncthreads();

        // Faraday: new B on the own sites, and B_x, B_z on the row y0 - 1
        T Bn[3] = {(T)0, (T)0, (T)0};
        if (live) {
            Bn[0] = Bo[0] - kB * (sX[cur][2][c0 + L] - sX[cur][2][c0] - sX[nxt][1][c0] + sX[cur][1][c0]);
            Bn[1] = Bo[1] - kB * (sX[nxt][0][c0] - sX[cur][0][c0] - sX[cur][2][yy * L + xp] + sX[cur][2][c0]);
            Bn[2] = Bo[2] - kB * (sX[cur][1][yy * L + xp] - sX[cur][1][c0] - sX[cur][0][c0 + L] + sX[cur][0][c0]);
#pragma unroll
            for (int d = 0; d < 3; ++d) sB[d][c0] = Bn[d];
            if (act) {
                const size_t off = zoff + (size_t)gy * L + x;
#pragma unroll
                for (int d = 0; d < 3; ++d) A.Bout[(size_t)d * Ns + off] = Bn[d];
            }
            if (r == 0) {
                sB[0][x] = hb0 - kB * (sX[cur][2][L + x] - sX[cur][2][x] - sX[nxt][1][x] + sX[cur][1][x]);
                sB[2][x] = hb1 - kB * (sX[cur][1][xp] - sX[cur][1][x] - sX[cur][0][L + x] + sX[cur][0][x]);
            }
        }
        __syncthreads();

        // Ampere: new D on the own sites
        if (live) {
            const T dx = Dc[0] + kD * (Bn[2] - sB[2][c0 - L] - Bn[1] + prevB[1]);
            const T dy = Dc[1] + kD * (Bn[0] - prevB[0] - Bn[2] + sB[2][yy * L + xm]);
            const T dz = Dc[2] + kD * (Bn[1] - sB[1][yy * L + xm] - Bn[0] + sB[0][c0 - L]);
            if (act) {
                const size_t off = zoff + (size_t)gy * L + x;
                A.Dout[off] = dx;
                A.Dout[Ns + off] = dy;
                A.Dout[2 * Ns + off] = dz;
            }
            prevB[0] = Bn[0];
            prevB[1] = Bn[1];
#pragma unroll
            for (int d = 0; d < 3; ++d) Dc[d] = pn.d[d];
        }
        cur = nxt;
    }
}

}  // namespace memd
