// ion_records.hpp -- the per-slot records of the fused deposit and the ion
// movers that write them (gfx950).
//
// A record holds what the leapfrog tiles need of one ion's move for the
// step: its start cell, per axis the link box the dimension-split move
// touches, and the values it adds to those links (the current of the move,
// assigned so that Gauss's law holds after the move, eq. constraint, with
// the transverse linear weights).
#pragma once

#include "device_util.hpp"
#include "ion_ops.hpp"
#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"
#include "philox.hpp"

namespace memd {

// The records of the fused deposit (leapfrog_tile.hpp), one per slot, and
// what decides whether an ion stays with the tiles: its cell at the last
// list build (cbin, packed) and whether it fitted the lists (list_fail).
template <typename T>
struct DepOut {
    int4 *head;
    DepCell<T> *con0, *con1;
    const int *cbin;
    const int *list_fail;
    double *du;  // [3n] by slot: the (sanitised) displacement the record was made for
    IonFQ<T> *fq;  // [n] by slot: fractional position in the start cell and charge
    int *icnt;     // non-null: the atomic-path ions of the records' step are appended here
    int *ilist;    // (their slots; irr_count)
    int *endc;     // non-null: [n] by slot, the cell the move ends in (packed)
};

// The record of one ion in slot s for the fused deposit (du already
// sanitised): the axes of the dimension-split move are taken in turn with
// the arithmetic of deposit_ion (bit for bit), giving per axis the link-box
// corner and the values -q (ub - ua)/a w w / a^2 (in the field type).
// Returns true, and writes a head of -1, when the ion is left to the atomic
// path: irregular, drifted more than one cell from its list cell along an
// axis, or missing from a list.
// (list_fail and cb: the slot's entries of O.list_fail and O.cbin.)
// WHOLE: the two cells' values are built in registers and stored whole with
// 16-byte stores (entries of an axis the move does not use are zero; the
// readers skip them by the axis flags; the second cell only when a move
// crosses a face), else each value is stored where it is formed.  A kernel
// that writes records on the path between two leapfrog launches (the ions'
// own dynamics) takes the first, whose stores leave the wavefront sooner;
// the movers beside the tiles the second, which writes fewer bytes.
template <typename T, bool WHOLE = false>
__device__ __forceinline__ bool write_record_at(int L, double a, double qi, const double (&u_in)[3],
                                                const double (&du)[3], int s, const DepOut<T> &O, int list_fail,
                                                int cb) {
#pragma unroll
    for (int d = 0; d < 3; ++d) O.du[3 * s + d] = du[d];
    double u[3] = {u_in[0], u_in[1], u_in[2]};
    int c0[3];
    double f0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) fold(u[d], a, L, c0[d], f0[d]);
    if (O.endc) {
        int ce[3];
        double fe;
#pragma unroll
        for (int d = 0; d < 3; ++d) fold(u_in[d] + du[d], a, L, ce[d], fe);
        O.endc[s] = pack_cell(ce[0], ce[1], ce[2]);
    }
    bool atomic_path = list_fail != 0 || !ion_regular(a, u_in, du);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        int off = c0[e] - ((cb >> (10 * e)) & 1023) + 1;
        off += off < 0 ? L : (off >= L ? -L : 0);
        atomic_path = atomic_path || off > 2;  // start cell within one cell of the list cell
    }
    if (atomic_path) {
        O.head[s] = make_int4(-1, 0, 0, 0);
        if (O.icnt) {
            // the tiles take these ions' moves and forces from the atomic-path list
            O.ilist[atomicAdd(O.icnt, 1)] = s;
            IonFQ<T> fq;
            fq.f[0] = (T)f0[0];
            fq.f[1] = (T)f0[1];
            fq.f[2] = (T)f0[2];
            fq.q = (T)qi;
            O.fq[s] = fq;
        }
        return true;
    }
    const double a2 = a * a;
    unsigned int g[3] = {0u, 0u, 0u};
    union {
        T v[12];
        uint4 w[kCellWords<T>];
    } cv[2];
    if constexpr (WHOLE) {
#pragma unroll
        for (int j = 0; j < 12; ++j) cv[0].v[j] = cv[1].v[j] = (T)0;
    }
    bool any_two = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
        const double u0 = u[d], u1 = u0 + du[d];
        if (u1 != u0) {
            int c1, c2;
            double f1, f2;
            fold(u[d1], a, L, c1, f1);
            fold(u[d2], a, L, c2, f2);
            const double lo_u = u0 < u1 ? u0 : u1, hi_u = u0 < u1 ? u1 : u0;
            const double sgn = u1 > u0 ? 1.0 : -1.0;
            const double klo = floor(div_a(lo_u, a)), khi = floor(div_a(hi_u, a));
            int corner[3];
            corner[d] = mod_cell(klo, L);
            corner[d1] = c1;
            corner[d2] = c2;
            const bool two = khi > klo;
            any_two = any_two || two;
            g[d] = (unsigned)pack_cell(corner[0], corner[1], corner[2]) | kGroupOn | (two ? kGroupTwo : 0u);
            // a regular move spans at most two cells along the axis
#pragma unroll
            for (int cell = 0; cell < 2; ++cell) {
                if (cell == 1 && !two) break;  // the second cell's values are only read when it is used
                const double kc = cell ? khi : klo;
                const double s0 = kc * a, s1 = (kc + 1.0) * a;
                const double sa = lo_u > s0 ? lo_u : s0;
                const double sb = hi_u < s1 ? hi_u : s1;
                const double len = sb - sa;
                const double amount = len > 0.0 ? div_a(qi * sgn * div_a(len, a), a2) : 0.0;
#pragma unroll
                for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                    for (int o1 = 0; o1 < 2; ++o1) {
                        const T val = (T)(-(amount * lin_w(o1, f1) * lin_w(o2, f2)));
                        if constexpr (WHOLE) cv[cell].v[4 * d + 2 * o2 + o1] = val;
                        else (cell ? O.con1 : O.con0)[s].v[4 * d + 2 * o2 + o1] = val;
                    }
            }
        }
        u[d] = u1;
    }
    if constexpr (WHOLE) {
        uint4 *d0 = reinterpret_cast<uint4 *>(&O.con0[s].v[0]);
#pragma unroll
        for (int q = 0; q < kCellWords<T>; ++q) d0[q] = cv[0].w[q];
        if (any_two) {
            uint4 *d1 = reinterpret_cast<uint4 *>(&O.con1[s].v[0]);
#pragma unroll
            for (int q = 0; q < kCellWords<T>; ++q) d1[q] = cv[1].w[q];
        }
    }
    O.head[s] = make_int4(pack_cell(c0[0], c0[1], c0[2]), (int)g[0], (int)g[1], (int)g[2]);
    IonFQ<T> fq;
    fq.f[0] = (T)f0[0];
    fq.f[1] = (T)f0[1];
    fq.f[2] = (T)f0[2];
    fq.q = (T)qi;
    O.fq[s] = fq;
    return false;
}

template <typename T>
__device__ __forceinline__ bool write_record(int L, double a, double qi, const double (&u_in)[3],
                                             const double (&du)[3], int s, const DepOut<T> &O) {
    return write_record_at<T>(L, a, qi, u_in, du, s, O, O.list_fail[s], O.cbin[s]);
}

// The displacement of storage index i for the step (the caller's index
// perm[i]), sanitised and counted.
__device__ __forceinline__ void step_displacement(int i, int L, double a, const double *__restrict__ disp,
                                                  const int *__restrict__ perm, unsigned int *bad, uint64_t seed,
                                                  uint32_t t, double sigma, double (&du)[3]) {
    const int ci = perm ? perm[i] : i;
    if (disp) {
        du[0] = disp[3 * ci];
        du[1] = disp[3 * ci + 1];
        du[2] = disp[3 * ci + 2];
    } else {
        philox_displacement(seed, t, (uint32_t)ci, sigma, du);
    }
    sanitize_move(du, a, L, bad);
}

// The ion movers of the fused leapfrog launch.  Nothing they read or write
// is touched by the tiles of the same launch: they move every ion to
// r^{n+1} = r^n + du (into r_out; r^n stays for the forces and the irregular
// ions' deposit that follow the launch), write one partial of q r^{n+1} per
// wavefront, and, with pack set, the next step's records into the second
// record set (the tiles read the first).  They run as workgroups of their
// own beside the tiles (nblocks of them, kMoverIons ions each; ahead: the
// first workgroups of the launch, else the last).
constexpr int kMoverPerThread = 1;  // ions per mover thread
constexpr int kMoverIons = 256 * kMoverPerThread;  // ions per mover workgroup

template <typename T>
struct MoverArgs {
    int nblocks;  // mover workgroups (0: none)
    int ahead;    // the movers are the launch's first workgroups (else its last)
    int n, L;
    double a;
    const double *q, *r;
    double *r_out;
    const int *order;  // null: ions stored in bin order
    const int *perm;   // storage index -> caller index (displacements), null: identity
    const double *du;  // [3n] by slot: this step's displacements (the current records')
    double *dip_out;   // one partial of q r^{n+1} per mover workgroup
    int pack;          // write the next step's records
    const double *disp_next;  // null: the Philox displacements of step t_next
    uint64_t seed;
    uint32_t t_next;
    double sigma;
    unsigned int *bad;
    int *atomic_next;  // [n] by slot: the next step's ion left to the atomic path
    DepOut<T> out;     // the next step's records (cbin, list_fail: the lists' state)
    // The forces of the state the previous launch started from, completed
    // here (Ft_prev null: not): lattice part and self force from that
    // launch's tiles (stamped fdone_prev == tag_prev), plus the dipole term
    // with P_prev, into F by storage index (the finisher's arithmetic).
    const double *Ft_prev;
    const unsigned int *fdone_prev;
    unsigned int tag_prev;
    const double *P_prev;
    const double *scal;
    double V;
    double *F;
};

// Slots [s0, s0 + count) by the workgroup's 256 threads, kMoverPerThread
// per thread (all of a thread's loads issued before any of its arithmetic);
// the workgroup's dipole partial to dip_out[part] (its four wavefront sums
// added in order through psum; zero for a workgroup without ions).
template <typename T>
__device__ __forceinline__ void move_ions(const MoverArgs<T> &M, int s0, int count, int part, double (*psum)[4]) {
    constexpr int K = kMoverPerThread;
    double P[3] = {0.0, 0.0, 0.0};
    const int s1 = min(s0 + count, M.n);
    int sk[K], ik[K], ck[K], lfail[K], lcell[K];
    bool live[K];
    double u[K][3], du[K][3], dn[K][3], qk[K];
    unsigned int fdp[K];  // the previous state's force stamp and result (Ft_prev)
    double ftp[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sk[k] = s0 + (int)threadIdx.x + 256 * k;
        live[k] = sk[k] < s1;
        const int s = live[k] ? sk[k] : s0;
        ik[k] = M.order ? M.order[s] : s;
        ck[k] = M.perm ? M.perm[ik[k]] : ik[k];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[k][d] = M.r[3 * ik[k] + d];
            du[k][d] = M.du[3 * s + d];
            dn[k][d] = 0.0;
        }
        qk[k] = M.q[ik[k]];
        lfail[k] = M.pack ? M.out.list_fail[s] : 0;
        lcell[k] = M.pack ? M.out.cbin[s] : 0;
        fdp[k] = M.Ft_prev ? M.fdone_prev[s] : 0u;
#pragma unroll
        for (int d = 0; d < 3; ++d) ftp[k][d] = M.Ft_prev ? M.Ft_prev[3 * s + d] : 0.0;
    }
    if (M.pack) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (M.disp_next) {
#pragma unroll
                for (int d = 0; d < 3; ++d) dn[k][d] = M.disp_next[3 * ck[k] + d];
            } else {
                philox_displacement(M.seed, M.t_next, (uint32_t)ck[k], M.sigma, dn[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!live[k]) continue;
        const int s = sk[k], i = ik[k];
        // the position deposit_ion leaves, bit for bit
#pragma unroll
        for (int d = 0; d < 3; ++d) u[k][d] = u[k][d] + du[k][d];
        M.r_out[3 * i] = u[k][0];
        M.r_out[3 * i + 1] = u[k][1];
        M.r_out[3 * i + 2] = u[k][2];
#pragma unroll
        for (int d = 0; d < 3; ++d) P[d] += qk[k] * u[k][d];
        if (M.pack) {
            sanitize_move(dn[k], M.a, M.L, M.bad);
            M.atomic_next[s] = write_record_at<T>(M.L, M.a, qk[k], u[k], dn[k], s, M.out, lfail[k], lcell[k]) ? 1 : 0;
        }
    }
    if (M.Ft_prev) {
        const double w = M.scal[S_DIPW];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!live[k] || fdp[k] != M.tag_prev) continue;
            double *F = M.F + 3 * (size_t)ik[k];
#pragma unroll
            for (int d = 0; d < 3; ++d) F[d] = ftp[k][d] + qk[k] * (w * M.P_prev[d]) / (M.V * M.scal[S_EPSH + d]);
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) P[d] = wave_sum(P[d]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int d = 0; d < 3; ++d) psum[d][threadIdx.x >> 6] = P[d];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = (int)threadIdx.x;
        M.dip_out[3 * part + d] = ((psum[d][0] + psum[d][1]) + psum[d][2]) + psum[d][3];
    }
}

// The records of the step about to run (next: the second set, which the
// movers fill for the step after it).
template <typename T>
inline DepOut<T> dep_out(const memd_ctx *c, bool next = false) {
    DepOut<T> O;
    O.head = next ? c->rec_head_nx : c->rec_head;
    O.con0 = (DepCell<T> *)(next ? c->rec_con_nx : c->rec_con);
    O.con1 = (DepCell<T> *)(next ? c->rec_con1_nx : c->rec_con1);
    O.cbin = c->cbin;
    O.list_fail = c->list_fail;
    O.du = next ? c->du_slot_nx : c->du_slot;
    O.fq = (IonFQ<T> *)(next ? c->fq_nx : c->fq);
    O.icnt = c->tile_irregular ? irr_count(c, c->step_index + (next ? 1 : 0)) : nullptr;
    O.ilist = O.icnt ? O.icnt + kIrrHead : nullptr;
    O.endc = c->endc;
    return O;
}

inline int mover_blocks(int n) { return n > 0 ? (n + kMoverIons - 1) / kMoverIons : 0; }


template <typename T>
inline MoverArgs<T> mover_args(const memd_ctx *c, const IonMoves &mv) {
    MoverArgs<T> M;
    M.nblocks = mover_blocks(c->n);
    M.ahead = 0;  // chosen at the launch
    M.n = c->n;
    M.L = c->L;
    M.a = c->a;
    M.q = c->q;
    M.r = c->r;
    M.r_out = c->r_alt;
    M.order = c->sorted ? nullptr : c->order;
    M.perm = c->perm;
    M.du = c->du_slot;
    M.dip_out = mv.dip_out;
    M.pack = mv.pack_next ? 1 : 0;
    M.disp_next = mv.disp_next;
    M.seed = mv.seed;
    M.t_next = mv.t_next;
    M.sigma = mv.sigma;
    M.bad = c->bad_moves;
    M.atomic_next = c->dep_atomic_nx;
    M.out = dep_out<T>(c, true);
    M.Ft_prev = nullptr;  // set by the launch when it completes the previous state's forces
    M.fdone_prev = nullptr;
    M.tag_prev = 0;
    M.P_prev = nullptr;
    M.scal = nullptr;
    M.V = 0.0;
    M.F = nullptr;
    return M;
}

}  // namespace memd
