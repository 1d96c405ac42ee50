// kernels_field.hip -- lattice-field kernels for gfx950: the fused leapfrog
// (Faraday + Ampere, body in leapfrog_tile.hpp), energy and Gauss-audit
// reductions, permittivity maps, the salt-dependent permittivity.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_util.hpp"
#include "ion_ops.hpp"
#include "ion_records.hpp"
#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"

namespace memd {

template <typename T, int EM, int R>
__global__ __launch_bounds__(256) void k_leapfrog(LfArgs<T> A) {
    __shared__ LfSmem<T, R> S;
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    const int tile_x = logical % A.ntx;
    const int rest = logical / A.ntx;
    leapfrog_tile<T, EM, R>(A, tile_x, rest % A.nty, rest / A.nty, S);
}

// The leapfrog with the deposit of the regular ions fused in (leapfrog_tile.hpp),
// and the ion movers (ion_records.hpp) as M.nblocks workgroups of their own:
// ahead of the tiles when every tile is resident at once (they take CU slots
// at the start, and the tiles they hold back fill the slots that tiles free
// at the end), else after them (they fill the last round's free slots).
template <typename T, int EM, int R, int TZ, bool CAP = false>
__global__ __launch_bounds__(256) void k_leapfrog_dep(LfArgs<T> A, DepArgs P, MoverArgs<T> M) {
    __shared__ LfSmem<T, R> S;
    __shared__ DepSmem<T, R, TZ> DS;
    const int b = (int)blockIdx.x, nt = (int)gridDim.x - M.nblocks;
    const int m = M.ahead ? b : b - nt;  // the mover index, for a mover workgroup
    if (m >= 0 && m < M.nblocks) {
        move_ions<T>(M, m * kMoverIons, kMoverIons, m, DS.psum);
        return;
    }
    const int logical = xcd_logical(M.ahead ? b - M.nblocks : b, nt);
    const int tile_x = logical % A.ntx;
    const int rest = logical / A.ntx;
    leapfrog_tile<T, EM, R, true, TZ, CAP>(A, tile_x, rest % A.nty, rest / A.nty, S, &P, &DS);
}

// Workgroups of the kernel the whole device holds at once (0: unknown).
static int resident_blocks(const void *kernel) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

// Measured once per kernel, on the first device that launches it (the
// devices a process drives are taken to be alike).
template <typename T, int EM, int R, int TZ, bool CAP = false>
static int dep_resident() {
    static const int slots = resident_blocks((const void *)k_leapfrog_dep<T, EM, R, TZ, CAP>);
    return slots;
}

template <typename T, int EM>
static hipError_t launch_lf_t(memd_ctx *c, const void *Din, const void *Bin, void *Dout, void *Bout,
                              hipEvent_t e0, hipEvent_t e1, const DepArgs *dep, const MoverArgs<T> *mv) {
    LfArgs<T> A;
    A.Din = (const T *)Din;
    A.Bin = (const T *)Bin;
    A.Dout = (T *)Dout;
    A.Bout = (T *)Bout;
    A.eta_link = (const T *)c->eta_link;
    A.eta_prof = (const T *)c->eta_prof;
    A.eta_uni = (T)c->eta_uni;
    A.kB = (T)(c->dt / c->a);
    A.kD = (T)(c->dt * c->c * c->c / c->a);
    A.L = c->L;
    A.Ns = c->Ns;
    const int R = c->lf_rows;
    const int TY = 4 * R;
    A.ntx = (c->L + 63) / 64;
    A.nty = (c->L + TY - 1) / TY;
    A.tz = c->lf_tz;
    const int nz = (c->L + A.tz - 1) / A.tz;
    const int nblk = A.ntx * A.nty * nz;
    if (dep) {
        MoverArgs<T> M{};
        if (mv) M = *mv;
        void (*kern)(LfArgs<T>, DepArgs, MoverArgs<T>) = nullptr;
        int slots = 0;
        if (dep->ecap && R == 1 && A.tz > kDepTZ) {
            kern = k_leapfrog_dep<T, EM, 1, kDepTZWide, true>;
            slots = dep_resident<T, EM, 1, kDepTZWide, true>();
        } else if (dep->ecap && R == 1) {
            kern = k_leapfrog_dep<T, EM, 1, kDepTZ, true>;
            slots = dep_resident<T, EM, 1, kDepTZ, true>();
        } else if (R == 1 && A.tz > kDepTZ) {
            kern = k_leapfrog_dep<T, EM, 1, kDepTZWide>;
            slots = dep_resident<T, EM, 1, kDepTZWide>();
        } else if (R == 1) {
            kern = k_leapfrog_dep<T, EM, 1, kDepTZ>;
            slots = dep_resident<T, EM, 1, kDepTZ>();
        } else if (dep->ecap) {
            kern = k_leapfrog_dep<T, EM, 2, kDepTZ, true>;
            slots = dep_resident<T, EM, 2, kDepTZ, true>();
        } else {
            kern = k_leapfrog_dep<T, EM, 2, kDepTZ>;
            slots = dep_resident<T, EM, 2, kDepTZ>();
        }
        M.ahead = nblk <= slots ? 1 : 0;
        DepArgs P = *dep;
        P.dip_block = M.ahead ? M.nblocks : 0;  // the first tile sums the dipole
        // (the extended launch only where events ride on it)
        if (e0 || e1)
            hipExtLaunchKernelGGL(kern, dim3(nblk + M.nblocks), dim3(256), 0, c->stream, e0, e1, 0, A, P, M);
        else
            hipLaunchKernelGGL(kern, dim3(nblk + M.nblocks), dim3(256), 0, c->stream, A, P, M);
        return hipGetLastError();
    }
    if (R == 1)
        hipExtLaunchKernelGGL((k_leapfrog<T, EM, 1>), dim3(nblk), dim3(256), 0, c->stream, e0, e1, 0, A);
    else if (R == 2)
        hipExtLaunchKernelGGL((k_leapfrog<T, EM, 2>), dim3(nblk), dim3(256), 0, c->stream, e0, e1, 0, A);
    else
        hipExtLaunchKernelGGL((k_leapfrog<T, EM, 4>), dim3(nblk), dim3(256), 0, c->stream, e0, e1, 0, A);
    return hipGetLastError();
}

int list_tiles(const memd_ctx *c) {
    const int TY = 4 * c->lf_rows;
    return ((c->L + 63) / 64) * ((c->L + TY - 1) / TY) * ((c->L + c->lf_tz - 1) / c->lf_tz);
}

int list_cap(const memd_ctx *c) {
    const int nt = list_tiles(c);
    const size_t cap = c->list_entries / (size_t)(nt > 0 ? nt : 1);
    return cap > (size_t)INT32_MAX ? INT32_MAX : (int)cap;
}

bool fused_deposit_ok(const memd_ctx *c) {
    const int tz_max = c->lf_rows == 1 ? kDepTZWide : kDepTZ;
    return c->fuse_deposit && c->n > 0 && c->list && c->L >= 16 && c->L <= 1024 && c->lf_tz <= tz_max &&
           c->lf_rows <= (c->fp32 ? 2 : 1) && list_tiles(c) <= c->list_tiles_max && list_cap(c) >= 16;
}

hipError_t launch_leapfrog(memd_ctx *c, const void *Din, const void *Bin, void *Dout, void *Bout, hipEvent_t e0,
                           hipEvent_t e1, const double *disp, uint64_t seed, uint32_t t, double sigma,
                           bool with_deposit, bool need_pack, const double *dip_prev, int dip_nparts,
                           IonMoves *moves, bool own_forces) {
    DepArgs P;
    const DepArgs *dp = nullptr;
    unsigned int tag_prev = 0;
    c->ecap_tag = 0u;
    if (with_deposit) {
        // the lists first (records read each ion's list cell), then the
        // records unless the previous launch's movers wrote them against these lists
        const bool rebuild = c->lists_key != c->lf_rows * 4096 + c->lf_tz;
        if (rebuild) {
            hipError_t e = launch_build_lists(c, true, disp, seed, t, sigma);
            if (e != hipSuccess) return e;
        } else if (need_pack) {
            hipError_t e = launch_pack_ions(c, disp, seed, t, sigma);
            if (e != hipSuccess) return e;
        }
        P.head = c->rec_head;
        P.con0 = c->rec_con;
        P.con1 = c->rec_con1;
        P.list = c->list;
        P.count = c->list_count;
        P.cap = list_cap(c);
        P.own_forces = own_forces ? 1 : 0;
        P.fq = c->fq;
        P.ecell = c->ecell;
        const bool odd = (c->step_index & 1) != 0;
        P.Ft = c->fold_step && odd ? c->Ft_alt : c->Ft;
        P.fdone = c->fold_step && odd ? c->fdone_alt : c->fdone;
        tag_prev = c->force_tag;
        if (++c->force_tag == 0) c->force_tag = 1;  // 0 never marks a result
        P.tag = c->force_tag;
        P.G = c->scal + S_G;
        P.a = c->a;
        P.dip_prev = dip_prev;
        // (a list build just now may have rewritten the ions' own dynamics'
        // position partials, with its own count)
        P.dip_nparts = c->md_pos && dip_prev ? c->pos_nb : dip_nparts;
        P.P = c->scal + (c->fold_step ? S_PB + 3 * (int)(c->step_index & 1) : S_P);
        P.ovf_mark = c->fold_step ? c->ovf_mark : nullptr;
        P.V = c->V;
        P.eta_uni = c->eta_uni;
        P.epsh = c->scal + S_EPSH;
        P.irr_cnt = c->tile_irregular ? irr_count(c, c->step_index) : nullptr;
        P.irr_zero = c->tile_irregular ? irr_count(c, c->step_index + 2) : nullptr;
        P.irr_r = c->r;
        P.irr_du = c->du_slot;
        P.irr_q = c->q;
        P.irr_order = c->sorted ? nullptr : c->order;
        // the ions' own dynamics capture the new state's field for the ion
        // kernel that follows (with the atomic path on the tiles' list and
        // the Green's-function self energy)
        const bool cap = !own_forces && c->ecap && c->tile_irregular && c->self_scheme == MEMD_SELF_GREEN;
        P.endc = cap ? c->endc : nullptr;
        P.ecap = cap ? c->ecap : nullptr;
        P.ecap_bad = cap ? c->ecap_bad : nullptr;
        c->ecap_tag = cap ? P.tag : 0u;
        dp = &P;
    }
    const bool with_moves = dp && moves;
    if (with_moves) moves->nparts = mover_blocks(c->n);
    // the movers complete the forces of the state the previous launch started from
    auto assemble = [&](auto &M) {
        if (!(with_moves && c->fold_step && moves->assemble)) return;
        const bool prev_odd = ((c->step_index - 1) & 1) != 0;
        M.Ft_prev = prev_odd ? c->Ft_alt : c->Ft;
        M.fdone_prev = prev_odd ? c->fdone_alt : c->fdone;
        M.tag_prev = tag_prev;
        M.P_prev = c->scal + S_PB + 3 * (prev_odd ? 1 : 0);
        M.scal = c->scal;
        M.V = c->V;
        M.F = c->F;
    };
    if (c->fp32) {
        MoverArgs<float> M{};
        if (with_moves) M = mover_args<float>(c, *moves);
        assemble(M);
        const MoverArgs<float> *mp = with_moves ? &M : nullptr;
        switch (c->eta_mode) {
            case ETA_UNIFORM: return launch_lf_t<float, ETA_UNIFORM>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
            case ETA_ZPROF: return launch_lf_t<float, ETA_ZPROF>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
            default: return launch_lf_t<float, ETA_LINK>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
        }
    }
    MoverArgs<double> M{};
    if (with_moves) M = mover_args<double>(c, *moves);
    assemble(M);
    const MoverArgs<double> *mp = with_moves ? &M : nullptr;
    switch (c->eta_mode) {
        case ETA_UNIFORM: return launch_lf_t<double, ETA_UNIFORM>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
        case ETA_ZPROF: return launch_lf_t<double, ETA_ZPROF>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
        default: return launch_lf_t<double, ETA_LINK>(c, Din, Bin, Dout, Bout, e0, e1, dp, mp);
    }
}

// ------------------------------------------------------------------ energy

// The site-loop kernels (energy, audit) walk the lattice by row chunks
// (64 sites along x at one (y, z)), one wavefront per chunk of a 256-thread
// block: chunk k has x0 = 64 (k mod nxc),
// y = (k / nxc) mod L, z = k / (nxc L), nxc = ceil(L / 64).
struct RowChunk {
    int x, y, z;
    bool live;
};
__device__ __forceinline__ RowChunk row_chunk(int k, int L) {
    const int nxc = (L + 63) >> 6;
    const int yz = k / nxc;
    RowChunk r;
    r.x = (k - yz * nxc) * 64 + (int)(threadIdx.x & 63);
    r.y = yz % L;
    r.z = yz / L;
    r.live = r.x < L;
    return r;
}

// (over the first nblk blocks of the grid)
template <typename F>
__device__ __forceinline__ void for_row_chunks(int L, int nblk, F &&body) {
    const int nch = ((L + 63) >> 6) * L * L;
    for (int k = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6))); k < nch;
         k += nblk * 4) {
        const RowChunk rc = row_chunk(k, L);
        if (rc.live) body(rc);
    }
}

template <typename T>
struct FieldView {
    const T *D;
    const T *B;
    const T *eta_link;
    const T *eta_prof;
    double eta_uni;
    int mode;
    int L;
    size_t Ns;
};

template <typename T>
__device__ __forceinline__ double eta_fv(const FieldView<T> &V, int d, int k, size_t off) {
    if (V.mode == ETA_UNIFORM) return V.eta_uni;
    if (V.mode == ETA_ZPROF) return (double)V.eta_prof[d * V.L + k];
    return (double)V.eta_link[(size_t)d * V.Ns + off];
}

template <typename T>
__device__ __forceinline__ double X_at(const FieldView<T> &V, int d, int i, int j, int k) {
    const size_t off = site_index(i, j, k, V.L);
    return eta_fv(V, d, k, off) * (double)V.D[(size_t)d * V.Ns + off];
}

template <typename T>
static FieldView<T> make_view(memd_ctx *c, const void *D, const void *B) {
    FieldView<T> V;
    V.D = (const T *)D;
    V.B = (const T *)B;
    V.eta_link = (const T *)c->eta_link;
    V.eta_prof = (const T *)c->eta_prof;
    V.eta_uni = c->eta_uni;
    V.mode = c->eta_mode;
    V.L = c->L;
    V.Ns = c->Ns;
    return V;
}

static int site_blocks(size_t Ns) {
    size_t b = (Ns + kThreads - 1) / kThreads;
    return (int)(b < (size_t)kSiteBlocks ? b : (size_t)kSiteBlocks);
}

// ------------------------------------------------------------------- audit

// R_v = a^2 sum_d [D_d(v) - D_d(v-e_d)] - rho_v in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_audit(const T *__restrict__ D, const double *__restrict__ rho,
                                               int L, size_t Ns, double a2, double *partials) {
    double mx = 0.0, ss = 0.0;
    for_row_chunks(L, (int)gridDim.x, [&](const RowChunk &rc) {
        const int i = rc.x, j = rc.y, k = rc.z;
        const size_t v = ((size_t)k * L + j) * L + i;
        const size_t vx = site_index(i == 0 ? L - 1 : i - 1, j, k, L);
        const size_t vy = site_index(i, j == 0 ? L - 1 : j - 1, k, L);
        const size_t vz = site_index(i, j, k == 0 ? L - 1 : k - 1, L);
        const double dv = ((double)D[v] - (double)D[vx]) + ((double)D[Ns + v] - (double)D[Ns + vy]) +
                          ((double)D[2 * Ns + v] - (double)D[2 * Ns + vz]);
        const double R = a2 * dv - rho[v];
        mx = fmax(mx, fabs(R));
        ss += R * R;
    });
    double s[1] = {ss};
    block_sum<1>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = m;
        partials[2 * blockIdx.x + 1] = s[0];
    }
}

hipError_t launch_audit_raw(hipStream_t s, const void *D, bool fp32, const double *rho, int L, double a,
                            double *partials, int *nblk) {
    const size_t Ns = (size_t)L * L * L;
    const int nb = site_blocks(Ns);
    *nblk = nb;
    const double a2 = a * a;
    if (fp32)
        hipLaunchKernelGGL(k_audit<float>, dim3(nb), dim3(kThreads), 0, s, (const float *)D, rho, L, Ns, a2,
                           partials);
    else
        hipLaunchKernelGGL(k_audit<double>, dim3(nb), dim3(kThreads), 0, s, (const double *)D, rho, L, Ns, a2,
                           partials);
    return hipGetLastError();
}

// The observables of the current state in one pass over the lattice, per
// block: with ENG, sum eta D^2 and sum B (B - (dt/a) C(eta D)) (W_E = 1/2 a^3
// of the first, W_B = (c^2/2) a^3 of the second: the leapfrog's shadow form
// B^{n+1/2} B^{n+3/2}, the later factor made here); with AUD, max |R| and
// sum R^2 of R_v = a^2 sum_d [D_d(v) - D_d(v-e_d)] - rho_v, the audit k_audit
// also forms.  Four partials per block (we, wb, max, sum).  With ENG the
// launch's last U.nb blocks compute the self-energy partials instead
// (self_energy_block), beside the field blocks.
template <typename T, bool AUD, bool ENG>
__global__ __launch_bounds__(256) void k_field_obs(FieldView<T> V, double kB, double a2, const double *__restrict__ rho,
                                                   double *partials, SelfEnergyArgs U) {
    const int L = V.L;
    const size_t Ns = V.Ns;
    const int nf = (int)gridDim.x - (ENG ? U.nb : 0);  // field blocks
    if (ENG && (int)blockIdx.x >= nf) {
        const EtaView<T> ev{V.mode, V.eta_uni, V.eta_prof, V.eta_link};
        self_energy_block<T>((int)blockIdx.x - nf, U, L, Ns, ev);
        return;
    }
    double we = 0.0, wb = 0.0, mx = 0.0, ss = 0.0;
    for_row_chunks(L, nf, [&](const RowChunk &rc) {
        const int i = rc.x, j = rc.y, k = rc.z;
        const size_t v = ((size_t)k * L + j) * L + i;
        double Dv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) Dv[d] = (double)V.D[(size_t)d * Ns + v];
        if constexpr (ENG) {
            const int ip = (i + 1 == L) ? 0 : i + 1, jp = (j + 1 == L) ? 0 : j + 1,
                      kp = (k + 1 == L) ? 0 : k + 1;
            double X[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                X[d] = eta_fv(V, d, k, v) * Dv[d];
                we += X[d] * Dv[d];
            }
            const double cx = X_at(V, 2, i, jp, k) - X[2] - X_at(V, 1, i, j, kp) + X[1];
            const double cy = X_at(V, 0, i, j, kp) - X[0] - X_at(V, 2, ip, j, k) + X[2];
            const double cz = X_at(V, 1, ip, j, k) - X[1] - X_at(V, 0, i, jp, k) + X[0];
            const double bx = (double)V.B[v], by = (double)V.B[Ns + v], bz = (double)V.B[2 * Ns + v];
            wb += bx * (bx - kB * cx) + by * (by - kB * cy) + bz * (bz - kB * cz);
        }
        if constexpr (AUD) {
            const size_t vx = site_index(i == 0 ? L - 1 : i - 1, j, k, L);
            const size_t vy = site_index(i, j == 0 ? L - 1 : j - 1, k, L);
            const size_t vz = site_index(i, j, k == 0 ? L - 1 : k - 1, L);
            const double dv = (Dv[0] - (double)V.D[vx]) + (Dv[1] - (double)V.D[Ns + vy]) +
                              (Dv[2] - (double)V.D[2 * Ns + vz]);
            const double R = a2 * dv - rho[v];
            mx = fmax(mx, fabs(R));
            ss += R * R;
        }
    });
    double s[3] = {we, wb, ss};
    block_sum<3>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        partials[4 * blockIdx.x] = s[0];
        partials[4 * blockIdx.x + 1] = s[1];
        partials[4 * blockIdx.x + 2] = m;
        partials[4 * blockIdx.x + 3] = s[2];
    }
}

// The observables pass runs 2048 blocks at most (four row chunks per
// wavefront at 128^3): at c4 it took 35.3 us on 8192 blocks (one chunk per
// wavefront, each block's reduction for 256 sites), 30.9 on 4096 and 27.7 on
// 2048, and its finaliser 13.2, 10.4 and 9.1 us over those partials.
constexpr int kObsBlocks = 2048;

hipError_t launch_field_obs(memd_ctx *c, bool audit, bool energy, double *partials, int *nblk, double *ipart,
                            int *iblk) {
    const int nb = site_blocks(c->Ns) < kObsBlocks ? site_blocks(c->Ns) : kObsBlocks;
    *nblk = nb;
    // the self energies ride on the energy launch as blocks of their own
    SelfEnergyArgs U{c->n, energy ? ion_blocks_x8(c->n, 1) : 0, c->a, c->q, c->r, c->scal + S_G, ipart};
    *iblk = U.nb;
    const int grid = nb + U.nb;
    const double kB = c->dt / c->a, a2 = c->a * c->a;
    const void *D = c->D[c->cur], *B = c->B[c->cur];
    if (c->fp32) {
        const auto V = make_view<float>(c, D, B);
        if (audit && energy)
            hipLaunchKernelGGL((k_field_obs<float, true, true>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
        else if (audit)
            hipLaunchKernelGGL((k_field_obs<float, true, false>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
        else
            hipLaunchKernelGGL((k_field_obs<float, false, true>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
    } else {
        const auto V = make_view<double>(c, D, B);
        if (audit && energy)
            hipLaunchKernelGGL((k_field_obs<double, true, true>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
        else if (audit)
            hipLaunchKernelGGL((k_field_obs<double, true, false>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
        else
            hipLaunchKernelGGL((k_field_obs<double, false, true>), dim3(grid), dim3(kThreads), 0, c->stream, V, kB, a2,
                               c->rho, partials, U);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ casts

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, size_t count) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = (D)src[t];
}

static int grid_for(size_t count) {
    size_t b = (count + kThreads - 1) / kThreads;
    if (b > 8192) b = 8192;
    return (int)(b ? b : 1);
}

hipError_t launch_cast(hipStream_t s, const double *src, void *dst, size_t count, bool to_fp32) {
    if (to_fp32)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(count)), dim3(kThreads), 0, s, src,
                           (float *)dst, count);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid_for(count)), dim3(kThreads), 0, s, src,
                           (double *)dst, count);
    return hipGetLastError();
}

hipError_t launch_uncast(hipStream_t s, const void *src, double *dst, size_t count, bool from_fp32) {
    if (from_fp32)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(count)), dim3(kThreads), 0, s,
                           (const float *)src, dst, count);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid_for(count)), dim3(kThreads), 0, s,
                           (const double *)src, dst, count);
    return hipGetLastError();
}

__global__ void k_fill(double *dst, double v, size_t count) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = v;
}

hipError_t launch_fill(hipStream_t s, double *dst, double v, size_t count) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(kThreads), 0, s, dst, v, count);
    return hipGetLastError();
}

// ------------------------------------------------------------ permittivity

// Fig. 2b / eq. dielectric-interpolation: mean of the two site values, or the
// harmonic combination on an interface link (ratio above `ratio`), decided in
// FP64.
__device__ __forceinline__ double link_eps(double e1, double e2, double ratio) {
    const double hi = e1 > e2 ? e1 : e2, lo = e1 > e2 ? e2 : e1;
    if (hi / lo > ratio) return 1.0 / (0.5 / e1 + 0.5 / e2);
    return 0.5 * (e1 + e2);
}

template <typename T>
__global__ void k_eta_site(const double *__restrict__ eps, double ratio, int L, size_t Ns,
                           T *__restrict__ eta) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(v % L), j = (int)((v / L) % L), k = (int)(v / ((size_t)L * L));
        const double e = eps[v];
        const double ex = eps[site_index(i + 1 == L ? 0 : i + 1, j, k, L)];
        const double ey = eps[site_index(i, j + 1 == L ? 0 : j + 1, k, L)];
        const double ez = eps[site_index(i, j, k + 1 == L ? 0 : k + 1, L)];
        eta[v] = (T)(1.0 / link_eps(e, ex, ratio));
        eta[Ns + v] = (T)(1.0 / link_eps(e, ey, ratio));
        eta[2 * Ns + v] = (T)(1.0 / link_eps(e, ez, ratio));
    }
}

template <typename T>
__global__ void k_eta_link(const double *__restrict__ eps, size_t count, T *__restrict__ eta) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < count;
         t += (size_t)gridDim.x * blockDim.x)
        eta[t] = (T)(1.0 / eps[t]);
}

// planar profile: x and y links lie inside one plane (both ends equal), z
// links join plane k to plane k+1.
template <typename T>
__global__ void k_eta_zprof(const double *__restrict__ epsz, double ratio, int L, T *__restrict__ prof) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L) return;
    const double e = epsz[k], en = epsz[k + 1 == L ? 0 : k + 1];
    const double inplane = 1.0 / link_eps(e, e, ratio);
    prof[k] = (T)inplane;
    prof[L + k] = (T)inplane;
    prof[2 * L + k] = (T)(1.0 / link_eps(e, en, ratio));
}

hipError_t launch_eta_from_link(memd_ctx *c, const double *eps_link, void *eta) {
    const size_t cnt = 3 * c->Ns;
    if (c->fp32)
        hipLaunchKernelGGL(k_eta_link<float>, dim3(grid_for(cnt)), dim3(kThreads), 0, c->stream, eps_link,
                           cnt, (float *)eta);
    else
        hipLaunchKernelGGL(k_eta_link<double>, dim3(grid_for(cnt)), dim3(kThreads), 0, c->stream, eps_link,
                           cnt, (double *)eta);
    return hipGetLastError();
}

hipError_t launch_eta_zprof(memd_ctx *c, const double *eps_z, double ratio, void *prof) {
    const int nb = (c->L + kThreads - 1) / kThreads;
    if (c->fp32)
        hipLaunchKernelGGL(k_eta_zprof<float>, dim3(nb), dim3(kThreads), 0, c->stream, eps_z, ratio, c->L,
                           (float *)prof);
    else
        hipLaunchKernelGGL(k_eta_zprof<double>, dim3(nb), dim3(kThreads), 0, c->stream, eps_z, ratio, c->L,
                           (double *)prof);
    return hipGetLastError();
}

hipError_t launch_eta_from_site(memd_ctx *c, const double *eps_site, double ratio, void *eta) {
    if (c->fp32)
        hipLaunchKernelGGL(k_eta_site<float>, dim3(grid_for(c->Ns)), dim3(kThreads), 0, c->stream, eps_site,
                           ratio, c->L, c->Ns, (float *)eta);
    else
        hipLaunchKernelGGL(k_eta_site<double>, dim3(grid_for(c->Ns)), dim3(kThreads), 0, c->stream, eps_site,
                           ratio, c->L, c->Ns, (double *)eta);
    return hipGetLastError();
}

// Per-block sums of eta_d over all d-links and the maximum eta (-> eps_min).
template <typename T>
__global__ __launch_bounds__(256) void k_eta_sums(const T *__restrict__ eta_link,
                                                  const T *__restrict__ eta_prof, double eta_uni,
                                                  int mode, int L, size_t Ns, double *partials) {
    double s[3] = {0.0, 0.0, 0.0};
    double mx = 0.0;
    const size_t LL = (size_t)L * L;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns;
         v += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double e;
            if (mode == ETA_UNIFORM) e = eta_uni;
            else if (mode == ETA_ZPROF) e = (double)eta_prof[d * L + (int)(v / LL)];
            else e = (double)eta_link[(size_t)d * Ns + v];
            s[d] += e;
            mx = fmax(mx, e);
        }
    }
    block_sum<3>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        partials[4 * blockIdx.x] = s[0];
        partials[4 * blockIdx.x + 1] = s[1];
        partials[4 * blockIdx.x + 2] = s[2];
        partials[4 * blockIdx.x + 3] = m;
    }
}

hipError_t launch_eta_sums(memd_ctx *c, double *partials, int *nblk) {
    const int nb = site_blocks(c->Ns);
    *nblk = nb;
    if (c->fp32)
        hipLaunchKernelGGL(k_eta_sums<float>, dim3(nb), dim3(kThreads), 0, c->stream,
                           (const float *)c->eta_link, (const float *)c->eta_prof, c->eta_uni, c->eta_mode,
                           c->L, c->Ns, partials);
    else
        hipLaunchKernelGGL(k_eta_sums<double>, dim3(nb), dim3(kThreads), 0, c->stream,
                           (const double *)c->eta_link, (const double *)c->eta_prof, c->eta_uni,
                           c->eta_mode, c->L, c->Ns, partials);
    return hipGetLastError();
}

// ---------------------------------------------------- salt permittivity

// Salt permittivity from the ion counts cnt (CIC number of ions per vertex):
//   nbar_v = (1/27) sum over the periodic 3x3x3 vertex box of cnt / a^3,
//   eps of a link = eps_w - slope * (mean of nbar at its two ends), at least
//   eps_floor; eta = 1 / eps stored per link; per site 12 / (sum of eta over
//   the 12 edges of its cell), as force_ion sums the stored values; per
//   block the sums of eta_d and the largest eta (4 partials).
// A workgroup takes tiles of 64 x 4 sites and marches through a chunk of
// kSaltTZ planes.  Per plane R it stages cnt with a one-site halo in LDS,
// forms the 3 x 3 sums over (x, y) for the 65 x 5 corners its cells need,
// keeps those of the last three planes in registers (each thread its own
// corners), and from them nbar of plane R-1 (two planes kept in LDS).  From nbar of planes P and P+1 (P = R-2) it computes eta of the own
// links of plane P's sites, the tile and a +1 halo in x and y, once each
// (two planes kept in LDS), and stores the tile's; 12 / (sum of eta over the
// 12 edges of a cell) of plane P-1 then reads them all from LDS.
constexpr int kSaltTZ = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_salt_tile(const double *__restrict__ cnt, int L, size_t Ns, double inv27, double eps_w, double slope,
                                                   double eps_floor, T *__restrict__ eta, T *__restrict__ ecell,
                                                   double *__restrict__ partials) {
    __shared__ double sc[7][67];      // cnt of plane R, x0-1 .. x0+65, y0-1 .. y0+5
    __shared__ double sN[2][5][65];   // nbar of two planes (ring by plane)
    __shared__ T sE[2][3][5][65];     // eta of the own links of two planes' sites (ring by plane)
    const int lx = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int ntx = (L + 63) >> 6, nty = (L + 3) >> 2, ntz = (L + kSaltTZ - 1) / kSaltTZ;
    const int tiles = ntx * nty * ntz;
    double s[3] = {0.0, 0.0, 0.0}, mx = 0.0;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int x0 = (tile % ntx) * 64, y0 = ((tile / ntx) % nty) * 4, z0 = (tile / (ntx * nty)) * kSaltTZ;
        const int z1 = min(z0 + kSaltTZ, L);
        // this thread's (up to) two entries of a staged plane, the next plane
        // in flight while the current one is processed
        auto fetch = [&](int R, double (&v)[2]) {
            const size_t zoff = (size_t)wrapc(R, L) * L * L;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = threadIdx.x + 256 * j;
                const int iy = t / 67, ix = t - iy * 67;
                v[j] = t < 7 * 67 ? cnt[zoff + (size_t)wrapc(y0 - 1 + iy, L) * L + wrapc(x0 - 1 + ix, L)] : 0.0;
            }
        };
        double pl[2];
        fetch(z0 - 1, pl);
        double bs1[2] = {0.0, 0.0}, bs2[2] = {0.0, 0.0};  // box sums of planes R - 1 and R - 2
        for (int R = z0 - 1; R <= z1 + 2; ++R) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = threadIdx.x + 256 * j;
                if (t < 7 * 67) (&sc[0][0])[t] = pl[j];
            }
            if (R <= z1 + 1) fetch(R + 1, pl);
            __syncthreads();
            // the box sums of plane R for this thread's entries (t, t + 256);
            // those of the two planes before stay in registers, so nbar of
            // plane Q = R - 1 follows without a barrier
            const int Q = R - 1;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int t = threadIdx.x + 256 * j;
                if (t < 5 * 65) {
                    const int iy = t / 65, ix = t - iy * 65;
                    double b = 0.0;
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx) b += sc[iy + dy][ix + dx];
                    if (Q >= z0) sN[(Q + 2) & 1][iy][ix] = (bs2[j] + bs1[j] + b) * inv27;
                    bs2[j] = bs1[j];
                    bs1[j] = b;
                }
            }
            __syncthreads();
            const int P = Q - 1;  // eta of plane P's own links from nbar of P and P + 1
            if (P >= z0 && P <= z1) {
                const int sp = (P + 2) & 1, sq = (P + 3) & 1;
                for (int t = threadIdx.x; t < 4 * 64 + 64 + 5; t += 256) {
                    // the tile's 4 x 64 sites first (t < 256: the thread's own
                    // site), then the +1 halo: row y0+4 (64 sites), column x0+64 (5)
                    int iy, ix;
                    if (t < 256) {
                        iy = t >> 6;
                        ix = t & 63;
                    } else if (t < 320) {
                        iy = 4;
                        ix = t - 256;
                    } else {
                        iy = t - 320;
                        ix = 64;
                    }
                    const double n0 = sN[sp][iy][ix];
                    const double nn[3] = {ix < 64 ? sN[sp][iy][ix + 1] : 0.0, iy < 4 ? sN[sp][iy + 1][ix] : 0.0,
                                          sN[sq][iy][ix]};
                    T e3[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        // the halo's own x-links (y-links) at the +x (+y) edge
                        // are never read; their partner corner lies outside
                        double e = eps_w - slope * (0.5 * (n0 + nn[d]));
                        e = e < eps_floor ? eps_floor : e;
                        e3[d] = (T)(1.0 / e);
                        sE[P & 1][d][iy][ix] = e3[d];
                    }
                    const int x = x0 + ix, y = y0 + iy;
                    if (t < 256 && P < z1 && x < L && y < L) {
                        const size_t v = ((size_t)P * L + y) * L + x;
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            eta[(size_t)d * Ns + v] = e3[d];
                            s[d] += (double)e3[d];
                            mx = fmax(mx, (double)e3[d]);
                        }
                    }
                }
            }
            __syncthreads();
            const int O = P - 1;  // 12 / sum of the cell's 12 edges, plane O (own links of O and O + 1)
            if (ecell && O >= z0 && O < z1) {
                const int x = x0 + lx, y = y0 + wy;
                if (x < L && y < L) {
                    double sum = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const int d1 = d == 2 ? 0 : d + 1, d2 = d == 0 ? 2 : d - 1;
#pragma unroll
                        for (int o2 = 0; o2 < 2; ++o2)
#pragma unroll
                            for (int o1 = 0; o1 < 2; ++o1) {
                                const int ox = (d1 == 0 ? o1 : 0) + (d2 == 0 ? o2 : 0);
                                const int oy = (d1 == 1 ? o1 : 0) + (d2 == 1 ? o2 : 0);
                                const int oz = (d1 == 2 ? o1 : 0) + (d2 == 2 ? o2 : 0);
                                sum += (double)sE[(O + oz) & 1][d][wy + oy][lx + ox];
                            }
                    }
                    ecell[((size_t)O * L + y) * L + x] = (T)(12.0 / sum);
                }
            }
        }
    }
    block_sum<3>(s);
    const double m = block_max(mx);
    if (threadIdx.x == 0) {
        partials[4 * blockIdx.x] = s[0];
        partials[4 * blockIdx.x + 1] = s[1];
        partials[4 * blockIdx.x + 2] = s[2];
        partials[4 * blockIdx.x + 3] = m;
    }
}

// ecell[c] = 12 / (sum of eta over the 12 edges of cell c): the d-links at
// c + o1 e_d1 + o2 e_d2, summed in the order force_ion sums them.
template <typename T>
__global__ void k_ecell(int L, size_t Ns, EtaView<T> ev, T *__restrict__ out) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < Ns; v += (size_t)gridDim.x * blockDim.x) {
        const int c[3] = {(int)(v % L), (int)((v / L) % L), (int)(v / ((size_t)L * L))};
        const int cp[3] = {c[0] + 1 == L ? 0 : c[0] + 1, c[1] + 1 == L ? 0 : c[1] + 1, c[2] + 1 == L ? 0 : c[2] + 1};
        double sum = 0.0;
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
                    sum += ev.at(d, x[2], site_index(x[0], x[1], x[2], L), L, Ns);
                }
        }
        out[v] = (T)(12.0 / sum);
    }
}

hipError_t launch_ecell(memd_ctx *c) {
    if (!c->ecell) return hipSuccess;
    const int g = grid_for(c->Ns);
    if (c->fp32) {
        const EtaView<float> ev{c->eta_mode, c->eta_uni, (const float *)c->eta_prof, (const float *)c->eta_link};
        hipLaunchKernelGGL(k_ecell<float>, dim3(g), dim3(kThreads), 0, c->stream, c->L, c->Ns, ev,
                           (float *)c->ecell);
    } else {
        const EtaView<double> ev{c->eta_mode, c->eta_uni, (const double *)c->eta_prof, (const double *)c->eta_link};
        hipLaunchKernelGGL(k_ecell<double>, dim3(g), dim3(kThreads), 0, c->stream, c->L, c->Ns, ev,
                           (double *)c->ecell);
    }
    return hipGetLastError();
}

hipError_t launch_salt(memd_ctx *c) {
    hipError_t e;
    double *cnt = c->salt_cnt;
    // (the audit that ended the previous step may have written the counts)
    if (c->salt_cnt_step != c->step_index && (e = launch_spread_dense(c, false, cnt)) != hipSuccess) return e;
    c->salt_cnt_step = -1;
    const double a3 = c->a * c->a * c->a;
    const int L = c->L;
    const int tiles = ((L + 63) / 64) * ((L + 3) / 4) * ((L + kSaltTZ - 1) / kSaltTZ);
    const int nb = tiles < kSiteBlocks ? tiles : kSiteBlocks;
    if (c->fp32)
        hipLaunchKernelGGL(k_salt_tile<float>, dim3(nb), dim3(kThreads), 0, c->stream, cnt, L, c->Ns,
                           1.0 / (27.0 * a3), c->salt_w, c->salt_slope, c->salt_floor, (float *)c->eta_link,
                           (float *)c->ecell, c->partials);
    else
        hipLaunchKernelGGL(k_salt_tile<double>, dim3(nb), dim3(kThreads), 0, c->stream, cnt, L, c->Ns,
                           1.0 / (27.0 * a3), c->salt_w, c->salt_slope, c->salt_floor, (double *)c->eta_link,
                           (double *)c->ecell, c->partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_finalize_epsh(c->stream, c->partials, nb, (double)c->Ns, c->scal + S_EPSH,
                                c->scal + S_ETAMAX);
}

}  // namespace memd
