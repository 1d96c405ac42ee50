// memd_internal.hpp -- context layout and launch interfaces shared by the
// translation units of libmemd (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/memd.h"

namespace memd {

// Offsets into the per-context device scalar block (FP64).
enum ScalarSlot : int {
    S_P = 0,        // dipole moment P[3]
    S_EPSH = 3,     // directional harmonic means eps_h[3]
    S_G = 6,        // lattice Green's function G[4] at (000),(100),(110),(111)
    S_AUDIT = 10,   // last audit: max, rms
    S_ENERGY = 12,  // last energy: 5 values
    S_CG = 20,      // conjugate-gradient scalars (20 slots)
    S_MEAN = 40,    // mean of D per direction [3]
    S_ETAMAX = 44,  // maximum eta over the links (1 / eps_min)
    S_DIPW = 45,    // weight of the dipole correction: 1 (on, the default) or 0 (off)
    S_PB = 46,      // P of the state a fused launch starts from, by the step's parity [2][3]
    S_COUNT = 64
};

enum EtaMode : int { ETA_UNIFORM = 0, ETA_ZPROF = 1, ETA_LINK = 2 };

enum Family : int {
    F_LEAPFROG = 0, F_DEPOSIT = 1, F_FORCES = 2, F_AUDIT = 3, F_ENERGY = 4, F_DIPOLE = 5,
    F_SALT = 6, F_NFAM = 7
};

constexpr int kRedBlocks = 1024;   // grid of the solver's reductions
constexpr int kSiteBlocks = 8192;  // grid of the field site-loop reductions (energy, audit, permittivity)
constexpr int kThreads = 256;      // threads per block of the plain kernels

struct EtaDesc {
    int mode;
    double uni;            // ETA_UNIFORM
    const void *prof;      // ETA_ZPROF: T[3*L]: eta_x(k), eta_y(k), eta_z(k)
    const void *link;      // ETA_LINK:  T[3*Ns]
};

struct ProfileEvents {
    std::vector<hipEvent_t> start, stop;
    std::vector<long> count;  // launches between start[k] and stop[k]
    std::vector<hipEvent_t> pool;  // made in advance, not yet used
    long seen = 0;  // launches of the family since the collection started
    bool open = false;  // a begin event is waiting for its end
};

}  // namespace memd

struct memd_ctx {
    void *arena;  // the one device allocation every fixed buffer below is carved from
    memd_params p;
    int n;
    int L;
    size_t Ns;
    double a, dt, c, V;
    bool fp32;
    size_t tsize;  // sizeof(T) of the field storage

    hipStream_t stream;
    bool own_stream;
    int device;

    // permittivity
    int eta_mode;
    double eta_uni;
    void *eta_prof;   // T[3L]
    void *eta_link;   // T[3Ns]
    double eps_h[3];
    double eps_min;
    bool c_fixed;
    int salt_every;
    bool dipole_correction;  // mirrors scal[S_DIPW]
    int self_scheme;         // memd_self_scheme
    double salt_w, salt_slope, salt_floor;
    double *salt_cnt;  // FP64 [Ns]: ion counts of the salt permittivity
    long salt_cnt_step;  // salt_cnt already holds the counts of the positions at this step (-1: none)

    // fields: ping-pong buffers, cur holds the live state
    void *D[2];
    void *B[2];
    int cur;

    // ions
    double *q;     // [n]
    double *r;     // [3n]
    double *F;     // [3n]
    int *order;    // [n] ion visiting order (binned by lattice row), refreshed every sort_every steps
    int *slot;     // [n] inverse of order: the slot of ion i
    // Storage order of the ion arrays r, q, F: the caller's order until the
    // first re-binning of a step loop, which moves them into bin order; perm
    // maps a storage index to the caller's index (identity while !sorted).
    int *perm;
    bool sorted;
    double *r_alt, *q_alt, *F_alt;  // targets of the re-binning's move
    int *perm_alt;
    int *bins;     // [3 L^2] bin counts, row starts, cursors
    // Fused deposit (leapfrog_tile.hpp): records by slot (rec_head, rec_con),
    // the tile lists built at re-binning for the tile shape lists_key
    // (rows * 4096 + planes; -1: none), list_entries entries shared by the
    // tiles, and per slot the cell at the build (cbin) and list_fail.
    int4 *rec_head;
    void *rec_con, *rec_con1;  // the records' first cells, second cells (one allocation)
    int *list, *list_count, *cbin, *list_fail;
    double *du_slot;  // [3n] by slot: the displacement each record was made for
    // The second record set (head, values, displacement, fq, dep_atomic):
    // the ion movers of a fused leapfrog launch fill it for the step after
    // the current one, and the two sets swap when that step starts.
    int4 *rec_head_nx;
    void *rec_con_nx, *rec_con1_nx, *fq_nx;
    double *du_slot_nx;
    int *dep_atomic_nx;
    // Forces computed by the leapfrog tiles (DepArgs): fractional positions
    // and charges by slot (fq), 12 / (sum of the cell's 12 eta) per site
    // (ecell), the tile results by slot (Ft) with their launch stamp (fdone,
    // compared with force_tag, which every fused leapfrog launch advances).
    void *fq, *ecell;
    double *Ft;
    unsigned int *fdone;
    unsigned int force_tag;
    // One launch per step (fold_step, set for each launch): the tile results
    // of state t go to the buffers of t's parity (Ft and fdone for even t,
    // Ft_alt and fdone_alt for odd), and the movers of the next launch
    // complete them into F; ovf_mark: the owned ions a tile gathers itself.
    double *Ft_alt;
    unsigned int *fdone_alt;
    unsigned int *ovf_mark;
    bool fold_step;
    size_t list_entries;
    int list_tiles_max;
    int lists_key;
    int list_zero_key;  // shape whose list counts are all zero (-1: none)
    int *dep_atomic;
    // The ions the atomic path holds, per step (index step mod 3): a count in
    // a 128-byte line of its own, then their slots (irr_list).  Whatever
    // writes a step's records appends its atomic-path ions; the leapfrog
    // tiles of that step deposit their moves on the links they own; the
    // leapfrog launch of step t clears the count of step t + 2.
    int *irr;
    bool tile_irregular;      // the tiles, not the finisher, deposit those ions' moves
    bool final_forces;        // a call ends with the forces of its final state (memd_set_final_forces)
    unsigned int *bad_moves;  // rejected displacement components (not finite or > L a)
    bool fuse_deposit;
    int sort_every;
    double *stage;       // FP64 staging buffer for host inputs / FP32 casts
    size_t stage_bytes;
    double *md_buf;      // ion dynamics: the step's move [3n], staged velocities [3n] and masses [n]
    // ion dynamics with the fused deposit: the field E = eta D of the new
    // state on the 12 links of each ion's end cell, captured by the leapfrog
    // tiles ([12n] field type, by slot), the launch tag of the ions whose
    // capture was incomplete ([n]), the end cell of each record's move ([n]);
    // one allocation (md_cap), made by the first memd_md_step
    void *md_cap;
    void *ecap;
    unsigned int *ecap_bad;
    int *endc;
    unsigned int ecap_tag;  // tag of the leapfrog launch that captured (0: none)
    long irr_zeroed;        // step whose atomic-path count the last re-binning cleared (-1: none)
    // the ions' own dynamics without movers in the leapfrog: a list build
    // that packs records also writes the moves' end positions (r_alt) and
    // their dipole partials (dip[step_index & 1], pos_nb of them)
    bool md_pos;
    int pos_nb;
    long perm_version;   // advanced whenever perm changes

    // reductions and audit
    double *rho;       // FP64 [Ns]: the charge assignment of the last audit
    int *drift;        // [n] by storage index: ion left to the atomic pass of the spread
    double *partials;  // FP64 reduction scratch (partial_doubles)
    double *dip[2];    // FP64 per-workgroup q r sums of the ion movers, alternating by step
    double *scal;      // FP64 [S_COUNT]
    double *hist_audit;   // FP64 [2*hist_cap]
    double *hist_energy;  // FP64 [5*hist_cap]
    int hist_cap;
    int hist_audit_n, hist_energy_n;

    bool ready;      // initial solve done or state set
    bool poisoned;
    long step_index;

    // leapfrog tiling
    int lf_rows;
    int lf_tz;

    // profiling
    bool prof_on;
    unsigned prof_mask;
    int prof_every;
    memd::ProfileEvents prof[memd::F_NFAM];
};

namespace memd {

// The ion movers of a fused leapfrog launch (ion_records.hpp): every ion
// moved by its record's displacement into r_alt, one dipole partial of
// q r^{n+1} per mover workgroup into dip_out (nparts, set by the launch),
// and with pack_next the next step's records (displacements disp_next, or
// the Philox stream at t_next) into the second record set.
// The count of the atomic-path ions of step `step` (its slots follow at +32).
constexpr int kIrrHead = 32;
inline int *irr_count(const memd_ctx *c, long step) {
    return c->irr ? c->irr + (step % 3) * (kIrrHead + (size_t)(c->n > 0 ? c->n : 1)) : nullptr;
}

// Sites per leapfrog work item of a lattice narrower than a wavefront (the
// batched leapfrog's tiles of whole rows: 256 / L rows of L < 64 sites).
constexpr int kRowSites = 256;

struct IonMoves {
    const double *disp_next;
    uint64_t seed;
    uint32_t t_next;
    double sigma;
    bool pack_next;
    double *dip_out;
    int nparts;
    bool assemble;  // (one launch per step) complete the previous state's forces
};

// ---- launchers (field kernels) ----
// ev0/ev1 (optional): events recorded at the kernel's start and end.
// with_deposit: the regular ions' deposit is fused in (displacements from disp,
// or from the Philox stream when disp is null); requires fused_deposit_ok(c).
// need_pack: write the deposit records first (false when the previous
// launch's movers already wrote them for this step).  dip_prev (nparts
// values of 3): the previous step's dipole partials, which the fused kernel
// sums into the scalars' P (null: P is already there).  moves (with the
// deposit only; null: none): the ion movers run in the same launch.
// own_forces: the tiles compute the forces of the ions whose start cell they
// own (off for the ions' own dynamics, which gathers forces after the step).
hipError_t launch_leapfrog(memd_ctx *c, const void *Din, const void *Bin, void *Dout, void *Bout,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, const double *disp = nullptr,
                           uint64_t seed = 0, uint32_t t = 0, double sigma = 0.0, bool with_deposit = false,
                           bool need_pack = true, const double *dip_prev = nullptr, int dip_nparts = 0,
                           IonMoves *moves = nullptr, bool own_forces = true);
bool fused_deposit_ok(const memd_ctx *c);
// Tiles of the current leapfrog tile shape, and the list capacity per tile.
int list_tiles(const memd_ctx *c);
int list_cap(const memd_ctx *c);
// Tile lists of the fused deposit for the current tile shape and positions.
hipError_t launch_build_lists(memd_ctx *c, bool pack, const double *disp, uint64_t seed, uint32_t t,
                              double sigma);
// 12 / (sum of eta over each cell's 12 edges), after any permittivity change
// (no-op when the context has no fused deposit).
hipError_t launch_ecell(memd_ctx *c);
hipError_t launch_pack_ions(memd_ctx *c, const double *disp, uint64_t seed, uint32_t t, double sigma);
// Clears the count of the atomic-path ions of the current step (before its
// records are written whole).
hipError_t launch_clear_irregular(memd_ctx *c);
// The ion side of a step after the fused leapfrog and its movers
// (k_ion_finish): forces of the state the step started from (tile results,
// or gathered from Dcur at r^n, plus the dipole term with the scalars' P),
// and the irregular ions of the current records deposited into Dnext with
// global atomics (from r^n, still in c->r).
// forces = false: only the irregular deposits (the ions' own dynamics gathers
// the new state's forces after the step).
hipError_t launch_ion_finish(memd_ctx *c, const void *Dcur, void *Dnext, bool forces = true);
// The dipole moment and the forces of the context's current state (D[cur],
// r), recomputed on its stream (the server, for a replica the batched kernels
// advanced).
hipError_t refresh_forces(memd_ctx *c);
// The ion side of a step of the ions' own dynamics (k_md_ions): the forces of
// the state in D (gather; else c->F as it is, dip_partials unused), `kicks`
// half kicks of v (caller order, masses too), with pack the next move dt v
// into disp (caller order), with records also its deposit records (the
// current set; the fused deposit only).
// with positions also the end position of each next move into r_alt and
// their dipole partials into dip[step_index & 1] (pos_nb of them), so that the
// next step's leapfrog runs no movers.
hipError_t launch_md_ions(memd_ctx *c, const void *D, const double *dip_partials, int dip_nblk, bool gather,
                          const double *mass, double *v, int kicks, double *disp, bool pack, bool records,
                          bool positions = false);
// grid of the sorted-order ion kernels (lanes_per_ion lanes per ion): a
// multiple of the 8 XCDs
inline int ion_blocks_x8(int n, int lanes_per_ion = 1) {
    const long long t = (long long)(n > 0 ? n : 1) * lanes_per_ion;
    const int b = (int)((t + kThreads - 1) / kThreads);
    return (b + 7) / 8 * 8;
}
// Energy and/or audit of the current state in one pass over the lattice
// (the audit reads c->rho): partials[4 nblk] = (we, wb, max |R|, sum R^2).
// (with energy also the self-energy partials into ipart, iblk of them)
hipError_t launch_field_obs(memd_ctx *c, bool audit, bool energy, double *partials, int *nblk, double *ipart,
                            int *iblk);
// The audit's site pass on any buffers: partials[2 * nblk] (max |R|, sum R^2
// per block) of R_v = a^2 div D(v) - rho_v; nblk <= kSiteBlocks.
hipError_t launch_audit_raw(hipStream_t s, const void *D, bool fp32, const double *rho, int L, double a,
                            double *partials, int *nblk);
hipError_t launch_cast(hipStream_t s, const double *src, void *dst, size_t count, bool to_fp32);
hipError_t launch_uncast(hipStream_t s, const void *src, double *dst, size_t count, bool from_fp32);
hipError_t launch_eta_from_link(memd_ctx *c, const double *eps_link, void *eta_link);
hipError_t launch_eta_from_site(memd_ctx *c, const double *eps_site, double ratio, void *eta_link);
hipError_t launch_eta_zprof(memd_ctx *c, const double *eps_z, double ratio, void *prof);
hipError_t launch_eta_sums(memd_ctx *c, double *partials, int *nblk);
hipError_t launch_salt(memd_ctx *c);
hipError_t launch_fill(hipStream_t s, double *dst, double v, size_t count);

// ---- launchers (ion kernels) ----
// disp == nullptr: displacements from the Philox stream (seed, step t, sigma)
hipError_t launch_deposit(memd_ctx *c, void *D, const double *disp, double *partials, int *nblk,
                          uint64_t seed = 0, uint32_t t = 0, double sigma = 0.0);
hipError_t launch_spread(memd_ctx *c, const double *charges_or_null, double *dst);
// dst += the linear assignment of q[i] (1 when q is null) at r[3i..3i+2], FP64 atomics.
hipError_t launch_spread_raw(hipStream_t s, int n, int L, double a, const double *q, const double *r,
                             double *dst);
// dst <- the assignment of every ion (charges, or 1 each without weighted);
// writes every vertex (no global atomics once the ions are in bin order).
hipError_t launch_spread_dense(memd_ctx *c, bool weighted, double *dst, double *dst2 = nullptr);
hipError_t launch_dipole(memd_ctx *c, double *partials, int *nblk);
// zero_irr: also clear the atomic-path count of the current step (which the
// next call's record pack then need not clear)
hipError_t launch_forces(memd_ctx *c, const void *D, const double *dip_partials, int dip_nblk,
                         bool zero_irr = false);
// Row binning of the ions (order, slot, row counts/starts); with
// reorder the ion arrays themselves move into bin order (see sorted).
// zero_irr: the re-binning's scan also clears the count of this step's
// atomic-path ions (the list build that follows it in the step then need not)
hipError_t launch_bin_ions(memd_ctx *c, bool reorder = false, bool zero_irr = false);
hipError_t launch_iota(hipStream_t s, int *dst, int n);
// out[perm[s] * w + k] = in[s * w + k] on the context's stream.
hipError_t launch_unpermute(memd_ctx *c, int w, const double *in, double *out);

// ---- launchers (reductions / finalisers) ----
// Sum `width` doubles per block over nblk partial blocks into dst[width] (fixed order).
hipError_t launch_finalize_sum(hipStream_t s, const double *partials, int nblk, int width,
                               double *dst);
// Audit finaliser: partials hold (max, sumsq) per block -> dst = (max, rms); also appends.
hipError_t launch_finalize_audit(hipStream_t s, const double *partials, int nblk, double Ns,
                                 double *dst, double *hist);
hipError_t launch_finalize_dipole(hipStream_t s, const double *partials, int nblk,
                                  double *P);
// Audit and/or energy from launch_field_obs's partials (4 per block), the
// self-energy partials and (null: P in the scalars) the movers' dipole
// partials; results into the scalars (S_AUDIT, S_ENERGY, S_P) and the
// history slots when given.
hipError_t launch_finalize_obs(memd_ctx *c, const double *fpart, int fblk, const double *ipart, int iblk,
                               const double *dip, int dipn, bool audit, bool energy, double *audit_hist,
                               double *energy_hist);
hipError_t launch_finalize_epsh(hipStream_t s, const double *partials, int nblk, double Ns,
                                double *epsh, double *etamax);
hipError_t launch_greens(memd_ctx *c, double *G);

// tile autotuner with a bound on the rows per thread (the batched kernel holds <= 2)
memd_status autotune_leapfrog(memd_ctx *c, int reps, const char *cache_path, int max_rows, int *rows_out,
                              int *planes_out, double *us_out);

// ---- initial solve (FP64) ----
hipError_t solve_recursion(memd_ctx *c, double *D);
hipError_t solve_mean_shift(memd_ctx *c, double *D);
// uniform or planar permittivity, 4 <= L <= 128: the relaxed field directly
bool planar_solve_ok(const memd_ctx *c);
hipError_t solve_planar(memd_ctx *c, double *D);
memd_status solve_relax(memd_ctx *c, double *D, double tol, int max_iter, int *iters,
                        double *res);


}  // namespace memd
