/*
 * memd.h -- C-ABI of the MI355X (gfx950) MEMD library: the per-timestep
 * lattice update of Maxwell Equations Molecular Dynamics with a spatially
 * varying permittivity (Fahrenberger & Holm, "Computing Coulomb Interaction
 * in Inhomogeneous Dielectric Media via a Local Electrostatics Lattice
 * Algorithm", arXiv:1309.7859).
 *
 * Lattice and fields
 *   L x L x L periodic cubic lattice, spacing a, volume V = (L a)^3, Ns = L^3.
 *   Site v = (i, j, k) sits at a*v; linear index v = i + L*(j + L*k), x fastest.
 *   Links carry D and the permittivity, plaquettes carry B, vertices carry
 *   the interpolated charges (section "Extension of the algorithm", Fig. 2a).
 *   Link (v, d) runs from v to v + e_d; plaquette (v, d) has corner v and
 *   normal d.  Field arrays crossing this boundary are FP64, structure of
 *   arrays, component-major: X[d*Ns + v], d = 0 (x), 1 (y), 2 (z).
 *   Positions are unfolded (never wrapped), xyz interleaved per ion: r[3*i + d].
 *   Units: eps0 = 1; Gauss's law a^2 * sum_d [D_d(v) - D_d(v - e_d)] = q_v.
 *
 * Pointers
 *   Every array argument may point to host memory or to device memory of the
 *   context's GPU; the library tells them apart itself.  Inputs are copied (or,
 *   for device pointers, consumed in stream order) before the call returns
 *   control of host memory: the caller keeps ownership and may reuse a host
 *   buffer at once.  A device input must stay valid until the context's
 *   stream has reached the call.  Outputs go to caller-allocated buffers.
 *
 * Ordering and threads
 *   A context owns one HIP stream (the caller's, or its own when NULL is given)
 *   and enqueues all work there.  memd_step returns once the work is enqueued.
 *   Calls that return results (forces, energy, residual, dipole, state, solve)
 *   wait for the stream.  A context is not thread-safe.
 *
 * Errors
 *   Every call returns a memd_status; no C++ exception crosses this boundary.
 *   After MEMD_EDEVICE the context is poisoned and only memd_destroy is valid.
 */
#ifndef MEMD_H
#define MEMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct memd_ctx memd_ctx;

typedef enum {
    MEMD_OK = 0,
    MEMD_EINVAL = -1,       /* bad argument (NULL pointer, L < 2, a <= 0, ...) */
    MEMD_ENOMEM = -2,       /* device allocation failed */
    MEMD_ENONNEUTRAL = -3,  /* |sum q| > 1e-12 sum |q|: no periodic solution of Gauss's law */
    MEMD_EUNSTABLE = -4,    /* Courant number c dt sqrt(3) / (a sqrt(eps_min)) >= 1 */
    MEMD_ESTATE = -5,       /* call out of order (e.g. step before the initial solve) */
    MEMD_ENOCONV = -6,      /* the relaxation did not reach the tolerance */
    MEMD_EDEVICE = -7,      /* a HIP call failed; the context is poisoned */
    MEMD_ESIZE = -8         /* input larger than the fixed scratch area of an allocation-free call */
} memd_status;

typedef enum {
    MEMD_FP64 = 0,        /* D, B, eta stored and propagated in FP64 */
    MEMD_FP32_MIXED = 1   /* D, B, eta in FP32; initial solve, dipole, energies and the
                             Gauss audit in FP64 */
} memd_precision;

typedef enum {
    MEMD_SELF_GREEN = 0,  /* lattice Green's-function self force, eps of the cell = harmonic mean of its
                             12 edges (the default) */
    MEMD_SELF_DIRECT = 1  /* direct subtraction of the self field on each of the cell's links */
} memd_self_scheme;

typedef enum {
    MEMD_EPS_UNIFORM = 0, /* eps[0]: one value everywhere */
    MEMD_EPS_SITE = 1,    /* eps[Ns]: one value per lattice site, mapped to links */
    MEMD_EPS_LINK = 2,    /* eps[3*Ns]: one value per link, component-major */
    MEMD_EPS_ZSITE = 3    /* eps[L]: site value per z plane (a planar profile), mapped to links */
} memd_eps_mode;

typedef struct {
    int L;              /* lattice points per side, >= 2 */
    double a;           /* lattice spacing, > 0 */
    double dt;          /* time step, > 0 */
    double c;           /* artificial speed of light, c^2 = 1/f_mass; <= 0: set at the first
                           memd_set_permittivity for a Courant number of 1/4 */
    int precision;      /* memd_precision */
    int audit_every;    /* Gauss audit every this many steps inside memd_step (0 = never) */
    int energy_every;   /* energy evaluation every this many steps inside memd_step (0 = never) */
} memd_params;

typedef struct {
    double W_E;          /* 1/2 a^3 sum_links D^2 / eps */
    double W_B;          /* (c^2/2) a^3 sum_plaquettes B^{n+1/2} B^{n+3/2} (leapfrog shadow form) */
    double U_self;       /* sum_i q_i^2 S(f_i) / (2 eps_cell a): lattice self energy */
    double U_dip;        /* sum_d P_d^2 / (2 V eps_h_d): uniform-mode energy removed by the
                            dipole correction */
    double E_corrected;  /* W_E + W_B - U_self - U_dip */
} memd_energy_t;

/* Create a context: lattice, ions and the device buffers.
 * Section "Extension of the algorithm" (the method's two parts: an initial
 * solution of Gauss's law, then its propagation).  q[n] charges, r0[3n]
 * unfolded positions.  hip_stream: a hipStream_t, or NULL for a stream of the
 * library's own.  The permittivity starts uniform, eps = 1.
 * Errors: EINVAL (bad params or pointers, n < 0, a position not finite or
 * beyond 2^40 L a in magnitude), ENONNEUTRAL, ENOMEM, EDEVICE. */
memd_status memd_init_lattice(memd_ctx **out, const memd_params *p, int n_ions,
                              const double *q, const double *r0, void *hip_stream);

/* Map a permittivity onto the links (section "Extension of the algorithm",
 * Fig. 2b and eq. dielectric-interpolation): for SITE and ZSITE modes the
 * link takes the mean of its two site values, or, where their ratio exceeds
 * interface_ratio (<= 0 selects 4), the harmonic combination
 * 1/eps = 1/(2 eps1) + 1/(2 eps2) of an interface link.  Also forms the
 * directional harmonic means used by the dipole correction.  Allowed during a
 * run: D and B are kept.  eps values must be > 0.
 * Errors: EINVAL (mode, NULL, eps <= 0), EUNSTABLE (Courant number >= 1), EDEVICE. */
memd_status memd_set_permittivity(memd_ctx *ctx, int mode, const double *eps,
                                  double interface_ratio);

/* Salt-dependent permittivity per link (the introduction: the permittivity
 * of water falls with the salt concentration): eps = eps_w - slope * c with c
 * the linear-interpolated ion count per a^3, averaged over the periodic
 * 3 x 3 x 3 vertex box and over the two ends of each link; floored at
 * eps_floor.  Evaluated now and, when every > 0, again inside memd_step
 * before every step whose index is a multiple of `every`.
 * Errors: EINVAL (eps_w <= 0, eps_floor <= 0, every < 0), EUNSTABLE, EDEVICE. */
memd_status memd_set_salt_permittivity(memd_ctx *ctx, double eps_w, double slope,
                                       double eps_floor, int every);

/* Initial solution of Gauss's law (Fig. 1: plane -> line -> vertex recursion),
 * the uniform mode set to -P/V (section "Periodicity"), then relaxation to
 * curl E = 0 by minimising the field energy (the paragraph after the
 * recursion), all in FP64 on the GPU; B is set to 0.  Stops when
 * a max|C(eta D)| <= tol max|eta D| (tol <= 0 selects 1e-13).
 * iters_out and curl_residual_out may be NULL.
 * Errors: ENOCONV (not converged within max_iter; the best D is kept), EDEVICE. */
memd_status memd_initial_gauss_solve(memd_ctx *ctx, double tol, int max_iter,
                                     int *iters_out, double *curl_residual_out);

/* Advance nsteps time steps with prescribed displacements disp[nsteps*n*3]
 * (step-major, then ion, then xyz).  Each step (eqs. faraday/ampere with
 * E = D/eps, eq. constraint): B -= dt C(eta D); D += dt c^2 C^T B; the ions
 * move by their displacement, axis by axis, depositing their currents on the
 * links so that Gauss's law holds exactly; then the dipole moment of the
 * unfolded positions and the corrected forces (eq. force without v x B,
 * self-energy and dipole corrections) are formed on the device.  Audit and
 * energy run at their configured cadence.  Asynchronous.
 * Errors: ESTATE (no initial solve or state yet), EINVAL, EDEVICE. */
memd_status memd_step(memd_ctx *ctx, const double *disp, int nsteps);

/* Same step as memd_step, with the displacements drawn on the device from the
 * counter-based stream of `seed` (Philox4x32-10 of Salmon et al. 2011; ion i,
 * step t = steps done since the initial solve, counters (i, t, 0, 0) and
 * (i, t, 1, 0), key = the two 32-bit halves of seed, 53-bit uniforms,
 * Box-Muller), times sigma.  memd_seeded_displacements returns the same
 * numbers for one step into out[3n] (host or device memory).
 * Errors: ESTATE, EINVAL (sigma < 0), EDEVICE. */
memd_status memd_step_seeded(memd_ctx *ctx, uint64_t seed, double sigma, int nsteps);

/* The ions' own dynamics: nsteps steps in which the ions obey Newton's
 * equation with the force memd_forces returns (the kinetic term of the
 * Lagrangian in section "Extension of the algorithm" and eq. force, without
 * the magnetic v x B part, as the paper's implementation omits it), by
 * velocity Verlet: a half kick v += (dt/2) F/m with the forces of the current
 * state, the memd_step step whose move is dt v (the move is the current the
 * step deposits), a second half kick with the forces of the new state.  The
 * conserved quantity is the kinetic energy plus E_corrected of memd_energy.
 * v[3n] (in/out, the ions' velocities, AoS, the caller's order) and mass[n]
 * (in, > 0) may be host or device memory; host velocities are copied back
 * before the call returns (device ones are updated in stream order).  The
 * forces of the current state are recomputed at the start of the call, so
 * the permittivity may have changed since the last step; with a salt
 * permittivity, a step's first half kick uses the forces from before that
 * step's permittivity update.  Audit and energy histories run at their
 * cadence.  The library keeps 7n doubles of device memory for this call until
 * the context is destroyed.
 * Errors: ESTATE, EINVAL (null v or mass with ions, a host mass <= 0 or not
 * finite), ENOMEM, EDEVICE. */
memd_status memd_md_step(memd_ctx *ctx, double *v, const double *mass, int nsteps);
memd_status memd_seeded_displacements(uint64_t seed, int step, int n, double sigma, double *out);

/* Forces on the ions at the current state: eq. force (the electric part
 * q_i E with E = D/eps; the magnetic v x B part is omitted, as the paper's
 * own implementation omits it), with E interpolated from the 4 links of each
 * axis of the ion's cell by the transverse linear weights (the partner of the
 * current assignment of the same cell), minus the lattice self force of
 * eq. greens (section "Self energy interaction": U = q^2 S(f)/(2 eps_cell a),
 * eps_cell the harmonic mean of the cell's 12 edges), plus the dipole term
 * q_i P_d/(V eps_h_d) of section "Periodicity".  F_out[3n] (host or device
 * memory, FP64, AoS xyz, the caller's ion order) is owned by the caller.
 * Waits for the context's stream.
 * Errors: EINVAL (F_out NULL with ions), EDEVICE. */
memd_status memd_forces(memd_ctx *ctx, double *F_out);

/* Energies of the current state, accumulated in FP64 on the device: the
 * field terms of eq. lagrangian, W_E = (1/2) a^3 sum_links D^2/eps (the
 * weight of eq. finalpartitionfunction) and the magnetic term in the
 * leapfrog's shadow form (c^2/2) a^3 sum B^{n+1/2} B^{n+3/2} (the later factor
 * made transiently, the state left unchanged), the lattice self energy
 * U_self of section "Self energy interaction", the uniform-mode energy U_dip
 * removed by the dipole correction of section "Periodicity", and
 * E_corrected = W_E + W_B - U_self - U_dip.  *out is owned by the caller.
 * Waits for the context's stream.
 * Errors: EINVAL (out NULL), EDEVICE. */
memd_status memd_energy(memd_ctx *ctx, memd_energy_t *out);

/* Gauss audit of the current state: Gauss's law as the recursion of Fig. 1
 * establishes it and every later update keeps it (section "Extension of the
 * algorithm", eq. constraint), R_v = a^2 sum_d [D_d(v) - D_d(v - e_d)] - q_v
 * with q_v the linear assignment of the ions' charges to the vertices;
 * returns max_v |R_v| and the rms over the Ns vertices, computed in FP64 on
 * the device (in FP32 mode from the stored FP32 values).  Either output may
 * be NULL.  Waits for the context's stream.
 * Errors: EDEVICE. */
memd_status memd_gauss_residual(memd_ctx *ctx, double *max_abs, double *rms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the audit of
 * memd_gauss_residual on caller-owned buffers, without a context and without
 * any allocation.  D[3 L^3] (FP64 for MEMD_FP64, FP32 for MEMD_FP32_MIXED,
 * component-major), q[n] and r[3n] (FP64, unfolded, AoS xyz) must be device
 * memory of the current device; out[2] receives (max_v |R_v|, rms) and may be
 * device memory (written in stream order, the call does not wait: usable
 * under graph capture) or host memory (the call waits for the stream).  Work
 * runs on hip_stream (NULL: the null stream).  The charge assignment and the
 * partial sums live in one fixed device array of 16.1 MiB per GPU (held from
 * the first call on that GPU until the process ends), which limits L to 128.
 * Every call on a GPU shares that array: calls that overlap on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller.
 * Errors: EINVAL (L < 2, a <= 0, n < 0, NULL or non-device pointers, bad
 * precision), ESIZE (L > 128), EDEVICE. */
memd_status memd_gauss_residual_noalloc(int L, double a, int n, const double *q, const double *r,
                                        const void *D, int precision, double *out, void *hip_stream);

/* Dipole moment of the unfolded positions, P = sum_i q_i r_i (FP64). */
memd_status memd_dipole(memd_ctx *ctx, double P[3]);

/* Results of the audits and energy evaluations run inside memd_step since the
 * last call (oldest first).  audit: 2 doubles per entry (max, rms); energy: 5
 * doubles per entry (memd_energy_t order).  *count receives the number of
 * entries available (capped at max_entries when copying).  Either buffer may
 * be NULL to query the count. */
memd_status memd_history(memd_ctx *ctx, double *audit, double *energy, int max_entries,
                         int *audit_count, int *energy_count);

/* Copy the state out / in: D[3*Ns], B[3*Ns] (B at the last half step), r[3n].
 * memd_set_state also marks the context ready to step (it replaces the
 * initial solve).  Any of the three may be NULL to skip it.  memd_set_state
 * returns EINVAL, changing nothing, when a position is not finite or beyond
 * 2^40 L a in magnitude. */
memd_status memd_get_state(memd_ctx *ctx, double *D, double *B, double *r);
memd_status memd_set_state(memd_ctx *ctx, const double *D, const double *B, const double *r);

/* Introspection: the context's stream (hipStream_t), the speed of light in use,
 * and the directional harmonic-mean permittivities eps_h[3]. */
memd_status memd_get_stream(memd_ctx *ctx, void **stream);
memd_status memd_get_params(memd_ctx *ctx, double *c, double eps_h[3], double *eps_min);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * launches of the kernel families (0 leapfrog, 1 deposit, 2 forces, 3 audit,
 * 4 energy, 5 dipole, 6 salt).  mask is a bit mask (1 << family) of the
 * families to time, -1 all of them, 0 stops timing; every >= 1 times one
 * launch in `every` of each family (the other families use marker events,
 * which cost several microseconds each).  The leapfrog family is timed in
 * runs: consecutive steps that are one fused launch and nothing else are
 * bracketed by one marker pair per run, and every launch of the run counts;
 * a leapfrog launch outside such runs gets events riding on its own launch,
 * the last of each `every` such launches, never the first launch of a call.
 * Each call starts a fresh collection.  memd_profile_read waits for the stream and returns the
 * total milliseconds and the number of timed launches of one family. */
memd_status memd_profile_enable(memd_ctx *ctx, int mask, int every);
memd_status memd_profile_read(memd_ctx *ctx, int family, double *total_ms, long *launches);

/* Tile configuration of the leapfrog kernel: rows per thread (1, 2 or 4: a
 * tile of 64 x 4*rows sites per plane) and planes per z-chunk (>= 1).
 * 0 keeps the current value. */
memd_status memd_set_tiling(memd_ctx *ctx, int rows_per_thread, int planes_per_chunk);

/* Options of the step.  fuse_deposit = 1 (default): on lattices of 16 or
 * more sites per side the current deposit of ions that move less than a per
 * axis (and stay within one row of where they were last binned) runs inside
 * the leapfrog kernel, each tile adding the contributions to the links it
 * owns; the other ions, and every ion when fuse_deposit = 0, deposit with
 * global atomics.  sort_every: steps between re-binnings of the ions by
 * lattice row (default 64; 0 = never after the first).  Both forms give the
 * same result up to the order of floating-point additions. */
memd_status memd_set_options(memd_ctx *ctx, int fuse_deposit, int sort_every);
/* Whether memd_step ends with the forces of the final state (on = 1, the
 * default).  With the fused deposit every step computes the forces of the
 * state it starts from inside the step (eq. force: the tiles gather the
 * lattice part and the self force of the ions whose start cell they own
 * while they hold E in LDS; the movers of the next step's launch add the
 * dipole term, or, with the direct self subtraction, a finisher after the
 * leapfrog computes them), and one more force launch after the last step
 * gives the final state's.  With on = 0 that launch is skipped, and
 * memd_forces returns the newest forces a step completed: those of the
 * state two steps before the end (calls of three steps or more; one step
 * before with the direct subtraction; on the plain path, which computes each
 * new state's forces in its step, those of the final state).  This exposes
 * the in-step force computation to checks.  Errors: EINVAL (on not 0 or 1). */
memd_status memd_set_final_forces(memd_ctx *ctx, int on);
/* The dipole correction of section "Periodicity" (on = 1, the default): the
 * uniform mode of D, which follows -P/V with P the dipole moment of the
 * unfolded positions, exerts -q_i P/(V eps_h) on each ion and holds P in a
 * harmonic well, the behaviour of a periodic system with eps = 0 at
 * infinity; the correction adds q_i P_d/(V eps_h_d) to every force (and
 * subtracts U_dip from E_corrected), the metallic boundary at infinity under
 * which P performs a free random walk.  on = 0 runs the plain lattice
 * algorithm: no dipole term in the forces, U_dip reported as 0.  The forces
 * of the current state are recomputed.  Waits for the context's stream.
 * Errors: EINVAL (on not 0 or 1), EDEVICE. */
memd_status memd_set_dipole_correction(memd_ctx *ctx, int on);

/* Self-energy treatment of the forces (section "Self energy interaction").
 * MEMD_SELF_GREEN (default): the lattice Green's-function scheme (eq. greens;
 * phi = q G/(a eps) with one eps per cell, the harmonic mean of its 12
 * edges): F_self = -grad of U_self = q^2 S(f)/(2 eps_cell a).
 * MEMD_SELF_DIRECT: the direct subtraction (eq. direct-subtraction, whose
 * printed form is garbled; reading): the ion's own linearly assigned charges
 * produce on each link of its cell the displacement field of a homogeneous
 * lattice (from the same Green's function, independent of eps), that field
 * divided by the link's own permittivity is interpolated to the ion like the
 * lattice field, and the result is subtracted.  It equals the Green's-function
 * self force wherever the cell's 12 edges share one permittivity, and
 * differs where the permittivity changes inside the cell.  It is not the
 * gradient of a potential there, so the energy keeps the Green's-function
 * U_self.  With the direct scheme every force is gathered after the step (the
 * leapfrog's own force pass uses the Green's function).  The forces of the
 * current state are recomputed.  Waits for the context's stream.
 * Errors: EINVAL (unknown scheme), EDEVICE. */
memd_status memd_set_self_scheme(memd_ctx *ctx, int scheme);

/* bad_moves: displacement components rejected so far (not finite, or longer
 * than (L + 1024) a; they are taken as 0).  fused_path: 1 if the next
 * step runs the fused deposit.  Either may be NULL. */
memd_status memd_counters(memd_ctx *ctx, unsigned long *bad_moves, int *fused_path);

/* Tile-shape autotuner of the leapfrog kernel: times every candidate shape
 * (reps launches each, HIP events) on the context's buffers without changing
 * its state, keeps the fastest, and appends it to the text cache at
 * cache_path (NULL: no cache).  A cache entry for the same lattice size,
 * precision and permittivity representation is used without measuring.
 * Outputs may be NULL. */
memd_status memd_autotune(memd_ctx *ctx, int reps, const char *cache_path, int *rows_out,
                          int *planes_out, double *us_out);

void memd_destroy(memd_ctx *ctx);
const char *memd_strerror(memd_status status);
int memd_version(void);

/* ------------------------------------------------------------------ serving
 * Continuous batching of independent replicas (FP32 fields; each replica is a
 * full MEMD system of its own: lattice size, ions, planar or uniform
 * permittivity, step count, displacement stream).  Requests queue on submit;
 * memd_server_progress admits queued requests while the device-memory budget
 * (resident buffers plus the FP64 solver's work vectors) and the slot count
 * allow, initialises them on worker threads (own streams: context,
 * permittivity, FP64 initial solve to solve_tol), joins initialised replicas
 * to the device-resident replica table, replays the captured step graph
 * `global_steps` times (every resident replica advances one step per replay:
 * two launches, the batched leapfrog and the batched deposit), and retires
 * finished replicas (forces, energies and Gauss residual of the final state
 * kept for memd_server_poll; device memory returned).  Times are seconds since
 * memd_server_create.  memd_server_create tunes the batched leapfrog's tile
 * depth on a synthetic batch of up to 16 lattices of 64^3 sites (about 200 MB
 * for a moment, fewer lattices under a smaller budget), or reads it from the
 * cache file tune_cache.  Not thread-safe: one caller drives a server. */
typedef struct memd_server memd_server;

typedef enum {
    MEMD_REQ_PENDING = 0, MEMD_REQ_INIT = 1, MEMD_REQ_READY = 2, MEMD_REQ_ACTIVE = 3,
    MEMD_REQ_DONE = 4, MEMD_REQ_FAILED = 5
} memd_request_state;

memd_status memd_server_create(memd_server **out, size_t hbm_budget_bytes, int max_slots,
                               int init_workers, double solve_tol, const char *tune_cache,
                               void *hip_stream);
/* eps_mode: MEMD_EPS_UNIFORM (eps[1]) or MEMD_EPS_ZSITE (eps[L]).  Inputs are
 * copied (host memory).  A request larger than the whole budget fails at once
 * (state FAILED, ENOMEM). */
memd_status memd_server_submit(memd_server *srv, const memd_params *p, int n, const double *q,
                               const double *r0, int eps_mode, const double *eps, int nsteps,
                               uint64_t seed, double sigma, uint64_t *req_id);
memd_status memd_server_progress(memd_server *srv, int global_steps, int *active, int *queued,
                                 int *finished);
/* state: memd_request_state.  F_out[3n], E_out and gauss_max are filled once
 * DONE; a FAILED request returns its error code. */
memd_status memd_server_poll(memd_server *srv, uint64_t req_id, int *state, double *F_out,
                             memd_energy_t *E_out, double *gauss_max, double *t_arrival,
                             double *t_done);
memd_status memd_server_stats(memd_server *srv, long *global_steps, long *replica_steps,
                              size_t *bytes_in_use);
memd_status memd_server_destroy(memd_server *srv);
/* Text of the last device error a server call returned (empty if none). */
const char *memd_server_last_error(memd_server *srv);

#ifdef __cplusplus
}
#endif
#endif
