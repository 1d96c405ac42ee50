// memd_api.hip -- the C-ABI of libmemd: context life cycle, argument checks,
// buffer ownership, stream ordering and the per-step launch sequence.  Every
// computation runs in the kernels of kernels_*.hip; this file only moves
// inputs and outputs and enqueues launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "leapfrog_tile.hpp"
#include "memd_internal.hpp"
#include "serve_internal.hpp"

using namespace memd;

namespace {

constexpr int kHistCap = 4096;

// Positions enter finite and within 2^40 box lengths of the origin; every
// accepted displacement component is at most one box length, so a cell index
// floor(u / a) stays below 2^51 L (where the device's fold is exact) for
// 2^50 steps.  r may be host or device memory.
constexpr double kPosBoxes = 1099511627776.0;  // 2^40

bool positions_ok(const double *r, size_t n, int L, double a) {
    if (n == 0) return true;
    std::vector<double> h(3 * n);
    if (hipMemcpy(h.data(), r, 3 * n * sizeof(double), hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const double lim = kPosBoxes * (double)L * a;
    for (double x : h)
        if (!(std::fabs(x) <= lim)) return false;
    return true;
}

#define CK(expr)                                  \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) {                   \
            c->poisoned = true;                   \
            return MEMD_EDEVICE;                  \
        }                                         \
    } while (0)

#define CHECK_CTX(c)                              \
    do {                                          \
        if (!(c)) return MEMD_EINVAL;             \
        if ((c)->poisoned) return MEMD_EDEVICE;   \
        if (hipSetDevice((c)->device) != hipSuccess) return MEMD_EDEVICE; \
    } while (0)

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice;
}

// Copy bytes from a host or device pointer into device memory, in stream
// order, and wait so that the caller may reuse a host buffer at once.
hipError_t copy_in(memd_ctx *c, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

hipError_t copy_out(memd_ctx *c, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return hipStreamSynchronize(c->stream);
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

hipError_t ensure_stage(memd_ctx *c, size_t bytes) {
    if (c->stage_bytes >= bytes) return hipSuccess;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    if (c->stage) hipFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    e = hipMalloc((void **)&c->stage, bytes);
    if (e != hipSuccess) return e;
    c->stage_bytes = bytes;
    return hipSuccess;
}

// Whether this launch of family fam is one of the timed ones.
constexpr int kProfPoolPairs = 64;  // event pairs made per family when profiling is enabled

static bool prof_take(memd_ctx *c, int fam) {
    if (!c->prof_on || !(c->prof_mask & (1u << fam))) return false;
    // the leapfrog's sampled launches (beside cadence work, where the host's
    // event recording can leave the GPU idle) are the last of each group of
    // `every`; other families take the first
    const long k = c->prof[fam].seen++ % c->prof_every;
    return k == (fam == F_LEAPFROG ? c->prof_every - 1 : 0);
}

// An event for a sample: from the pool made when profiling was enabled (so
// that a sampled launch costs the host no event creation), else a new one.
static hipError_t prof_event(memd_ctx *c, int fam, hipEvent_t *e) {
    auto &pool = c->prof[fam].pool;
    if (!pool.empty()) {
        *e = pool.back();
        pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// A marker event opening a timed interval of family fam on the stream.
static void prof_open(memd_ctx *c, int fam) {
    auto &P = c->prof[fam];
    hipEvent_t e;
    if (prof_event(c, fam, &e) == hipSuccess) {
        if (hipEventRecord(e, c->stream) == hipSuccess) {
            P.start.push_back(e);
            P.count.push_back(0);
            P.open = true;
        } else {
            hipEventDestroy(e);
        }
    }
}

void prof_begin(memd_ctx *c, int fam) {
    auto &P = c->prof[fam];
    P.open = false;
    if (!prof_take(c, fam)) return;
    prof_open(c, fam);
    if (P.open) P.count.back() = 1;
}

void prof_end(memd_ctx *c, int fam) {
    auto &P = c->prof[fam];
    if (!P.open) return;
    P.open = false;
    hipEvent_t e = nullptr;
    if (prof_event(c, fam, &e) == hipSuccess && hipEventRecord(e, c->stream) == hipSuccess) {
        P.stop.push_back(e);
    } else {
        if (e) hipEventDestroy(e);
        hipEventDestroy(P.start.back());
        P.start.pop_back();
        P.count.pop_back();
    }
}

// Runs of leapfrog launches with no other launch between them (steps that
// do nothing but the one fused launch) are timed whole: a marker before the
// first launch of the run and one after its last, so that the interval holds
// those launches back to back and nothing else.  Only the launches of such
// runs are counted.
static void prof_run_enter(memd_ctx *c) {
    if (!c->prof_on || !(c->prof_mask & (1u << F_LEAPFROG))) return;
    if (!c->prof[F_LEAPFROG].open) prof_open(c, F_LEAPFROG);
    if (c->prof[F_LEAPFROG].open) ++c->prof[F_LEAPFROG].count.back();
}

static void prof_run_close(memd_ctx *c) {
    if (c->prof[F_LEAPFROG].open) prof_end(c, F_LEAPFROG);
}

// A start/stop event pair attached to one launch (hipExtLaunchKernelGGL
// records them at the kernel's own start and end, with no marker packets).
void prof_pair(memd_ctx *c, int fam, hipEvent_t *e0, hipEvent_t *e1) {
    *e0 = *e1 = nullptr;
    if (!prof_take(c, fam)) return;
    if (prof_event(c, fam, e0) != hipSuccess) return;
    if (prof_event(c, fam, e1) != hipSuccess) {
        hipEventDestroy(*e0);
        *e0 = nullptr;
        return;
    }
    c->prof[fam].start.push_back(*e0);
    c->prof[fam].stop.push_back(*e1);
    c->prof[fam].count.push_back(1);
}

void prof_clear(memd_ctx *c) {
    for (int f = 0; f < F_NFAM; ++f) {
        for (auto e : c->prof[f].start) hipEventDestroy(e);
        for (auto e : c->prof[f].stop) hipEventDestroy(e);
        for (auto e : c->prof[f].pool) hipEventDestroy(e);
        c->prof[f].start.clear();
        c->prof[f].stop.clear();
        c->prof[f].count.clear();
        c->prof[f].pool.clear();
        c->prof[f].seen = 0;
        c->prof[f].open = false;
    }
}

double courant(const memd_ctx *c) {
    return c->c * c->dt * std::sqrt(3.0) / (c->a * std::sqrt(c->eps_min));
}

// Reduction scratch: the solver's partials (<= 8 per block of kRedBlocks),
// site-loop partials (<= 4 per block of kSiteBlocks), the deposit's dipole
// partials (3 per block of 16 ions), the self-energy partials (1 per block
// of 64 ions, from offset kSiteBlocks * 4).
size_t partial_doubles(int n) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t dep = 3 * (nn / 16 + 16);
    const size_t us = (size_t)kSiteBlocks * 4 + nn / 64 + 16;
    size_t m = (size_t)kRedBlocks * 8;
    if (dep > m) m = dep;
    if (us > m) m = us;
    return m + 64;
}

double *ion_partials(memd_ctx *c) { return c->partials + (size_t)kSiteBlocks * 4; }

// Read eps_h and the largest eta back, fix c on first use, check Courant.
memd_status finish_permittivity(memd_ctx *c) {
    double h[4];
    CK(hipMemcpyAsync(h, c->scal + S_EPSH, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CK(hipMemcpyAsync(h + 3, c->scal + S_ETAMAX, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    c->eps_h[0] = h[0];
    c->eps_h[1] = h[1];
    c->eps_h[2] = h[2];
    c->eps_min = 1.0 / h[3];
    if (!c->c_fixed) {
        c->c = 0.25 * (c->a / c->dt) * std::sqrt(c->eps_min / 3.0);
        c->c_fixed = true;
    }
    if (!(courant(c) < 1.0)) return MEMD_EUNSTABLE;
    return MEMD_OK;
}

memd_status refresh_eta(memd_ctx *c) {
    int nb = 0;
    CK(launch_eta_sums(c, c->partials, &nb));
    CK(launch_ecell(c));
    CK(launch_finalize_epsh(c->stream, c->partials, nb, (double)c->Ns, c->scal + S_EPSH, c->scal + S_ETAMAX));
    return finish_permittivity(c);
}

memd_status ensure_eta_link(memd_ctx *c) {
    if (c->eta_link) return MEMD_OK;
    CK(hipMalloc(&c->eta_link, 3 * c->Ns * c->tsize));
    return MEMD_OK;
}

// Energy of the current state into dst (and hist when given).
// The Gauss audit and/or the energies of the current state: the charge
// assignment (for the audit), one pass over the lattice for both, the self
// energies (for the energy), one finaliser; results in the scalars (S_AUDIT,
// S_ENERGY) and in the history slots when given.  dip (nparts partials):
// the movers' dipole partials of the state, summed into P by the finaliser;
// null: P is in the scalars already.
// cnt (with audit): the same charge-assignment pass also writes the ion
// counts of the salt permittivity there (for a recompute that follows on
// the same positions).
hipError_t enqueue_observables(memd_ctx *c, bool audit, bool energy, double *audit_hist, double *energy_hist,
                               const double *dip = nullptr, int dipn = 0, double *cnt = nullptr) {
    hipError_t e;
    int fb = 0, ib = 0;
    prof_begin(c, audit ? F_AUDIT : F_ENERGY);
    if (audit && (e = launch_spread_dense(c, true, c->rho, cnt)) != hipSuccess) return e;
    if ((e = launch_field_obs(c, audit, energy, c->partials, &fb, ion_partials(c), &ib)) != hipSuccess) return e;
    e = launch_finalize_obs(c, c->partials, fb, ion_partials(c), ib, dip, dipn, audit, energy, audit_hist,
                            energy_hist);
    prof_end(c, audit ? F_AUDIT : F_ENERGY);
    return e;
}

hipError_t enqueue_dipole_forces(memd_ctx *c) {
    hipError_t e;
    int nb = 0;
    prof_begin(c, F_DIPOLE);
    if ((e = launch_dipole(c, c->partials, &nb)) != hipSuccess) return e;
    if ((e = launch_finalize_dipole(c->stream, c->partials, nb, c->scal + S_P)) != hipSuccess) return e;
    prof_end(c, F_DIPOLE);
    prof_begin(c, F_FORCES);
    e = launch_forces(c, c->D[c->cur], nullptr, 0);
    prof_end(c, F_FORCES);
    return e;
}

}  // namespace

namespace memd {

hipError_t refresh_forces(memd_ctx *c) {
    const hipError_t e = hipSetDevice(c->device);
    return e != hipSuccess ? e : enqueue_dipole_forces(c);
}

}  // namespace memd

extern "C" {

int memd_version(void) { return 1; }

const char *memd_strerror(memd_status s) {
    switch (s) {
        case MEMD_OK: return "ok";
        case MEMD_EINVAL: return "invalid argument";
        case MEMD_ENOMEM: return "device allocation failed";
        case MEMD_ENONNEUTRAL: return "charges are not neutral";
        case MEMD_EUNSTABLE: return "Courant number c dt sqrt(3)/(a sqrt(eps_min)) >= 1";
        case MEMD_ESTATE: return "call out of order";
        case MEMD_ENOCONV: return "relaxation did not converge";
        case MEMD_EDEVICE: return "HIP device error";
        case MEMD_ESIZE: return "input larger than the fixed scratch area of an allocation-free call";
    }
    return "unknown status";
}

void memd_destroy(memd_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    if (c->stream) hipStreamSynchronize(c->stream);
    prof_clear(c);
    // the arena holds every fixed buffer; the rest were made on demand
    void *bufs[] = {c->arena, c->eta_link, c->stage, c->salt_cnt, c->md_buf, c->md_cap};
    for (void *b : bufs)
        if (b) hipFree(b);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    delete c;
}

memd_status memd_init_lattice(memd_ctx **out, const memd_params *p, int n, const double *q, const double *r0,
                              void *hip_stream) {
    if (!out || !p) return MEMD_EINVAL;
    *out = nullptr;
    if (p->L < 2 || !(p->a > 0.0) || !(p->dt > 0.0) || n < 0 ||
        (p->precision != MEMD_FP64 && p->precision != MEMD_FP32_MIXED) || p->audit_every < 0 ||
        p->energy_every < 0 || !std::isfinite(p->a) || !std::isfinite(p->dt) || !std::isfinite(p->c))
        return MEMD_EINVAL;
    if (n > 0 && (!q || !r0)) return MEMD_EINVAL;
    const size_t Ns = (size_t)p->L * p->L * p->L;
    if (p->L > 2048) return MEMD_EINVAL;

    memd_ctx *c = new (std::nothrow) memd_ctx();
    if (!c) return MEMD_ENOMEM;
    c->p = *p;
    c->n = n;
    c->prof_every = 1;
    c->irr_zeroed = -1;
    c->L = p->L;
    c->Ns = Ns;
    c->a = p->a;
    c->dt = p->dt;
    c->V = std::pow(p->L * p->a, 3);
    c->fp32 = p->precision == MEMD_FP32_MIXED;
    c->tsize = c->fp32 ? sizeof(float) : sizeof(double);
    c->lf_rows = c->fp32 ? 2 : 1;
    c->lf_tz = 4;
    c->sort_every = 64;
    c->dipole_correction = true;
    c->final_forces = true;
    c->salt_cnt_step = -1;
    c->irr = nullptr;
    c->Ft_alt = nullptr;
    c->fdone_alt = nullptr;
    c->ovf_mark = nullptr;
    c->fold_step = false;
    c->self_scheme = MEMD_SELF_GREEN;
    c->fuse_deposit = true;
    c->hist_cap = kHistCap;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MEMD_EDEVICE;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return MEMD_EDEVICE;
        }
        c->own_stream = true;
    }

    auto fail = [&](memd_status s) {
        memd_destroy(c);
        return s;
    };

    // neutrality (needs the charges on the host)
    std::vector<double> hq((size_t)n);
    if (n > 0) {
        if (hipMemcpy(hq.data(), q, (size_t)n * sizeof(double), hipMemcpyDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MEMD_EINVAL);
        }
        double s = 0.0, sa = 0.0;
        for (double x : hq) {
            if (!std::isfinite(x)) return fail(MEMD_EINVAL);
            s += x;
            sa += std::fabs(x);
        }
        if (std::fabs(s) > 1e-12 * sa) return fail(MEMD_ENONNEUTRAL);
        if (!positions_ok(r0, (size_t)n, p->L, p->a)) return fail(MEMD_EINVAL);
    }

    const size_t fb = 3 * Ns * c->tsize;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t dip_parts = nn / 64 + 32;  // dipole partials: one per mover workgroup of 256 ions (room for 4)
    // Every fixed buffer of the context is carved from one allocation (each
    // piece 256-byte aligned): one hipMalloc here and one hipFree at destroy,
    // which matters to a server creating and destroying contexts while other
    // work runs.  The buffers made later on demand (per-link eta, staging,
    // salt counts, the ion-dynamics buffers) are allocations of their own.
    std::vector<std::pair<void **, size_t>> pieces;
    auto piece = [&](auto **ptr, size_t bytes) { pieces.push_back({(void **)ptr, bytes}); };
    piece(&c->D[0], fb);
    piece(&c->D[1], fb);
    piece(&c->B[0], fb);
    piece(&c->B[1], fb);
    piece(&c->eta_prof, 3 * (size_t)c->L * c->tsize);
    piece(&c->q, nn * sizeof(double));
    piece(&c->r, 3 * nn * sizeof(double));
    piece(&c->F, 3 * nn * sizeof(double));
    piece(&c->order, nn * sizeof(int));
    piece(&c->slot, nn * sizeof(int));
    piece(&c->perm, nn * sizeof(int));
    piece(&c->perm_alt, nn * sizeof(int));
    piece(&c->r_alt, 3 * nn * sizeof(double));
    piece(&c->q_alt, nn * sizeof(double));
    piece(&c->F_alt, 3 * nn * sizeof(double));
    piece(&c->bins, 3 * (size_t)p->L * p->L * sizeof(int));
    piece(&c->dep_atomic, nn * sizeof(int));
    piece(&c->bad_moves, sizeof(unsigned int));
    piece(&c->rho, Ns * sizeof(double));
    piece(&c->drift, nn * sizeof(int));
    piece(&c->partials, partial_doubles(n) * sizeof(double));
    piece(&c->dip[0], 3 * dip_parts * sizeof(double));
    piece(&c->dip[1], 3 * dip_parts * sizeof(double));
    piece(&c->scal, S_COUNT * sizeof(double));
    piece(&c->hist_audit, 2 * (size_t)kHistCap * sizeof(double));
    piece(&c->hist_energy, 5 * (size_t)kHistCap * sizeof(double));
    // Fused deposit: records by slot (two sets), and tile lists sized for the
    // smallest fused tile shape (64 x 4 x 2): twelve entries per ion plus 64
    // per tile.
    c->lists_key = -1;
    c->list_zero_key = -1;
    const size_t rec = 2 * (c->fp32 ? sizeof(DepCell<float>) : sizeof(DepCell<double>));
    const size_t fqb = c->fp32 ? sizeof(IonFQ<float>) : sizeof(IonFQ<double>);
    const bool fused_bufs = n > 0 && p->L >= 16 && p->L <= 1024;
    if (fused_bufs) {
        const size_t L = (size_t)p->L;
        const size_t tiles = ((L + 63) / 64) * ((L + 3) / 4) * ((L + 1) / 2);
        c->list_tiles_max = (int)tiles;
        c->list_entries = 12 * nn + 64 * tiles;
        piece(&c->rec_head, nn * sizeof(int4));
        piece(&c->rec_con, nn * rec);
        piece(&c->list, c->list_entries * sizeof(int));
        piece(&c->list_count, tiles * kCountStride * sizeof(int));
        piece(&c->cbin, nn * sizeof(int));
        piece(&c->list_fail, nn * sizeof(int));
        piece(&c->du_slot, 3 * nn * sizeof(double));
        piece(&c->fq, nn * fqb);
        piece(&c->ecell, Ns * c->tsize);
        piece(&c->Ft, 3 * nn * sizeof(double));
        piece(&c->fdone, nn * sizeof(unsigned int));
        piece(&c->rec_head_nx, nn * sizeof(int4));
        piece(&c->rec_con_nx, nn * rec);
        piece(&c->du_slot_nx, 3 * nn * sizeof(double));
        piece(&c->fq_nx, nn * fqb);
        piece(&c->dep_atomic_nx, nn * sizeof(int));
        piece(&c->irr, 3 * (kIrrHead + nn) * sizeof(int));
        piece(&c->Ft_alt, 3 * nn * sizeof(double));
        piece(&c->fdone_alt, nn * sizeof(unsigned int));
        piece(&c->ovf_mark, nn * sizeof(unsigned int));
    }
    size_t arena_bytes = 0;
    for (const auto &pc : pieces) arena_bytes += (pc.second + 255) / 256 * 256;
    if (hipMalloc(&c->arena, arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        c->arena = nullptr;
        return fail(MEMD_ENOMEM);
    }
    {
        char *at = (char *)c->arena;
        for (const auto &pc : pieces) {
            *pc.first = at;
            at += (pc.second + 255) / 256 * 256;
        }
    }
    if (fused_bufs) {
        c->rec_con1 = (char *)c->rec_con + nn * (rec / 2);
        c->rec_con1_nx = (char *)c->rec_con_nx + nn * (rec / 2);
    }
    hipStream_t s = c->stream;
    if (c->fdone) hipMemsetAsync(c->fdone, 0, nn * sizeof(unsigned int), s);  // no launch is stamped 0
    c->tile_irregular = c->irr != nullptr;
    if (c->irr) hipMemsetAsync(c->irr, 0, 3 * (kIrrHead + nn) * sizeof(int), s);
    if (c->fdone_alt) hipMemsetAsync(c->fdone_alt, 0, nn * sizeof(unsigned int), s);
    if (c->ovf_mark) hipMemsetAsync(c->ovf_mark, 0, nn * sizeof(unsigned int), s);
    for (int b = 0; b < 2; ++b) {
        hipMemsetAsync(c->D[b], 0, fb, s);
        hipMemsetAsync(c->B[b], 0, fb, s);
    }
    hipMemsetAsync(c->rho, 0, Ns * sizeof(double), s);
    hipMemsetAsync(c->bad_moves, 0, sizeof(unsigned int), s);
    hipMemsetAsync(c->bins, 0, (size_t)c->L * c->L * sizeof(int), s);  // bin counts: kept zero between binnings
    hipMemsetAsync(c->scal, 0, S_COUNT * sizeof(double), s);
    if (launch_fill(s, c->scal + S_DIPW, 1.0, 1) != hipSuccess) return fail(MEMD_EDEVICE);
    hipMemsetAsync(c->F, 0, 3 * nn * sizeof(double), s);
    c->sorted = false;
    if (launch_iota(s, c->perm, n) != hipSuccess) return fail(MEMD_EDEVICE);
    if (n > 0) {
        if (copy_in(c, c->q, q, (size_t)n * sizeof(double)) != hipSuccess ||
            copy_in(c, c->r, r0, 3 * (size_t)n * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MEMD_EINVAL);
        }
        if (launch_bin_ions(c) != hipSuccess) return fail(MEMD_EDEVICE);
    }
    // permittivity 1 everywhere until set
    c->eta_mode = ETA_UNIFORM;
    c->eta_uni = 1.0;
    c->eps_min = 1.0;
    c->c = p->c;
    c->c_fixed = p->c > 0.0;
    if (launch_greens(c, c->scal + S_G) != hipSuccess) return fail(MEMD_EDEVICE);
    memd_status st = refresh_eta(c);
    if (st == MEMD_EDEVICE) return fail(st);
    if (!c->c_fixed) c->c = 0.25 * (c->a / c->dt) * std::sqrt(1.0 / 3.0);
    c->c_fixed = p->c > 0.0;  // a default c is chosen again at the first memd_set_permittivity
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MEMD_EDEVICE);
    *out = c;
    return MEMD_OK;
}

memd_status memd_set_permittivity(memd_ctx *c, int mode, const double *eps, double ratio) {
    CHECK_CTX(c);
    if (!eps) return MEMD_EINVAL;
    if (!(ratio > 0.0)) ratio = 4.0;
    size_t count;
    switch (mode) {
        case MEMD_EPS_UNIFORM: count = 1; break;
        case MEMD_EPS_SITE: count = c->Ns; break;
        case MEMD_EPS_LINK: count = 3 * c->Ns; break;
        case MEMD_EPS_ZSITE: count = (size_t)c->L; break;
        default: return MEMD_EINVAL;
    }
    std::vector<double> h(count);
    if (hipMemcpy(h.data(), eps, count * sizeof(double), hipMemcpyDefault) != hipSuccess) {
        (void)hipGetLastError();
        return MEMD_EINVAL;
    }
    for (double x : h)
        if (!(x > 0.0) || !std::isfinite(x)) return MEMD_EINVAL;
    c->salt_every = 0;
    if (mode == MEMD_EPS_UNIFORM) {
        c->eta_mode = ETA_UNIFORM;
        c->eta_uni = 1.0 / h[0];
    } else {
        CK(ensure_stage(c, count * sizeof(double)));
        CK(copy_in(c, c->stage, h.data(), count * sizeof(double)));
        if (mode == MEMD_EPS_ZSITE) {
            CK(launch_eta_zprof(c, c->stage, ratio, c->eta_prof));
            c->eta_mode = ETA_ZPROF;
        } else {
            memd_status st = ensure_eta_link(c);
            if (st != MEMD_OK) return st;
            if (mode == MEMD_EPS_SITE)
                CK(launch_eta_from_site(c, c->stage, ratio, c->eta_link));
            else
                CK(launch_eta_from_link(c, c->stage, c->eta_link));
            c->eta_mode = ETA_LINK;
        }
    }
    return refresh_eta(c);
}

memd_status memd_set_salt_permittivity(memd_ctx *c, double eps_w, double slope, double eps_floor, int every) {
    CHECK_CTX(c);
    if (!(eps_w > 0.0) || !(eps_floor > 0.0) || every < 0 || !std::isfinite(slope)) return MEMD_EINVAL;
    memd_status st = ensure_eta_link(c);
    if (st != MEMD_OK) return st;
    if (!c->salt_cnt) {
        CK(hipMalloc((void **)&c->salt_cnt, c->Ns * sizeof(double)));
    }
    c->salt_w = eps_w;
    c->salt_slope = slope;
    c->salt_floor = eps_floor;
    c->eta_mode = ETA_LINK;
    CK(launch_salt(c));
    st = finish_permittivity(c);
    c->salt_every = every;
    return st;
}

memd_status memd_initial_gauss_solve(memd_ctx *c, double tol, int max_iter, int *iters_out, double *res_out) {
    CHECK_CTX(c);
    if (!(tol > 0.0)) tol = 1e-13;
    if (max_iter <= 0) max_iter = 1000000;
    if (!c->c_fixed) {
        c->c = 0.25 * (c->a / c->dt) * std::sqrt(c->eps_min / 3.0);
        c->c_fixed = true;
    }
    if (!(courant(c) < 1.0)) return MEMD_EUNSTABLE;
    const size_t M = 3 * c->Ns;
    double *Dw = nullptr;
    if (c->fp32) {
        CK(hipMallocAsync((void **)&Dw, M * sizeof(double), c->stream));
    } else {
        Dw = (double *)c->D[c->cur];
    }
    if (planar_solve_ok(c)) {
        // the minimiser itself; the relaxation then only checks it
        CK(solve_planar(c, Dw));
    } else {
        CK(solve_recursion(c, Dw));
        CK(solve_mean_shift(c, Dw));
    }
    memd_status st = solve_relax(c, Dw, tol, max_iter, iters_out, res_out);
    if (st == MEMD_EDEVICE || st == MEMD_ENOMEM) {
        if (st == MEMD_EDEVICE) c->poisoned = true;
        return st;
    }
    if (c->fp32) {
        CK(launch_cast(c->stream, Dw, c->D[c->cur], M, true));
        CK(hipFreeAsync(Dw, c->stream));
    }
    CK(hipMemsetAsync(c->B[c->cur], 0, M * c->tsize, c->stream));
    CK(enqueue_dipole_forces(c));
    CK(hipStreamSynchronize(c->stream));
    c->ready = true;
    c->step_index = 0;
    c->salt_cnt_step = -1;
    return st;
}

}  // extern "C"

namespace {

// The records the movers wrote for the step after the current one become
// the current ones.
void swap_record_sets(memd_ctx *c) {
    std::swap(c->rec_head, c->rec_head_nx);
    std::swap(c->rec_con, c->rec_con_nx);
    std::swap(c->rec_con1, c->rec_con1_nx);
    std::swap(c->du_slot, c->du_slot_nx);
    std::swap(c->fq, c->fq_nx);
    std::swap(c->dep_atomic, c->dep_atomic_nx);
}

// The per-step launch sequence (displacements from disp, or from the Philox
// stream of `seed` when disp is null).
//
// With the fused deposit a step is two kernels: the leapfrog (with the
// tile-owned deposit of the regular ions, and the ion movers, which also
// write the next step's deposit records) and the ion finisher, which
// computes the forces of the state the step started from and deposits the
// irregular ions.  The first step of a call skips those forces
// (the previous call, or the solve or set_state, left them in F), and after
// the last step one force launch gives the forces of the final state, so
// each state's forces are computed once.  Otherwise: leapfrog, the atomic
// deposit, forces.
// One step of the ions' own dynamics hands its end over to the caller:
// recs_ready (in): the caller wrote this step's records (k_md_ions); out:
// whether the forces of the new state were gathered here (the plain path),
// else the movers' dipole partials the caller's gather sums into P.
// pos_ready (in): the caller also wrote where this step's moves end (r_alt)
// and their dipole partials (dip[step_index & 1], pos_nb of them), so the
// leapfrog runs no movers; its first tile sums those partials into P of the
// new state.
struct MdHandoff {
    bool recs_ready;
    bool gathered;
    const double *dip;
    int nb;
    bool pos_ready;
};

memd_status run_steps(memd_ctx *c, const double *dd, int nsteps, uint64_t seed, double sigma,
                      MdHandoff *md = nullptr) {
    const size_t per = 3 * (size_t)c->n;
    // the deposit records of this step were written by the previous step's
    // movers (or, for the ions' own dynamics, by the caller)
    bool recs_ready = md && md->recs_ready;
    const bool md_pos = md && md->pos_ready;
    const double *dip_prev = nullptr;
    int dip_nb = 0;
    bool alone = false;
    for (int t = 0; t < nsteps; ++t) {
        {
            // a step that is its one fused launch and nothing else continues
            // the current timed run of leapfrog launches; any other ends it
            const long nx_i = c->step_index + 1;
            const bool fold0 = fused_deposit_ok(c) && !md && c->tile_irregular && c->self_scheme == MEMD_SELF_GREEN;
            alone = fold0 && recs_ready && c->lists_key == c->lf_rows * 4096 + c->lf_tz &&
                    !(c->salt_every > 0 && c->step_index % c->salt_every == 0) &&
                    !(c->sort_every > 0 && c->step_index % c->sort_every == 0) &&
                    !(c->p.audit_every > 0 && nx_i % c->p.audit_every == 0) &&
                    !(c->p.energy_every > 0 && nx_i % c->p.energy_every == 0);
            if (!alone) prof_run_close(c);
        }
        if (c->salt_every > 0 && c->step_index % c->salt_every == 0) {
            prof_begin(c, F_SALT);
            CK(launch_salt(c));
            prof_end(c, F_SALT);
        }
        const int nx = c->cur ^ 1;
        const long next = c->step_index + 1;
        const bool audit_now = c->p.audit_every > 0 && next % c->p.audit_every == 0;
        const bool energy_now = c->p.energy_every > 0 && next % c->p.energy_every == 0;
        const double *dstep = dd ? dd + per * t : nullptr;
        const uint32_t tstep = (uint32_t)c->step_index;
        int nb = 0;
        if (c->sort_every > 0 && c->step_index % c->sort_every == 0) {
            CK(launch_bin_ions(c, true, true));
            recs_ready = false;
        }
        const bool fused = fused_deposit_ok(c);
        // with the fused deposit, the movers write the next step's records
        // only when it exists in this call and does not re-bin first
        const bool pack_next = fused && t + 1 < nsteps && !(c->sort_every > 0 && next % c->sort_every == 0);
        // One launch per step: the tiles deposit every ion's move and compute
        // every owned ion's lattice and self force, the movers of the next
        // launch add the dipole term (from the third step of a call on: the
        // first launch of a call has no dipole of its start state).  The
        // direct self subtraction and the ions' own dynamics keep their own
        // force paths.
        const bool fold = fused && !md && c->tile_irregular && c->self_scheme == MEMD_SELF_GREEN;
        IonMoves mv{dd && pack_next ? dd + per * (t + 1) : nullptr, seed, tstep + 1u, sigma, pack_next,
                    c->dip[c->step_index & 1], 0, fold && t >= 2};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (alone) {
            prof_run_enter(c);
        } else if (t > 0) {
            // (the first launch of a call is not sampled: the GPU may be idle
            // and its start event taken before the host has issued the kernel)
            prof_pair(c, F_LEAPFROG, &e0, &e1);
        }
        c->fold_step = fold;
        if (md_pos && fused) {
            // the end positions and their partials are ready (or are written
            // by the list build that a re-binning brings on)
            dip_prev = c->dip[c->step_index & 1];
            dip_nb = c->pos_nb;
        }
        c->md_pos = md_pos && fused;
        const hipError_t lf = launch_leapfrog(c, c->D[c->cur], c->B[c->cur], c->D[nx], c->B[nx], e0, e1, dstep,
                                              seed, tstep, sigma, fused, !recs_ready, fused ? dip_prev : nullptr,
                                              dip_nb, fused && !md_pos ? &mv : nullptr, !md);
        c->md_pos = false;
        c->fold_step = false;
        CK(lf);
        if (fused) {
            // (with the tiles depositing the atomic path, only the direct self
            // subtraction's forces need the finisher)
            if (!fold && (!md || !c->tile_irregular)) {
                prof_begin(c, F_DEPOSIT);
                CK(launch_ion_finish(c, c->D[c->cur], c->D[nx], !md));
                prof_end(c, F_DEPOSIT);
            }
            std::swap(c->r, c->r_alt);  // the movers' (or the caller's) positions are now the current ones
            if (pack_next) swap_record_sets(c);
            recs_ready = pack_next;
            if (md_pos) {
                dip_nb = c->pos_nb;  // (dip_prev: the partials of those positions)
            } else {
                dip_prev = mv.dip_out;
                dip_nb = mv.nparts;
            }
            c->cur = nx;
        } else {
            prof_begin(c, F_DEPOSIT);
            CK(launch_deposit(c, c->D[nx], dstep, c->partials, &nb, seed, tstep, sigma));
            prof_end(c, F_DEPOSIT);
            c->cur = nx;
            prof_begin(c, F_FORCES);
            // every force block sums the deposit's per-block q r partials into
            // P (block 0 also stores it)
            CK(launch_forces(c, c->D[c->cur], c->partials, nb));
            prof_end(c, F_FORCES);
            dip_prev = nullptr;
        }
        if (audit_now || energy_now) {
            double *ah = nullptr, *eh = nullptr;
            if (audit_now) {
                const int slot = c->hist_audit_n < c->hist_cap ? c->hist_audit_n : c->hist_cap - 1;
                ah = c->hist_audit + 2 * (size_t)slot;
                if (c->hist_audit_n < c->hist_cap) ++c->hist_audit_n;
            }
            if (energy_now) {
                const int slot = c->hist_energy_n < c->hist_cap ? c->hist_energy_n : c->hist_cap - 1;
                eh = c->hist_energy + 5 * (size_t)slot;
                if (c->hist_energy_n < c->hist_cap) ++c->hist_energy_n;
            }
            // with the fused deposit, P of this state is in the movers' partials;
            // when the next step starts with the salt permittivity, the audit's
            // charge assignment also gives its ion counts (same positions)
            double *cnt = audit_now && c->salt_cnt && c->salt_every > 0 && next % c->salt_every == 0
                              ? c->salt_cnt
                              : nullptr;
            CK(enqueue_observables(c, audit_now, energy_now, ah, eh, energy_now ? dip_prev : nullptr,
                                   energy_now ? dip_nb : 0, cnt));
            c->salt_cnt_step = cnt ? next : -1;
        }
        c->step_index = next;
    }
    prof_run_close(c);
    if (md) {
        md->gathered = dip_prev == nullptr;  // the plain path gathered them after its deposit
        md->dip = dip_prev;
        md->nb = dip_nb;
    } else if (dip_prev && c->final_forces) {
        // forces (and P) of the final state
        prof_begin(c, F_FORCES);
        CK(launch_forces(c, c->D[c->cur], dip_prev, dip_nb, true));
        prof_end(c, F_FORCES);
    }
    return MEMD_OK;
}

}  // namespace

extern "C" {

memd_status memd_step(memd_ctx *c, const double *disp, int nsteps) {
    CHECK_CTX(c);
    if (!c->ready) return MEMD_ESTATE;
    if (nsteps < 0) return MEMD_EINVAL;
    if (nsteps == 0) return MEMD_OK;
    if (c->n > 0 && !disp) return MEMD_EINVAL;
    const size_t per = 3 * (size_t)c->n;
    const double *dd = disp;
    if (c->n > 0 && !is_device_ptr(disp)) {
        CK(ensure_stage(c, per * nsteps * sizeof(double)));
        CK(copy_in(c, c->stage, disp, per * nsteps * sizeof(double)));
        dd = c->stage;
    }
    memd_status st = run_steps(c, c->n > 0 ? dd : nullptr, nsteps, 0, 0.0);
    if (st != MEMD_OK) return st;
    if (dd != disp) CK(hipStreamSynchronize(c->stream));  // the staging buffer is reused
    return MEMD_OK;
}

memd_status memd_step_seeded(memd_ctx *c, uint64_t seed, double sigma, int nsteps) {
    CHECK_CTX(c);
    if (!c->ready) return MEMD_ESTATE;
    if (nsteps < 0 || !(sigma >= 0.0) || !std::isfinite(sigma)) return MEMD_EINVAL;
    return run_steps(c, nullptr, nsteps, seed, sigma);
}

memd_status memd_md_step(memd_ctx *c, double *v, const double *mass, int nsteps) {
    CHECK_CTX(c);
    if (!c->ready) return MEMD_ESTATE;
    if (nsteps < 0) return MEMD_EINVAL;
    if (nsteps == 0) return MEMD_OK;
    if (c->n == 0) return run_steps(c, nullptr, nsteps, 0, 0.0);
    if (!v || !mass) return MEMD_EINVAL;
    const size_t n = (size_t)c->n, per = 3 * n;
    const bool v_dev = is_device_ptr(v), m_dev = is_device_ptr(mass);
    if (!m_dev)
        for (size_t i = 0; i < n; ++i)
            if (!(mass[i] > 0.0) || !std::isfinite(mass[i])) return MEMD_EINVAL;
    if (!c->md_buf) {
        CK(hipStreamSynchronize(c->stream));
        if (hipMalloc((void **)&c->md_buf, (2 * per + n) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            c->md_buf = nullptr;
            return MEMD_ENOMEM;
        }
    }
    double *disp = c->md_buf;
    double *dv = v_dev ? v : c->md_buf + per;
    const double *dm = m_dev ? mass : c->md_buf + 2 * per;
    if (!v_dev) CK(copy_in(c, dv, v, per * sizeof(double)));
    if (!m_dev) CK(copy_in(c, c->md_buf + 2 * per, mass, n * sizeof(double)));
    // With the fused deposit the records of a step are written by the ion
    // kernel that ends the step before (k_md_ions: forces of the new state,
    // the closing half kick of the step and the opening one of the next with
    // the same forces, the next move and its records); the step itself then
    // runs the leapfrog (its tiles compute no forces) and the irregular
    // deposits.  The plain path gathers the forces in the step, and the ion
    // kernel only kicks and writes the move.
    const bool records = fused_deposit_ok(c);
    // with the atomic path on the tiles' list, the ion kernel also writes the
    // positions the next moves end at, and the leapfrog runs no movers
    const bool pos = records && c->tile_irregular;
    if (records && !c->md_cap) {
        // the capture buffers of the fused path: E on the 12 links of each
        // ion's end cell (field type), the incomplete-capture stamps (0 marks
        // none), the end cells
        const size_t eb = (12 * n * c->tsize + 255) / 256 * 256;
        const size_t bytes = eb + 2 * n * sizeof(int);
        CK(hipStreamSynchronize(c->stream));
        if (hipMalloc(&c->md_cap, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->md_cap = nullptr;
            return MEMD_ENOMEM;
        }
        CK(hipMemsetAsync(c->md_cap, 0, bytes, c->stream));
        c->ecap = c->md_cap;
        c->ecap_bad = (unsigned int *)((char *)c->md_cap + eb);
        c->endc = (int *)(c->ecap_bad + n);
    }
    // forces of the current state (the permittivity may have changed since
    // the last ones were computed), the opening half kick, the first move
    CK(enqueue_dipole_forces(c));
    if (records && c->tile_irregular) CK(launch_clear_irregular(c));
    c->irr_zeroed = -1;  // (the ion kernel below appends to that count)
    CK(launch_md_ions(c, c->D[c->cur], nullptr, 0, false, dm, dv, 1, disp, true, records, pos));
    for (int t = 0; t < nsteps; ++t) {
        MdHandoff h{records, false, nullptr, 0, pos};
        const memd_status st = run_steps(c, disp, 1, 0, 0.0, &h);
        if (st != MEMD_OK) return st;
        const bool last = t + 1 == nsteps;
        // The move in caller order (disp) is read by the plain path's deposit
        // and, with records, only by the list build of a re-binning step (the
        // step about to run is c->step_index now; the first step of a call
        // has it from the kernel before the loop, in case its lists are
        // built then).
        const bool rebin_next = c->sort_every > 0 && c->step_index % c->sort_every == 0;
        const bool pack = !last && (!records || rebin_next);
        // (with pos the leapfrog's first tile has summed P of the new state)
        CK(launch_md_ions(c, c->D[c->cur], pos ? nullptr : h.dip, pos ? 0 : h.nb, !h.gathered, dm, dv,
                          last ? 1 : 2, disp, pack, records && !last, pos && !last));
    }
    if (!v_dev) CK(copy_out(c, v, dv, per * sizeof(double)));
    return MEMD_OK;
}

memd_status memd_seeded_displacements(uint64_t seed, int step, int n, double sigma, double *out) {
    if (n < 0 || step < 0 || !(sigma >= 0.0) || (n > 0 && !out)) return MEMD_EINVAL;
    if (n == 0) return MEMD_OK;
    double *d = nullptr;
    if (hipMalloc((void **)&d, 3 * (size_t)n * sizeof(double)) != hipSuccess) return MEMD_ENOMEM;
    memd_status st = MEMD_OK;
    if (launch_philox_disp(nullptr, seed, (uint32_t)step, n, sigma, d) != hipSuccess ||
        hipMemcpy(out, d, 3 * (size_t)n * sizeof(double), hipMemcpyDefault) != hipSuccess)
        st = MEMD_EDEVICE;
    hipFree(d);
    return st;
}

memd_status memd_forces(memd_ctx *c, double *F_out) {
    CHECK_CTX(c);
    if (!F_out && c->n > 0) return MEMD_EINVAL;
    if (!c->ready) return MEMD_ESTATE;
    const size_t bytes = 3 * (size_t)c->n * sizeof(double);
    if (c->sorted) {
        CK(ensure_stage(c, bytes));
        CK(launch_unpermute(c, 3, c->F, c->stage));
        CK(copy_out(c, F_out, c->stage, bytes));
    } else {
        CK(copy_out(c, F_out, c->F, bytes));
    }
    return MEMD_OK;
}

memd_status memd_energy(memd_ctx *c, memd_energy_t *out) {
    CHECK_CTX(c);
    if (!out) return MEMD_EINVAL;
    CK(enqueue_observables(c, false, true, nullptr, nullptr));
    double h[5];
    CK(copy_out(c, h, c->scal + S_ENERGY, 5 * sizeof(double)));
    out->W_E = h[0];
    out->W_B = h[1];
    out->U_self = h[2];
    out->U_dip = h[3];
    out->E_corrected = h[4];
    return MEMD_OK;
}

memd_status memd_gauss_residual(memd_ctx *c, double *max_abs, double *rms) {
    CHECK_CTX(c);
    CK(enqueue_observables(c, true, false, nullptr, nullptr));
    double h[2];
    CK(copy_out(c, h, c->scal + S_AUDIT, 2 * sizeof(double)));
    if (max_abs) *max_abs = h[0];
    if (rms) *rms = h[1];
    return MEMD_OK;
}

memd_status memd_dipole(memd_ctx *c, double P[3]) {
    CHECK_CTX(c);
    if (!P) return MEMD_EINVAL;
    int nb = 0;
    CK(launch_dipole(c, c->partials, &nb));
    CK(launch_finalize_dipole(c->stream, c->partials, nb, c->scal + S_P));
    CK(copy_out(c, P, c->scal + S_P, 3 * sizeof(double)));
    return MEMD_OK;
}

memd_status memd_history(memd_ctx *c, double *audit, double *energy, int max_entries, int *audit_count,
                         int *energy_count) {
    CHECK_CTX(c);
    const int na = c->hist_audit_n, ne = c->hist_energy_n;
    if (audit_count) *audit_count = na;
    if (energy_count) *energy_count = ne;
    if (audit && max_entries > 0) {
        const int k = na < max_entries ? na : max_entries;
        CK(copy_out(c, audit, c->hist_audit, 2 * (size_t)k * sizeof(double)));
    }
    if (energy && max_entries > 0) {
        const int k = ne < max_entries ? ne : max_entries;
        CK(copy_out(c, energy, c->hist_energy, 5 * (size_t)k * sizeof(double)));
    }
    if (audit || energy) {
        c->hist_audit_n = 0;
        c->hist_energy_n = 0;
    }
    return MEMD_OK;
}

memd_status memd_get_state(memd_ctx *c, double *D, double *B, double *r) {
    CHECK_CTX(c);
    const size_t M = 3 * c->Ns;
    if (D || B) CK(ensure_stage(c, M * sizeof(double)));
    if (D) {
        CK(launch_uncast(c->stream, c->D[c->cur], c->stage, M, c->fp32));
        CK(copy_out(c, D, c->stage, M * sizeof(double)));
    }
    if (B) {
        CK(launch_uncast(c->stream, c->B[c->cur], c->stage, M, c->fp32));
        CK(copy_out(c, B, c->stage, M * sizeof(double)));
    }
    if (r) {
        const size_t bytes = 3 * (size_t)c->n * sizeof(double);
        if (c->sorted) {
            CK(ensure_stage(c, bytes));
            CK(launch_unpermute(c, 3, c->r, c->stage));
            CK(copy_out(c, r, c->stage, bytes));
        } else {
            CK(copy_out(c, r, c->r, bytes));
        }
    }
    return MEMD_OK;
}

memd_status memd_set_state(memd_ctx *c, const double *D, const double *B, const double *r) {
    CHECK_CTX(c);
    const size_t M = 3 * c->Ns;
    if (D || B) CK(ensure_stage(c, M * sizeof(double)));
    if (D) {
        CK(copy_in(c, c->stage, D, M * sizeof(double)));
        CK(launch_cast(c->stream, c->stage, c->D[c->cur], M, c->fp32));
    }
    if (B) {
        CK(hipStreamSynchronize(c->stream));
        CK(copy_in(c, c->stage, B, M * sizeof(double)));
        CK(launch_cast(c->stream, c->stage, c->B[c->cur], M, c->fp32));
    }
    if (r && !positions_ok(r, (size_t)c->n, c->L, c->a)) return MEMD_EINVAL;
    if (r) {
        if (c->sorted) {
            // back to the caller's order: q moves, perm becomes the identity
            CK(launch_unpermute(c, 1, c->q, c->q_alt));
            std::swap(c->q, c->q_alt);
            CK(launch_iota(c->stream, c->perm, c->n));
            ++c->perm_version;
            c->sorted = false;
        }
        CK(copy_in(c, c->r, r, 3 * (size_t)c->n * sizeof(double)));
        CK(launch_bin_ions(c));
        c->salt_cnt_step = -1;  // counts of the old positions
    }
    if (!c->c_fixed) {
        c->c = 0.25 * (c->a / c->dt) * std::sqrt(c->eps_min / 3.0);
        c->c_fixed = true;
    }
    CK(enqueue_dipole_forces(c));
    CK(hipStreamSynchronize(c->stream));
    c->ready = true;
    return MEMD_OK;
}

memd_status memd_get_stream(memd_ctx *c, void **stream) {
    CHECK_CTX(c);
    if (!stream) return MEMD_EINVAL;
    *stream = (void *)c->stream;
    return MEMD_OK;
}

memd_status memd_get_params(memd_ctx *c, double *cc, double eps_h[3], double *eps_min) {
    CHECK_CTX(c);
    if (cc) *cc = c->c;
    if (eps_h) {
        double h[3];
        CK(copy_out(c, h, c->scal + S_EPSH, 3 * sizeof(double)));
        eps_h[0] = h[0];
        eps_h[1] = h[1];
        eps_h[2] = h[2];
    }
    if (eps_min) *eps_min = c->eps_min;
    return MEMD_OK;
}

memd_status memd_profile_enable(memd_ctx *c, int mask, int every) {
    CHECK_CTX(c);
    if (every < 1) return MEMD_EINVAL;
    CK(hipStreamSynchronize(c->stream));
    prof_clear(c);
    c->prof_on = mask != 0;
    c->prof_mask = (unsigned)mask;
    c->prof_every = every;
    for (int f = 0; f < F_NFAM; ++f) {
        if (!(c->prof_mask & (1u << f))) continue;
        for (int k = 0; k < 2 * kProfPoolPairs; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                break;
            }
            c->prof[f].pool.push_back(e);
        }
    }
    return MEMD_OK;
}

memd_status memd_profile_read(memd_ctx *c, int family, double *total_ms, long *launches) {
    CHECK_CTX(c);
    if (family < 0 || family >= F_NFAM) return MEMD_EINVAL;
    CK(hipStreamSynchronize(c->stream));
    const auto &P = c->prof[family];
    const size_t m = P.start.size() < P.stop.size() ? P.start.size() : P.stop.size();
    double tot = 0.0;
    long cnt = 0;
    for (size_t t = 0; t < m; ++t) {
        float ms = 0.0f;
        CK(hipEventElapsedTime(&ms, P.start[t], P.stop[t]));
        tot += ms;
        cnt += P.count[t];
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return MEMD_OK;
}

}  // extern "C"

// Tile-shape autotuner of the leapfrog kernel.  Each candidate (rows per
// thread x planes per z-chunk) is launched `reps` times on the context's own
// buffers and timed with HIP events; the leapfrog writes only the inactive
// ping-pong buffers, so the state is untouched.  The winner is kept in the
// context and, when cache_path is given, in a text cache keyed by lattice
// size, precision and permittivity representation.
memd_status memd::autotune_leapfrog(memd_ctx *c, int reps, const char *cache_path, int max_rows, int *rows_out,
                                    int *planes_out, double *us_out) {
    CHECK_CTX(c);
    if (reps <= 0) reps = 10;
    char key[112];
    snprintf(key, sizeof(key), "leapfrog L=%d prec=%d eta=%d rmax=%d", c->L, c->fp32 ? 1 : 0, c->eta_mode,
             max_rows);
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[256];
            int br = 0, bp = 0;
            double bu = 0.0;
            bool hit = false;
            while (fgets(line, sizeof(line), f)) {
                const size_t kl = strlen(key);
                if (strncmp(line, key, kl) == 0 && line[kl] == ' ') {
                    int rr = 0, pp = 0;
                    double uu = 0.0;
                    if (sscanf(line + kl, " rows=%d planes=%d us=%lf", &rr, &pp, &uu) == 3 &&
                        (rr == 1 || rr == 2 || rr == 4) && rr <= max_rows && pp >= 1) {
                        br = rr;
                        bp = pp;
                        bu = uu;
                        hit = true;
                    }
                }
            }
            fclose(f);
            if (hit) {
                c->lf_rows = br;
                c->lf_tz = bp;
                if (rows_out) *rows_out = br;
                if (planes_out) *planes_out = bp;
                if (us_out) *us_out = bu;
                return MEMD_OK;
            }
        }
    }
    const int rows_c[3] = {1, 2, 4};
    const int planes_c[6] = {2, 4, 8, 16, 32, 64};
    // with ions on a lattice of 16 or more, the step runs the leapfrog with the
    // deposit fused in: only its tile shapes are candidates, and it is timed
    // with Philox displacements (sigma = 0.02 a) into the inactive buffer
    const bool want_fused = c->fuse_deposit && c->n > 0 && c->L >= 16;
    const int saved_rows = c->lf_rows, saved_tz = c->lf_tz;
    int best_r = c->lf_rows, best_p = c->lf_tz;
    double best_us = HUGE_VAL;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    const int nx = c->cur ^ 1;
    for (int ri = 0; ri < 3; ++ri)
        for (int pi = 0; pi < 6; ++pi) {
            if (rows_c[ri] > max_rows) continue;
            const int pl = planes_c[pi];
            if (pl > c->L && pi > 0) continue;
            c->lf_rows = rows_c[ri];
            c->lf_tz = pl;
            if (want_fused && !fused_deposit_ok(c)) continue;
            const double sg = want_fused ? 0.02 * c->a : 0.0;
            CK(launch_leapfrog(c, c->D[c->cur], c->B[c->cur], c->D[nx], c->B[nx], nullptr, nullptr, nullptr, 0, 0,
                               sg, want_fused));
            CK(hipEventRecord(e0, c->stream));
            for (int t = 0; t < reps; ++t)
                CK(launch_leapfrog(c, c->D[c->cur], c->B[c->cur], c->D[nx], c->B[nx], nullptr, nullptr, nullptr, 0,
                                   0, sg, want_fused));
            CK(hipEventRecord(e1, c->stream));
            CK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CK(hipEventElapsedTime(&ms, e0, e1));
            const double us = 1e3 * ms / reps;
            if (us < best_us) {
                best_us = us;
                best_r = rows_c[ri];
                best_p = pl;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best_us == HUGE_VAL) {
        best_r = saved_rows;
        best_p = saved_tz;
    }
    c->lf_rows = best_r;
    c->lf_tz = best_p;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s rows=%d planes=%d us=%.3f\n", key, best_r, best_p, best_us);
            fclose(f);
        }
    }
    if (rows_out) *rows_out = best_r;
    if (planes_out) *planes_out = best_p;
    if (us_out) *us_out = best_us;
    return MEMD_OK;
}

extern "C" {

memd_status memd_autotune(memd_ctx *c, int reps, const char *cache_path, int *rows_out, int *planes_out,
                          double *us_out) {
    return autotune_leapfrog(c, reps, cache_path, 4, rows_out, planes_out, us_out);
}

memd_status memd_set_options(memd_ctx *c, int fuse_deposit, int sort_every) {
    CHECK_CTX(c);
    if (fuse_deposit < 0 || fuse_deposit > 1 || sort_every < 0) return MEMD_EINVAL;
    c->fuse_deposit = fuse_deposit != 0;
    c->sort_every = sort_every;
    return MEMD_OK;
}

memd_status memd_set_final_forces(memd_ctx *c, int on) {
    CHECK_CTX(c);
    if (on < 0 || on > 1) return MEMD_EINVAL;
    c->final_forces = on != 0;
    return MEMD_OK;
}

memd_status memd_set_dipole_correction(memd_ctx *c, int on) {
    CHECK_CTX(c);
    if (on < 0 || on > 1) return MEMD_EINVAL;
    c->dipole_correction = on != 0;
    CK(launch_fill(c->stream, c->scal + S_DIPW, on ? 1.0 : 0.0, 1));
    if (c->ready) CK(enqueue_dipole_forces(c));  // the current state's forces under the new setting
    CK(hipStreamSynchronize(c->stream));
    return MEMD_OK;
}

memd_status memd_set_self_scheme(memd_ctx *c, int scheme) {
    CHECK_CTX(c);
    if (scheme != MEMD_SELF_GREEN && scheme != MEMD_SELF_DIRECT) return MEMD_EINVAL;
    c->self_scheme = scheme;
    if (c->ready) CK(enqueue_dipole_forces(c));  // the current state's forces under the new scheme
    CK(hipStreamSynchronize(c->stream));
    return MEMD_OK;
}

memd_status memd_counters(memd_ctx *c, unsigned long *bad_moves, int *fused_path) {
    CHECK_CTX(c);
    unsigned int h = 0;
    CK(copy_out(c, &h, c->bad_moves, sizeof(unsigned int)));
    if (bad_moves) *bad_moves = h;
    if (fused_path) *fused_path = fused_deposit_ok(c) ? 1 : 0;
    return MEMD_OK;
}

memd_status memd_set_tiling(memd_ctx *c, int rows, int planes) {
    CHECK_CTX(c);
    if (rows != 0 && rows != 1 && rows != 2 && rows != 4) return MEMD_EINVAL;
    if (planes < 0) return MEMD_EINVAL;
    if (rows) c->lf_rows = rows;
    if (planes) c->lf_tz = planes;
    return MEMD_OK;
}

}  // extern "C"
