// server.hip -- continuous-batching server of independent MEMD replicas.
//
// Requests (lattice size, ions, permittivity profile, step count, seed of the
// displacement stream) are queued on submit.  Admission is by device-memory
// budget and slot count: an admitted request is initialised by a worker thread
// on a stream of its own (context, permittivity, FP64 initial solve, tile
// autotune), which overlaps with the batched steps of the resident replicas.
// Each global step advances every resident replica by one time step with one
// replay of a captured HIP graph of two launches (batched leapfrog, then the
// batched deposit, which also advances the step counters); the replica table
// the graph reads lives in device memory and is rewritten between replays
// when replicas join or leave.  Finished replicas are retired on a worker
// thread (forces, energy and Gauss audit of the final state computed on the
// replica's own stream and copied out, memory returned) and their slots
// reused.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "memd_internal.hpp"
#include "serve_internal.hpp"

using namespace memd;

namespace {

enum ReqState { Q_PENDING = 0, Q_INIT = 1, Q_READY = 2, Q_ACTIVE = 3, Q_DONE = 4, Q_FAILED = 5 };

struct Request {
    uint64_t id;
    memd_params p;
    int n;
    std::vector<double> q, r0, eps;
    int eps_mode;
    int nsteps;
    uint64_t seed;
    double sigma;
    double t_arrival = 0.0, t_admit = 0.0, t_ready = 0.0, t_done = 0.0;
    int state = Q_PENDING;
    memd_status error = MEMD_OK;
    memd_ctx *ctx = nullptr;
    size_t bytes_resident = 0, bytes_peak = 0;
    int slot = -1;
    std::vector<double> F;
    memd_energy_t E{};
    double gauss = 0.0;
};

size_t resident_bytes(int L, int n) {
    const size_t Ns = (size_t)L * L * L;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t b = 4 * 3 * Ns * sizeof(float)            // D, B ping-pong
               + Ns * sizeof(double)                 // rho
               + 3 * (size_t)L * L * sizeof(int)     // bins
               + nn * (14 * sizeof(double) + 7 * sizeof(int))  // ion arrays and their re-binning targets
               + (2 + 5) * 4096 * sizeof(double)     // histories
               + 3 * (size_t)L * sizeof(float) + (1 << 16)
               + ((size_t)kSiteBlocks * 4 + nn / 16 * 3 + 4096) * sizeof(double);  // reduction scratch
    if (n > 0 && L >= 16 && L <= 1024) {  // the fused deposit (FP32 fields)
        const size_t tiles = (((size_t)L + 63) / 64) * (((size_t)L + 3) / 4) * (((size_t)L + 1) / 2);
        // two record sets: head, both cells' values, displacement, fq, flag
        b += 2 * nn * (16 + 24 * sizeof(float) + 24 + 16 + 4);
        b += (12 * nn + 64 * tiles) * sizeof(int) + tiles * 128;  // tile lists and their counts
        b += nn * (2 * sizeof(int) + 24 + 4);                     // cbin, list_fail, Ft, fdone
        b += nn * (24 + 2 * 4 + 3 * 4) + 3 * 32 * 4;              // Ft_alt, fdone_alt, ovf_mark, atomic-path lists
        b += Ns * sizeof(float);                                  // 12 / sum(eta) per site
    }
    return b;
}

size_t solve_bytes(int L) {
    const size_t Ns = (size_t)L * L * L;
    return (8 * 3 + 3) * Ns * sizeof(double);  // CG work vectors + the FP64 D being solved
}

}  // namespace

struct memd_server {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    size_t budget = 0, used = 0;
    int max_slots = 0;
    int slots_used = 0;       // admitted and not yet retired
    double solve_tol = 1e-8;
    std::string tune_cache;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::deque<Request *> init_queue;   // admitted, waiting for a worker
    std::deque<Request *> retire_queue; // finished, results to be taken out by a worker
    std::deque<Request *> pending;      // waiting for admission
    std::vector<Request *> ready;       // initialised, waiting to join the table
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Request *> active;      // resident replicas (table order)
    uint64_t next_id = 1;

    RepDesc *d_tab = nullptr;
    int *d_hdr = nullptr;
    int *d_steps = nullptr;       // two counters per slot (RepDesc::steps)
    RepDesc *h_tab = nullptr;     // pinned mirrors
    int *h_hdr = nullptr;
    int *h_steps = nullptr;
    std::vector<int> free_slots;
    bool table_dirty = true;

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int lf_grid = 2048, dep_grid = 2048;
    int batch_tz = 8;  // planes per z-chunk of every replica's leapfrog tiles (tune_batch_depth)

    long global_steps = 0, replica_steps = 0, done_count = 0, failed_count = 0;
    char last_error[160] = {0};

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void finish_request(memd_server *s, Request *rq);

void worker_main(memd_server *s) {
    hipSetDevice(s->device);
    for (;;) {
        Request *rq = nullptr;
        bool retiring = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stopping || !s->init_queue.empty() || !s->retire_queue.empty(); });
            if (s->stopping) return;
            // finished replicas first: their memory admits the next requests
            retiring = !s->retire_queue.empty();
            std::deque<Request *> &q = retiring ? s->retire_queue : s->init_queue;
            rq = q.front();
            q.pop_front();
        }
        if (retiring) {
            finish_request(s, rq);
            continue;
        }
        memd_status st = memd_init_lattice(&rq->ctx, &rq->p, rq->n, rq->q.data(), rq->r0.data(), nullptr);
        if (st == MEMD_OK) st = memd_set_permittivity(rq->ctx, rq->eps_mode, rq->eps.data(), 4.0);
        if (st == MEMD_OK) st = memd_initial_gauss_solve(rq->ctx, s->solve_tol, 0, nullptr, nullptr);
        std::lock_guard<std::mutex> lk(s->mu);
        rq->t_ready = s->now();
        if (st == MEMD_OK) {
            rq->state = Q_READY;
            s->ready.push_back(rq);
            s->used -= (rq->bytes_peak - rq->bytes_resident);
        } else {
            rq->state = Q_FAILED;
            rq->error = st;
            rq->t_done = rq->t_ready;
            if (rq->ctx) memd_destroy(rq->ctx);
            rq->ctx = nullptr;
            s->used -= rq->bytes_peak;
            --s->slots_used;
            ++s->failed_count;
        }
    }
}

// Admission: pending requests join the init queue, in arrival order, while
// device memory (peak need: resident buffers plus the solver's work vectors)
// and slots allow.
void admit(memd_server *s) {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->pending.empty()) {
        Request *rq = s->pending.front();
        if (s->slots_used >= s->max_slots) break;
        if (s->used + rq->bytes_peak > s->budget) break;
        s->pending.pop_front();
        s->used += rq->bytes_peak;
        ++s->slots_used;
        rq->state = Q_INIT;
        rq->t_admit = s->now();
        s->init_queue.push_back(rq);
    }
    s->cv.notify_all();
}

void fill_desc(const Request *rq, int slot, int *d_steps, int tz, RepDesc &d) {
    memd_ctx *c = rq->ctx;
    d.L = c->L;
    d.n = c->n;
    d.rows = 1;  // the batched leapfrog holds tiles of one row per thread
    d.tz = std::min(tz, c->L);
    // a lattice narrower than a wavefront: tiles of whole rows, 256 / L of them
    d.xrows = c->L < 64 ? kRowSites / c->L : 0;
    d.ntx = d.xrows > 0 ? 1 : (c->L + 63) / 64;
    d.nty = d.xrows > 0 ? (c->L + d.xrows - 1) / d.xrows : (c->L + 4 * d.rows - 1) / (4 * d.rows);
    d.nzc = (c->L + d.tz - 1) / d.tz;
    d.tiles = d.ntx * d.nty * d.nzc;
    d.dblocks = c->n > 0 ? (c->n + kDepIons - 1) / kDepIons : 1;
    d.eta_mode = c->eta_mode;
    d.nsteps = rq->nsteps;
    d.eta_uni = (float)c->eta_uni;
    d.kB = (float)(c->dt / c->a);
    d.kD = (float)(c->dt * c->c * c->c / c->a);
    d.a = c->a;
    d.V = c->V;
    d.sigma = rq->sigma;
    d.seed = rq->seed;
    d.D[0] = (float *)c->D[0];
    d.D[1] = (float *)c->D[1];
    d.B[0] = (float *)c->B[0];
    d.B[1] = (float *)c->B[1];
    d.eta_prof = (const float *)c->eta_prof;
    d.q = c->q;
    d.r = c->r;
    d.steps = d_steps + 2 * slot;
}

hipError_t upload_table(memd_server *s) {
    int toff = 0, doff = 0;
    for (size_t k = 0; k < s->active.size(); ++k) {
        Request *rq = s->active[k];
        RepDesc &d = s->h_tab[k];
        fill_desc(rq, rq->slot, s->d_steps, s->batch_tz, d);
        d.tile_off = toff;
        d.dep_off = doff;
        s->h_hdr[kHdrInts + RANGE_TILES * s->max_slots + k] = toff;
        s->h_hdr[kHdrInts + RANGE_DEP * s->max_slots + k] = doff;
        toff += d.tiles;
        doff += d.dblocks;
    }
    s->h_hdr[0] = (int)s->active.size();
    s->h_hdr[1] = toff;
    s->h_hdr[2] = s->max_slots;
    s->h_hdr[3] = doff;
    hipError_t e;
    if (!s->active.empty())
        if ((e = hipMemcpyAsync(s->d_tab, s->h_tab, s->active.size() * sizeof(RepDesc), hipMemcpyHostToDevice,
                                s->stream)) != hipSuccess)
            return e;
    if ((e = hipMemcpyAsync(s->d_hdr, s->h_hdr, hdr_ints(s->max_slots) * sizeof(int), hipMemcpyHostToDevice,
                            s->stream)) !=
        hipSuccess)
        return e;
    s->table_dirty = false;
    return hipSuccess;
}

// The step graph reads the replica table from device memory, so it is
// captured once, when the server is created (before any worker runs).
hipError_t capture_graph(memd_server *s) {
    hipError_t e;
    if ((e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    launch_batch_step(s->stream, s->d_tab, s->d_hdr, s->max_slots, s->lf_grid, s->dep_grid);
    if ((e = hipStreamEndCapture(s->stream, &s->graph)) != hipSuccess) return e;
    return hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0);
}

// The tile depth of the batched leapfrog (planes per z-chunk), one for every
// replica, picked by timing the batched kernel itself on a synthetic batch
// that fills the device as a live one does: up to 16 lattices of 64^3 sites
// (4.2M sites, fewer under a small budget), zero fields (the kernel's time
// does not depend on the values), uniform permittivity.  Depths 2..32, ten
// launches each after two untimed ones; the pick is cached in tune_cache.
// Tuning replicas one at a time, alone on the device, favours shallow tiles
// (more of them to fill the device) where the full batch is faster with
// deeper ones, whose z halo costs less.
hipError_t tune_batch_depth(memd_server *s) {
    const char *key = "batch_leapfrog fp32";
    if (!s->tune_cache.empty()) {
        if (FILE *f = fopen(s->tune_cache.c_str(), "r")) {
            char line[256];
            int tz = 0;
            while (fgets(line, sizeof(line), f)) {
                int t = 0;
                if (strncmp(line, key, strlen(key)) == 0 && sscanf(line + strlen(key), " planes=%d", &t) == 1 &&
                    t >= 1)
                    tz = t;
            }
            fclose(f);
            if (tz > 0) {
                s->batch_tz = tz;
                return hipSuccess;
            }
        }
    }
    constexpr int L = 64;
    const size_t Ns = (size_t)L * L * L, per = 12 * Ns * sizeof(float);  // D, B and their next values
    const int M = (int)std::max<size_t>(1, std::min<size_t>(16, s->budget / per));
    float *fields = nullptr;
    RepDesc *d_tab = nullptr;
    int *d_hdr = nullptr, *d_cnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<RepDesc> tab(M);
    std::vector<int> hdr(hdr_ints(M), 0);
    hipError_t e = hipMalloc((void **)&fields, M * per);
    if (e == hipSuccess) e = hipMalloc((void **)&d_tab, M * sizeof(RepDesc));
    if (e == hipSuccess) e = hipMalloc((void **)&d_hdr, hdr.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&d_cnt, 2 * (size_t)M * sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(fields, 0, M * per, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_cnt, 0, 2 * (size_t)M * sizeof(int), s->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best_us = HUGE_VAL;
    for (int tz = 2; tz <= 32 && e == hipSuccess; tz *= 2) {
        int toff = 0;
        for (int k = 0; k < M; ++k) {
            RepDesc &d = tab[k];
            memset(&d, 0, sizeof(d));
            d.L = L;
            d.rows = 1;
            d.xrows = 0;
            d.tz = tz;
            d.ntx = 1;
            d.nty = L / 4;
            d.nzc = L / tz;
            d.tiles = d.ntx * d.nty * d.nzc;
            d.dblocks = 1;
            d.tile_off = toff;
            d.dep_off = k;
            d.eta_mode = ETA_UNIFORM;
            d.nsteps = 1 << 30;
            d.eta_uni = 1.0f;
            d.kB = 0.01f;
            d.kD = 0.01f;
            d.a = 1.0;
            d.V = (double)Ns;
            float *f = fields + 12 * Ns * k;
            d.D[0] = f;
            d.D[1] = f + 3 * Ns;
            d.B[0] = f + 6 * Ns;
            d.B[1] = f + 9 * Ns;
            d.steps = d_cnt + 2 * k;
            hdr[kHdrInts + RANGE_TILES * M + k] = toff;
            hdr[kHdrInts + RANGE_DEP * M + k] = k;
            toff += d.tiles;
        }
        hdr[0] = M;
        hdr[1] = toff;
        hdr[2] = M;
        hdr[3] = M;
        e = hipMemcpyAsync(d_tab, tab.data(), M * sizeof(RepDesc), hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_hdr, hdr.data(), hdr.size() * sizeof(int), hipMemcpyHostToDevice, s->stream);
        for (int t = 0; t < 12 && e == hipSuccess; ++t) {
            if (t == 2) e = hipEventRecord(e0, s->stream);
            if (e == hipSuccess) e = launch_batch_leapfrog(s->stream, d_tab, d_hdr, M, s->lf_grid);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);  // the host copies above are reused next round
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && 100.0 * ms < best_us) {
            best_us = 100.0 * ms;  // us per launch
            s->batch_tz = tz;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(fields);
    hipFree(d_tab);
    hipFree(d_hdr);
    hipFree(d_cnt);
    if (e == hipSuccess && !s->tune_cache.empty())
        if (FILE *f = fopen(s->tune_cache.c_str(), "a")) {
            fprintf(f, "%s planes=%d us=%.3f\n", key, s->batch_tz, best_us);
            fclose(f);
        }
    return e;
}

memd_status fail_dev(memd_server *s, const char *what, hipError_t e) {
    snprintf(s->last_error, sizeof(s->last_error), "%s: %s", what, hipGetErrorString(e));
    return MEMD_EDEVICE;
}

// Join initialised replicas (slot, zeroed step counters).
hipError_t join_ready(memd_server *s) {
    std::vector<Request *> joining;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        joining.swap(s->ready);
    }
    for (Request *rq : joining) {
        rq->slot = s->free_slots.back();
        s->free_slots.pop_back();
        int *hs = s->h_steps + 2 * rq->slot;
        hs[0] = 0;
        hs[1] = 0;
        hipError_t e = hipMemcpyAsync(s->d_steps + 2 * rq->slot, hs, 2 * sizeof(int), hipMemcpyHostToDevice,
                                      s->stream);
        if (e != hipSuccess) return e;
        rq->state = Q_ACTIVE;
        s->active.push_back(rq);
        s->table_dirty = true;
    }
    return hipSuccess;
}

// Retire finished replicas: out of the table (their slot is free for the
// next one to join); a worker takes their results out and frees their
// memory, off this thread, so the step graph keeps its queue.
hipError_t retire(memd_server *s) {
    std::vector<Request *> keep;
    bool any = false;
    for (Request *rq : s->active) {
        if (s->h_steps[2 * rq->slot + 1] < rq->nsteps) {
            keep.push_back(rq);
            continue;
        }
        s->free_slots.push_back(rq->slot);
        s->table_dirty = true;
        std::lock_guard<std::mutex> lk(s->mu);
        s->retire_queue.push_back(rq);
        any = true;
    }
    s->active.swap(keep);
    if (any) s->cv.notify_all();
    return hipSuccess;
}

// Results of a finished replica (forces, energy, Gauss audit of its final
// state, on its context's own stream), then its context destroyed and its
// memory returned to the budget.
void finish_request(memd_server *s, Request *rq) {
    memd_ctx *c = rq->ctx;
    c->cur = rq->nsteps & 1;
    c->step_index = rq->nsteps;
    rq->F.assign(3 * (size_t)rq->n, 0.0);
    memd_status ms = refresh_forces(c) == hipSuccess ? MEMD_OK : MEMD_EDEVICE;
    if (ms == MEMD_OK) ms = memd_forces(c, rq->F.data());
    if (ms == MEMD_OK) ms = memd_energy(c, &rq->E);
    if (ms == MEMD_OK) ms = memd_gauss_residual(c, &rq->gauss, nullptr);
    bool finite = std::isfinite(rq->E.E_corrected);
    for (double f : rq->F) finite = finite && std::isfinite(f);
    memd_destroy(c);
    std::lock_guard<std::mutex> lk(s->mu);
    rq->ctx = nullptr;
    rq->t_done = s->now();
    rq->state = (ms == MEMD_OK && finite) ? Q_DONE : Q_FAILED;
    rq->error = ms != MEMD_OK ? ms : (finite ? MEMD_OK : MEMD_EDEVICE);
    s->used -= rq->bytes_resident;
    --s->slots_used;
    if (rq->state == Q_DONE) ++s->done_count;
    else ++s->failed_count;
}

}  // namespace

extern "C" {

memd_status memd_server_create(memd_server **out, size_t hbm_budget_bytes, int max_slots, int init_workers,
                               double solve_tol, const char *tune_cache, void *hip_stream) {
    if (!out || hbm_budget_bytes == 0 || max_slots <= 0 || init_workers <= 0 || init_workers > 64)
        return MEMD_EINVAL;
    *out = nullptr;
    memd_server *s = new (std::nothrow) memd_server();
    if (!s) return MEMD_ENOMEM;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->solve_tol = solve_tol > 0.0 ? solve_tol : 1e-8;
    if (tune_cache) s->tune_cache = tune_cache;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return MEMD_EDEVICE;
    }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return MEMD_EDEVICE;
        }
        s->own_stream = true;
    }
    if (hipMalloc((void **)&s->d_tab, (size_t)max_slots * sizeof(RepDesc)) != hipSuccess ||
        hipMalloc((void **)&s->d_hdr, hdr_ints(max_slots) * sizeof(int)) != hipSuccess ||
        hipMalloc((void **)&s->d_steps, 2 * (size_t)max_slots * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void **)&s->h_tab, (size_t)max_slots * sizeof(RepDesc), 0) != hipSuccess ||
        hipHostMalloc((void **)&s->h_hdr, hdr_ints(max_slots) * sizeof(int), 0) != hipSuccess ||
        hipHostMalloc((void **)&s->h_steps, 2 * (size_t)max_slots * sizeof(int), 0) != hipSuccess) {
        memd_server_destroy(s);
        return MEMD_ENOMEM;
    }
    memset(s->h_hdr, 0, hdr_ints(max_slots) * sizeof(int));
    memset(s->h_steps, 0, 2 * (size_t)max_slots * sizeof(int));
    for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
    if (tune_batch_depth(s) != hipSuccess || upload_table(s) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess || capture_graph(s) != hipSuccess) {
        memd_server_destroy(s);
        return MEMD_EDEVICE;
    }
    for (int w = 0; w < init_workers; ++w) s->workers.emplace_back(worker_main, s);
    *out = s;
    return MEMD_OK;
}

memd_status memd_server_submit(memd_server *s, const memd_params *p, int n, const double *q, const double *r0,
                               int eps_mode, const double *eps, int nsteps, uint64_t seed, double sigma,
                               uint64_t *req_id) {
    if (!s || !p || !req_id || n < 0 || nsteps < 0 || (n > 0 && (!q || !r0)) || !eps || !(sigma >= 0.0))
        return MEMD_EINVAL;
    if (eps_mode != MEMD_EPS_UNIFORM && eps_mode != MEMD_EPS_ZSITE) return MEMD_EINVAL;
    if (p->L < 2 || p->L > 1024) return MEMD_EINVAL;
    auto rq = std::make_unique<Request>();
    rq->p = *p;
    rq->p.precision = MEMD_FP32_MIXED;
    rq->p.audit_every = 0;
    rq->p.energy_every = 0;
    rq->n = n;
    rq->q.assign(q, q + n);
    rq->r0.assign(r0, r0 + 3 * (size_t)n);
    const size_t ne = eps_mode == MEMD_EPS_UNIFORM ? 1 : (size_t)p->L;
    rq->eps.assign(eps, eps + ne);
    rq->eps_mode = eps_mode;
    rq->nsteps = nsteps;
    rq->seed = seed;
    rq->sigma = sigma;
    rq->bytes_resident = resident_bytes(p->L, n);
    rq->bytes_peak = rq->bytes_resident + solve_bytes(p->L);
    std::lock_guard<std::mutex> lk(s->mu);
    rq->id = s->next_id++;
    rq->t_arrival = s->now();
    *req_id = rq->id;
    if (rq->bytes_peak > s->budget) {
        rq->state = Q_FAILED;
        rq->error = MEMD_ENOMEM;
        rq->t_done = rq->t_arrival;
        ++s->failed_count;
    } else {
        s->pending.push_back(rq.get());
    }
    s->all[rq->id] = std::move(rq);
    return MEMD_OK;
}

memd_status memd_server_progress(memd_server *s, int global_steps, int *active, int *pending, int *done) {
    if (!s || global_steps < 0) return MEMD_EINVAL;
    hipError_t e;
    if ((e = hipSetDevice(s->device)) != hipSuccess) return fail_dev(s, "hipSetDevice", e);
    admit(s);
    if ((e = join_ready(s)) != hipSuccess) return fail_dev(s, "join", e);
    if (s->table_dirty) {
        if ((e = upload_table(s)) != hipSuccess) return fail_dev(s, "table upload", e);
        if (s->active.empty() && (e = hipStreamSynchronize(s->stream)) != hipSuccess)
            return fail_dev(s, "table sync", e);
    }
    if (!s->active.empty() && global_steps > 0) {
        for (int t = 0; t < global_steps; ++t)
            if ((e = hipGraphLaunch(s->exec, s->stream)) != hipSuccess) return fail_dev(s, "hipGraphLaunch", e);
        s->global_steps += global_steps;
        if ((e = hipMemcpyAsync(s->h_steps, s->d_steps, 2 * (size_t)s->max_slots * sizeof(int),
                                hipMemcpyDeviceToHost, s->stream)) != hipSuccess)
            return fail_dev(s, "step counters", e);
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return fail_dev(s, "step sync", e);
        if ((e = retire(s)) != hipSuccess) return fail_dev(s, "retire", e);
        admit(s);
    } else if (s->active.empty()) {
        // nothing resident: let the workers run
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (active) *active = (int)s->active.size();
    // queued: waiting for admission, or admitted and not yet resident
    if (pending) *pending = (int)s->pending.size() + s->slots_used - (int)s->active.size();
    if (done) *done = (int)(s->done_count + s->failed_count);
    return MEMD_OK;
}

const char *memd_server_last_error(memd_server *s) { return s ? s->last_error : ""; }

memd_status memd_server_poll(memd_server *s, uint64_t req_id, int *state, double *F_out, memd_energy_t *E_out,
                             double *gauss_max, double *t_arrival, double *t_done) {
    if (!s) return MEMD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(req_id);
    if (it == s->all.end()) return MEMD_EINVAL;
    Request *rq = it->second.get();
    if (state) *state = rq->state;
    if (t_arrival) *t_arrival = rq->t_arrival;
    if (t_done) *t_done = rq->t_done;
    if (rq->state == Q_DONE) {
        if (F_out && !rq->F.empty()) memcpy(F_out, rq->F.data(), rq->F.size() * sizeof(double));
        if (E_out) *E_out = rq->E;
        if (gauss_max) *gauss_max = rq->gauss;
    }
    if (rq->state == Q_FAILED) return rq->error;
    return MEMD_OK;
}

memd_status memd_server_stats(memd_server *s, long *global_steps, long *replica_steps, size_t *bytes_in_use) {
    if (!s) return MEMD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    long rs = 0;
    for (const auto &kv : s->all)
        if (kv.second->state == Q_DONE) rs += kv.second->nsteps;
    if (global_steps) *global_steps = s->global_steps;
    if (replica_steps) *replica_steps = rs;
    if (bytes_in_use) *bytes_in_use = s->used;
    return MEMD_OK;
}

memd_status memd_server_destroy(memd_server *s) {
    if (!s) return MEMD_EINVAL;
    hipSetDevice(s->device);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv.notify_all();
    for (auto &t : s->workers) t.join();
    if (s->stream) hipStreamSynchronize(s->stream);
    for (auto &kv : s->all) {
        Request *rq = kv.second.get();
        if (rq->ctx) memd_destroy(rq->ctx);
    }
    if (s->exec) hipGraphExecDestroy(s->exec);
    if (s->graph) hipGraphDestroy(s->graph);
    if (s->d_tab) hipFree(s->d_tab);
    if (s->d_hdr) hipFree(s->d_hdr);
    if (s->d_steps) hipFree(s->d_steps);
    if (s->h_tab) hipHostFree(s->h_tab);
    if (s->h_hdr) hipHostFree(s->h_hdr);
    if (s->h_steps) hipHostFree(s->h_steps);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    delete s;
    return MEMD_OK;
}

}  // extern "C"
