"""Request loop over the continuous-batching server of libmemd.

Replicas arrive at their (Poisson) arrival times in wall-clock seconds; the
loop submits each on arrival and drives memd_server_progress, which admits
requests by memory budget and slots, initialises them on worker threads while
the resident replicas keep stepping, and retires finished ones.  Latency is
completion minus arrival, both on the server's clock.
"""
from __future__ import annotations

import time

import numpy as np

from . import memd
from . import workloads as W


def replica_request(spec: W.ReplicaSpec, a=1.0, dt=W.DT, sigma=0.02):
    q, r0 = W.replica_inputs(spec, a)
    if spec.eps_kind == "uniform":
        mode, eps = memd.EPS_UNIFORM, np.array([spec.eps_value])
    else:
        mode, eps = memd.EPS_ZSITE, np.asarray(spec.eps_z, dtype=np.float64)
    params = memd.make_params(spec.L, a, dt, 0.0, memd.FP32_MIXED)
    return params, q, r0, mode, eps, sigma


def run_stream(specs, budget_bytes: int, max_slots: int = 512, workers: int = 4,
               poll_steps: int = 4, solve_tol: float = 1e-8, tune_cache: str | None = None,
               time_limit: float = 600.0, sigma: float = 0.02):
    """Serve `specs` (arrival times in seconds from now).  Returns per-request
    results and the aggregate throughput."""
    srv = memd.memd_server_create(budget_bytes, max_slots, workers, solve_tol, tune_cache)
    order = sorted(specs, key=lambda s: s.arrival)
    reqs = {}
    k = 0
    t_start = time.perf_counter()
    try:
        while True:
            now = time.perf_counter() - t_start
            while k < len(order) and order[k].arrival <= now:
                sp = order[k]
                params, q, r0, mode, eps, sg = replica_request(sp, sigma=sigma)
                rid = memd.memd_server_submit(srv, params, q, r0, mode, eps, sp.steps, sp.seed, sg)
                reqs[rid] = sp
                k += 1
            active, queued, finished = memd.memd_server_progress(srv, poll_steps)
            if k == len(order) and finished == len(order):
                break
            if active == 0 and queued == 0 and k < len(order):
                wait = order[k].arrival - (time.perf_counter() - t_start)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            if time.perf_counter() - t_start > time_limit:
                raise TimeoutError("serving stream did not finish in time")
        makespan = time.perf_counter() - t_start
        results = {}
        for rid, sp in reqs.items():
            st, status, F, E, g, ta, td = memd.memd_server_poll(srv, rid, sp.n)
            results[sp.index] = dict(state=st, status=status, F=F, E=E, gauss=g, t_arrival=ta,
                                     t_done=td, latency=td - ta, steps=sp.steps, L=sp.L, n=sp.n)
        gsteps, rsteps, _ = memd.memd_server_stats(srv)
    finally:
        memd.memd_server_destroy(srv)
    lat = np.array([r["latency"] for r in results.values() if r["state"] == memd.REQ_DONE])
    site_steps = sum(r["steps"] * r["L"] ** 3 for r in results.values() if r["state"] == memd.REQ_DONE)
    return dict(results=results, makespan=makespan, global_steps=gsteps, replica_steps=rsteps,
                replica_steps_per_s=rsteps / makespan, site_updates_per_s=site_steps / makespan,
                p50=float(np.percentile(lat, 50)) if len(lat) else None,
                p99=float(np.percentile(lat, 99)) if len(lat) else None,
                done=int(len(lat)), failed=int(sum(1 for r in results.values() if r["state"] != memd.REQ_DONE)))


def run_sequential_fp64(specs, sigma: float = 0.02, solve_tol: float = 1e-8):
    """The plain FP64 single-system path, one replica after another in arrival
    order (a single FIFO server): latency = completion - arrival."""
    order = sorted(specs, key=lambda s: s.arrival)
    t_start = time.perf_counter()
    lat = []
    rsteps = 0
    site_steps = 0
    for sp in order:
        now = time.perf_counter() - t_start
        if sp.arrival > now:
            time.sleep(sp.arrival - now)
        q, r0 = W.replica_inputs(sp)
        with memd.Context(sp.L, q, r0, dt=W.DT, precision=memd.FP64) as G:
            if sp.eps_kind == "uniform":
                G.set_permittivity(memd.EPS_UNIFORM, [sp.eps_value])
            else:
                G.set_permittivity(memd.EPS_ZSITE, sp.eps_z)
            G.solve(solve_tol)
            memd.memd_step_seeded(G.ctx, sp.seed, sigma, sp.steps)
            G.forces()
        lat.append(time.perf_counter() - t_start - sp.arrival)
        rsteps += sp.steps
        site_steps += sp.steps * sp.L ** 3
    makespan = time.perf_counter() - t_start
    lat = np.array(lat)
    return dict(makespan=makespan, replica_steps_per_s=rsteps / makespan,
                site_updates_per_s=site_steps / makespan, p50=float(np.percentile(lat, 50)),
                p99=float(np.percentile(lat, 99)), done=len(lat))
