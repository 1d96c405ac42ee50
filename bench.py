"""MEMD step throughput on one MI355X.

Workload c4: 128^3 periodic lattice, 10^5 ions (45 000 x (+-1), 5 000 x (+-2))
at seeded uniform positions, salt-dependent permittivity per link
(eps = 80 - 15 c_local, c_local the 3x3x3-smoothed linear-interpolated ion
density) recomputed every 50 steps, seeded Gaussian prescribed displacements
(sigma = 0.02 a), FP32 fields with FP64 positions, dipole, Gauss audit and
energies.  One step = leapfrog (Faraday + Ampere) + ion move and current
deposit + dipole + corrected forces; every 50 steps the permittivity
recompute, the Gauss audit and the energy evaluation, every 100 the
re-binning of the ions.  The timed window starts on the last step of a
100-step period (extra untimed steps after the warm-up align it), so it
holds at least one of each of these whatever its length.  Inputs (including all displacements)
are resident in HBM before timing.

Prints one JSON line: value = lattice-site updates per second (whole job),
plus ion-steps/s, the leapfrog kernel's roofline object (HIP events over the
runs of one-launch steps in the timed region) on the algorithmic bytes per site and
per ion, an on-box stream-copy ceiling, and the FP64 CPU oracle's throughput
on a bounded sample of the same workload; beside them the FP64 variant over
the same trajectory (and the FP32 path's error on each output against it),
the same recipe at 256^3, the same system moved by its own forces (velocity
Verlet) and the batched serving stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MEMD lattice-site updates/s + ion-steps/s; p50/p99 latency for batched replicas"
HBM_PEAK_GBS = 8000.0
CADENCE = 50
# the ions are re-binned (and the tile lists rebuilt) every REBIN_EVERY steps,
# a multiple of the cadence, so that re-binnings fall on cadence steps
REBIN_EVERY = 2 * CADENCE
# under their own dynamics the ions move ballistically and leave the tile
# lists' one-cell margin sooner: re-binned every MD_REBIN_EVERY steps
MD_REBIN_EVERY = 16
PROFILE_EVERY = 10

# Algorithmic bytes of a step (each value read once and written once):
#   per site: D[3], B[3] read and written, the per-link eta[3] read
#     (15 values: 60 B FP32, 120 B FP64)
#   per ion: r and the displacement read, r written, q read, the 12-link
#     current read-modify-write, the 12-link gather of D (and eta), the force
#     written: about 250 B FP32, 490 B FP64
SITE_BYTES = {"fp32": 60, "fp64": 120}
ION_BYTES = {"fp32": 250, "fp64": 490}


def algorithmic_bytes(precision: str, sites: int, ions: int) -> int:
    return SITE_BYTES[precision] * sites + ION_BYTES[precision] * ions


# Bytes this implementation moves per launch of the fused leapfrog, counted
# the same way (each value once): the algorithmic field bytes, and per ion
# the tiles' share (its record: a 16-byte head and the 12 first-cell values
# in the field type; the fractional position, charge and 12/sum(eta) for the
# force the tile computes, which it writes with a 4-byte stamp) and the
# movers' share (mover_bytes_per_ion).


def leapfrog_bytes_per_site(fp32: bool, per_link_eps: bool) -> int:
    t = 4 if fp32 else 8
    return (15 if per_link_eps else 12) * t


def mover_bytes_per_ion(fp32: bool) -> int:
    """The movers of the fused launch: read r, q, the record's displacement,
    list_fail, cbin, perm and the next displacement (given by the caller);
    write r^{n+1} and the next record (16-byte head, the first cell's 12
    values, the displacement, the fractional position and charge, the
    atomic-path flag); and, completing the force of the state the previous
    launch started from, read that launch's tile force with its stamp and
    write the whole force."""
    t = 4 if fp32 else 8
    return ((24 + 8 + 24 + 4 + 4 + 4 + 24) + (24 + 16 + 12 * t + 24 + 4 * t + 4)
            + (24 + 4) + 24)


def implementation_bytes(fp32: bool, sites: int, ions: int, fused: bool) -> int:
    t = 4 if fp32 else 8
    rec = 16 + 12 * t + 5 * t + 24 + 4 + mover_bytes_per_ion(fp32)
    return leapfrog_bytes_per_site(fp32, True) * sites + (rec * ions if fused else 0)


def kernel_source_hash() -> str:
    """Hash of the sources of the leapfrog kernels (plain and with the fused deposit)."""
    h = hashlib.sha256()
    for f in ("kernels_field.hip", "leapfrog_tile.hpp", "ion_records.hpp", "ion_ops.hpp", "device_util.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1309_7859_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(precision: str):
    """HBM bytes per leapfrog launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"leapfrog_c4_{precision}_hbm_traffic.md")
    if not os.path.exists(p):
        return None
    text = open(p).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    h = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    if not m or not h or h.group(1) != kernel_source_hash():
        return None
    return float(m.group(1))


def align_steps(warmup: int) -> int:
    """Untimed steps after the warm-up that put the first timed step on the
    last step of a re-binning period (step index -1 mod REBIN_EVERY, a
    multiple of CADENCE): that step ends with the audit and the energy
    evaluation, and the next one starts with the permittivity recompute and
    the re-binning, so a window of two or more steps holds each of them."""
    return (REBIN_EVERY - 1 - warmup) % REBIN_EVERY


def cadence_counts(first: int, steps: int) -> dict:
    idx = range(first, first + steps)
    return {"permittivity_recompute": sum(1 for t in idx if t % CADENCE == 0),
            "rebinning": sum(1 for t in idx if t % REBIN_EVERY == 0),
            "audit": sum(1 for t in idx if (t + 1) % CADENCE == 0),
            "energy": sum(1 for t in idx if (t + 1) % CADENCE == 0)}


def gpu_run(w, steps, warmup, precision, copy_mb=0, tile=None, solve_tol=1e-12, outputs=False):
    import torch
    from paper_1309_7859_amd import memd
    from paper_1309_7859_amd import workloads as W

    fp32 = precision == "fp32"
    pre = warmup + align_steps(warmup)
    s = W.make_system(w, steps=0)
    stream = W.DisplacementStream(w)
    disp = torch.from_numpy(stream.take(pre + steps)).to("cuda").contiguous()
    torch.cuda.synchronize()
    if copy_mb:
        # a plain copy of known size: calibrates the HBM byte counters under rocprofv3
        src = torch.empty(copy_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    G = memd.Context(w.L, s["q"], s["r0"], a=w.a, dt=w.dt, c=0.0,
                     precision=memd.FP32_MIXED if fp32 else memd.FP64,
                     audit_every=CADENCE, energy_every=CADENCE)
    G.set_salt(80.0, 15.0, 1.0, every=CADENCE)
    t0 = time.perf_counter()
    st, iters, res = G.solve(solve_tol, check=False)
    t_solve = time.perf_counter() - t0
    if tile:
        memd.memd_set_tiling(G.ctx, tile[0], tile[1])
        tile_used = tuple(tile) + (None,)
    else:
        tile_used = memd.memd_autotune(G.ctx, 10, None)
    memd.memd_set_options(G.ctx, 1, REBIN_EVERY)  # re-binning on a multiple of the cadence
    c_used, eps_h, eps_min = G.params_in_use()
    per = 3 * w.n
    base = disp.data_ptr()
    if pre:
        memd.memd_step(G.ctx, base, pre)
    torch.cuda.synchronize()
    # The steps that are one leapfrog launch and nothing else are timed in
    # runs (an event pair around each run of them, every launch counted);
    # the last of every PROFILE_EVERY other leapfrog launches (those beside
    # the cadence work) carries events of its own, never the first of the call
    memd.memd_profile_enable(G.ctx, ["leapfrog"], PROFILE_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    memd.memd_step(G.ctx, base + 8 * per * pre, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lf_ms, lf_n = memd.memd_profile_read(G.ctx, "leapfrog")
    memd.memd_profile_enable(G.ctx, [])
    bad_moves, fused = memd.memd_counters(G.ctx)
    audits, energies = G.history()
    gauss_max = float(np.max(audits[:, 0])) if len(audits) else None
    gauss_final, _ = G.gauss_residual()  # the state the window ends on, after the timing
    out = dict(wall=wall, lf_ms=lf_ms, lf_n=lf_n, solve_s=t_solve, solve_iters=iters, tile=tile_used,
               fused=bool(fused), bad_moves=bad_moves, pre=pre,
               solve_res=res, solve_status=st, c=c_used, eps_min=eps_min, gauss_max=gauss_max,
               gauss_final=gauss_final, cadence=cadence_counts(pre, steps),
               energy_last=energies[-1].tolist() if len(energies) else None)
    if outputs:
        out["F"] = G.forces()
        out["E"] = G.energy()
        out["P"] = G.dipole()
    G.close()
    return out


def output_error(r32, r64) -> dict:
    """Error of each output of the FP32-field run against the FP64 run of the
    same trajectory (the FP64 path matches the FP64 oracle to 1e-10)."""
    F, F64 = r32["F"], r64["F"]
    rms = float(np.sqrt(np.mean(np.sum(F64 ** 2, axis=1))))
    e, e64 = r32["E"], r64["E"]
    out = {"force_max_over_rms": float(np.max(np.abs(F - F64)) / rms)}
    for k in ("W_E", "W_B", "U_self", "U_dip"):
        out[k] = abs(e[k] - e64[k]) / max(abs(e64[k]), 1e-300)
    out["E_corrected_over_W_E"] = abs(e["E_corrected"] - e64["E_corrected"]) / abs(e64["W_E"])
    out["dipole"] = float(np.max(np.abs(r32["P"] - r64["P"])) / max(1.0, np.max(np.abs(r64["P"]))))
    out["gauss_max"] = r32["gauss_final"]
    out["gauss_max_fp64"] = r64["gauss_final"]
    return {k: float("%.3g" % v) for k, v in out.items()}


def stream_copy_gbs(mb: int = 1024, reps: int = 10) -> dict:
    """On-box bandwidth ceiling: a device-to-device copy of mb MiB (torch's
    copy kernel), timed with events, median of reps; bytes = read + write."""
    import torch
    n = (mb << 20) // 4
    src = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    t = float(np.median(times))
    return {"GBps": round(2 * n * 4 / t / 1e9, 1), "bytes_per_copy": 2 * n * 4, "median_s": t,
            "reps": reps}


def md_run(w, steps, warmup, tile=None):
    """The c4 system with the ions' own dynamics instead of prescribed moves
    (memd_md_step: velocity Verlet under the MEMD forces; mass 100 and
    initial velocities N(0, 2) per component, so that a step moves an ion
    about as far as the prescribed displacements do).  Per step: the
    leapfrog with the deposit of the step's move, then the forces of the new
    state with both half kicks and the next move's records.  The ions move
    ballistically here, so they are re-binned every MD_REBIN_EVERY = 16
    steps (measured over 400 steps: 0.0552 ms per step at 12, 0.0549 at 16,
    0.0551 at 20, 0.0579 at 24)."""
    import torch
    from paper_1309_7859_amd import memd
    from paper_1309_7859_amd import workloads as W

    s = W.make_system(w, steps=0)
    G = memd.Context(w.L, s["q"], s["r0"], a=w.a, dt=w.dt, c=0.0, precision=memd.FP32_MIXED,
                     audit_every=CADENCE, energy_every=CADENCE)
    G.set_salt(80.0, 15.0, 1.0, every=CADENCE)
    G.solve(1e-6, check=False)
    if tile:
        memd.memd_set_tiling(G.ctx, tile[0], tile[1])
    else:
        memd.memd_autotune(G.ctx, 10, None)
    memd.memd_set_options(G.ctx, 1, MD_REBIN_EVERY)
    rng = np.random.default_rng(w.seed + 1)
    v = torch.from_numpy(rng.normal(0.0, 2.0, size=(w.n, 3))).to("cuda").contiguous()
    m = torch.full((w.n,), 100.0, dtype=torch.float64, device="cuda")
    pre = warmup + align_steps(warmup)
    if pre:
        G.md_step(v, m, pre)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.md_step(v, m, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    audits, _ = G.history()
    gauss_max = float(np.max(audits[:, 0])) if len(audits) else None
    gauss_final, _ = G.gauss_residual()
    G.close()
    return dict(wall=wall, gauss_max=gauss_max, gauss_final=gauss_final)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, sample_steps: int, single_steps: int):
    """The FP64 oracle on a bounded sample of the same workload: per step the
    leapfrog, the deposit, the dipole and the forces, timed over sample_steps
    steps three times (the median is taken) with all of the oracle's threads,
    and over single_steps steps three times with one thread; the permittivity
    recompute, the Gauss audit and the energy evaluation are timed once at
    each thread count and amortised at the GPU cadence of one per 50 steps.
    The oracle starts from the recursion solution (its CG relaxation at 128^3
    is a one-off that is not part of a step)."""
    import oracle
    from paper_1309_7859_amd import workloads as W

    s = W.make_system(w, steps=0)
    disp = W.DisplacementStream(w).take(3 * sample_steps + 3 * single_steps)
    S = oracle.System(w.L, w.a, w.dt, 1.0, s["q"], s["r0"])
    S.set_eps_salt()
    S.c = W.default_c(w.a, w.dt, float(np.min(1.0 / S.eta)))
    S.recursion_only()
    cursor = [0]

    def steps_time(k):
        t0 = time.perf_counter()
        for _ in range(k):
            S.step(disp[cursor[0]])
            S.forces()
            cursor[0] += 1
        return (time.perf_counter() - t0) / k

    def cadence_time():
        t0 = time.perf_counter()
        S.set_eps_salt()
        S.gauss_residual()
        S.energy()
        return time.perf_counter() - t0

    threads = oracle.threads()
    t_start = time.perf_counter()
    multi = [steps_time(sample_steps) for _ in range(3)]
    cad_multi = cadence_time()
    oracle.set_threads(1)
    try:
        single = [steps_time(single_steps) for _ in range(3)]
        cad_single = cadence_time()
    finally:
        oracle.set_threads(threads)
    total = time.perf_counter() - t_start
    per_multi = float(np.median(multi)) + cad_multi / CADENCE
    per_single = float(np.median(single)) + cad_single / CADENCE
    return dict(per_step=per_multi, per_step_single=per_single, cores=threads, total=total,
                runs=[round(x * 1e3, 1) for x in multi], runs_single=[round(x * 1e3, 1) for x in single])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--fp64", type=int, default=1,
                    help="1: run the FP64 variant over the same trajectory and report the FP32 "
                         "path's error on each output against it (0 = skip)")
    ap.add_argument("--cpu-steps", type=int, default=30,
                    help="oracle sample: steps per timed run with all threads (0 = skip)")
    ap.add_argument("--cpu-single-steps", type=int, default=2,
                    help="oracle sample: steps per timed run with one thread")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter calibration)")
    ap.add_argument("--stream-mb", type=int, default=1024,
                    help="size of the on-box stream-copy ceiling measurement (0 = skip)")
    ap.add_argument("--tile", type=str, default="", help="rows,planes of the leapfrog tile")
    ap.add_argument("--md-steps", type=int, default=400,
                    help="steps of the c4 system under its own dynamics (0 = skip; the default, 400, "
                         "is a whole number of cadence periods (50) and re-binning periods (16))")
    ap.add_argument("--diag256-steps", type=int, default=50,
                    help="steps of the same workload at 256^3 (8e5 ions), whose fields exceed the "
                         "256 MB Infinity Cache (0 = skip)")
    ap.add_argument("--serve-count", type=int, default=512,
                    help="replicas in the serving stream (0 = skip the serving measurement)")
    ap.add_argument("--serve-rate", type=float, default=500.0, help="Poisson arrival rate (1/s)")
    ap.add_argument("--serve-fp64-count", type=int, default=512,
                    help="replicas of the same stream run one by one on the FP64 single-system path")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build measures the "
              "single-GPU path; sharding across GPUs is described in DESIGN.md, not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1309_7859_amd import workloads as W

    w = W.WORKLOADS["c4"]
    tile = tuple(int(x) for x in args.tile.split(",")) if args.tile else None
    fp32 = args.precision == "fp32"
    copy = stream_copy_gbs(args.stream_mb) if args.stream_mb > 0 else None
    r = gpu_run(w, args.steps, args.warmup, args.precision, args.copy_mb, tile, outputs=True)
    sites = w.sites
    value = sites * args.steps / r["wall"]
    ion_steps = w.n * args.steps / r["wall"]

    # (a one-step window times no leapfrog launch: the first of a call is never sampled)
    lf_avg_s = r["lf_ms"] / 1e3 / r["lf_n"] if r["lf_n"] else None
    alg = algorithmic_bytes(args.precision, sites, w.n)
    impl = implementation_bytes(fp32, sites, w.n, r["fused"])
    achieved = alg / lf_avg_s / 1e9 if lf_avg_s else None
    traffic = load_traffic(args.precision)

    def per_launch(x, nd):
        return round(x, nd) if lf_avg_s else None
    roof = {"bound": "hbm", "achieved": per_launch(achieved or 0.0, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": per_launch((achieved or 0.0) / HBM_PEAK_GBS, 4),
            "traffic": (round(traffic / lf_avg_s / 1e9, 1) if traffic and lf_avg_s else None),
            "kernel": ("k_leapfrog_dep (Faraday + Ampere + tile-owned current deposit + forces + ion movers)" if r["fused"]
                       else "k_leapfrog (Faraday + Ampere)"),
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_bytes_rule": f"{SITE_BYTES[args.precision]} B/site + {ION_BYTES[args.precision]} B/ion",
            "avg_launch_us": per_launch((lf_avg_s or 0.0) * 1e6, 2),
            "launches": r["lf_n"],
            "timing": "HIP events around each run of one-launch steps in the timed window (all their "
                      f"launches), plus the last of every {PROFILE_EVERY} launches beside cadence work",
            "implementation_bytes_per_launch": impl,
            "implementation_frac": per_launch(impl / (lf_avg_s or 1.0) / 1e9 / HBM_PEAK_GBS, 4),
            "tile": {"x": 64, "y": 4 * r["tile"][0], "z_chunk": r["tile"][1],
                     "autotuned_us": r["tile"][2]}}
    if traffic:
        roof["traffic_bytes_per_launch"] = traffic
    if copy and achieved:
        roof["frac_of_stream_copy"] = round(achieved / copy["GBps"], 4)
    ms_step = r["wall"] * 1e3 / args.steps
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "site-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 fields, f64 positions/reductions" if fp32 else "f64",
        "data": "synthetic: seeded uniform ions, Gaussian displacements (c4 recipe)",
        "config": {"workload": f"c4: 128^3 lattice, 1e5 ions (10% +-2), salt eps per link, audit and "
                               f"energy every {CADENCE} steps, re-binning every {REBIN_EVERY}",
                   "L": w.L, "n_ions": w.n, "precision": args.precision, "c": r["c"],
                   "dt": w.dt, "sigma": w.sigma},
        "ion_steps_per_s": round(ion_steps, 1),
        "step_hbm_frac": round(alg / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "timed_window": {"first_step_index": r["pre"], "align_steps": r["pre"] - args.warmup,
                         "cadence_work_inside": r["cadence"]},
        "gauss_residual_max": r["gauss_max"],
        "gauss_residual_final": r["gauss_final"],
        "initial_solve": {"seconds": round(r["solve_s"], 3), "iterations": r["solve_iters"],
                          "curl_residual": r["solve_res"], "status": r["solve_status"]},
    }
    if copy:
        out["stream_copy"] = {"GBps": copy["GBps"], "frac_of_peak": round(copy["GBps"] / HBM_PEAK_GBS, 4),
                              "kind": f"device copy of {args.stream_mb} MiB (torch), median of {copy['reps']}"}
    if fp32 and args.fp64 > 0:
        r64 = gpu_run(w, args.steps, args.warmup, "fp64", outputs=True)
        lf64 = r64["lf_ms"] / 1e3 / r64["lf_n"] if r64["lf_n"] else float("nan")
        b64 = algorithmic_bytes("fp64", sites, w.n)
        out["fp64_variant"] = {
            "value": round(sites * args.steps / r64["wall"], 1),
            "ion_steps_per_s": round(w.n * args.steps / r64["wall"], 1),
            "ms_per_step": round(r64["wall"] * 1e3 / args.steps, 5),
            "leapfrog_avg_us": round(lf64 * 1e6, 2),
            "leapfrog_frac": round(b64 / lf64 / 1e9 / HBM_PEAK_GBS, 4),
            "step_hbm_frac": round(b64 / (r64["wall"] / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
            "steps": args.steps, "gauss_residual_final": r64["gauss_final"]}
        out["fp32_error_vs_fp64"] = dict(steps=r["pre"] + args.steps, **output_error(r, r64))
    if fp32 and args.diag256_steps > 0:
        # the same recipe at 256^3 with 8x the ions (same density): 604 MB of
        # fields per step, more than the Infinity Cache holds
        w2 = W.Workload("c4@256", 256, w.a, w.dt, tuple(8 * c for c in w.counts), "salt", 0.0, w.sigma,
                        args.diag256_steps, 105, salt_every=CADENCE)
        r2 = gpu_run(w2, args.diag256_steps, 10, "fp32", solve_tol=1e-6)
        lf2 = r2["lf_ms"] / 1e3 / r2["lf_n"] if r2["lf_n"] else float("nan")
        b2 = algorithmic_bytes("fp32", w2.sites, w2.n)
        out["diag_256"] = {
            "workload": f"c4 recipe at 256^3: 8e5 ions (10% +-2), salt eps, audit and energy every {CADENCE} "
                        f"steps, re-binning every {REBIN_EVERY}, FP32 fields",
            "value": round(w2.sites * args.diag256_steps / r2["wall"], 1), "unit": "site-updates/s",
            "ms_per_step": round(r2["wall"] * 1e3 / args.diag256_steps, 5),
            "steps": args.diag256_steps,
            "step_hbm_frac": round(b2 / (r2["wall"] / args.diag256_steps) / 1e9 / HBM_PEAK_GBS, 4),
            "leapfrog": {"avg_launch_us": round(lf2 * 1e6, 2), "algorithmic_bytes_per_launch": b2,
                         "achieved": round(b2 / lf2 / 1e9, 1),
                         "frac": round(b2 / lf2 / 1e9 / HBM_PEAK_GBS, 4),
                         "implementation_bytes_per_launch": implementation_bytes(True, w2.sites, w2.n, r2["fused"]),
                         "tile": {"x": 64, "y": 4 * r2["tile"][0], "z_chunk": r2["tile"][1]},
                         "fused": r2["fused"]},
            "gauss_residual_final": r2["gauss_final"]}
    if fp32 and args.md_steps > 0:
        rm = md_run(w, args.md_steps, 10, tile=tile)
        out["md"] = {
            "workload": "c4 with the ions' own dynamics (velocity Verlet under the MEMD forces, mass 100, "
                        "initial velocities N(0, 2)), FP32 fields, salt eps + audit + energy every 50 steps, "
                        "re-binning every 16 steps",
            "value": round(sites * args.md_steps / rm["wall"], 1), "unit": "site-updates/s",
            "ion_steps_per_s": round(w.n * args.md_steps / rm["wall"], 1),
            "ms_per_step": round(rm["wall"] * 1e3 / args.md_steps, 5), "steps": args.md_steps,
            "gauss_residual_max": rm["gauss_max"], "gauss_residual_final": rm["gauss_final"]}
    if args.cpu_steps > 0:
        cb = cpu_baseline(w, args.cpu_steps, args.cpu_single_steps)
        out["cpu_baseline"] = {
            "value": round(sites / cb["per_step"], 1), "unit": "site-updates/s",
            "cores": cb["cores"], "kind": "oracle",
            "sample": f"c4, FP64, from the recursion solution: 3 runs of {args.cpu_steps} steps (leapfrog, "
                      f"deposit, dipole, forces) with {cb['cores']} threads, median, plus one permittivity "
                      f"recompute, audit and energy amortised at 1/50; the same with 1 thread over 3 runs "
                      f"of {args.cpu_single_steps} step(s); {cb['total']:.1f} s of CPU work",
            "ion_steps_per_s": round(w.n / cb["per_step"], 1),
            "cpu_model": cpu_model(),
            "ms_per_step_runs": cb["runs"],
            "single_thread": {"value": round(sites / cb["per_step_single"], 1),
                              "ion_steps_per_s": round(w.n / cb["per_step_single"], 1),
                              "ms_per_step_runs": cb["runs_single"]}}
    if args.serve_count > 0:
        out["serving"] = serving_run(args.serve_count, args.serve_rate, args.serve_fp64_count)
    print(json.dumps(out), flush=True)


def serving_run(count, rate, fp64_count):
    """Workload c5: a Poisson stream of independent replicas (L in {16, 24, 32,
    48, 64}, ion counts log-uniform in [100, 8000], uniform or tanh-slab eps in
    [2, 80], 100-2000 steps each, sigma = 0.02 a), served by the batched FP32
    server under a 200 GB budget; beside it the first fp64_count replicas of
    the same stream run one after another on the plain FP64 single-system path."""
    from paper_1309_7859_amd import serve
    from paper_1309_7859_amd import workloads as W

    specs = W.serving_stream(count, rate)
    tune_cache = os.path.join(ROOT, "_build_tune_cache.txt")
    if os.path.exists(tune_cache):
        os.remove(tune_cache)
    r = serve.run_stream(specs, 200 << 30, max_slots=count, workers=8, poll_steps=4,
                         tune_cache=tune_cache)
    if os.path.exists(tune_cache):
        os.remove(tune_cache)
    out = {"workload": f"c5: {count} replicas, Poisson {rate:g}/s, L in (16,24,32,48,64), "
                       "n 100-8000, uniform or tanh-slab eps, 100-2000 steps, FP32, 200 GB budget",
           "replica_steps_per_s": round(r["replica_steps_per_s"], 1),
           "site_updates_per_s": round(r["site_updates_per_s"], 1),
           "p50_latency_s": round(r["p50"], 4), "p99_latency_s": round(r["p99"], 4),
           "makespan_s": round(r["makespan"], 3), "done": r["done"], "failed": r["failed"],
           "global_steps": r["global_steps"]}
    if fp64_count > 0:
        b = serve.run_sequential_fp64(specs[:fp64_count])
        out["fp64_single_system_baseline"] = {
            "replicas": fp64_count, "replica_steps_per_s": round(b["replica_steps_per_s"], 1),
            "site_updates_per_s": round(b["site_updates_per_s"], 1),
            "p50_latency_s": round(b["p50"], 4), "p99_latency_s": round(b["p99"], 4),
            "makespan_s": round(b["makespan"], 3)}
    return out


if __name__ == "__main__":
    main()
