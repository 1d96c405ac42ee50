"""The continuous-batching server: seeded displacement stream, results of a
replica alone and in a mix, admission by memory budget, failure isolation,
and a served replica against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd, serve
from paper_1309_7859_amd import workloads as W
from tests.gpu_helpers import energy_err, force_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def spec(index, L, n, steps, kind="uniform", eps=20.0, arrival=0.0, seed=None, eps_pair=(70.0, 3.0)):
    ez = W.slab_between(L, *eps_pair) if kind == "zsite" else None
    return W.ReplicaSpec(index, L, n, kind, eps if kind == "uniform" else 0.0, ez, steps,
                         seed if seed is not None else 7000 + index, arrival)


def test_seeded_displacements_match_oracle():
    for seed, t, n in [(1, 0, 10), (2 ** 40 + 17, 123, 1000)]:
        g = memd.memd_seeded_displacements(seed, t, n, 0.02)
        o = oracle.seeded_displacements(seed, t, n, 0.02)
        assert np.max(np.abs(g - o)) <= 1e-15


def test_seeded_step_matches_oracle():
    """FP64 single-system step with device-drawn displacements vs the oracle
    drawing the same stream."""
    L, n, steps, seed, sigma = 12, 60, 25, 99, 0.05
    rng = np.random.default_rng(4)
    q = np.repeat([1.0, -1.0], n // 2)
    r = rng.uniform(0, L, size=(n, 3))
    c = W.default_c(1.0, 0.01, 5.0)
    S = oracle.System(L, 1.0, 0.01, c, q, r)
    S.set_eps_uniform(5.0)
    S.initial_solve(1e-13)
    G = memd.Context(L, q, r, c=c)
    G.set_permittivity(memd.EPS_UNIFORM, [5.0])
    G.set_state(*S.state())
    memd.memd_step_seeded(G.ctx, seed, sigma, steps)
    for t in range(steps):
        S.step(oracle.seeded_displacements(seed, t, n, sigma))
    assert force_err(G.forces(), S.forces()[0]) <= 1e-10
    assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12


@pytest.mark.parametrize("prec", [memd.FP32_MIXED, memd.FP64])
def test_seeded_fused_step_matches_oracle(prec):
    """Device-drawn displacements on the fused path (L >= 16): the movers of
    each leapfrog launch draw the next step's displacements themselves, over
    two calls and re-binnings every 4 steps."""
    L, n, seed, sigma = 24, 400, 2024, 0.05
    rng = np.random.default_rng(11)
    q = np.repeat([1.0, -1.0], n // 2)
    r = rng.uniform(0, L, size=(n, 3))
    c = W.default_c(1.0, 0.01, 5.0)
    S = oracle.System(L, 1.0, 0.01, c, q, r)
    S.set_eps_uniform(5.0)
    S.initial_solve(1e-13)
    G = memd.Context(L, q, r, c=c, precision=prec)
    try:
        G.set_permittivity(memd.EPS_UNIFORM, [5.0])
        G.set_state(*S.state())
        memd.memd_set_options(G.ctx, 1, 4)
        assert memd.memd_counters(G.ctx)[1] == 1
        memd.memd_step_seeded(G.ctx, seed, sigma, 6)
        memd.memd_step_seeded(G.ctx, seed, sigma, 9)
        for t in range(15):
            S.step(oracle.seeded_displacements(seed, t, n, sigma))
        fp32 = prec == memd.FP32_MIXED
        assert force_err(G.forces(), S.forces()[0]) <= (1e-4 if fp32 else 1e-10)
        assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12 * L
        m, _ = G.gauss_residual()
        assert m <= (1e-5 if fp32 else 1e-12)
    finally:
        G.close()


def _served(specs, budget=8 << 30, **kw):
    out = serve.run_stream(specs, budget, max_slots=64, workers=2, poll_steps=3, **kw)
    return out


def test_alone_equals_in_the_mix():
    """A replica served alone and the same replica served among others that
    arrive earlier and later (different sizes, ion counts, profiles) give the
    same forces and energies within the FP32 tolerance."""
    target = spec(0, 24, 300, 40, kind="zsite", eps_pair=(60.0, 4.0), seed=4242)
    alone = _served([target])["results"][0]
    others = [spec(1, 16, 120, 60, "uniform", 30.0, 0.0), spec(2, 32, 800, 25, "zsite", 0.0, 0.0),
              spec(3, 48, 2000, 35, "uniform", 75.0, 0.01), spec(4, 16, 100, 15, "zsite", 0.0, 0.02),
              spec(5, 24, 500, 80, "uniform", 2.5, 0.0)]
    t = W.ReplicaSpec(**{**target.__dict__, "index": 9, "arrival": 0.005})
    mix = _served(others + [t])
    assert mix["done"] == 6 and mix["failed"] == 0
    inmix = mix["results"][9]
    assert alone["state"] == memd.REQ_DONE and inmix["state"] == memd.REQ_DONE
    assert force_err(inmix["F"], alone["F"]) <= 1e-4
    errs = energy_err(inmix["E"], alone["E"])
    assert max(errs.values()) <= 1e-4, errs
    assert alone["gauss"] <= 1e-5 and inmix["gauss"] <= 1e-5


def test_served_replica_matches_oracle():
    """One served FP32 replica against the FP64 oracle fed the same seeded
    displacements (FP32 tolerances)."""
    sp = spec(0, 16, 200, 30, kind="zsite", eps_pair=(50.0, 5.0), seed=31337)
    res = _served([sp], solve_tol=1e-12)["results"][0]
    q, r0 = W.replica_inputs(sp)
    c = W.default_c(1.0, W.DT, float(np.min(sp.eps_z)))
    S = oracle.System(sp.L, 1.0, W.DT, c, q, r0)
    S.set_eps_zsite(sp.eps_z)
    S.initial_solve(1e-12)
    for t in range(sp.steps):
        S.step(oracle.seeded_displacements(sp.seed, t, sp.n, 0.02))
    assert force_err(res["F"], S.forces()[0]) <= 1e-4
    errs = energy_err(res["E"], S.energy())
    assert max(errs.values()) <= 1e-4, errs


def test_admission_respects_budget():
    """Under a 64 MiB budget the replicas cannot all be resident; they are
    admitted as memory frees up and all finish."""
    specs = [spec(k, 32, 400, 30, "uniform", 10.0 + k, 0.0) for k in range(10)]
    out = _served(specs, budget=64 << 20)
    assert out["done"] == 10 and out["failed"] == 0
    # a 32^3 replica needs ~8 MiB resident and ~14 MiB more while solving: the
    # completions must be spread over several admission rounds
    t_done = sorted(r["t_done"] for r in out["results"].values())
    assert t_done[-1] > t_done[0]


def test_failures_are_isolated():
    """A request whose Courant number is too large fails at initialisation and
    a request larger than the whole budget fails at submit; the others finish."""
    good = [spec(k, 16, 100, 20, "uniform", 20.0, 0.0) for k in range(3)]
    srv = memd.memd_server_create(256 << 20, 16, 2)
    try:
        ids = []
        for sp in good:
            params, q, r0, mode, eps, sg = serve.replica_request(sp)
            ids.append(memd.memd_server_submit(srv, params, q, r0, mode, eps, sp.steps, sp.seed, sg))
        bad = spec(10, 16, 100, 20, "uniform", 20.0, 0.0)
        params, q, r0, mode, eps, sg = serve.replica_request(bad)
        params.c = 1e4  # Courant number far above 1
        bad_id = memd.memd_server_submit(srv, params, q, r0, mode, eps, bad.steps, bad.seed, sg)
        huge = spec(11, 1024, 100, 20, "uniform", 20.0, 0.0)
        params, q, r0, mode, eps, sg = serve.replica_request(huge)
        huge_id = memd.memd_server_submit(srv, params, q, r0, mode, eps, huge.steps, huge.seed, sg)
        for _ in range(2000):
            a, p, f = memd.memd_server_progress(srv, 2)
            if f == 5:
                break
        st, status, *_ = memd.memd_server_poll(srv, bad_id, bad.n)
        assert st == memd.REQ_FAILED and status == memd.EUNSTABLE
        st, status, *_ = memd.memd_server_poll(srv, huge_id, huge.n)
        assert st == memd.REQ_FAILED and status == memd.ENOMEM
        for rid, sp in zip(ids, good):
            st, status, F, E, g, *_ = memd.memd_server_poll(srv, rid, sp.n)
            assert st == memd.REQ_DONE and status == memd.OK
            assert np.all(np.isfinite(F)) and g <= 1e-5
    finally:
        memd.memd_server_destroy(srv)


def test_served_equals_single_system_fp32():
    """The batched kernels and the single-system FP32 kernels compute the same
    step (same arithmetic, different launch structure)."""
    sp = spec(0, 32, 600, 20, kind="uniform", eps=12.0, seed=555)
    res = _served([sp])["results"][0]
    q, r0 = W.replica_inputs(sp)
    with memd.Context(sp.L, q, r0, dt=W.DT, precision=memd.FP32_MIXED) as G:
        G.set_permittivity(memd.EPS_UNIFORM, [12.0])
        G.solve(1e-8)
        memd.memd_step_seeded(G.ctx, sp.seed, 0.02, sp.steps)
        F = G.forces()
    assert force_err(res["F"], F) <= 1e-5


def test_short_replicas_match_oracle():
    """Replicas of 0, 1 and 2 steps in one mix (their final forces come from
    the leapfrog launch after their last deposit, or from the initial solve
    for no steps) against the oracle."""
    specs = [spec(k, L, n, steps, "zsite" if k % 2 else "uniform", 15.0, 0.0, seed=900 + k)
             for k, (L, n, steps) in enumerate([(16, 60, 0), (24, 90, 1), (16, 120, 2), (32, 40, 1)])]
    _check_against_oracle(specs)


def _check_against_oracle(specs):
    """Serves the replicas in one mix and compares each with the oracle fed
    the same seeded displacements (FP32 tolerances)."""
    out = _served(specs, solve_tol=1e-12)
    assert out["done"] == len(specs) and out["failed"] == 0
    for k, sp in enumerate(specs):
        q, r0 = W.replica_inputs(sp)
        eps_min = 15.0 if sp.eps_kind == "uniform" else float(np.min(sp.eps_z))
        S = oracle.System(sp.L, 1.0, W.DT, W.default_c(1.0, W.DT, eps_min), q, r0)
        if sp.eps_kind == "uniform":
            S.set_eps_uniform(15.0)
        else:
            S.set_eps_zsite(sp.eps_z)
        S.initial_solve(1e-12)
        for t in range(sp.steps):
            S.step(oracle.seeded_displacements(sp.seed, t, sp.n, 0.02))
        res = out["results"][k]
        assert force_err(res["F"], S.forces()[0]) <= 1e-4, (k, sp.steps)
        errs = energy_err(res["E"], S.energy())
        assert max(errs.values()) <= 1e-4, (k, errs)


def test_narrow_row_tiles_match_oracle():
    """Lattices narrower than a wavefront run as tiles of 256 // L whole rows:
    L = 8 (one tile holds every row), 20 and 40 (a shorter last tile), 63
    (four rows per tile, three in the last), in one mix with both
    permittivity kinds, against the oracle."""
    specs = [spec(k, L, n, steps, "zsite" if k % 2 else "uniform", 15.0, 0.0, seed=950 + k)
             for k, (L, n, steps) in enumerate([(8, 30, 12), (20, 80, 10), (40, 300, 8), (63, 500, 6)])]
    _check_against_oracle(specs)


def test_batch_depth_tuned_and_cached(tmp_path):
    """memd_server_create times the batched leapfrog for each tile depth on a
    synthetic batch and caches the pick; a second server reads it back (no
    new line) and serves a replica with it."""
    cache = str(tmp_path / "tune.txt")
    srv = memd.memd_server_create(1 << 30, 8, 1, 1e-8, cache)
    memd.memd_server_destroy(srv)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch_leapfrog fp32 planes=")
    assert int(lines[0].split("planes=")[1].split()[0]) in (2, 4, 8, 16, 32)
    sp = spec(0, 24, 100, 10, "uniform", 20.0, 0.0)
    out = serve.run_stream([sp], 1 << 30, max_slots=8, workers=1, poll_steps=2, tune_cache=cache)
    assert out["done"] == 1
    assert open(cache).read().splitlines() == lines
