"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Step parity starts from a shared state (the oracle's initial solution is
uploaded with memd_set_state), so solver termination differences do not enter
the step path; the initial solve is compared separately.  Tolerances: forces
max|dF| / RMS|F| <= 1e-10 (FP64), 1e-4 (FP32); Gauss residual <= 1e-12
(FP64), and in FP32 1e-5 per unit of the largest vertex charge magnitude,
max(max|q|, max_v sum_i |q_i| w_v) (fp32_gauss_bar); energies relative 1e-10
(FP64); dipole 1e-12.
"""
import numpy as np
import pytest

import oracle

from paper_1309_7859_amd import memd
from paper_1309_7859_amd import workloads as W
from tests.gpu_helpers import (apply_eps, energy_err, force_err, fp32_gauss_bar, output_errors, pair,
                               record, rel, require_gpu, share_state)

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _rng_system(seed, n, L, valence2=False):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.array([1.0 if i % 2 == 0 else -1.0 for i in range(n)])
    if valence2:
        q[:2] *= 2
    return rng, q, r


# ------------------------------------------------------------ initial solve

@pytest.mark.parametrize("case", ["c1", "site12", "zsite16", "link10", "uniform12", "zsite24", "link16", "site32",
                                  "link8_contrast"])
def test_initial_solve_parity(case):
    """The GPU initial solution against the oracle's relaxation.  Uniform and
    planar permittivities (c1, zsite16, uniform12, zsite24: lattice sides
    that are and are not powers of two) are solved directly (a 2-D DFT and a
    tridiagonal solve per mode), so the relaxation that follows has nothing
    left to do; per-site and per-link ones are relaxed: with the diagonal
    preconditioner on sides that are not powers of two (site12, link10), with
    the spectral one (FFT of the inverse lattice Laplacian) on the others
    (link16, site32, and link8_contrast with a permittivity contrast of 1000)."""
    if case == "c1":
        w = W.WORKLOADS["c1"]
        s = W.make_system(w, steps=0)
        q, r, L = s["q"], s["r0"], w.L
        S, G = pair(L, q, r)
        apply_eps(S, G, "uniform", 1.0)
    elif case == "site12":
        L = 12
        rng, q, r = _rng_system(5, 10, L, True)
        eps = 2.0 + 60.0 * rng.uniform(size=L ** 3) ** 2
        S, G = pair(L, q, r, eps_min=eps.min())
        apply_eps(S, G, "site", eps_site=eps)
    elif case == "zsite16":
        L = 16
        rng, q, r = _rng_system(6, 12, L)
        ez = W.tanh_slab(L, 1.0)
        S, G = pair(L, q, r, eps_min=ez.min())
        apply_eps(S, G, "zsite", eps_z=ez)
    elif case == "uniform12":
        L = 12
        rng, q, r = _rng_system(8, 14, L, True)
        S, G = pair(L, q, r, eps_min=5.0)
        apply_eps(S, G, "uniform", 5.0)
    elif case == "zsite24":
        L = 24
        rng, q, r = _rng_system(9, 40, L, True)
        ez = W.tanh_slab(L, 1.0)
        S, G = pair(L, q, r, eps_min=ez.min())
        apply_eps(S, G, "zsite", eps_z=ez)
    elif case == "link16":
        L = 16
        rng, q, r = _rng_system(17, 30, L, True)
        el = 1.0 + 9.0 * rng.uniform(size=3 * L ** 3)
        S, G = pair(L, q, r, eps_min=el.min())
        apply_eps(S, G, "link", eps_link=el)
    elif case == "site32":
        L = 32
        rng, q, r = _rng_system(18, 60, L, True)
        eps = 20.0 + 60.0 * rng.uniform(size=L ** 3)
        S, G = pair(L, q, r, eps_min=eps.min())
        apply_eps(S, G, "site", eps_site=eps)
    elif case == "link8_contrast":
        L = 8
        rng, q, r = _rng_system(19, 6, L)
        el = np.exp(np.log(1000.0) * rng.uniform(size=3 * L ** 3))
        S, G = pair(L, q, r, eps_min=el.min())
        apply_eps(S, G, "link", eps_link=el)
    else:
        L = 10
        rng, q, r = _rng_system(7, 8, L)
        el = 1.0 + 9.0 * rng.uniform(size=3 * L ** 3)
        S, G = pair(L, q, r, eps_min=el.min())
        apply_eps(S, G, "link", eps_link=el)
    rc, it, res = S.initial_solve(1e-13)
    assert rc == 0
    st, git, gres = G.solve(1e-13)
    assert st == memd.OK and gres <= 1e-13
    if case in ("c1", "zsite16", "uniform12", "zsite24"):
        assert git == 0  # the direct solution is the minimiser already
    record("initial_solve", label=case, L=L, gpu_iterations=git, oracle_iterations=it)
    D, B, rr = G.state()
    E = S.eta * D
    Eref = S.eta * S.D
    assert np.max(np.abs(E - Eref)) <= 1e-9 * np.max(np.abs(Eref))
    assert np.max(np.abs(B)) == 0.0
    m, _ = G.gauss_residual()
    assert m <= 1e-12
    assert force_err(G.forces(), S.forces()[0]) <= 1e-8


# -------------------------------------------------------------- step parity

def run_parity(S, G, disp, checks, ftol, gtol, etol, audit_each=False):
    """Step both sides one step at a time.  gtol is the Gauss bound, or
    "fp32" for fp32_gauss_bar over the start and current positions."""
    n = disp.shape[0]
    r_start = S.r.copy()
    for t in range(n):
        S.step(disp[t])
        G.step(disp[t], 1)
        if audit_each or (t + 1) in checks:
            m, _ = G.gauss_residual()
            bar = fp32_gauss_bar(S.L, S.a, S.q, r_start, S.r) if gtol == "fp32" else gtol
            assert m <= bar, (t, m, bar)
        if (t + 1) in checks:
            Fo, _ = S.forces()
            assert force_err(G.forces(), Fo) <= ftol, t
            P = G.dipole()
            Po = S.dipole()
            assert np.max(np.abs(P - Po)) <= 1e-12 * max(1.0, np.max(np.abs(Po)))
            if etol is not None:
                errs = energy_err(G.energy(), S.energy())
                assert max(errs.values()) <= etol, (t, errs)


def test_c1_fp64_full_run():
    """Plain FP64 MEMD on the 8^3 two-charge workload, all 200 steps."""
    w = W.WORKLOADS["c1"]
    s = W.make_system(w)
    S, G = pair(w.L, s["q"], s["r0"])
    apply_eps(S, G, "uniform", 1.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    run_parity(S, G, s["disp"], {1, 50, 100, 150, 200}, 1e-10, 1e-12, 1e-10, audit_each=True)


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_c2_parity(prec):
    """32^3, 1000 ions, eps = 80: the first 100 of the 1000 steps."""
    w = W.WORKLOADS["c2"]
    s = W.make_system(w, steps=100)
    S, G = pair(w.L, s["q"], s["r0"], eps_min=80.0, precision=prec)
    apply_eps(S, G, "uniform", 80.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    if prec == memd.FP64:
        run_parity(S, G, s["disp"], {1, 10, 100}, 1e-10, 1e-12, 1e-10)
    else:
        run_parity(S, G, s["disp"], {1, 10, 100}, 1e-4, "fp32", 1e-4)


def run_full_length(name, S, G, disp, calls, prec):
    """Advance both sides over disp in len(calls) calls of the given lengths
    (the multi-step pipeline: deposit records one step ahead, forces of each
    state once, re-binning at its cadence) and compare every output against
    the oracle after each call; the errors are recorded per call."""
    fp32 = prec == memd.FP32_MIXED
    ftol, etol = (1e-4, 1e-4) if fp32 else (1e-10, 1e-10)
    r_start = S.r.copy()
    t0 = 0
    for k, nst in enumerate(calls):
        d = disp[t0:t0 + nst]
        G.step(d, nst)
        for t in range(nst):
            S.step(d[t])
        t0 += nst
        err = output_errors(G, S)
        bar = fp32_gauss_bar(S.L, S.a, S.q, r_start, S.r) if fp32 else 1e-12
        record(name, precision="fp32" if fp32 else "fp64", steps=t0, gauss_bar=bar, **err)
        assert err["gauss_max"] <= bar, (t0, err)
        assert err["gauss_max_oracle"] <= 1e-12
        assert err["force"] <= ftol, (t0, err)
        assert max(err[k] for k in ("W_E", "W_B_vs_W_E", "U_self", "U_dip", "E_corrected")) <= etol, (t0, err)
        assert err["dipole"] <= 1e-12 and err["position"] <= 1e-12, (t0, err)
    assert t0 == disp.shape[0]


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_c2_all_1000_steps(prec):
    """32^3, 1000 ions, eps = 80 over the workload's full 1000 steps, taken
    in calls of 250 steps; every output against the FP64 oracle after each
    call."""
    w = W.WORKLOADS["c2"]
    s = W.make_system(w)
    assert s["disp"].shape[0] == 1000
    S, G = pair(w.L, s["q"], s["r0"], eps_min=80.0, precision=prec)
    apply_eps(S, G, "uniform", 80.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    run_full_length("c2", S, G, s["disp"], [250] * 4, prec)


def test_c3_fp32_all_1000_steps():
    """64^3, 10^4 ions, tanh slab 2 -> 80 (site profile per plane), FP32
    fields, over the workload's full 1000 steps in calls of 250; every
    output against the FP64 oracle after each call."""
    w = W.WORKLOADS["c3"]
    s = W.make_system(w)
    assert s["disp"].shape[0] == 1000
    ez = s["eps_z"]
    S, G = pair(w.L, s["q"], s["r0"], eps_min=ez.min(), precision=memd.FP32_MIXED)
    apply_eps(S, G, "zsite", eps_z=ez)
    S.initial_solve(1e-12)
    share_state(S, G)
    run_full_length("c3", S, G, s["disp"], [250] * 4, memd.FP32_MIXED)


def test_zsite_equals_site_mode():
    """A planar profile given per plane and the same profile given per site
    produce the same run."""
    L = 16
    rng, q, r = _rng_system(8, 20, L)
    ez = W.slab_between(L, 70.0, 3.0)
    c = W.default_c(1.0, 0.01, ez.min())
    A = memd.Context(L, q, r, c=c)
    B = memd.Context(L, q, r, c=c)
    A.set_permittivity(memd.EPS_ZSITE, ez)
    B.set_permittivity(memd.EPS_SITE, np.repeat(ez, L * L))
    A.solve()
    B.solve()
    disp = rng.normal(0, 0.05, size=(10, 20, 3))
    for t in range(10):
        A.step(disp[t], 1)
        B.step(disp[t], 1)
    assert force_err(A.forces(), B.forces()) <= 1e-12


def test_salt_permittivity_parity():
    """Salt-dependent eps per link recomputed every 5 steps (FP64)."""
    L = 16
    rng = np.random.default_rng(9)
    n = 400
    r = rng.uniform(0, L, size=(n, 3))
    q = np.repeat([1.0, -1.0, 2.0, -2.0], n // 4)
    S, G = pair(L, q, r, eps_min=70.0)
    S.set_eps_salt()
    G.set_salt(80.0, 15.0, 1.0, every=5)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.normal(0, 0.05, size=(15, n, 3))
    for t in range(15):
        if t % 5 == 0:
            S.set_eps_salt()
        S.step(disp[t])
        G.step(disp[t], 1)
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= 1e-10
    errs = energy_err(G.energy(), S.energy())
    assert max(errs.values()) <= 1e-10


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_salt_counts_from_the_audit(prec):
    """When an audit inside a call ends the step before a salt recompute, its
    charge-assignment pass also writes the ion counts that the recompute then
    uses: within a call (salt every 4 steps, audit every 2), across a call
    boundary, and not after memd_set_state has moved ions in between (the
    recompute then assigns the new positions itself)."""
    L, n = 16, 400
    rng = np.random.default_rng(19)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.repeat([1.0, -1.0, 2.0, -2.0], n // 4)
    S, G = pair(L, q, r, eps_min=70.0, precision=prec, audit_every=2)
    S.set_eps_salt()
    G.set_salt(80.0, 15.0, 1.0, every=4)
    S.initial_solve(1e-13)
    share_state(S, G)
    fp32 = prec == memd.FP32_MIXED
    disp = rng.normal(0, 0.05, size=(16, n, 3))

    def oracle_steps(t0, t1):
        for t in range(t0, t1):
            if t % 4 == 0:
                S.set_eps_salt()
            S.step(disp[t])

    G.step(disp[:8], 8)
    oracle_steps(0, 8)
    G.step(disp[8:12], 4)
    oracle_steps(8, 12)
    # move a quarter of the ions by half a spacing: the counts the last
    # audit wrote are stale
    D, B, rr = S.state()
    rr = rr.reshape(-1, 3).copy()
    rr[::4, 0] += 0.5
    S.set_state(D, B, rr)
    share_state(S, G)
    G.step(disp[12:], 4)
    oracle_steps(12, 16)
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= (1e-4 if fp32 else 1e-10)
    errs = energy_err(G.energy(), S.energy())
    assert max(errs.values()) <= (1e-4 if fp32 else 1e-10), errs
    E = S.eta * G.state()[0]
    assert np.max(np.abs(E - S.eta * S.D)) <= (1e-4 if fp32 else 1e-10) * np.max(np.abs(S.eta * S.D))


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_large_moves_wraparound(L):
    """Face crossings of several cells per axis, wrap-around, unfolded positions."""
    rng, q, r = _rng_system(10 + L, 6, L, True)
    el = 1.0 + 4.0 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, dt=0.05, c=3.0)
    apply_eps(S, G, "link", eps_link=el)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.uniform(-2.5, 2.5, size=(20, 6, 3)) * (rng.uniform(size=(20, 6, 1)) < 0.6)
    run_parity(S, G, disp, {5, 20}, 1e-10, 1e-12, 1e-10, audit_each=True)
    assert np.allclose(G.state()[2], S.r, rtol=0, atol=1e-12)


@pytest.mark.parametrize("L,rows,tz", [(17, 1, 3), (24, 2, 16), (48, 4, 5), (65, 2, 7), (70, 1, 64)])
def test_leapfrog_ragged_tiles(L, rows, tz):
    """The fused leapfrog on lattice sizes that do not divide into tiles, from a
    random field state, against the oracle's Faraday + Ampere (no ions)."""
    rng = np.random.default_rng(L)
    q = np.zeros(0)
    r = np.zeros((0, 3))
    el = 1.0 + 3.0 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, dt=0.05, c=2.0)
    apply_eps(S, G, "link", eps_link=el)
    memd.memd_set_tiling(G.ctx, rows, tz)
    D = rng.normal(size=3 * L ** 3)
    B = rng.normal(size=3 * L ** 3)
    S.set_state(D, B, r)
    G.set_state(D, B, r.reshape(-1))
    for _ in range(3):
        S.faraday()
        S.ampere()
    G.step(np.zeros(0), 3)
    Dg, Bg, _ = G.state()
    assert np.max(np.abs(Dg - S.D)) <= 1e-12 * np.max(np.abs(S.D))
    assert np.max(np.abs(Bg - S.B)) <= 1e-12 * np.max(np.abs(S.B))


def test_tilings_bitwise_identical():
    """Every tile shape computes the same arithmetic: results agree bit for bit."""
    L = 32
    rng = np.random.default_rng(3)
    D = rng.normal(size=3 * L ** 3)
    B = rng.normal(size=3 * L ** 3)
    ez = W.tanh_slab(L, 1.0)
    outs = []
    for rows, tz in [(1, 1), (2, 16), (4, 32), (2, 5)]:
        G = memd.Context(L, np.zeros(0), np.zeros((0, 3)), dt=0.05, c=1.0)
        G.set_permittivity(memd.EPS_ZSITE, ez)
        memd.memd_set_tiling(G.ctx, rows, tz)
        G.set_state(D, B, np.zeros(0))
        G.step(np.zeros(0), 4)
        outs.append(G.state()[:2])
        G.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_history_matches_explicit_calls():
    L = 12
    rng, q, r = _rng_system(11, 30, L)
    G = memd.Context(L, q, r, audit_every=2, energy_every=3)
    G.set_permittivity(memd.EPS_UNIFORM, [4.0])
    G.solve()
    disp = rng.normal(0, 0.05, size=(6, 30, 3))
    G.step(disp, 6)
    A, E = G.history()
    assert A.shape == (3, 2) and E.shape == (2, 5)
    assert np.all(A[:, 0] <= 1e-12)
    e = G.energy()
    assert E[-1, 0] == pytest.approx(e["W_E"], rel=1e-14)
    assert E[-1, 4] == pytest.approx(e["E_corrected"], rel=1e-12, abs=1e-14)


def test_device_pointer_inputs():
    """Inputs and outputs given as device memory (torch tensors) behave like
    host arrays."""
    import torch
    L = 8
    rng, q, r = _rng_system(12, 6, L)
    disp = rng.normal(0, 0.1, size=(5, 6, 3))
    Gh = memd.Context(L, q, r)
    Gh.solve()
    Gh.step(disp, 5)
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    rd = torch.tensor(r.reshape(-1), dtype=torch.float64, device="cuda")
    dd = torch.tensor(disp.reshape(-1), dtype=torch.float64, device="cuda")
    Gd = memd.Context(L, qd, rd)
    Gd.solve()
    memd.memd_step(Gd.ctx, dd, 5)
    Fd = torch.zeros(18, dtype=torch.float64, device="cuda")
    memd.memd_forces(Gd.ctx, Fd)
    assert force_err(Fd.cpu().numpy().reshape(6, 3), Gh.forces()) <= 1e-12


def test_error_codes():
    L = 8
    q = np.array([1.0, -1.0])
    r = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    with pytest.raises(memd.MemdError) as e:
        memd.Context(L, np.array([1.0, 1.0]), r)
    assert e.value.status == memd.ENONNEUTRAL
    with pytest.raises(memd.MemdError) as e:
        memd.Context(1, q, r)
    assert e.value.status == memd.EINVAL
    for bad in (np.nan, np.inf, 2.0 ** 41 * L):  # positions: finite, within 2^40 L a
        rb = r.copy()
        rb[1, 2] = bad
        with pytest.raises(memd.MemdError) as e:
            memd.Context(L, q, rb)
        assert e.value.status == memd.EINVAL
    G = memd.Context(L, q, r)
    rb = r.copy()
    rb[0, 0] = -np.inf
    with pytest.raises(memd.MemdError) as e:
        G.set_state(None, None, rb)
    assert e.value.status == memd.EINVAL
    with pytest.raises(memd.MemdError) as e:
        G.step(np.zeros((2, 3)), 1)
    assert e.value.status == memd.ESTATE
    with pytest.raises(memd.MemdError) as e:
        G.set_permittivity(memd.EPS_UNIFORM, [-1.0])
    assert e.value.status == memd.EINVAL
    H = memd.Context(L, q, r, c=1000.0)
    with pytest.raises(memd.MemdError) as e:
        H.set_permittivity(memd.EPS_UNIFORM, [1.0])
    assert e.value.status == memd.EUNSTABLE
    with pytest.raises(memd.MemdError) as e:
        memd.memd_set_tiling(G.ctx, 3, 0)
    assert e.value.status == memd.EINVAL
    G.set_state(None, None, r + 2.0 ** 39 * L)  # far from the origin, but inside the bound
    G.step(np.zeros((2, 3)), 1)


def test_autotune_keeps_state_and_caches(tmp_path):
    """The autotuner leaves the state alone, picks a valid tile and reuses its cache."""
    L = 32
    rng, q, r = _rng_system(13, 40, L)
    G = memd.Context(L, q, r)
    G.set_permittivity(memd.EPS_UNIFORM, [2.0])
    G.solve()
    before = G.state()
    cache = str(tmp_path / "tiles.txt")
    rows, planes, us = memd.memd_autotune(G.ctx, 3, cache)
    assert rows in (1, 2, 4) and planes >= 1 and us > 0
    after = G.state()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    assert open(cache).read().count("leapfrog L=32") == 1
    rows2, planes2, _ = memd.memd_autotune(G.ctx, 3, cache)
    assert (rows2, planes2) == (rows, planes)
    assert open(cache).read().count("leapfrog L=32") == 1
    disp = rng.normal(0, 0.05, size=(3, 40, 3))
    G.step(disp, 3)
    m, _ = G.gauss_residual()
    assert m <= 1e-12


def _mixed_moves(rng, steps, n, big_frac=0.05):
    """Small Gaussian moves with a fraction of components replaced by jumps of
    up to 2.5 a (ions that the fused deposit leaves to the atomic path)."""
    d = rng.normal(0, 0.05, size=(steps, n, 3))
    big = rng.uniform(size=d.shape) < big_frac
    d[big] = rng.uniform(-2.5, 2.5, size=int(big.sum()))
    return d


@pytest.mark.parametrize("prec,tile,L", [(memd.FP64, None, 32), (memd.FP32_MIXED, None, 32),
                                         (memd.FP32_MIXED, (1, 8), 44), (memd.FP32_MIXED, (2, 4), 44),
                                         (memd.FP64, (1, 2), 44), (memd.FP64, (1, 8), 44)])
def test_fused_deposit_matches_atomic_path_and_oracle(prec, tile, L):
    """The deposit fused into the leapfrog (tile-owned links) and the global
    atomic deposit give the oracle's result, with jumps of up to 2.5 a mixed
    in, for several fused tile shapes (ragged tiles and z-chunks at L = 44)."""
    n = 600
    rng = np.random.default_rng(21)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    el = 2.0 + 20.0 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, dt=0.01, eps_min=el.min(), precision=prec)
    c = W.default_c(1.0, 0.01, el.min())
    H = memd.Context(L, q, r, c=c, precision=prec)
    apply_eps(S, G, "link", eps_link=el)
    H.set_permittivity(memd.EPS_LINK, el)
    memd.memd_set_options(H.ctx, 0, 8)
    S.initial_solve(1e-13)
    share_state(S, G)
    H.set_state(*S.state())
    if tile:
        memd.memd_set_tiling(G.ctx, *tile)
    assert memd.memd_counters(G.ctx)[1] == 1 and memd.memd_counters(H.ctx)[1] == 0
    disp = _mixed_moves(rng, 12, n)
    fp32 = prec == memd.FP32_MIXED
    ftol = 1e-4 if fp32 else 1e-10
    for t in range(12):
        S.step(disp[t])
        G.step(disp[t], 1)
        H.step(disp[t], 1)
        gtol = fp32_gauss_bar(L, 1.0, q, r, S.r) if fp32 else 1e-12
        assert G.gauss_residual()[0] <= gtol
        assert H.gauss_residual()[0] <= gtol
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= ftol
    assert force_err(H.forces(), Fo) <= ftol
    assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12


@pytest.mark.parametrize("prec,L", [(memd.FP64, 32), (memd.FP32_MIXED, 32), (memd.FP64, 17),
                                    (memd.FP32_MIXED, 65)])
def test_fused_mixed_moves_in_one_call(prec, L):
    """The same mixed moves (jumps of up to 2.5 a among small steps) taken in
    one call, re-binning every 5 steps: the records of most steps are then
    written by the previous launch's movers into the other record set, and
    the jumping ions they mark reach D^{n+1} through the finisher's atomic
    deposit.  L = 17 and 65 leave ragged tiles in every direction."""
    n, steps = 600, 13
    rng = np.random.default_rng(24)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    el = 2.0 + 20.0 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, dt=0.01, eps_min=el.min(), precision=prec)
    apply_eps(S, G, "link", eps_link=el)
    S.initial_solve(1e-13)
    share_state(S, G)
    memd.memd_set_options(G.ctx, 1, 5)
    assert memd.memd_counters(G.ctx)[1] == 1
    disp = _mixed_moves(rng, steps, n)
    G.step(disp, steps)
    for t in range(steps):
        S.step(disp[t])
    fp32 = prec == memd.FP32_MIXED
    assert G.gauss_residual()[0] <= (fp32_gauss_bar(L, 1.0, q, r, S.r) if fp32 else 1e-12)
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= (1e-4 if fp32 else 1e-10)
    assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12 * L
    assert np.max(np.abs(G.dipole() - S.dipole())) <= 1e-12 * max(1.0, np.max(np.abs(S.dipole())))


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_fused_two_ions_smallest_lattice(prec):
    """Two opposite charges on the smallest lattice with the fused deposit
    (L = 16), 30 steps in one call, re-binning every 4 steps, moves of up to
    0.9 a that carry both ions across the periodic faces: one mover
    workgroup with two live threads, tiles with empty lists."""
    L = 16
    q = np.array([1.0, -1.0])
    r = np.array([[15.6, 0.3, 7.9], [0.2, 15.7, 8.4]])
    S, G = pair(L, q, r, dt=0.01, eps_min=3.0, precision=prec)
    apply_eps(S, G, "uniform", 3.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    memd.memd_set_options(G.ctx, 1, 4)
    assert memd.memd_counters(G.ctx)[1] == 1
    rng = np.random.default_rng(41)
    disp = rng.uniform(-0.9, 0.9, size=(30, 2, 3))
    G.step(disp, 30)
    for t in range(30):
        S.step(disp[t])
    fp32 = prec == memd.FP32_MIXED
    assert G.gauss_residual()[0] <= (fp32_gauss_bar(L, 1.0, q, r, S.r) if fp32 else 1e-12)
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= (1e-4 if fp32 else 1e-10)
    assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12 * L
    assert np.max(np.abs(S.r.reshape(-1, 3) - r)) > 1.0  # the ions did move


def test_fused_deposit_with_stale_bins():
    """Bins never refreshed (sort_every = 0) while ions drift several rows: the
    drifted ions fall back to the atomic path and the result stays exact."""
    L, n = 24, 300
    rng = np.random.default_rng(22)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, dt=0.01, eps_min=5.0)
    apply_eps(S, G, "uniform", 5.0)
    memd.memd_set_options(G.ctx, 1, 0)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.normal(0, 0.4, size=(25, n, 3))
    run_parity(S, G, disp, {5, 25}, 1e-10, 1e-12, 1e-10, audit_each=True)


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_dense_spread_with_drifted_ions(prec):
    """Ions stay in the bin order of the first step (re-binning every 1000
    steps) while they drift several rows: the charge assignment of every
    audit and the ion counts of the salt permittivity (every 3 steps) take
    the ions that left their bin rows through the atomic pass, and stay
    exact."""
    L, n = 24, 300
    rng = np.random.default_rng(23)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    S, G = pair(L, q, r, dt=0.01, eps_min=70.0, precision=prec)
    S.set_eps_salt()
    G.set_salt(80.0, 15.0, 1.0, every=3)
    memd.memd_set_options(G.ctx, 1, 1000)
    S.initial_solve(1e-13)
    share_state(S, G)
    fp32 = prec == memd.FP32_MIXED
    disp = rng.normal(0, 0.4, size=(24, n, 3))
    for t in range(24):
        if t % 3 == 0:
            S.set_eps_salt()
        S.step(disp[t])
        G.step(disp[t], 1)
        m, _ = G.gauss_residual()
        assert m <= (fp32_gauss_bar(L, 1.0, q, r, S.r) if fp32 else 1e-12), (t, m)
    drift = np.abs(G.state()[2].reshape(-1, 3) - r).max()
    assert drift > 2.0  # ions left their bin rows
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= (1e-4 if fp32 else 1e-10)
    if not fp32:
        errs = energy_err(G.energy(), S.energy())
        assert max(errs.values()) <= 1e-10, errs


@pytest.mark.parametrize("prec", [memd.FP32_MIXED, memd.FP64])
def test_fused_deposit_list_overflow(prec):
    """2000 ions packed into a 3 x 3 x 3 cell corner of a 32^3 lattice: the
    tile lists there overflow their capacity, the ions that did not fit are
    deposited by the atomic path, and the run still matches the oracle."""
    L, n = 32, 2000
    rng = np.random.default_rng(31)
    r = 30.5 + rng.uniform(0, 3.0, size=(n, 3))  # wraps across the periodic corner
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, dt=0.01, eps_min=10.0, precision=prec)
    apply_eps(S, G, "uniform", 10.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    memd.memd_set_tiling(G.ctx, 1, 8 if prec == memd.FP32_MIXED else 4)
    assert memd.memd_counters(G.ctx)[1] == 1
    disp = rng.normal(0, 0.05, size=(40, n, 3))
    G.step(disp, 40)
    for t in range(40):
        S.step(disp[t])
    # about 70 ions per cell: the FP32 bound scales with the vertex charge
    # magnitude (fp32_gauss_bar), the same rule as every other FP32 case
    fp32 = prec == memd.FP32_MIXED
    ftol, gtol = (1e-4, fp32_gauss_bar(L, 1.0, q, r, S.r)) if fp32 else (1e-10, 1e-12)
    m = G.gauss_residual()[0]
    record("list_overflow", precision="fp32" if fp32 else "fp64", gauss_max=m, gauss_bar=gtol,
           max_abs_q=1.0)
    assert m <= gtol
    Fo, _ = S.forces()
    assert force_err(G.forces(), Fo) <= ftol
    assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12 * np.max(np.abs(S.r))


def test_rejected_moves_are_counted_and_taken_as_zero():
    L, n = 16, 40
    rng = np.random.default_rng(23)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, dt=0.01, eps_min=3.0)
    apply_eps(S, G, "uniform", 3.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.normal(0, 0.05, size=(3, n, 3))
    disp[1, 3, 0] = np.nan
    disp[2, 7, 2] = 1e9
    clean = disp.copy()
    clean[1, 3, 0] = 0.0
    clean[2, 7, 2] = 0.0
    for t in range(3):
        S.step(clean[t])
        G.step(disp[t], 1)
    assert memd.memd_counters(G.ctx)[0] == 2
    assert force_err(G.forces(), S.forces()[0]) <= 1e-10
    assert G.gauss_residual()[0] <= 1e-12
