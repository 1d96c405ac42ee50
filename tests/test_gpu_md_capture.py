"""The ions' own dynamics on the fused path, where the leapfrog tiles capture
E = eta D of the new state on the 12 links of the cell each move ends in and
the ion kernel forms the forces from those values instead of gathering the
field: against the oracle's System.md_step (velocity Verlet under the MEMD
forces) where the tiles' capture lists overflow (ions packed into a few
cells, gathered instead), where moves longer than a cell take the atomic
path (captured from the tiles' list of them), on lattices whose side is not
a multiple of the tile, and with the direct self subtraction (which gathers
every force)."""
import numpy as np
import pytest

from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, fp32_gauss_bar, force_err, pair, record, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _run(name, L, r, q, m, v0, prec, calls, rebin=4, direct=False, seed=0, tile=None):
    rng = np.random.default_rng(seed)
    eps = 2.0 + 6.0 * rng.uniform(size=L ** 3)
    S, G = pair(L, q, r, dt=0.01, eps_min=2.0, precision=prec)
    try:
        apply_eps(S, G, "site", eps_site=eps)
        if direct:
            S.self_scheme = "direct"
            G.set_self_scheme(memd.SELF_DIRECT)
        S.initial_solve(1e-13)
        share_state(S, G)
        memd.memd_set_options(G.ctx, 1, rebin)
        if tile:
            memd.memd_set_tiling(G.ctx, *tile)
        assert memd.memd_counters(G.ctx)[1] == 1  # the fused path
        vg, vo = v0.copy(), v0.copy()
        for k in calls:
            G.md_step(vg, m, k)
            for _ in range(k):
                S.md_step(vo, m)
        fp32 = prec == memd.FP32_MIXED
        Fo, _ = S.forces()
        fe = force_err(G.forces(), Fo)
        vrms = np.sqrt(np.mean(vo ** 2))
        ve = np.max(np.abs(vg - vo)) / vrms
        pe = np.max(np.abs(G.state()[2] - S.r))
        gm = G.gauss_residual()[0]
        record(name, force=fe, velocity=ve, position=pe, gauss=gm)
        assert fe <= (1e-4 if fp32 else 1e-10), fe
        assert ve <= (1e-5 if fp32 else 1e-11), ve
        assert pe <= (1e-8 if fp32 else 1e-12 * L), pe
        assert gm <= (fp32_gauss_bar(L, 1.0, S.q, S.r, r) if fp32 else 1e-12), gm
        return S, G
    finally:
        G.close()


@pytest.mark.parametrize("prec,tile", [(memd.FP64, (1, 4)), (memd.FP32_MIXED, (1, 8)), (memd.FP32_MIXED, (2, 4))])
def test_md_capture_overflowing_lists(prec, tile):
    """768 of 1024 ions packed into 27 cells: the tiles' deposit lists and
    capture lists overflow, so most ions take the atomic path and many forces
    are gathered rather than captured."""
    L, n = 16, 1024
    rng = np.random.default_rng(310)
    r = np.concatenate([rng.uniform(2.0, 5.0, size=(768, 3)), rng.uniform(0, L, size=(256, 3))])
    q = np.tile([1.0, -1.0], n // 2)
    m = rng.uniform(20.0, 60.0, size=n)
    v = rng.normal(0, 0.05, size=(n, 3))
    _run("md_capture_overflow", L, r, q, m, v, prec, (5, 7), seed=311, tile=tile)


@pytest.mark.parametrize("prec,tile", [(memd.FP64, (1, 4)), (memd.FP32_MIXED, (1, 8)), (memd.FP32_MIXED, (2, 4))])
def test_md_capture_long_moves(prec, tile):
    """Every 8th ion moves about 1.5 cells a step (the atomic path, whose end
    cells the tiles find from the irregular list), the rest slowly."""
    L, n = 16, 96
    rng = np.random.default_rng(320)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    m = rng.uniform(20.0, 60.0, size=n)
    v = rng.normal(0, 0.05, size=(n, 3))
    v[::8] = rng.normal(0, 90.0, size=(n // 8, 3))
    _run("md_capture_long_moves", L, r, q, m, v, prec, (6, 9), seed=321, tile=tile)


@pytest.mark.parametrize("prec,L,tile", [(memd.FP64, 20, (1, 4)), (memd.FP32_MIXED, 20, (1, 8)),
                                         (memd.FP32_MIXED, 27, (2, 4)), (memd.FP64, 27, (1, 4))])
def test_md_capture_ragged_lattices(prec, L, tile):
    """Lattice sides that leave the last tile partly outside along x, y and z."""
    n = 80
    rng = np.random.default_rng(330 + L)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    m = rng.uniform(20.0, 60.0, size=n)
    v = rng.normal(0, 0.2, size=(n, 3))
    _run(f"md_capture_L{L}", L, r, q, m, v, prec, (5, 8), rebin=3, seed=331, tile=tile)


def test_md_direct_scheme_gathers():
    """With the direct self subtraction the ion kernel gathers every force
    (the tiles capture nothing) and still follows the oracle."""
    L, n = 16, 64
    rng = np.random.default_rng(340)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    m = rng.uniform(20.0, 60.0, size=n)
    v = rng.normal(0, 0.1, size=(n, 3))
    _run("md_direct", L, r, q, m, v, memd.FP64, (4, 6), direct=True, seed=341)
