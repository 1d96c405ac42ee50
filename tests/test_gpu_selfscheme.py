"""The direct self subtraction (memd_set_self_scheme(MEMD_SELF_DIRECT),
section "Self energy interaction") against the oracle's: a per-link random
permittivity (every cell's edges differ), on the fused path (L = 16, the
finisher gathers every force) and the plain one (L = 12), FP64 and FP32, over
two calls and back to the Green's-function scheme; and ions inside the cells
that straddle a dielectric wall, where the two schemes differ most."""
import numpy as np
import pytest

from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, energy_err, force_err, pair, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("prec,L", [(memd.FP64, 16), (memd.FP32_MIXED, 16), (memd.FP64, 12)])
def test_direct_scheme_matches_oracle(prec, L):
    n = 48
    rng = np.random.default_rng(70 + L)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    el = 1.5 + 6.5 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, eps_min=el.min(), precision=prec)
    apply_eps(S, G, "link", eps_link=el)
    S.initial_solve(1e-13)
    share_state(S, G)
    memd.memd_set_options(G.ctx, 1, 4)
    assert memd.memd_counters(G.ctx)[1] == (1 if L >= 16 else 0)
    fp32 = prec == memd.FP32_MIXED
    ftol, etol = (1e-4, 1e-4) if fp32 else (1e-10, 1e-10)
    Fg = S.forces()[0]
    S.self_scheme = "direct"
    G.set_self_scheme(memd.SELF_DIRECT)
    Fd = S.forces()[0]
    assert force_err(Fd, Fg) > 1e-3  # the schemes differ on this permittivity
    assert force_err(G.forces(), Fd) <= ftol
    for k in (5, 8):
        disp = rng.normal(0, 0.1, size=(k, n, 3))
        G.step(disp, k)
        for t in range(k):
            S.step(disp[t])
        assert force_err(G.forces(), S.forces()[0]) <= ftol
        errs = energy_err(G.energy(), S.energy())
        assert max(errs.values()) <= etol, errs
    S.self_scheme = "green"
    G.set_self_scheme(memd.SELF_GREEN)
    assert force_err(G.forces(), S.forces()[0]) <= ftol
    disp = rng.normal(0, 0.1, size=(3, n, 3))
    G.step(disp, 3)
    for t in range(3):
        S.step(disp[t])
    assert force_err(G.forces(), S.forces()[0]) <= ftol


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_direct_scheme_at_a_wall(prec):
    """Ions inside and beside the cells that straddle the walls of a water
    slab (eps 80 on the vertex planes 1..20 of 32, eps 2 elsewhere)."""
    L = 32
    ez = np.full(L, 2.0)
    ez[1:21] = 80.0
    xs = [8.1, 8.25, 8.4, 12.2, 16.35, 20.45]
    zs = [0.7, 0.9, 1.3, 20.3, 20.7, 10.3]
    r = np.array([[x, 8.5 + 3 * i, z] for i, (x, z) in enumerate(zip(xs, zs))])
    q = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    S, G = pair(L, q, r, eps_min=2.0, precision=prec)
    apply_eps(S, G, "zsite", eps_z=ez)
    S.initial_solve(1e-12)
    share_state(S, G)
    S.self_scheme = "direct"
    G.set_self_scheme(memd.SELF_DIRECT)
    fp32 = prec == memd.FP32_MIXED
    assert force_err(G.forces(), S.forces()[0]) <= (1e-4 if fp32 else 1e-10)
    zero = np.zeros((10, 6, 3))
    G.step(zero, 10)
    for t in range(10):
        S.step(zero[t])
    assert force_err(G.forces(), S.forces()[0]) <= (1e-4 if fp32 else 1e-10)
