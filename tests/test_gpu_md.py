"""The ions' own dynamics (memd_md_step: velocity Verlet under the MEMD
forces) against the oracle's System.md_step on the same start: positions,
velocities, forces and energies after several calls, on the fused path (with
re-binning inside a call) and the plain one, FP64 and FP32 fields; and the
conserved total K + E_corrected on the GPU."""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, energy_err, force_err, fp32_gauss_bar, pair, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _system(L, n, prec, seed):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    eps = 2.0 + 6.0 * rng.uniform(size=L ** 3)
    S, G = pair(L, q, r, dt=0.01, eps_min=2.0, precision=prec)
    apply_eps(S, G, "site", eps_site=eps)
    S.initial_solve(1e-13)
    share_state(S, G)
    m = rng.uniform(20.0, 60.0, size=n)
    v = rng.normal(0, 0.05, size=(n, 3))
    return S, G, m, v


@pytest.mark.parametrize("prec,L,fused", [(memd.FP64, 16, 1), (memd.FP32_MIXED, 16, 1), (memd.FP64, 8, 0)])
def test_md_matches_oracle(prec, L, fused):
    n = 48
    S, G, m, v0 = _system(L, n, prec, 50 + L)
    try:
        memd.memd_set_options(G.ctx, 1, 4)
        assert memd.memd_counters(G.ctx)[1] == fused
        vg = v0.copy()
        vo = v0.copy()
        for k in (6, 9, 10):  # three calls
            G.md_step(vg, m, k)
            for _ in range(k):
                S.md_step(vo, m)
        fp32 = prec == memd.FP32_MIXED
        Fo, _ = S.forces()
        assert force_err(G.forces(), Fo) <= (1e-4 if fp32 else 1e-10)
        vrms = np.sqrt(np.mean(vo ** 2))
        assert np.max(np.abs(vg - vo)) <= (1e-5 if fp32 else 1e-11) * vrms
        assert np.max(np.abs(G.state()[2] - S.r)) <= (1e-8 if fp32 else 1e-12 * L)
        assert G.gauss_residual()[0] <= (fp32_gauss_bar(L, 1.0, S.q, S.r) if fp32 else 1e-12)
        if not fp32:
            errs = energy_err(G.energy(), S.energy())
            assert max(errs.values()) <= 1e-10, errs
    finally:
        G.close()


def test_md_device_velocities_and_energy_conservation():
    """Velocities and masses in device memory give the host-memory result;
    with uniform permittivity and ions crossing many cell faces the GPU run
    keeps K + E_corrected as the oracle does (FP64 fields)."""
    import torch
    L, n = 16, 48
    rng = np.random.default_rng(78)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, dt=0.01, eps_min=4.0)
    apply_eps(S, G, "uniform", 4.0)
    c = S.c
    H = memd.Context(L, q, r, c=c, precision=memd.FP64)
    try:
        S.initial_solve(1e-13)
        share_state(S, G)
        H.set_permittivity(memd.EPS_UNIFORM, [4.0])
        H.set_state(*S.state())
        m = np.full(n, 30.0)
        v0 = rng.normal(0, 0.3, size=(n, 3))
        vd = torch.from_numpy(v0.copy()).to("cuda")
        md = torch.from_numpy(m.copy()).to("cuda")
        vh = v0.copy()
        vo = v0.copy()
        tot, toto = [], []
        for _ in range(6):
            G.md_step(vd, md, 25)
            H.md_step(vh, m, 25)
            for _ in range(25):
                S.md_step(vo, m)
            torch.cuda.synchronize()
            tot.append(0.5 * float(np.sum(m[:, None] * vh * vh)) + H.energy()["E_corrected"])
            toto.append(0.5 * float(np.sum(m[:, None] * vo * vo)) + S.energy()["E_corrected"])
        vrms = np.sqrt(np.mean(vo ** 2))
        assert np.max(np.abs(vd.cpu().numpy() - vh)) <= 1e-13 * vrms
        assert np.max(np.abs(G.state()[2] - H.state()[2])) <= 1e-12 * L
        assert np.max(np.abs(vh - vo)) <= 1e-10 * vrms
        tot, toto = np.array(tot), np.array(toto)
        assert np.max(np.abs(tot - toto)) <= 1e-10 * abs(toto[0])
        assert np.max(np.abs(H.state()[2].reshape(-1, 3) - r)) > 1.0  # ions crossed cell faces
        assert np.ptp(tot) <= 2e-5 * abs(tot[0])
    finally:
        G.close()
        H.close()


def test_md_error_codes():
    """Before a state exists, with missing buffers, non-positive or non-finite
    host masses, or a negative step count, memd_md_step refuses and leaves the
    context usable."""
    L = 8
    q = np.array([1.0, -1.0])
    r = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    v = np.zeros((2, 3))
    G = memd.Context(L, q, r)
    try:
        with pytest.raises(memd.MemdError) as e:
            G.md_step(v, np.ones(2), 1)
        assert e.value.status == memd.ESTATE
        G.set_permittivity(memd.EPS_UNIFORM, [2.0])
        G.solve(1e-12)
        for mass in (np.array([1.0, 0.0]), np.array([1.0, -2.0]), np.array([1.0, np.nan])):
            with pytest.raises(memd.MemdError) as e:
                G.md_step(v, mass, 1)
            assert e.value.status == memd.EINVAL
        with pytest.raises(memd.MemdError) as e:
            memd.memd_md_step(G.ctx, None, np.ones(2), 1)
        assert e.value.status == memd.EINVAL
        with pytest.raises(memd.MemdError) as e:
            G.md_step(v, np.ones(2), -1)
        assert e.value.status == memd.EINVAL
        G.md_step(v, np.ones(2), 0)  # nothing to do
        v[0, 0] = 0.1
        G.md_step(v, np.ones(2), 3)  # still usable
        assert G.gauss_residual()[0] <= 1e-12
    finally:
        G.close()
