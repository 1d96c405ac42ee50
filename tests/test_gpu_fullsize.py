"""Parity at the full size of the timed workload: 128^3 lattice, 10^5 ions,
salt-dependent permittivity per link recomputed every 50 steps, in the launch
configuration the bench times (autotuned tile shape, the leapfrog with the
fused deposit and its ion movers, several steps per call so that the
finisher computes the forces of the state each step starts from and the
movers write the next step's records), with the ions re-binned every 8
steps and the run split over two calls, so that records are built by the
re-binning, by the pack at a call's start and by the movers, on both
record sets.

Both sides start from the oracle's recursion solution (its CG relaxation at
128^3 is a one-off outside the step) and take the same seeded displacements.
Every force, position, the dipole, the energies and the Gauss residual are
compared, not a sample: the oracle runs these 20 steps in seconds.
"""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from paper_1309_7859_amd import workloads as W
from tests.gpu_helpers import energy_err, force_err, require_gpu

pytestmark = pytest.mark.gpu

STEPS = 20
SPLIT = 7  # the first call's steps
CADENCE = 10


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("prec", [memd.FP32_MIXED, memd.FP64])
def test_c4_full_size_parity(prec):
    w = W.WORKLOADS["c4"]
    s = W.make_system(w, steps=0)
    disp = W.DisplacementStream(w).take(STEPS)
    S = oracle.System(w.L, w.a, w.dt, 1.0, s["q"], s["r0"])
    S.set_eps_salt()
    S.c = W.default_c(w.a, w.dt, float(np.min(1.0 / S.eta)))
    S.recursion_only()
    D0, B0, r0 = S.state()
    G = memd.Context(w.L, s["q"], s["r0"], a=w.a, dt=w.dt, c=S.c, precision=prec,
                     audit_every=CADENCE, energy_every=CADENCE)
    try:
        G.set_salt(80.0, 15.0, 1.0, every=50)
        G.set_state(D0, B0, r0)
        memd.memd_autotune(G.ctx, 3, None)
        memd.memd_set_options(G.ctx, 1, 8)
        assert memd.memd_counters(G.ctx)[1] == 1  # the fused path, as in the bench
        G.step(disp[:SPLIT], SPLIT)
        G.step(disp[SPLIT:], STEPS - SPLIT)
        gauss = []
        for t in range(STEPS):
            if t % 50 == 0:
                S.set_eps_salt()
            S.step(disp[t])
            if (t + 1) % CADENCE == 0:
                gauss.append(S.gauss_residual()[0])
        Fo, _ = S.forces()
        F = G.forces()
        D, B, r = G.state()
        audits, energies = G.history()
        fp32 = prec == memd.FP32_MIXED
        ftol, gtol, etol = (1e-4, 2e-5, 1e-4) if fp32 else (1e-10, 1e-12, 1e-10)
        assert np.max(np.abs(r - S.r)) <= 1e-12 * max(1.0, np.max(np.abs(S.r)))
        assert force_err(F, Fo) <= ftol
        P, Po = G.dipole(), S.dipole()
        assert np.max(np.abs(P - Po)) <= 1e-12 * max(1.0, np.max(np.abs(Po)))
        assert len(audits) == STEPS // CADENCE and len(energies) == STEPS // CADENCE
        assert np.all(audits[:, 0] <= gtol), audits
        assert max(gauss) <= 1e-12
        m, _ = G.gauss_residual()
        assert m <= gtol
        errs = energy_err(G.energy(), S.energy())
        assert max(errs.values()) <= etol, errs
        E = S.eta * D
        Eo = S.eta * S.D
        assert np.max(np.abs(E - Eo)) <= (1e-4 if fp32 else 1e-10) * np.max(np.abs(Eo))
    finally:
        G.close()
