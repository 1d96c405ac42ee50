"""Parity at the full size of the timed workload: 128^3 lattice, 10^5 ions,
salt-dependent permittivity per link recomputed every 50 steps, in the launch
configuration the bench times (autotuned tile shape, the leapfrog with the
fused deposit and its ion movers, several steps per call so that the
finisher computes the forces of the state each step starts from and the
movers write the next step's records, re-binning and the permittivity
recompute every 50 steps, audit and energy at their cadence), over 63 steps
split into calls of 27 and 36 steps, so that the step-50 permittivity
recompute and re-binning run inside a call.

Both precisions start from the oracle's recursion solution (its CG
relaxation at 128^3 is a one-off outside the step) and take the same seeded
displacements; the oracle runs once for both.  Every force, position, the
dipole, the energies and the Gauss residual are compared, not a sample.
"""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from paper_1309_7859_amd import workloads as W
from tests.gpu_helpers import (energy_err, force_err, fp32_gauss_bar, output_errors, record,
                               require_gpu)

pytestmark = pytest.mark.gpu

CALLS = (27, 36)
STEPS = sum(CALLS)
CADENCE = 50    # permittivity recompute and re-binning, as in the bench
AUDIT = 9       # audit and energy histories inside the calls


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def c4_oracle():
    """The oracle's run of the 63 steps: its start state, the displacements,
    and the finished System with the Gauss residuals at the audit cadence."""
    w = W.WORKLOADS["c4"]
    s = W.make_system(w, steps=0)
    disp = W.DisplacementStream(w).take(STEPS)
    S = oracle.System(w.L, w.a, w.dt, 1.0, s["q"], s["r0"])
    S.set_eps_salt()
    S.c = W.default_c(w.a, w.dt, float(np.min(1.0 / S.eta)))
    S.recursion_only()
    start = S.state()
    gauss = []
    for t in range(STEPS):
        if t % CADENCE == 0:
            S.set_eps_salt()
        S.step(disp[t])
        if (t + 1) % AUDIT == 0:
            gauss.append(S.gauss_residual()[0])
    return dict(w=w, s=s, disp=disp, S=S, start=start, gauss=gauss)


@pytest.mark.parametrize("prec", [memd.FP32_MIXED, memd.FP64])
def test_c4_full_size_parity(prec, c4_oracle):
    w, s, disp, S = c4_oracle["w"], c4_oracle["s"], c4_oracle["disp"], c4_oracle["S"]
    D0, B0, r0 = c4_oracle["start"]
    G = memd.Context(w.L, s["q"], s["r0"], a=w.a, dt=w.dt, c=S.c, precision=prec,
                     audit_every=AUDIT, energy_every=AUDIT)
    try:
        G.set_salt(80.0, 15.0, 1.0, every=CADENCE)
        G.set_state(D0, B0, r0)
        memd.memd_autotune(G.ctx, 3, None)
        memd.memd_set_options(G.ctx, 1, CADENCE)
        assert memd.memd_counters(G.ctx)[1] == 1  # the fused path, as in the bench
        G.step(disp[:CALLS[0]], CALLS[0])
        G.step(disp[CALLS[0]:], CALLS[1])
        fp32 = prec == memd.FP32_MIXED
        ftol, etol = (1e-4, 1e-4) if fp32 else (1e-10, 1e-10)
        gtol = fp32_gauss_bar(w.L, w.a, s["q"], r0, S.r) if fp32 else 1e-12
        D, B, r = G.state()
        audits, energies = G.history()
        err = output_errors(G, S)
        record("c4", precision="fp32" if fp32 else "fp64", steps=STEPS, gauss_bar=gtol,
               audit_history_max=float(np.max(audits[:, 0])), **err)
        assert err["position"] <= 1e-12
        assert err["force"] <= ftol, err
        assert err["dipole"] <= 1e-12
        assert len(audits) == STEPS // AUDIT and len(energies) == STEPS // AUDIT
        assert np.all(audits[:, 0] <= gtol), audits
        assert max(c4_oracle["gauss"]) <= 1e-12
        assert err["gauss_max"] <= gtol
        errs = energy_err(G.energy(), S.energy())
        assert max(errs.values()) <= etol, errs
        E = S.eta * D
        Eo = S.eta * S.D
        assert np.max(np.abs(E - Eo)) <= (1e-4 if fp32 else 1e-10) * np.max(np.abs(Eo))
    finally:
        G.close()


def test_c4_initial_solve_at_full_size():
    """The FP64 initial solve at 128^3 with 10^5 ions and the salt
    permittivity (CG relaxation, 600+ iterations), checked with the oracle's
    operators: the relaxed field is the unique minimiser of the field energy
    over the fields that obey Gauss's law with mean D = -P/V (the paragraph
    after the recursion; section "Periodicity"), so it is pinned at any size by
    those three properties: the Gauss residual at round-off, the mean, and a
    curl-free E = eta D (a max|C(eta D)| / max|eta D| within the solve's
    tolerance, measured by the oracle)."""
    w = W.WORKLOADS["c4"]
    s = W.make_system(w, steps=0)
    S = oracle.System(w.L, w.a, w.dt, 1.0, s["q"], s["r0"])
    S.set_eps_salt()
    S.c = W.default_c(w.a, w.dt, float(np.min(1.0 / S.eta)))
    G = memd.Context(w.L, s["q"], s["r0"], a=w.a, dt=w.dt, c=S.c, precision=memd.FP64)
    try:
        G.set_salt(80.0, 15.0, 1.0, every=0)
        st, iters, res = G.solve(1e-12)
        assert st == memd.OK and iters > 0 and res <= 1e-12
        D, B, r = G.state()
        assert np.max(np.abs(B)) == 0.0
        S.set_state(D, B, r)
        curl = S.curl_measure()
        gmax, _ = S.gauss_residual()
        P = S.dipole()
        mean = D.reshape(3, -1).mean(axis=1)
        record("c4_solve", iterations=iters, gpu_curl=res, oracle_curl=curl, gauss=gmax)
        assert curl <= 1.01e-12, curl
        assert gmax <= 1e-12, gmax
        assert np.max(np.abs(mean + P / S.V)) <= 1e-12 * max(1.0, np.max(np.abs(P / S.V)))
    finally:
        G.close()
