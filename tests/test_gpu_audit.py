"""The Gauss audit measures real violations of Gauss's law.

After the recursion (section "Extension of the algorithm") Gauss's law holds
by construction and every later update keeps it, so a correct run leaves the
audit near zero, and the parity tests can only bound it from above.  Here a
field with known violations is uploaded with memd_set_state: a few links get
an extra amount delta, which moves R_v = a^2 div D(v) - q_v by +a^2 delta at
the link's lower end and by -a^2 delta at its upper end.  The audit's max|R|
and rms R must then equal the oracle's on the same field and positions to
1e-12 relative, in FP64 and in FP32 (the FP32 field is the oracle's rounded
to FP32 on both sides, so both audit the same values), with the charge
assignment done by the atomic pass (ions in the caller's order) and by the
tile pass over binned ions (L >= 16 after a step).
"""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, pair, record, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("prec,L,binned", [(memd.FP64, 12, False), (memd.FP32_MIXED, 12, False),
                                           (memd.FP64, 24, True), (memd.FP32_MIXED, 24, True),
                                           (memd.FP32_MIXED, 33, True)])
def test_audit_reports_known_violation(prec, L, binned):
    rng = np.random.default_rng(100 + L)
    n = 60
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    S, G = pair(L, q, r, eps_min=3.0, precision=prec)
    apply_eps(S, G, "uniform", 3.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    if binned:
        # a few steps on both sides: the context then holds its ions in bin order
        disp = rng.normal(0, 0.1, size=(3, n, 3))
        G.step(disp, 3)
        for t in range(3):
            S.step(disp[t])
        assert np.max(np.abs(G.state()[2] - S.r)) <= 1e-12 * L
    Ns = L ** 3
    D = S.D.copy()
    links = rng.choice(3 * Ns, 9, replace=False)
    delta = rng.uniform(0.05, 0.4, size=9) * rng.choice([-1.0, 1.0], size=9)
    D[links] += delta
    if prec == memd.FP32_MIXED:
        D = D.astype(np.float32).astype(np.float64)
    S.set_state(D, S.B, S.r)
    G.set_state(D, None, None)  # the context keeps its own (binned) positions
    m, rms = G.gauss_residual()
    mo, rmso = S.gauss_residual()
    record("audit_violation", precision="fp32" if prec == memd.FP32_MIXED else "fp64", L=L,
           binned=binned, gpu_max=m, oracle_max=mo, gpu_rms=rms, oracle_rms=rmso)
    # the planted amounts dominate: max|R| is at least the smallest |delta|
    assert mo >= 0.05 * 0.99
    assert abs(m - mo) <= 1e-12 * mo, (m, mo)
    assert abs(rms - rmso) <= 1e-12 * rmso, (rms, rmso)


def test_audit_history_reports_violation():
    """The audits that run inside memd_step record the residual of the state
    they see: a violation planted before the call persists (the leapfrog and
    the deposit keep div D - rho unchanged), so every history entry equals
    the oracle's residual of the same trajectory."""
    L, n = 16, 40
    rng = np.random.default_rng(7)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, eps_min=2.0, audit_every=2)
    apply_eps(S, G, "uniform", 2.0)
    S.initial_solve(1e-13)
    D = S.D.copy()
    D[5] += 0.25
    D[3 * L ** 3 - 7] -= 0.125
    S.set_state(D, S.B, S.r)
    share_state(S, G)
    disp = rng.normal(0, 0.05, size=(6, n, 3))
    G.step(disp, 6)
    ref = []
    for t in range(6):
        S.step(disp[t])
        if (t + 1) % 2 == 0:
            ref.append(S.gauss_residual())
    A, _ = G.history()
    assert A.shape == (3, 2)
    for (m, rms), (mo, rmso) in zip(A, ref):
        assert mo >= 0.25 * 0.99
        assert abs(m - mo) <= 1e-12 * mo and abs(rms - rmso) <= 1e-12 * rmso
