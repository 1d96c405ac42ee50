"""memd_gauss_residual_noalloc (the audit for callers that cannot allocate)
against memd_gauss_residual of a context holding the same state, and the
oracle: two calls in a row, the second on a smaller lattice with fewer ions
and FP32 fields, then the first input again with the result in host memory.
The fields carry planted violations of Gauss's law, so max and rms are far
from zero; both sides audit in FP64, so they agree to 1e-12 relative."""
import numpy as np
import pytest

from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, pair, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _case(L, n, prec, seed):
    """A context after a few steps (ions binned for L >= 16) whose field gets
    planted violations; returns its audit, the oracle's, and device copies of
    the charges, positions (caller order) and field."""
    import torch
    rng = np.random.default_rng(seed)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    S, G = pair(L, q, r, eps_min=4.0, precision=prec)
    apply_eps(S, G, "uniform", 4.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.normal(0, 0.1, size=(3, n, 3))
    G.step(disp, 3)
    for t in range(3):
        S.step(disp[t])
    D = S.D.copy()
    links = rng.choice(3 * L ** 3, 7, replace=False)
    D[links] += rng.uniform(0.05, 0.3, size=7) * rng.choice([-1.0, 1.0], size=7)
    fp32 = prec == memd.FP32_MIXED
    if fp32:
        D = D.astype(np.float32).astype(np.float64)
    S.set_state(D, S.B, S.r)
    G.set_state(D, None, None)
    ctx_audit = G.gauss_residual()
    rg = G.state()[2]
    G.close()
    dev = dict(q=torch.tensor(q, dtype=torch.float64, device="cuda"),
               r=torch.tensor(rg, dtype=torch.float64, device="cuda"),
               D=torch.tensor(D, dtype=torch.float32 if fp32 else torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return dict(L=L, n=n, prec=prec, ctx=ctx_audit, orc=S.gauss_residual(), dev=dev)


def _close(x, ref):
    return abs(x - ref) <= 1e-12 * abs(ref)


def test_noalloc_audit_matches_context_audit():
    import torch
    big = _case(40, 200, memd.FP64, 11)
    small = _case(12, 32, memd.FP32_MIXED, 12)
    out_dev = torch.zeros(2, dtype=torch.float64, device="cuda")
    d = big["dev"]
    memd.memd_gauss_residual_noalloc(40, 1.0, 200, d["q"], d["r"], d["D"], memd.FP64, out_dev)
    torch.cuda.synchronize()
    first = out_dev.cpu().numpy()
    out_host = np.zeros(2)
    d = small["dev"]
    memd.memd_gauss_residual_noalloc(12, 1.0, 32, d["q"], d["r"], d["D"], memd.FP32_MIXED, out_host)
    second = out_host.copy()
    d = big["dev"]
    memd.memd_gauss_residual_noalloc(40, 1.0, 200, d["q"], d["r"], d["D"], memd.FP64, out_host)
    third = out_host.copy()
    for res, case in ((first, big), (second, small), (third, big)):
        m, rms = case["ctx"]
        mo, rmso = case["orc"]
        assert mo >= 0.05 * 0.99  # the planted violations dominate
        assert _close(res[0], m) and _close(res[1], rms), (res, case["ctx"])
        assert _close(res[0], mo) and _close(res[1], rmso), (res, case["orc"])


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    q = torch.zeros(2, dtype=torch.float64, device="cuda")
    r = torch.zeros(6, dtype=torch.float64, device="cuda")
    D = torch.zeros(24, dtype=torch.float64, device="cuda")
    out = np.zeros(2)
    with pytest.raises(memd.MemdError) as e:
        memd.memd_gauss_residual_noalloc(129, 1.0, 2, q, r, D, memd.FP64, out)
    assert e.value.status == memd.ESIZE
    with pytest.raises(memd.MemdError) as e:  # host memory for the field
        memd.memd_gauss_residual_noalloc(2, 1.0, 2, q, r, np.zeros(24), memd.FP64, out)
    assert e.value.status == memd.EINVAL
