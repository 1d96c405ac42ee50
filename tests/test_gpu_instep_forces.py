"""The forces each step computes inside itself on the fused path (eq. force)
against the oracle.  With the Green's-function self energy a step is one
launch: its tiles compute the lattice part and the self force of every ion
whose start cell they own (the atomic-path ions and those beyond a tile's
LDS list gathered from D^n), and the movers of the next launch add the
dipole term; with the direct subtraction the finisher computes them after
the leapfrog.  memd_step normally ends with one more force launch for the
final state, which hides them; memd_set_final_forces(0) skips it, so that
memd_forces returns the newest forces a step completed: those of the state
two steps before the end (one step before, with the direct subtraction)."""
import numpy as np
import pytest

from paper_1309_7859_amd import memd
from tests.gpu_helpers import apply_eps, force_err, pair, record, require_gpu, share_state

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _check(S, G, disp, ftol, label, prec, lag=2):
    """Steps both sides through disp; the GPU with its final force launch
    off must hold the oracle's forces of the state `lag` steps before the end."""
    k = disp.shape[0]
    G.set_final_forces(False)
    G.step(disp, k)
    for t in range(k - lag):
        S.step(disp[t])
    F_before = S.forces()[0]
    err = force_err(G.forces(), F_before)
    for t in range(k - lag, k):
        S.step(disp[t])
    G.set_final_forces(True)
    record("instep_forces", label=label, precision="fp32" if prec == memd.FP32_MIXED else "fp64", force_err=err)
    assert err <= ftol, (label, err)
    # the state itself is the same either way: the next call (final forces
    # on) ends with the final state's forces
    G.step(np.zeros((1,) + disp.shape[1:]), 1)
    S.step(np.zeros(disp.shape[1:]))
    assert force_err(G.forces(), S.forces()[0]) <= ftol


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_instep_forces_link_eps(prec):
    """Random per-link permittivity, L = 16 (fused path), 6 steps."""
    L, n = 16, 60
    rng = np.random.default_rng(81)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0, 2.0, -2.0], n // 4)
    el = 2.0 + 6.0 * rng.uniform(size=3 * L ** 3)
    S, G = pair(L, q, r, eps_min=el.min(), precision=prec)
    apply_eps(S, G, "link", eps_link=el)
    S.initial_solve(1e-13)
    share_state(S, G)
    assert memd.memd_counters(G.ctx)[1] == 1
    disp = rng.normal(0, 0.1, size=(6, n, 3))
    _check(S, G, disp, 1e-4 if prec == memd.FP32_MIXED else 1e-10, "link16", prec)


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_instep_forces_irregular_and_crowded(prec):
    """Ions the tiles do not take: 2000 ions in a 3 x 3 x 3 cell corner of a
    32^3 lattice (more than a tile holds, lists overflowing) and moves of
    more than a lattice spacing (the atomic path), with the direct self
    subtraction off and on."""
    L, n = 32, 2000
    rng = np.random.default_rng(82)
    r = 30.5 + rng.uniform(0, 3.0, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, dt=0.01, eps_min=10.0, precision=prec)
    apply_eps(S, G, "uniform", 10.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    memd.memd_set_tiling(G.ctx, 1, 8 if prec == memd.FP32_MIXED else 4)
    assert memd.memd_counters(G.ctx)[1] == 1
    disp = rng.normal(0, 0.05, size=(5, n, 3))
    disp[:, ::97, :] *= 40.0  # every 97th ion jumps about 2 a
    ftol = 1e-4 if prec == memd.FP32_MIXED else 1e-10
    _check(S, G, disp, ftol, "crowded", prec)
    S.self_scheme = "direct"
    G.set_self_scheme(memd.SELF_DIRECT)
    disp = rng.normal(0, 0.05, size=(4, n, 3))
    _check(S, G, disp, ftol, "crowded_direct", prec, lag=1)


def test_instep_forces_first_step_of_a_call():
    """A call of one step completes no forces inside it: with the final
    launch off, the forces stay those the previous call (here the state's
    upload) left, of the state the step started from."""
    L, n = 16, 40
    rng = np.random.default_rng(83)
    r = rng.uniform(0, L, size=(n, 3))
    q = np.tile([1.0, -1.0], n // 2)
    S, G = pair(L, q, r, eps_min=4.0)
    apply_eps(S, G, "uniform", 4.0)
    S.initial_solve(1e-13)
    share_state(S, G)
    disp = rng.normal(0, 0.1, size=(1, n, 3))
    G.set_final_forces(False)
    G.step(disp, 1)
    assert force_err(G.forces(), S.forces()[0]) <= 1e-10
    assert memd.load().memd_set_final_forces(G.ctx, 2) == memd.EINVAL
