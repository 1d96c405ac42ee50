"""The dielectric-walls check of section "Validation" (Fig. 6) on the GPU: a
+1/-1 pair inside a water slab (eps_W = 80, vertex planes 1..20 of a 32^3
periodic box) between walls of eps_C = 2 (the other planes), dragged slowly
from the slab's centre towards the lower wall under the MEMD dynamics and held
still for 1000 steps at 6, 4 and 2 lattice spacings from it.  The GPU run
(FP64 and FP32 fields, planar permittivity) matches the oracle's force and
positions at the end of every rest, and the mean force of each rest (second
half) is the analytic multiple-image force within 5 %, as the oracle's is."""
import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from tests.gpu_helpers import force_err, record, require_gpu

pytestmark = pytest.mark.gpu

L, EW, EC = 32, 80.0, 2.0
Z_LO, Z_HI = 0.5, 20.5
CHECKPOINTS = (6.5, 4.5, 2.5)
REST, SPEED, NU, DT = 1000, 0.002, 0.9, 0.01


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _profile():
    ez = np.full(L, EC)
    ez[1:21] = EW
    return ez


def _analytic(z0):
    return oracle.wall_image_force_z([(1.0, 8.5, 8.5), (-1.0, 24.5, 24.5)], z0, Z_LO, Z_HI, EW, EC,
                                     period=L, lateral=30)


def _legs():
    """(displacement per step, steps) of each drag leg, from z = 10.5."""
    z, legs = 10.5, []
    for zc in CHECKPOINTS:
        nst = int(round((z - zc) / SPEED))
        legs.append((-(z - zc) / nst, nst))
        z = zc
    return legs


@pytest.fixture(scope="module")
def wall_oracle():
    r0 = np.array([[8.5, 8.5, 10.5], [24.5, 24.5, 10.5]])
    c = oracle.default_c(1.0, DT, EC, NU)
    S = oracle.System(L, 1.0, DT, c, [1.0, -1.0], r0)
    S.set_eps_zsite(_profile())
    assert S.initial_solve(1e-12)[0] == 0
    start = S.state()
    out = []
    for dz, nst in _legs():
        dd = np.zeros((2, 3))
        dd[:, 2] = dz
        for _ in range(nst):
            S.step(dd)
        f = []
        for _ in range(REST):
            S.step(np.zeros((2, 3)))
            f.append(S.forces()[0][0, 2])
        out.append(dict(F=S.forces()[0], r=S.r.copy(), mean=float(np.mean(f[REST // 2:]))))
    return dict(c=c, start=start, r0=r0, cps=out)


@pytest.mark.parametrize("prec", [memd.FP64, memd.FP32_MIXED])
def test_dielectric_walls_drag(prec, wall_oracle):
    fp32 = prec == memd.FP32_MIXED
    G = memd.Context(L, np.array([1.0, -1.0]), wall_oracle["r0"], dt=DT, c=wall_oracle["c"], precision=prec)
    try:
        G.set_permittivity(memd.EPS_ZSITE, _profile())
        G.set_state(*wall_oracle["start"])
        zero = np.zeros((2, 3))
        for (dz, nst), ref in zip(_legs(), wall_oracle["cps"]):
            d = np.zeros((nst, 2, 3))
            d[:, :, 2] = dz
            G.step(d, nst)
            f = []
            for _ in range(REST):
                G.step(zero, 1)
                f.append(G.forces()[0, 2])
            F = G.forces()
            assert force_err(F, ref["F"]) <= (1e-4 if fp32 else 1e-10)
            assert np.max(np.abs(G.state()[2] - ref["r"])) <= 1e-12 * L
            mean = float(np.mean(f[REST // 2:]))
            z0 = ref["r"][2]
            pred = _analytic(z0)
            record("walls", precision="fp32" if fp32 else "fp64", z0=z0, distance=z0 - Z_LO, gpu_mean=mean,
                   oracle_mean=ref["mean"], analytic=pred)
            assert abs(mean - pred) <= 0.05 * pred, (z0, mean, pred)
            assert abs(mean - ref["mean"]) <= (1e-3 if fp32 else 1e-9) * pred
    finally:
        G.close()
