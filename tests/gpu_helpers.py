"""Helpers shared by the GPU tests: building matching oracle and HIP systems
from the same seeded inputs, the parity metrics, and a recorder of measured
errors."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from paper_1309_7859_amd import memd
from paper_1309_7859_amd import workloads as W


def require_gpu():
    try:
        import torch
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
    except ImportError:
        pytest.skip("no torch")
    memd.load()


def force_err(F, Fref):
    """max_i |F_i - Fref_i| / RMS_i |Fref_i|."""
    rms = np.sqrt(np.mean(np.sum(Fref ** 2, axis=1)))
    return np.max(np.abs(F - Fref)) / rms


def fp32_gauss_bar(L, a, q, *positions):
    """Gauss-residual bound of the FP32-field path: 1e-5 per unit of the
    largest vertex charge magnitude, max(max_i |q_i|, max_v sum_i |q_i| w_v(r_i))
    over the given position sets (w_v the linear assignment weights).

    Why this scale: the audit is FP64 arithmetic on FP32-stored D, so its
    residual is the sum, over the six links of a vertex, of the rounding
    errors those stored values carry.  Each step rounds a link once in the
    leapfrog store and once per ion whose current lands on it, each time by
    at most half an ulp of |D|; the number of depositing ions at a vertex
    grows with sum_i |q_i| w_v / max|q|.  For dilute ions the bound is
    1e-5 max|q| times a factor of order 1 (1.6 at 32^3 with 1000 ions)."""
    qa = np.abs(np.asarray(q, dtype=np.float64))
    if qa.size == 0:
        return 1e-5
    qv = max(float(np.max(oracle.spread(L, a, qa, r))) for r in positions) if positions else 0.0
    return 1e-5 * max(float(qa.max()), qv)


def record(name, **values):
    """Append measured errors of one case to the JSON-lines file named by
    MEMD_PARITY_LOG (nothing when it is unset)."""
    path = os.environ.get("MEMD_PARITY_LOG")
    if not path:
        return
    row = {"case": name}
    for k, v in values.items():
        row[k] = v.tolist() if isinstance(v, np.ndarray) else v
    with open(path, "a") as f:
        f.write(json.dumps(row) + "\n")


def output_errors(G, S):
    """Every output of a run against the oracle: force max|dF|/RMS F, the
    relative error of each energy term (W_B also, and E_corrected only,
    against |W_E|: the metric of energy_err), the GPU
    Gauss residual (max, rms), the oracle's, and the dipole's relative
    error."""
    Fo, _ = S.forces()
    e, eo = G.energy(), S.energy()
    out = {"force": force_err(G.forces(), Fo)}
    for k in ("W_E", "W_B", "U_self", "U_dip"):
        out[k] = abs(e[k] - eo[k]) / max(abs(eo[k]), 1e-300)
    out["W_B_vs_W_E"] = abs(e["W_B"] - eo["W_B"]) / abs(eo["W_E"])
    out["E_corrected"] = abs(e["E_corrected"] - eo["E_corrected"]) / abs(eo["W_E"])
    out["gauss_max"], out["gauss_rms"] = G.gauss_residual()
    out["gauss_max_oracle"] = S.gauss_residual()[0]
    P, Po = G.dipole(), S.dipole()
    out["dipole"] = float(np.max(np.abs(P - Po)) / max(1.0, np.max(np.abs(Po))))
    out["position"] = float(np.max(np.abs(G.state()[2] - S.r)) / max(1.0, np.max(np.abs(S.r))))
    return out


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def energy_err(e, eref, keys=("W_E", "W_B", "U_self", "U_dip", "E_corrected"), scale=None):
    """Relative error of each energy component; W_B (which starts at zero) and
    E_corrected are measured against the scale of W_E."""
    out = {}
    s = scale if scale is not None else abs(eref["W_E"])
    for k in keys:
        den = abs(eref[k]) if k in ("W_E", "U_self", "U_dip") else s
        out[k] = abs(e[k] - eref[k]) / max(den, 1e-300)
    return out


def pair(L, q, r0, a=1.0, dt=0.01, c=None, eps_min=1.0, precision=memd.FP64, audit_every=0,
         energy_every=0):
    """An oracle system and a HIP context with identical parameters."""
    if c is None:
        c = W.default_c(a, dt, eps_min)
    S = oracle.System(L, a, dt, c, q, r0)
    G = memd.Context(L, q, r0, a=a, dt=dt, c=c, precision=precision, audit_every=audit_every,
                     energy_every=energy_every)
    return S, G


def apply_eps(S, G, kind, value=None, eps_z=None, eps_site=None, eps_link=None):
    if kind == "uniform":
        S.set_eps_uniform(value)
        G.set_permittivity(memd.EPS_UNIFORM, [value])
    elif kind == "zsite":
        S.set_eps_zsite(eps_z)
        G.set_permittivity(memd.EPS_ZSITE, eps_z)
    elif kind == "site":
        S.set_eps_site(eps_site)
        G.set_permittivity(memd.EPS_SITE, eps_site)
    elif kind == "link":
        S.set_eps_link(eps_link)
        G.set_permittivity(memd.EPS_LINK, eps_link)
    else:
        raise ValueError(kind)


def share_state(S, G):
    """Upload the oracle's state to the HIP context (the shared start of a
    step-parity run)."""
    D, B, r = S.state()
    G.set_state(D, B, r)
