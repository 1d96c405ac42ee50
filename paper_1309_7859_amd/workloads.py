"""Seeded synthetic inputs for the MEMD workloads.

This module only draws random numbers and lays out configuration values; it
holds none of the method's arithmetic, so both the HIP path and the CPU oracle
can be fed from it.  Draw order for one system, from one
``numpy.random.Generator(PCG64(seed))``: positions, then the charge
permutation, then the displacements one step at a time (steps x n x 3).

Workloads (the paper gives no datasets for this path; every input is synthetic):
  c1  8^3,  a = 1, eps = 1 uniform, one +1 and one -1 ion, sigma = 0.01 a, 200 steps
  c2  32^3, 500 x (+1) and 500 x (-1), eps = 80 uniform, sigma = 0.02 a, 1000 steps
  c3  64^3, 5000 x (+1) and 5000 x (-1), site permittivity
      eps(z) = 41 + 39 tanh((z - L a / 2) / (2 a)) sampled at the vertex planes
      (80 on one side, 2 on the other), sigma = 0.02 a, 1000 steps
  c4  128^3, 45000 x (+-1) and 5000 x (+-2) ions, salt-dependent link permittivity
      eps = 80 - 15 c_local recomputed every 50 steps, sigma = 0.02 a, 500 steps
The time step is dt = 0.01 in every workload.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DT = 0.01


@dataclasses.dataclass
class Workload:
    name: str
    L: int
    a: float
    dt: float
    counts: tuple  # (n(+1), n(-1), n(+2), n(-2))
    eps_kind: str  # "uniform" | "zsite" | "salt"
    eps_value: float
    sigma: float
    steps: int
    seed: int
    salt_every: int = 0

    @property
    def n(self) -> int:
        return int(sum(self.counts))

    @property
    def sites(self) -> int:
        return self.L ** 3


WORKLOADS = {
    "c1": Workload("c1", 8, 1.0, DT, (1, 1, 0, 0), "uniform", 1.0, 0.01, 200, 101),
    "c2": Workload("c2", 32, 1.0, DT, (500, 500, 0, 0), "uniform", 80.0, 0.02, 1000, 102),
    "c3": Workload("c3", 64, 1.0, DT, (5000, 5000, 0, 0), "zsite", 0.0, 0.02, 1000, 103),
    "c4": Workload("c4", 128, 1.0, DT, (45000, 45000, 5000, 5000), "salt", 0.0, 0.02, 500, 104,
                   salt_every=50),
}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def positions(rng: np.random.Generator, n: int, L: int, a: float) -> np.ndarray:
    """Uniform positions in [0, L a)^3, shape (n, 3), FP64."""
    return rng.uniform(0.0, L * a, size=(n, 3))


def charges(rng: np.random.Generator, counts) -> np.ndarray:
    """A random permutation of n(+1) ones, n(-1) minus ones, n(+2) twos, n(-2) minus twos."""
    npos, nneg, npos2, nneg2 = counts
    q = np.concatenate([np.full(npos, 1.0), np.full(nneg, -1.0),
                        np.full(npos2, 2.0), np.full(nneg2, -2.0)])
    return q[rng.permutation(q.size)]


def displacements(rng: np.random.Generator, steps: int, n: int, sigma: float) -> np.ndarray:
    """Independent N(0, sigma^2) per component, per ion, per step: (steps, n, 3)."""
    return rng.normal(0.0, sigma, size=(steps, n, 3))


def tanh_slab(L: int, a: float, eps_mid: float = 41.0, amp: float = 39.0,
              width: float = 2.0) -> np.ndarray:
    """Site permittivity per vertex plane z = k a: eps_mid + amp tanh((z - L a/2)/(width a))."""
    z = np.arange(L, dtype=np.float64) * a
    return eps_mid + amp * np.tanh((z - 0.5 * L * a) / (width * a))


def slab_between(L: int, eps1: float, eps2: float, a: float = 1.0) -> np.ndarray:
    """A tanh slab running from eps2 (low z) to eps1 (high z)."""
    mid, amp = 0.5 * (eps1 + eps2), 0.5 * (eps1 - eps2)
    return tanh_slab(L, a, mid, amp, 2.0)


def make_system(w: Workload, steps: int | None = None, rng_state=None):
    """Draw one system: returns dict(q, r0, disp, eps_z) in the documented order."""
    rng = rng_for(w.seed)
    r0 = positions(rng, w.n, w.L, w.a)
    q = charges(rng, w.counts)
    nsteps = w.steps if steps is None else steps
    disp = displacements(rng, nsteps, w.n, w.sigma) if nsteps > 0 else np.zeros((0, w.n, 3))
    eps_z = tanh_slab(w.L, w.a) if w.eps_kind == "zsite" else None
    return dict(q=q, r0=r0, disp=disp, eps_z=eps_z)


class DisplacementStream:
    """Draws the same displacement sequence as ``make_system`` in chunks of steps."""

    def __init__(self, w: Workload):
        self.w = w
        self.rng = rng_for(w.seed)
        positions(self.rng, w.n, w.L, w.a)
        charges(self.rng, w.counts)

    def take(self, steps: int) -> np.ndarray:
        return displacements(self.rng, steps, self.w.n, self.w.sigma)


def default_c(a: float, dt: float, eps_min: float, nu: float = 0.25) -> float:
    """c for a Courant number nu = c dt sqrt(3) / (a sqrt(eps_min)) (configuration value)."""
    return nu * (a / dt) * math.sqrt(eps_min / 3.0)


# ------------------------------------------------------------ serving stream

SERVE_SIZES = (16, 24, 32, 48, 64)


@dataclasses.dataclass
class ReplicaSpec:
    index: int
    L: int
    n: int
    eps_kind: str  # "uniform" or "zsite"
    eps_value: float
    eps_z: np.ndarray | None
    steps: int
    seed: int
    arrival: float


def serving_stream(count: int = 512, rate: float = 500.0, seed: int = 105,
                   steps_range=(100, 2000), n_range=(100, 8000)) -> list:
    """Poisson arrivals of independent replicas (sizes, ion counts, eps profiles)."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        L = int(SERVE_SIZES[rng.integers(0, len(SERVE_SIZES))])
        n = 2 * int(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]))) // 2)
        n = max(n, 2)
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        if rng.uniform() < 0.5:
            kind, val, ez = "uniform", float(rng.uniform(2.0, 80.0)), None
        else:
            e1, e2 = rng.uniform(2.0, 80.0, size=2)
            kind, val, ez = "zsite", 0.0, slab_between(L, float(e1), float(e2))
        out.append(ReplicaSpec(k, L, n, kind, val, ez, steps, seed * 1_000_000 + k, t))
    return out


def replica_inputs(spec: ReplicaSpec, a: float = 1.0):
    """Positions and charges of one serving replica (half +1, half -1)."""
    rng = rng_for(spec.seed)
    r0 = positions(rng, spec.n, spec.L, a)
    q = charges(rng, (spec.n // 2, spec.n // 2, 0, 0))
    return q, r0
