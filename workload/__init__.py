"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and
the benchmark.

This module holds no arithmetic of the evolution method: it only draws random
numbers and states the workload shapes.  Everything here is a plain input
(product-state spinors, Gaussian tensors, bath parameters).  Both the CPU oracle
(``oracle/``) and the HIP path consume these inputs; neither side imports the
other.

Seed convention: ``numpy.random.default_rng(1000 * cfg + replicate)``.

Workloads (the paper's Heisenberg chain and Anderson impurity model):

* ``heis10``   -- Heisenberg S=1/2 open chain, L=10, chi<=32 (exact), backward
                 Euler type step, geometric grid 0.01 * 1.5**k -> 100.
* ``heis64``   -- L=64, chi<=256, SVD cutoff 1e-10, geometric grid 0.01 -> 1000,
                 ratio 1.3.
* ``heis100``  -- L=100, chi=1024 (contraction bound), Neel + 0.1 perturbation.
* ``aim60``    -- Anderson impurity, 1 impurity + 59 bath sites (d=4), chi<=512,
                 cutoff 1e-9, grid 0.01 -> 1e4, ratio 1.3.
* ``serve256`` -- 256 independent Heisenberg evolutions with random L, chi and
                 target beta/2, Poisson arrivals at 20 requests/s.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "rng_for",
    "random_spinors",
    "neel_spinors",
    "random_isometry_mps",
    "gaussian",
    "aim_bath",
    "Workload",
    "WORKLOADS",
    "serving_requests",
]


def rng_for(cfg: int, replicate: int = 0) -> np.random.Generator:
    """PCG64 generator for workload ``cfg`` and replicate ``replicate``."""
    return np.random.default_rng(1000 * int(cfg) + int(replicate))


def random_spinors(rng: np.random.Generator, L: int, d: int) -> list[np.ndarray]:
    """``L`` real spinors with i.i.d. N(0,1) entries, each scaled to unit norm."""
    out = []
    for _ in range(L):
        v = rng.standard_normal(d)
        out.append(v / np.linalg.norm(v))
    return out


def neel_spinors(rng: np.random.Generator, L: int, eps: float = 0.1) -> list[np.ndarray]:
    """Neel pattern e_(i mod 2) plus ``eps`` * N(0,1) noise, unit norm (d=2)."""
    out = []
    for i in range(L):
        v = np.zeros(2)
        v[i % 2] = 1.0
        v = v + eps * rng.standard_normal(2)
        out.append(v / np.linalg.norm(v))
    return out


def gaussian(rng: np.random.Generator, *shape: int) -> np.ndarray:
    """I.i.d. N(0,1) array of the given shape (float64, C order)."""
    return rng.standard_normal(shape)


def full_bond_dims(L: int, d: int, chi_max: int) -> list[int]:
    """Bond dimensions D_0..D_L = min(d^i, d^(L-i), chi_max) (D_0 = D_L = 1)."""
    dims = []
    for i in range(L + 1):
        e = min(i, L - i)
        dims.append(int(min(chi_max, d ** e if e < 63 else chi_max)))
    return dims


def random_isometry_mps(rng: np.random.Generator, L: int, d: int, chi_max: int,
                        distinct: int | None = None) -> list[np.ndarray]:
    """A random right-orthonormal MPS at full bond dimensions.

    Site tensor i has shape (D_(i-1), d, D_i); reshaped to D_(i-1) x (d D_i) its
    rows are orthonormal (the Q factor of a Gaussian matrix, i.e. a Haar-random
    isometry).  With ``distinct`` set, only that many different interior tensors
    of each shape are drawn and then reused, which keeps set-up time small for
    the largest chains.
    """
    dims = full_bond_dims(L, d, chi_max)
    cache: dict[tuple[int, int], list[np.ndarray]] = {}
    out = []
    for i in range(L):
        dl, dr = dims[i], dims[i + 1]
        key = (dl, dr)
        pool = cache.setdefault(key, [])
        if distinct is not None and len(pool) >= distinct:
            out.append(pool[i % distinct].copy())
            continue
        g = rng.standard_normal((d * dr, dl))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        a = np.ascontiguousarray(q.T).reshape(dl, d, dr)
        pool.append(a)
        out.append(a)
    return out


def aim_bath(n_bath: int = 59, gamma: float = 0.1) -> tuple[np.ndarray, np.ndarray]:
    """Bath energies on the midpoint grid of [-1, 1] and equal couplings.

    eps_k = -1 + (k - 1/2) * dE, dE = 2 / n_bath, V_k = sqrt(gamma * dE / pi),
    k = 1..n_bath, ascending in energy.
    """
    de = 2.0 / n_bath
    eps = np.array([-1.0 + (k - 0.5) * de for k in range(1, n_bath + 1)])
    v = np.full(n_bath, math.sqrt(gamma * de / math.pi))
    return eps, v


@dataclass(frozen=True)
class Workload:
    name: str
    model: str              # "heisenberg" or "aim"
    L: int
    d: int
    w: int                  # MPO bond dimension
    chi_max: int
    cutoff: float
    scheme: str             # "be" or "trap"
    tau0: float
    tau1: float
    ratio: float
    init: str               # "random", "neel", "isometry"
    extra: dict = field(default_factory=dict)


WORKLOADS: dict[str, Workload] = {
    "heis10": Workload("heis10", "heisenberg", 10, 2, 5, 32, 0.0, "be", 0.01, 100.0, 1.5,
                       "random", {"cfg": 0, "tol_loc": 1e-12, "pad_full": True}),
    "heis64": Workload("heis64", "heisenberg", 64, 2, 5, 256, 1e-10, "trap", 0.01, 1000.0, 1.3,
                       "random", {"cfg": 1}),
    "heis100": Workload("heis100", "heisenberg", 100, 2, 5, 1024, 0.0, "trap", 0.01, 1000.0, 1.3,
                        "neel", {"cfg": 2}),
    "aim60": Workload("aim60", "aim", 60, 4, 6, 512, 1e-9, "trap", 0.01, 1e4, 1.3,
                      "random", {"cfg": 3, "U": (2.0, 4.0, 6.0, 8.0), "gamma": 0.1}),
}


def serving_requests(n: int = 256, rate: float = 20.0, seed: int = 4000, Ls=(32, 48, 64, 96, 128),
                     chis=(64, 128, 256, 512), tau_range=(1.0, 1000.0)):
    """Request stream: (arrival_s, L, chi_max, tau_final, seed) tuples.

    Defaults: L uniform in {32,48,64,96,128}, chi_max uniform in
    {64,128,256,512}, tau_final = beta/2 log-uniform in [1, 1000], Poisson
    arrivals at ``rate``/s.  Ls, chis and tau_range give scaled-down streams of
    the same structure.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log10(tau_range[0]), math.log10(tau_range[1])
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        L = int(rng.choice(list(Ls)))
        chi = int(rng.choice(list(chis)))
        tau = float(10 ** rng.uniform(lo, hi))
        out.append((t, L, chi, tau, seed + 1 + i))
    return out
