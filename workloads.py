"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload parameters and random-number draws only: no part
of the Coulomb method's arithmetic (basis, mesh, tables, sums) lives here, so
the oracle and the GPU path can both take their inputs from it without
sharing any computation.  Callers pass in the basis size N and occupied size
M that their own side computed.

The workloads follow the paper's uniform-electron-gas setting (Sec. III):
planewaves in a cube, a Fermi sphere of occupied orbitals, and streams of
(i, j, k, l) index quadruples into the planewave basis.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    L: float                 # box side (bohr)
    n2max: int               # basis: |n|^2 <= n2max
    n2occ: int               # occupied Fermi sphere: |n|^2 <= n2occ
    n_nodes: int             # quadrature nodes Q (default Mesh 2: Q = 8 q + 8)
    n_quads: int             # length of the quadruple stream (0: none)
    seed: int = 0
    note: str = ""


# The five measured workloads.  "tiny" is a unit-test fixture.
TINY = Workload("tiny", 1.0, 2, 1, 16, 0, 7, "basis |n|^2<=2 (19 PW), Q=16")
C1_PLAIN = Workload("plain_fp64_123pw", 1.0, 9, 2, 48, 19 ** 4, 0,
                    "123 PW, occupied 19, Q=48; all 19^4 occupied quadruples")
C2_SPLIT = Workload("split_fp32_1045pw", 1.0, 40, 9, 64, 10_000_000, 1502,
                    "1045 PW, occupied 123, Q=64; 1e7 uniform quadruples")
C3_PAPER = Workload("paper_scale_9171pw", 1.0, 169, 36, 96, 0, 0,
                    "9171 PW, occupied 925, Q=96; exchange over all occupied pairs")
C4_STREAM = Workload("lookup_stream_9171pw", 1.0, 169, 36, 96, 100_000_000, 8043,
                     "9171 PW, Q=96; 1e8 quadruples, half uniform over the basis, "
                     "half over the occupied sphere")
STRETCH_9171 = Workload("exchange_9171occ", 1.0, 169, 169, 96, 0, 0,
                        "9171 PW all occupied: 8.41e7 ordered pairs")

ALL = {w.name: w for w in (TINY, C1_PLAIN, C2_SPLIT, C3_PAPER, C4_STREAM, STRETCH_9171)}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_quads(N: int, n: int, seed: int, hi: Optional[int] = None) -> np.ndarray:
    """n quadruples (i, j, k, l), each index uniform on [0, hi or N); int32 [n, 4]."""
    hi = N if hi is None else hi
    if n < 0 or hi < 1 or hi > N:
        raise ValueError("bad quadruple request")
    return rng(seed).integers(0, hi, size=(n, 4), dtype=np.int32)


def all_quads(M: int) -> np.ndarray:
    """Every (i, j, k, l) in [0, M)^4 in lexicographic order; int32 [M^4, 4]."""
    g = np.indices((M, M, M, M), dtype=np.int32).reshape(4, -1).T
    return np.ascontiguousarray(g)


def lookup_stream(N: int, M: int, n: int, seed: int) -> np.ndarray:
    """The mixed lookup stream: first half uniform over [0, N)^4, second over [0, M)^4."""
    h = n // 2
    g = rng(seed)
    a = g.integers(0, N, size=(h, 4), dtype=np.int32)
    b = g.integers(0, M, size=(n - h, 4), dtype=np.int32)
    return np.concatenate([a, b], axis=0)


def occupations(M: int, seed: int, lo: float = 0.25, hi: float = 1.0) -> np.ndarray:
    """Non-uniform occupation weights f_i in [lo, hi) (the paper uses all ones)."""
    return rng(seed).uniform(lo, hi, size=M)


def sample_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct row indices out of n, sorted (for sampled parity checks)."""
    k = min(k, n)
    return np.sort(rng(seed).choice(n, size=k, replace=False))


# ---------------------------------------------------------------------------
# Separable Gaussian basis: one-dimensional s-type Gaussians on a line of
# centers, several exponents per center (the same set along x, y and z).

@dataclass(frozen=True)
class GaussianSet:
    name: str
    n_centers: int
    exponents: tuple         # per center (bohr^-2)
    spacing: float           # bohr between neighbouring centers
    jitter: float            # uniform jitter of each center (bohr)
    seed: int
    n_nodes: int = 0         # default mesh node count for this set (0: caller's)


GAUSS_SMALL = GaussianSet("gauss_12x2", 6, (0.6, 2.5), 1.4, 0.2, 31)
GAUSS_BENCH = GaussianSet("gauss_24x2", 12, (0.8, 3.0), 1.5, 0.2, 1502)


def gaussian_set(gs: GaussianSet):
    """(exponents a [n1], centers A [n1]) with n1 = n_centers * len(exponents),
    ordered by center, then exponent."""
    g = rng(gs.seed)
    centers = gs.spacing * np.arange(gs.n_centers) + g.uniform(-gs.jitter, gs.jitter, gs.n_centers)
    a = np.array([e for _ in range(gs.n_centers) for e in gs.exponents], dtype=np.float64)
    A = np.repeat(centers, len(gs.exponents)).astype(np.float64)
    return a, A


# ---------------------------------------------------------------------------
# Serving workload: a Poisson stream of requests over many (L, cutoff, Q) keys.

@dataclass
class Request:
    t_arrival: float         # seconds from stream start
    kind: int                # 0 reconstruct, 1 energies
    L: float
    n2max: int
    n_nodes: int
    n_quads: int = 0         # reconstruct: stream length
    n2occ: int = 0           # energies: occupied sphere
    seed: int = 0


@dataclass
class ServingMix:
    n_requests: int = 2000
    seed: int = 2015
    rate_hz: float = 1000.0
    L_values: tuple = tuple(float(x) for x in np.geomspace(0.5, 4.0, 8))
    R_range: tuple = (5, 20)
    Q_values: tuple = (32, 48, 64, 96, 128)
    frac_reconstruct: float = 0.8
    n_range: tuple = (10_000, 1_000_000)
    zipf_s: float = 1.1
    keys: list = field(default_factory=list)


def serving_stream(mix: ServingMix) -> list:
    """Poisson arrivals; keys drawn Zipf-like over a seeded permutation of the key grid."""
    g = rng(mix.seed)
    keys = [(L, R * R, Q) for L in mix.L_values
            for R in range(mix.R_range[0], mix.R_range[1] + 1) for Q in mix.Q_values]
    perm = g.permutation(len(keys))
    ranks = np.arange(1, len(keys) + 1, dtype=np.float64)
    p = ranks ** (-mix.zipf_s)
    p /= p.sum()
    t = np.cumsum(g.exponential(1.0 / mix.rate_hz, size=mix.n_requests))
    out = []
    for r in range(mix.n_requests):
        L, n2max, Q = keys[perm[g.choice(len(keys), p=p)]]
        seed = int(g.integers(0, 2 ** 31 - 1))
        if g.uniform() < mix.frac_reconstruct:
            lo, hi = np.log(mix.n_range[0]), np.log(mix.n_range[1])
            n = int(np.exp(g.uniform(lo, hi)))
            out.append(Request(float(t[r]), 0, L, n2max, Q, n_quads=n, seed=seed))
        else:
            R = int(round(n2max ** 0.5))
            Ro = int(g.integers(1, max(1, R // 2) + 1))
            out.append(Request(float(t[r]), 1, L, n2max, Q, n2occ=Ro * Ro, seed=seed))
    mix.keys = keys
    return out
