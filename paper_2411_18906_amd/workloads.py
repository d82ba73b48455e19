"""Seeded synthetic inputs for SRO evaluation and the Monte Carlo search.

This module only makes inputs: compositions, initial configurations, target
SRO matrices, shell weights and job mixes.  It holds none of the method's
arithmetic (no pair counting, no alpha, no objective), so the library, the
oracle and the benchmark can all draw the same inputs from it.

Shapes follow the paper's workloads: FCC/BCC supercells of A*L^3 sites (A = 4
for FCC, 2 for BCC; Sec. 2.2, Table 1), 3-6 species at 5-35 % (Sec. 1), up to
three coordination shells, targets that are user-supplied alpha matrices
(Sec. 4.4).  The paper measures only its own synthetic lattices, so these
generated inputs are the workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FCC, BCC = 0, 1
BASIS_PER_CELL = {FCC: 4, BCC: 2}


@dataclass
class Problem:
    lattice: int
    L: tuple
    M: int
    S: int
    target: np.ndarray  # [S][M][M] float64
    weight: np.ndarray  # [S] float64
    species: np.ndarray  # [N] int8
    seed: int = 1
    chain_id: int = 0
    n_trials: int = 0
    B: int = 64
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return BASIS_PER_CELL[self.lattice] * self.L[0] * self.L[1] * self.L[2]


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), stream & (2**64 - 1)]))


def largest_remainder(N: int, conc) -> np.ndarray:
    """Integer species counts summing to N: floor(c_j N), leftovers to the
    largest fractional parts (ties to the lower species index)."""
    c = np.asarray(conc, dtype=np.float64)
    c = c / c.sum()
    raw = c * N
    n = np.floor(raw).astype(np.int64)
    left = N - int(n.sum())
    frac = raw - n
    order = sorted(range(len(c)), key=lambda j: (-frac[j], j))
    for j in order[:left]:
        n[j] += 1
    return n


def shuffled_config(N: int, n_per_species, seed: int, chain_id: int) -> np.ndarray:
    """A uniformly random arrangement of the given multiset of species."""
    n = np.asarray(n_per_species, dtype=np.int64)
    assert int(n.sum()) == N
    base = np.repeat(np.arange(len(n), dtype=np.int8), n)
    return _rng(seed, (chain_id << 8) | 1).permutation(base).astype(np.int8)


def projected_target(S: int, M: int, conc, seed: int, stream: int = 7, scale: float = 0.2):
    """Per shell: symmetric matrix with entries U(-scale, scale) on and above the
    diagonal, mirrored, then projected A' = P A P, P = I - c c^T/|c|^2, so that
    A' c = 0 (i.e. sum_j c_j alpha_ij = 0) and A' stays symmetric."""
    c = np.asarray(conc, dtype=np.float64)
    rng = _rng(seed, (stream << 8) | 2)
    P = np.eye(M) - np.outer(c, c) / float(c @ c)
    out = np.zeros((S, M, M))
    for k in range(S):
        U = rng.uniform(-scale, scale, size=(M, M))
        A = np.triu(U) + np.triu(U, 1).T
        out[k] = P @ A @ P
    return out


def cells_for(lattice: int, n_target: float) -> int:
    return max(3, int(round((n_target / BASIS_PER_CELL[lattice]) ** (1.0 / 3.0))))


# --------------------------------------------------------------------------
# The five workloads: shapes, compositions and budgets.
# --------------------------------------------------------------------------

def fcc4_chain(seed: int = 1, chain_id: int = 0) -> Problem:
    """FCC 4x4x4 (256 sites), 4 equiatomic species, shells 1-2, alpha target 0,
    unit weights, 10^4 trials, B = 64 (the paper's 64-task preset)."""
    L = (4, 4, 4)
    sp = shuffled_config(256, [64] * 4, seed, chain_id)
    return Problem(FCC, L, 4, 2, np.zeros((2, 4, 4)), np.ones(2), sp, seed, chain_id, 10**4, 64)


def fcc20_chain(seed: int = 1, chain_id: int = 0) -> Problem:
    """FCC 20x20x20 (32,000 sites), 5 equiatomic species, shells 1-3, target 0,
    unit weights, 10^6 trials."""
    L = (20, 20, 20)
    sp = shuffled_config(32000, [6400] * 5, seed, chain_id)
    return Problem(FCC, L, 5, 3, np.zeros((3, 5, 5)), np.ones(3), sp, seed, chain_id, 10**6, 64)


def fcc40_chain(seed: int = 1, chain_id: int = 0) -> Problem:
    """FCC 40x40x40 (256,000 sites), 4 species at 0.25, shells 1-2, projected
    random target in [-0.2, 0.2], weights (1.0, 0.5), 10^7 trials."""
    L = (40, 40, 40)
    c = np.full(4, 0.25)
    sp = shuffled_config(256000, [64000] * 4, seed, chain_id)
    tgt = projected_target(2, 4, c, seed)
    return Problem(FCC, L, 4, 2, tgt, np.array([1.0, 0.5]), sp, seed, chain_id, 10**7, 64)


def dirichlet_conc(rng: np.random.Generator, M: int, lo: float = 0.05, hi: float = 0.35):
    """Dirichlet(1,...,1) concentrations, resampled until all lie in [lo, hi]."""
    while True:
        c = rng.dirichlet(np.ones(M))
        if np.all(c >= lo) and np.all(c <= hi):
            return c


def random_chain(rng: np.random.Generator, seed: int, chain_id: int, n_lo: float, n_hi: float,
                 n_trials: int, B: int = 64, S: int = 2) -> Problem:
    lattice = FCC if rng.uniform() < 0.5 else BCC
    n_star = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
    Lc = cells_for(lattice, n_star)
    M = int(rng.integers(3, 7))
    c = dirichlet_conc(rng, M)
    N = BASIS_PER_CELL[lattice] * Lc**3
    n = largest_remainder(N, c)
    sp = shuffled_config(N, n, seed, chain_id)
    tgt = projected_target(S, M, n / N, seed, stream=chain_id + 1000)
    w = np.array([1.0, 0.5, 0.25, 0.125][:S])
    return Problem(lattice, (Lc, Lc, Lc), M, S, tgt, w, sp, seed, chain_id, n_trials, B)


def mixed_chains(n_chains: int = 512, seed: int = 4, n_trials: int = 10**5) -> list:
    """Batched: FCC/BCC at 50/50, 250-16,000 sites log-uniform, 3-6 species at
    5-35 % (Dirichlet, rounded by largest remainder), projected targets, shell
    weights (1.0, 0.5), 10^5 trials per chain."""
    rng = _rng(seed, 4 << 8)
    return [random_chain(rng, seed, i, 250, 16000, n_trials) for i in range(n_chains)]


def served_jobs(n_jobs: int = 2000, seed: int = 5, n_lo: float = 2e3, n_hi: float = 2e6,
                 t_lo: float = 1e4, t_hi: float = 1e7) -> list:
    """Serving: job sizes 2,000-2,000,000 sites log-uniform, FCC/BCC, 3-6
    species, trial budgets log-uniform in [10^4, 10^7].  The job id is the
    chain id, so a job's trajectory depends only on its own inputs."""
    rng = _rng(seed, 5 << 8)
    jobs = []
    for i in range(n_jobs):
        T = int(round(math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))))
        jobs.append(random_chain(rng, seed, i, n_lo, n_hi, T))
    return jobs


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = _rng(seed, 6 << 8)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def random_configs(N: int, n_per_species, K: int, seed: int) -> np.ndarray:
    """K independent random arrangements of one composition, [K][N] int8."""
    rng = _rng(seed, 3 << 8)
    base = np.repeat(np.arange(len(n_per_species), dtype=np.int8), n_per_species)
    out = np.empty((K, N), np.int8)
    for k in range(K):
        out[k] = rng.permutation(base)
    return out


def iid_configs(N: int, M: int, K: int, seed: int) -> np.ndarray:
    """K configurations of N sites with species drawn i.i.d. uniform on [0, M),
    [K][N] int8 (a full-evaluation batch; every species is present with
    overwhelming probability for N in the thousands)."""
    rng = _rng(seed, 8 << 8)
    return rng.integers(0, M, size=(K, N), dtype=np.int8)
