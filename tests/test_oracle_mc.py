"""Pins of the oracle's Monte Carlo search (Sec. 4.2, Algorithms 2-3, Eq. 6).

The search is a heuristic, so there is no true result to compare with; the
oracle's trajectory is pinned by independent re-implementations of the rules
that recount everything from scratch (no incremental update), by invariants,
and by the global minimum of a tiny cell found by enumeration.
"""
from itertools import combinations

import numpy as np
import pytest

import bruteforce as bf
from oracle import oracle as orc
from paper_2411_18906_amd import workloads as wl


def _problem(lattice, L, S, M, seed, conc=None):
    N = orc.n_sites(lattice, L)
    rng = np.random.default_rng(seed)
    if conc is None:
        conc = wl.dirichlet_conc(rng, M, 0.1, 0.6) if M > 2 else np.array([0.4, 0.6])
    n = wl.largest_remainder(N, conc)
    sp = wl.shuffled_config(N, n, seed, 0)
    tgt = wl.projected_target(S, M, n / N, seed)
    w = np.array([1.0, 0.7, 0.4, 0.2][:S])
    return N, sp, tgt, w


class FullRecountChain:
    """Reference search that recomputes S from scratch for every trial."""

    def __init__(self, lattice, L, S, M, tgt, w, sp):
        self.tabs = bf.neighbor_table(lattice, L, S)
        self.M, self.tgt, self.w, self.z = M, tgt, w, bf.Z[lattice]
        self.sp = sp.copy()

    def S_of(self, sp):
        return bf.objective(bf.counts_by_offsets(self.tabs, self.M, sp), sp, self.tgt, self.w,
                            self.z)

    def near(self, x, y):
        return x == y or any(y in t[x] for t in self.tabs)

    def run(self, seed, chain, T, B, mode, tau=0.0):
        N = len(self.sp)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        log, step, done = [], 0, 0
        while done < T:
            tasks = min(B, T - done)
            S_cur = self.S_of(self.sp)
            cand = []
            for slot in range(tasks):
                x = orc.philox4x32_10([slot, step, chain, 0], key)
                p, q = (int(x[0]) * N) >> 32, (int(x[1]) * N) >> 32
                if self.sp[p] == self.sp[q]:
                    continue
                s2 = self.sp.copy()
                s2[p], s2[q] = s2[q], s2[p]
                dS = self.S_of(s2) - S_cur
                if dS < -tau:
                    cand.append((dS, slot, p, q))
            done += tasks
            cand.sort()
            committed = []
            for dS, slot, p, q in cand:
                if mode == orc.MODE_BEST and committed:
                    break
                if any(self.near(c, p) or self.near(c, q) for c in committed):
                    continue
                if committed:
                    s2 = self.sp.copy()
                    s2[p], s2[q] = s2[q], s2[p]
                    if not (self.S_of(s2) - self.S_of(self.sp) < -tau):
                        continue
                self.sp[p], self.sp[q] = self.sp[q], self.sp[p]
                committed += [p, q]
                log.append((step, slot, p, q))
            step += 1
        return np.array(log, dtype=np.uint32).reshape(-1, 4)


@pytest.mark.parametrize("lattice,L,S,M,B,mode", [
    (bf.FCC, (3, 3, 3), 2, 3, 1, orc.MODE_BEST),      # B = 1, improve-only: Algorithm 2
    (bf.BCC, (4, 4, 4), 3, 4, 16, orc.MODE_BEST),     # Algorithm 3 with Eq. 6
    (bf.FCC, (3, 3, 4), 2, 4, 16, orc.MODE_DISJOINT),
    (bf.BCC, (4, 3, 4), 4, 3, 32, orc.MODE_DISJOINT),
    (bf.FCC, (2, 2, 2), 3, 3, 8, orc.MODE_DISJOINT),  # multigraph cell
])
def test_chain_matches_full_recount_reference(lattice, L, S, M, B, mode):
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=17)
    T = 40 * B if B > 1 else 300
    sp_o, log_o, st, cnt = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=99, chain_id=3,
                                      n_trials=T, B=B, mode=mode)
    ref = FullRecountChain(lattice, L, S, M, tgt, w, sp)
    log_r = ref.run(99, 3, T, B, mode)
    assert len(log_r) > 3
    np.testing.assert_array_equal(log_o, log_r)
    np.testing.assert_array_equal(sp_o, ref.sp)
    assert st["trials"] == T and st["commits"] == len(log_r)


def test_chain_invariants():
    lattice, L, S, M = bf.FCC, (4, 4, 4), 3, 5
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=2)
    sp_o, log, st, cnt = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=5, chain_id=0,
                                    n_trials=4000, B=64)
    np.testing.assert_array_equal(np.bincount(sp_o, minlength=M), np.bincount(sp, minlength=M))
    tabs = bf.neighbor_table(lattice, L, S)
    np.testing.assert_array_equal(cnt, bf.counts_by_offsets(tabs, M, sp_o))
    # replaying the log: S never increases along the commits
    cur = sp.copy()
    S_prev = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
    S_first = S_prev
    for step, slot, p, q in log:
        cur[p], cur[q] = cur[q], cur[p]
        S_now = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
        assert S_now < S_prev + 1e-12
        S_prev = S_now
    np.testing.assert_array_equal(cur, sp_o)
    assert st["S"] == pytest.approx(S_prev, rel=1e-12)
    assert st["S"] < 0.5 * S_first
    assert st["trials"] == 4000 and st["steps"] == 63       # last step partial (4000 = 62*64+32)
    assert st["null_trials"] > 0


def test_best_commit_is_disjoint_first_commit():
    lattice, L, S, M = bf.BCC, (4, 4, 4), 2, 3
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=6)
    hits = 0
    for seed in range(40):
        _, lb, _, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=seed, chain_id=1,
                                 n_trials=32, B=32, mode=orc.MODE_BEST)
        _, ld, _, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=seed, chain_id=1,
                                 n_trials=32, B=32, mode=orc.MODE_DISJOINT)
        assert len(lb) == min(1, len(ld))
        if len(lb):
            np.testing.assert_array_equal(lb[0], ld[0])
            hits += 1
    assert hits > 10


def test_tiny_cell_reaches_global_minimum():
    """BCC 2x2x2 with 8/8 atoms: the search never goes below the exhaustive
    minimum of S and reaches it for most seeds."""
    lattice, L, S, M = bf.BCC, (2, 2, 2), 2, 2
    N = 16
    tgt = np.zeros((S, M, M))
    tgt[0] = [[-0.5, 0.5], [0.5, -0.5]]
    w = np.array([1.0, 0.5])
    tabs = bf.neighbor_table(lattice, L, S)
    best = np.inf
    for ones in combinations(range(N), 8):
        sp = np.zeros(N, np.int8)
        sp[list(ones)] = 1
        c = orc.counts(lattice, L, M, S, sp)
        best = min(best, orc.alpha_objective(lattice, L, M, S, sp, c, tgt, w)[2])
    reached = 0
    for seed in range(20):
        sp0 = wl.shuffled_config(N, [8, 8], seed, 0)
        _, _, st, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp0, seed=seed, chain_id=0,
                                 n_trials=3000, B=16)
        assert st["S"] >= best - 1e-12
        reached += st["S"] <= best + 1e-12
    assert reached >= 10
    assert bf.objective(bf.counts_by_offsets(tabs, M, sp0), sp0, tgt, w, bf.Z[lattice]) >= best


def test_depth_limit_stops_the_chain():
    lattice, L, S, M = bf.FCC, (3, 3, 3), 2, 3
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=1)
    sp1, _, st, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=1, chain_id=0, n_trials=10**6,
                               B=8, depth_limit=10)
    assert st["stop_reason"] == 1 and st["trials"] < 10**6
    assert st["trials"] == 8 * st["steps"]
    # the same run without the limit agrees up to the stop
    _, log_full, _, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=1, chain_id=0,
                                   n_trials=st["trials"], B=8)
    assert len(log_full) == st["commits"]


def test_tau_threshold():
    """A positive tau only commits swaps that improve S by more than tau."""
    lattice, L, S, M = bf.FCC, (3, 3, 3), 2, 3
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=4)
    tabs = bf.neighbor_table(lattice, L, S)
    tau = 1e-3
    sp1, log, st, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=3, chain_id=0, n_trials=2000,
                                 B=16, mode=orc.MODE_BEST, tau=tau)
    cur = sp.copy()
    for _, _, p, q in log:
        S0 = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
        cur[p], cur[q] = cur[q], cur[p]
        S1 = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
        assert S1 - S0 < -tau + 1e-12


@pytest.mark.parametrize("lattice,L,S,M,B,mode", [
    (bf.FCC, (3, 3, 3), 2, 3, 16, orc.MODE_BEST),       # Algorithm 3 with its threshold
    (bf.BCC, (4, 4, 4), 2, 4, 32, orc.MODE_DISJOINT),
    (bf.FCC, (3, 3, 3), 2, 3, 1, orc.MODE_BEST),        # B = 1: Algorithm 2 with its threshold
])
def test_threshold_acceptance_matches_full_recount_reference(lattice, L, S, M, B, mode):
    """tau < 0 (Algorithms 2-3 accept a swap that worsens S by less than the
    threshold): the oracle's log equals the full-recount reference's, every
    commit has S(after) - S(before) < -tau, and some commits do worsen S."""
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=23)
    tabs = bf.neighbor_table(lattice, L, S)
    T = 60 * B if B > 1 else 400
    # the threshold: a fifth of the median |dS| of random swaps of the start
    rng = np.random.default_rng(1)
    S0 = bf.objective(bf.counts_by_offsets(tabs, M, sp), sp, tgt, w, bf.Z[lattice])
    ds = []
    for _ in range(200):
        p, q = rng.integers(0, N, size=2)
        if sp[p] != sp[q]:
            s2 = sp.copy()
            s2[p], s2[q] = s2[q], s2[p]
            ds.append(abs(bf.objective(bf.counts_by_offsets(tabs, M, s2), s2, tgt, w, bf.Z[lattice]) - S0))
    tau = -0.2 * float(np.median(ds))
    sp_o, log_o, st, cnt = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=31, chain_id=2,
                                      n_trials=T, B=B, mode=mode, tau=tau)
    ref = FullRecountChain(lattice, L, S, M, tgt, w, sp)
    log_r = ref.run(31, 2, T, B, mode, tau=tau)
    np.testing.assert_array_equal(log_o, log_r)
    np.testing.assert_array_equal(sp_o, ref.sp)
    np.testing.assert_array_equal(cnt, bf.counts_by_offsets(tabs, M, sp_o))
    cur = sp.copy()
    worse = 0
    for _, _, p, q in log_o:
        a = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
        cur[p], cur[q] = cur[q], cur[p]
        b = bf.objective(bf.counts_by_offsets(tabs, M, cur), cur, tgt, w, bf.Z[lattice])
        assert b - a < -tau + 1e-12
        worse += b - a > 1e-12
    assert worse > 0 and len(log_o) > 5


def test_threshold_acceptance_never_commits_a_null_draw():
    """With tau < 0 a draw of two equal species (dS = 0 < -tau) is still a
    null trial: it is counted and never committed."""
    lattice, L, S, M = bf.FCC, (3, 3, 3), 2, 2
    N, sp, tgt, w = _problem(lattice, L, S, M, seed=8)
    sp_o, log, st, _ = orc.mc_run(lattice, L, M, S, tgt, w, sp, seed=4, chain_id=0, n_trials=640,
                                  B=64, mode=orc.MODE_DISJOINT, tau=-1.0)
    assert st["null_trials"] > 0
    for _, _, p, q in log:
        assert p != q
    # a huge threshold accepts every non-null draw that does not conflict
    assert st["commits"] > 0
    cur = sp.copy()
    for _, _, p, q in log:
        assert cur[p] != cur[q]
        cur[p], cur[q] = cur[q], cur[p]
    np.testing.assert_array_equal(cur, sp_o)
