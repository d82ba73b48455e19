"""Pins of the oracle's non-incremental baseline (two full evaluations per
swap): it agrees with the incremental closed form (pinned separately against
recounts) to rounding, is exactly zero for null swaps and exactly antisymmetric
under undoing the swap."""
import numpy as np
import pytest

from oracle import oracle as orc


@pytest.mark.parametrize("lattice,L,M,S", [(orc.FCC, (3, 3, 3), 4, 2), (orc.BCC, (4, 3, 3), 3, 3),
                                           (orc.FCC, (4, 4, 4), 5, 3)])
def test_recount_dS_matches_incremental(lattice, L, M, S):
    rng = np.random.default_rng(M * 10 + S)
    N = orc.n_sites(lattice, L)
    sp = rng.integers(0, M, N).astype(np.int8)
    sp[:M] = np.arange(M)
    t = rng.uniform(-0.2, 0.2, (S, M, M))
    w = rng.uniform(0.2, 1.0, S)
    _, _, S0, _ = orc.alpha_objective(lattice, L, M, S, sp, orc.counts(lattice, L, M, S, sp), t, w)
    for _ in range(40):
        p, q = (int(x) for x in rng.integers(0, N, 2))
        d_full = orc.swap_dS_recount(lattice, L, M, S, sp, p, q, t, w)
        d_inc = orc.swap_dS(lattice, L, M, S, sp, p, q, t, w)
        if sp[p] == sp[q]:
            assert d_full == 0.0 and d_inc == 0.0
            continue
        assert abs(d_full - d_inc) <= 1e-12 * max(1.0, abs(S0))
        sw = sp.copy()
        sw[p], sw[q] = sw[q], sw[p]
        assert orc.swap_dS_recount(lattice, L, M, S, sw, p, q, t, w) == -d_full
