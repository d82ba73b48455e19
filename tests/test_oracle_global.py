"""Pins of the oracle's global search (Sec. 4.1, Algorithm 1) and of its random
new solutions: properties the algorithm and a random arrangement must have,
and special cases that reduce to simpler, separately pinned computations."""
import numpy as np
import pytest

from oracle import oracle as orc


@pytest.mark.parametrize("N,comp", [(1, [1]), (2, [1, 1]), (5, [2, 3]), (256, [64] * 4),
                                    (108, [50, 30, 28]), (1000, [100, 200, 300, 400]),
                                    (4097, [1, 4096])])
def test_random_config_is_an_arrangement_of_the_composition(N, comp):
    c = orc.random_config(N, comp, seed=7, iteration=1, slot=3)
    assert c.min() >= 0                                   # every site written once
    np.testing.assert_array_equal(np.bincount(c, minlength=len(comp)), comp)
    np.testing.assert_array_equal(c, orc.random_config(N, comp, seed=7, iteration=1, slot=3))


def test_random_configs_differ_by_slot_iteration_and_seed():
    comp = [64] * 4
    base = orc.random_config(256, comp, seed=1, iteration=0, slot=0)
    for kw in [dict(seed=2, iteration=0, slot=0), dict(seed=1, iteration=1, slot=0),
               dict(seed=1, iteration=0, slot=1)]:
        assert not np.array_equal(base, orc.random_config(256, comp, **kw))


def test_random_config_sites_are_uniform():
    # over many draws each site holds species j with frequency c_j / N
    N, comp = 50, [10, 40]
    hits = np.zeros(N)
    n = 2000
    for s in range(n):
        hits += orc.random_config(N, comp, seed=11, iteration=0, slot=s) == 0
    p = 10 / 50
    sd = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(hits / n - p) < 5 * sd)


def test_random_config_rejects_bad_composition():
    with pytest.raises(ValueError):
        orc.random_config(10, [3, 3], seed=1, iteration=0, slot=0)


def test_retained_count():
    assert orc.retained_count(32, 0.5) == 16
    assert orc.retained_count(32, 0.25) == 16     # at most half of the refined
    assert orc.retained_count(32, 0.75) == 8
    assert orc.retained_count(5, 0.5) == 2
    assert orc.retained_count(4, 1.0) == 0


P1 = dict(lattice=orc.FCC, L=(4, 4, 4), M=4, S=2)


def _problem(rng=None):
    t = np.zeros((2, 4, 4)) if rng is None else rng.uniform(-0.2, 0.2, (2, 4, 4))
    return t, np.array([1.0, 0.5])


def test_no_refinement_is_the_best_random_draw():
    # with a zero trial budget the search keeps the best of its random draws
    t, w = _problem()
    kw = dict(n_solutions=6, iterations=3, n_refine=4, discard_frac=0.5, seed=5, B=16, n_trials=0)
    best, S, F, hist, st = orc.global_search(P1["lattice"], P1["L"], 4, 2, t, w, [64] * 4, **kw)
    R = orc.retained_count(4, 0.5)
    Fs = []
    for it in range(3):
        for s in range(0 if it == 0 else R, 6):
            c = orc.random_config(256, [64] * 4, seed=5, iteration=it, slot=s)
            Fs.append(orc.alpha_objective(P1["lattice"], P1["L"], 4, 2, c, orc.counts(P1["lattice"], P1["L"], 4, 2, c), t, w)[3])
    assert F == min(Fs) and st["trials"] == 0 and st["evaluations"] == 18


def test_one_solution_one_iteration_is_one_chain():
    t, w = _problem(np.random.default_rng(2))
    best, S, F, hist, st = orc.global_search(P1["lattice"], P1["L"], 4, 2, t, w, [64] * 4, n_solutions=1,
                                             iterations=1, n_refine=1, discard_frac=0.5, seed=9, B=32,
                                             n_trials=3000)
    c0 = orc.random_config(256, [64] * 4, seed=9, iteration=0, slot=0)
    sp, _, ms, _ = orc.mc_run(P1["lattice"], P1["L"], 4, 2, t, w, c0, seed=9, chain_id=0, n_trials=3000, B=32)
    np.testing.assert_array_equal(best, sp)
    assert F == ms["F"] and S == ms["S"] and st["trials"] == ms["trials"]


def test_search_invariants():
    t, w = _problem(np.random.default_rng(3))
    trace = []
    best, S, F, hist, st = orc.global_search(P1["lattice"], P1["L"], 4, 2, t, w, [64] * 4, n_solutions=8,
                                             iterations=4, n_refine=4, discard_frac=0.5, seed=21, B=16,
                                             n_trials=2000, depth_limit=6, trace=trace)
    R = orc.retained_count(4, 0.5)
    assert np.all(np.diff(hist) <= 0) and hist[-1] == F
    np.testing.assert_array_equal(np.bincount(best, minlength=4), [64] * 4)
    cnt = orc.counts(P1["lattice"], P1["L"], 4, 2, best)
    _, _, S1, F1 = orc.alpha_objective(P1["lattice"], P1["L"], 4, 2, best, cnt, t, w)
    assert S1 == S and F1 == F
    assert F == min(min(tr["refined_F"]) for tr in trace)
    for i, tr in enumerate(trace):
        Fp, top = np.array(tr["F"]), tr["top"]
        rest = [s for s in range(8) if s not in top]
        assert Fp[top].max() <= Fp[rest].min()                      # the best are refined
        # local search never worsens a solution
        assert sorted(tr["refined_F"]) == tr["refined_F"]
        assert min(tr["refined_F"]) <= Fp[top].min()
        if i + 1 < len(trace):                                      # seeds carried over
            np.testing.assert_array_equal(np.array(trace[i + 1]["F"][:R]), tr["refined_F"][:R])
