"""Global search (Sec. 4.1, Algorithm 1) and its random solutions on the GPU,
against the oracle: bit-exact random configurations, best solution, objective,
per-iteration history and counters."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2411_18906_amd import binding as pb
from paper_2411_18906_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("N,comp,it,slot0,n", [(1, [1], 0, 0, 2), (5, [2, 3], 3, 7, 4),
                                             (256, [64] * 4, 0, 0, 8), (108, [50, 30, 28], 2, 5, 3),
                                             (4097, [1, 4096], 1, 0, 2), (32000, [6400] * 5, 5, 12, 4),
                                             (1000, [0, 400, 600], 0, 1, 2)])
def test_random_configs_match_oracle(N, comp, it, slot0, n):
    out = torch.full((n, N), -1, dtype=torch.int8, device="cuda")
    pb.pyhea_random_configs(N, comp, 1234567, it, slot0, out)
    got = out.cpu().numpy()
    for c in range(n):
        want = orc.random_config(N, comp, seed=1234567, iteration=it, slot=slot0 + c)
        np.testing.assert_array_equal(got[c], want)


def _case(lattice, L, M, S, comp, rng_seed, **kw):
    rng = np.random.default_rng(rng_seed)
    t = rng.uniform(-0.2, 0.2, (S, M, M))
    t = (t + t.transpose(0, 2, 1)) / 2 if rng_seed % 2 == 0 else t
    w = rng.uniform(0.2, 1.0, S)
    N = orc.n_sites(lattice, L)
    best = torch.full((N,), -1, dtype=torch.int8, device="cuda")
    st, hist = pb.pyhea_global_search(lattice, L, M, S, t, w, comp, best, **kw)
    b_o, S_o, F_o, hist_o, st_o = orc.global_search(lattice, L, M, S, t, w, comp, **kw)
    np.testing.assert_array_equal(best.cpu().numpy(), b_o)
    assert st["S"] == S_o and st["F"] == F_o
    np.testing.assert_array_equal(hist, hist_o)
    for f in ["evaluations", "trials", "commits"]:
        assert st[f] == st_o[f], f


GLOBAL_CASES = [
    (orc.FCC, (4, 4, 4), 4, 2, [64] * 4, 2,
     dict(n_solutions=8, iterations=3, n_refine=4, discard_frac=0.5, seed=21, B=16, n_trials=2000,
          depth_limit=6)),
    (orc.BCC, (5, 5, 4), 3, 2, [70, 70, 60], 3,
     dict(n_solutions=6, iterations=2, n_refine=6, discard_frac=0.25, seed=5, B=64, n_trials=5000)),
    (orc.FCC, (3, 3, 3), 5, 3, [20, 20, 20, 24, 24], 4,
     dict(n_solutions=5, iterations=4, n_refine=2, discard_frac=1.0, seed=9, B=32, n_trials=800,
          mode=orc.MODE_BEST, tau=1e-3)),
    (orc.FCC, (4, 4, 4), 4, 2, [100, 60, 60, 36], 6,
     dict(n_solutions=7, iterations=2, n_refine=3, discard_frac=0.0, seed=3, B=8, n_trials=0)),
]


@pytest.mark.parametrize("case", range(len(GLOBAL_CASES)))
def test_global_search_matches_oracle(case):
    lattice, L, M, S, comp, rs, kw = GLOBAL_CASES[case]
    _case(lattice, L, M, S, comp, rs, **kw)


def test_global_search_rejects_bad_parameters():
    N = orc.n_sites(orc.FCC, (3, 3, 3))
    best = torch.zeros(N, dtype=torch.int8, device="cuda")
    t, w = np.zeros((2, 3, 3)), np.ones(2)
    base = dict(n_solutions=4, iterations=1, n_refine=2, discard_frac=0.5, seed=1, B=16, n_trials=10)
    for bad in [dict(n_refine=5), dict(n_refine=0), dict(iterations=0), dict(discard_frac=1.5)]:
        with pytest.raises(pb.PyheaError) as e:
            pb.pyhea_global_search(orc.FCC, (3, 3, 3), 3, 2, t, w, [36, 36, 36], best, **{**base, **bad})
        assert e.value.code == pb.EINVAL
    for comp in ([36, 36, 35], [0, 54, 54]):
        with pytest.raises(pb.PyheaError):
            pb.pyhea_global_search(orc.FCC, (3, 3, 3), 3, 2, t, w, comp, best, **base)


def test_global_search_fcc20_performance_preset_properties():
    # the paper's Performance-Optimized preset on the FCC 20^3 5-species problem
    p = wl.fcc20_chain()
    comp = np.bincount(p.species, minlength=p.M)
    best = torch.full((p.N,), -1, dtype=torch.int8, device="cuda")
    st, hist = pb.pyhea_global_search(p.lattice, p.L, p.M, p.S, p.target, p.weight, comp, best,
                                      n_solutions=64, iterations=6, n_refine=32, discard_frac=0.5,
                                      seed=p.seed, B=64, n_trials=10**5, depth_limit=8)
    b = best.cpu().numpy()
    np.testing.assert_array_equal(np.bincount(b, minlength=p.M), comp)
    cnt = orc.counts(p.lattice, p.L, p.M, p.S, b)
    _, _, S1, F1 = orc.alpha_objective(p.lattice, p.L, p.M, p.S, b, cnt, p.target, p.weight)
    assert st["S"] == S1 and st["F"] == F1 and hist[-1] == F1
    assert np.all(np.diff(hist) <= 0) and st["evaluations"] == 64 * 6 and st["trials"] > 0
