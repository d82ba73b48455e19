"""The measuring autotuner of the MC launch shapes: a chain's shape is chosen
by timing candidate shapes on a scratch copy, recorded in the statistics, kept
in the cache file across processes, and the chain's results are those of the
oracle whatever shape was chosen (shapes never change trajectories)."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2411_18906_amd import binding as pb
from paper_2411_18906_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def chain_stats(p, T, measure=True):
    pb.pyhea_tune_measure(measure)
    try:
        d = torch.from_numpy(p.species).cuda()
        st, _ = pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, d,
                                pb.make_params(p.seed, p.chain_id, T, p.B), None)
        return st, d.cpu().numpy()
    finally:
        pb.pyhea_tune_measure(True)


def test_measured_shape_is_reported_and_results_unchanged():
    p = wl.fcc4_chain()
    st, sp = chain_stats(p, 3000)
    assert st["shape_measured"] == 1 and st["shape"] > 0
    sp_o, _, st_o, _ = orc.mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species, seed=p.seed,
                                  chain_id=p.chain_id, n_trials=3000, B=p.B)
    np.testing.assert_array_equal(sp, sp_o)
    assert st["S"] == st_o["S"] and st["commits"] == st_o["commits"]
    st2, _ = chain_stats(p, 3000, measure=False)
    assert st2["shape_measured"] == 0


def test_batch_reports_model_shapes():
    """Batches keep the cost model's shapes (reported, not measured)."""
    chains = wl.mixed_chains(n_chains=8, seed=21, n_trials=2000)
    species = np.concatenate([c.species for c in chains])
    offsets = np.concatenate([[0], np.cumsum([c.N for c in chains])])
    d = torch.from_numpy(species).cuda()
    probs = [(c.lattice, c.L, c.M, c.S, c.target, c.weight) for c in chains]
    pars = [pb.make_params(c.seed, c.chain_id, c.n_trials, c.B) for c in chains]
    stats = pb.pyhea_mc_batch(probs, d, offsets, pars)
    assert all(s["shape_measured"] == 0 and s["shape"] > 0 for s in stats)
    fin = d.cpu().numpy()
    for i, c in enumerate(chains[:3]):
        sp_o, _, _, _ = orc.mc_run(c.lattice, c.L, c.M, c.S, c.target, c.weight, c.species, seed=c.seed,
                                   chain_id=c.chain_id, n_trials=c.n_trials, B=c.B)
        np.testing.assert_array_equal(fin[offsets[i]:offsets[i + 1]], sp_o)


CHILD = textwrap.dedent("""
    import sys
    sys.path.insert(0, {root!r})
    import torch
    from paper_2411_18906_amd import binding as pb
    from paper_2411_18906_amd import workloads as wl
    p = wl.fcc4_chain(seed=3)
    d = torch.from_numpy(p.species).cuda()
    st, _ = pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, d,
                            pb.make_params(p.seed, 0, 2000, p.B), None)
    print(st["shape"], st["shape_measured"])
""")


def test_shapes_persist_across_processes(tmp_path):
    cache = tmp_path / "shapes.txt"
    env = dict(os.environ, PYHEA_TUNE_CACHE=str(cache))
    code = CHILD.format(root=ROOT)
    out1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert out1.returncode == 0, out1.stderr
    lines1 = cache.read_text().splitlines()
    assert len(lines1) >= 1 and "gfx" in lines1[0]
    out2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert out2.returncode == 0, out2.stderr
    assert out1.stdout.split() == out2.stdout.split()            # same shape, measured (cached)
    assert out2.stdout.split()[1] == "1"
    assert cache.read_text().splitlines() == lines1              # nothing re-measured
