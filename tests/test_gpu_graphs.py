"""Recorded device work of chain calls: the second call of a structure records
its launches as a graph and later calls replay it with new descriptors.  Every
call, recorded, replayed or eager, must equal the oracle; replays are checked
one by one with the program's own eager GPU work and synchronizations between
them, and with the seeds, trial counts and configurations changed between
calls of one structure."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2411_18906_amd import binding as pb
from paper_2411_18906_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _batch(chains, seeds, T):
    species = np.concatenate([c.species for c in chains])
    offsets = np.concatenate([[0], np.cumsum([c.N for c in chains])])
    d = torch.from_numpy(species).cuda()
    probs = [(c.lattice, c.L, c.M, c.S, c.target, c.weight) for c in chains]
    pars = [pb.make_params(int(s), c.chain_id, T, c.B) for c, s in zip(chains, seeds)]
    stats = pb.pyhea_mc_batch(probs, d, offsets, pars)
    return stats, d.cpu().numpy(), offsets


def _check(chains, seeds, T, fin, offsets, stats, which):
    for i in which:
        c = chains[i]
        sp_o, _, st_o, _ = orc.mc_run(c.lattice, c.L, c.M, c.S, c.target, c.weight, c.species, seed=int(seeds[i]),
                                      chain_id=c.chain_id, n_trials=T, B=c.B)
        np.testing.assert_array_equal(fin[offsets[i]:offsets[i + 1]], sp_o, err_msg=f"chain {i}")
        assert stats[i]["S"] == st_o["S"] and stats[i]["commits"] == st_o["commits"]


def test_batch_replays_equal_oracle_with_new_seeds():
    chains = wl.mixed_chains(n_chains=12, seed=31, n_trials=1500)
    scratch = torch.zeros(1 << 20, device="cuda")
    flags = []
    for call in range(5):
        seeds = [1000 * call + i for i in range(len(chains))]
        T = 1500 if call % 2 == 0 else 1100   # trial counts change between calls of one structure
        stats, fin, offsets = _batch(chains, seeds, T)
        flags.append(int(stats[0]["graph"]))
        _check(chains, seeds, T, fin, offsets, stats, range(0, len(chains), 3))
        scratch.add_(1.0)              # eager work between replays
        torch.cuda.synchronize()
    assert flags == [0, 1, 1, 1, 1]
    assert float(scratch[0]) == 5.0


def test_graphs_off_runs_eagerly_and_equal():
    chains = wl.mixed_chains(n_chains=6, seed=32, n_trials=1200)
    seeds = [7 + i for i in range(len(chains))]
    pb.pyhea_tune_graphs(False)
    try:
        outs = [_batch(chains, seeds, 1200) for _ in range(3)]
    finally:
        pb.pyhea_tune_graphs(True)
    for stats, fin, offsets in outs:
        assert all(int(s["graph"]) == 0 for s in stats)
        np.testing.assert_array_equal(fin, outs[0][1])
    _check(chains, seeds, 1200, outs[0][1], outs[0][2], outs[0][0], range(len(chains)))
    # the same structure with graphs on: first call eager, then recorded and replayed
    for k in range(3):
        stats, fin, offsets = _batch(chains, seeds, 1200)
        assert int(stats[0]["graph"]) == (0 if k == 0 else 1)
        np.testing.assert_array_equal(fin, outs[0][1])


def test_single_chain_replays_and_logs():
    p = wl.fcc4_chain(seed=9)
    logs = []
    for call in range(4):
        d = torch.from_numpy(p.species).cuda()
        log = torch.zeros((4096, 4), dtype=torch.int32, device="cuda")
        st, _ = pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, d,
                                pb.make_params(p.seed + call, p.chain_id, 4000, p.B), log)
        assert st["graph"] == (0 if call == 0 else 1)
        sp_o, log_o, st_o, _ = orc.mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species,
                                          seed=p.seed + call, chain_id=p.chain_id, n_trials=4000, B=p.B)
        np.testing.assert_array_equal(d.cpu().numpy(), sp_o)
        n = int(st["log_len"])
        np.testing.assert_array_equal(log.cpu().numpy().view(np.uint32)[:n], np.asarray(log_o)[:n])
        logs.append(n)


@pytest.mark.skip(reason="dropping recorded plans (destroying an executable graph and freeing its "
                         "arena) ended in a host segmentation fault whose cause was not found; the "
                         "library no longer drops plans")
def test_many_structures_evict_and_stay_correct():
    """More structures than are kept: each is seen twice in turn (recorded, then
    dropped as others come), and the first one is right again at the end."""
    sets = [wl.mixed_chains(n_chains=3 + k, seed=40 + k, n_trials=800) for k in range(6)]
    for rep in range(2):
        for k, chains in enumerate(sets):
            seeds = [rep * 100 + k * 10 + i for i in range(len(chains))]
            stats, fin, offsets = _batch(chains, seeds, 800)
            _check(chains, seeds, 800, fin, offsets, stats, [0, len(chains) - 1])
    chains = sets[0]
    seeds = [5, 6, 7]
    for _ in range(3):
        stats, fin, offsets = _batch(chains, seeds, 800)
        _check(chains, seeds, 800, fin, offsets, stats, range(len(chains)))


def test_many_structures_record_and_replay():
    """Ten structures, three calls each: the first call of each runs eagerly,
    the later ones replay its recording (or, past the 32 recorded structures a
    process keeps, run eagerly too), and every call equals the oracle."""
    for k in range(10):
        chains = wl.mixed_chains(n_chains=2 + k, seed=60 + k, n_trials=600)
        seeds = [k * 10 + i for i in range(len(chains))]
        flags = []
        for _ in range(3):
            stats, fin, offsets = _batch(chains, seeds, 600)
            flags.append(int(stats[0]["graph"]))
            _check(chains, seeds, 600, fin, offsets, stats, [0, len(chains) - 1])
        assert flags[0] == 0 and flags[1] == flags[2]
