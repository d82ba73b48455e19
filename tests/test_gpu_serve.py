"""Serving: continuous batching of MC jobs.  Each job's result must be the
same alone (pyhea_mc_run) and in the mix, bit for bit; admission must respect
the HBM budget; errors and cancellation are reported per job."""
import threading
import time

import numpy as np
import pytest

from paper_2411_18906_amd import binding as pb
from paper_2411_18906_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def alone(p, T):
    d = torch.from_numpy(p.species).cuda()
    st, _ = pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, d,
                            pb.make_params(p.seed, p.chain_id, T, p.B))
    return d.cpu().numpy(), st


def mixed_jobs(n, seed=21):
    rng = np.random.Generator(np.random.Philox(seed))
    jobs = []
    for i in range(n):
        hi = 40000 if i % 5 else 420000          # every 5th job is large (HBM-resident)
        p = wl.random_chain(rng, seed, 100 + i, 2000, hi, int(rng.integers(2000, 30000)))
        jobs.append(p)
    return jobs


def test_each_job_same_alone_and_in_the_mix():
    jobs = mixed_jobs(12)
    with pb.Server(hbm_budget_bytes=64 << 20, max_slots=6, steps_per_round=37) as srv:
        for p in jobs:
            srv.pyhea_serve_submit(p.chain_id, p.lattice, p.L, p.M, p.S, p.target, p.weight,
                                   p.species, pb.make_params(p.seed, 0, p.n_trials, p.B))
        results = {p.chain_id: srv.pyhea_serve_poll(p.chain_id, p.N) for p in jobs}
        c = srv.pyhea_serve_counters()
    assert c["finished"] == len(jobs) and c["admitted"] == len(jobs) and c["rounds"] > 1
    for p in jobs:
        code, sp, st, times = results[p.chain_id]
        assert code == pb.OK
        sp_a, st_a = alone(p, p.n_trials)
        np.testing.assert_array_equal(sp, sp_a)
        for f in ["trials", "null_trials", "commits", "steps", "S", "F"]:
            assert st[f] == st_a[f], f
        assert times[0] <= times[1] <= times[2]


def test_budget_forces_queueing_and_is_never_exceeded():
    jobs = mixed_jobs(6, seed=5)
    jobs = [j for j in jobs if j.N < 100000]
    budget = max(j.N for j in jobs) + 16384     # room for about one job at a time
    seen = []
    with pb.Server(hbm_budget_bytes=budget * 2, max_slots=8, steps_per_round=16) as srv:
        for p in jobs:
            srv.pyhea_serve_submit(p.chain_id, p.lattice, p.L, p.M, p.S, p.target, p.weight,
                                   p.species, pb.make_params(p.seed, 0, p.n_trials, p.B))
        done = False
        while not done:
            c = srv.pyhea_serve_counters()
            seen.append(c)
            done = c["finished"] == len(jobs)
            time.sleep(0.002)
        for p in jobs:
            code, sp, st, _ = srv.pyhea_serve_poll(p.chain_id, p.N)
            assert code == pb.OK
            sp_a, st_a = alone(p, p.n_trials)
            np.testing.assert_array_equal(sp, sp_a)
    assert all(c["bytes_resident"] <= budget * 2 for c in seen)
    assert max(c["queued"] for c in seen) >= 1


def test_errors_cancel_and_unknown_ids():
    p = wl.fcc4_chain()
    with pb.Server(hbm_budget_bytes=128 << 10, max_slots=2, steps_per_round=8) as srv:
        bad = p.species.copy()
        bad[0] = 9
        with pytest.raises(pb.PyheaError) as e:
            srv.pyhea_serve_submit(1, p.lattice, p.L, p.M, p.S, p.target, p.weight, bad,
                                   pb.make_params(1, 0, 100))
        assert e.value.code == pb.EINVAL
        with pytest.raises(pb.PyheaError):        # too big for the budget
            big = wl.fcc40_chain()
            srv.pyhea_serve_submit(2, big.lattice, big.L, big.M, big.S, big.target, big.weight,
                                   big.species, pb.make_params(1, 0, 100))
        srv.pyhea_serve_submit(3, p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species,
                               pb.make_params(1, 0, 10**9))
        srv.pyhea_serve_submit(4, p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species,
                               pb.make_params(1, 0, 5000))
        with pytest.raises(pb.PyheaError):        # duplicate id
            srv.pyhea_serve_submit(4, p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species,
                                   pb.make_params(1, 0, 5000))
        time.sleep(0.05)
        assert srv.pyhea_serve_cancel(3) == pb.OK
        code, _, _, _ = srv.pyhea_serve_poll(3, p.N)
        assert code == pb.ECANCELLED
        code, sp, st, _ = srv.pyhea_serve_poll(4, p.N)
        assert code == pb.OK
        sp_a, st_a = alone(wl.Problem(p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species,
                                      1, 4, 5000, 64), 5000)
        np.testing.assert_array_equal(sp, sp_a)
        code, _, _, _ = srv.pyhea_serve_poll(4, p.N)
        assert code == pb.ENOENT
        c = srv.pyhea_serve_counters()
        assert c["rejected"] == 3


def test_jobs_submitted_while_others_run_join_later_rounds():
    jobs = mixed_jobs(8, seed=9)
    jobs = [j for j in jobs if j.N < 100000]
    with pb.Server(hbm_budget_bytes=256 << 20, max_slots=16, steps_per_round=8) as srv:
        first = jobs[: len(jobs) // 2]
        for p in first:
            srv.pyhea_serve_submit(p.chain_id, p.lattice, p.L, p.M, p.S, p.target, p.weight,
                                   p.species, pb.make_params(p.seed, 0, p.n_trials * 10, p.B))
        time.sleep(0.02)
        rounds_before = srv.pyhea_serve_counters()["rounds"]
        late = jobs[len(jobs) // 2:]
        for p in late:
            srv.pyhea_serve_submit(p.chain_id, p.lattice, p.L, p.M, p.S, p.target, p.weight,
                                   p.species, pb.make_params(p.seed, 0, p.n_trials, p.B))
        res = {p.chain_id: srv.pyhea_serve_poll(p.chain_id, p.N) for p in jobs}
    # late jobs finish before the long early ones: their work overlapped
    assert max(res[p.chain_id][3][2] for p in late) < max(res[p.chain_id][3][2] for p in first)
    assert rounds_before >= 1
    for p in late:
        sp_a, _ = alone(p, p.n_trials)
        np.testing.assert_array_equal(res[p.chain_id][1], sp_a)


@pytest.mark.parametrize("base_steps", [3, 50])
def test_launch_shapes_take_their_own_step_counts_and_stay_exact(base_steps):
    # small jobs held in LDS beside large HBM-resident ones: the faster shapes
    # run more steps per round (sized from their measured step times), so rounds
    # cut every job at other places than a fixed count would; each result must
    # still be the job's result alone
    rng = np.random.Generator(np.random.Philox(77))
    jobs = []
    for i in range(8):
        hi = 3000 if i % 2 else 300000
        jobs.append(wl.random_chain(rng, 77, 300 + i, 2000, hi, int(rng.integers(3000, 20000))))
    with pb.Server(hbm_budget_bytes=256 << 20, max_slots=8, steps_per_round=base_steps) as srv:
        for p in jobs:
            srv.pyhea_serve_submit(p.chain_id, p.lattice, p.L, p.M, p.S, p.target, p.weight,
                                   p.species, pb.make_params(p.seed, 0, p.n_trials, p.B))
        results = {p.chain_id: srv.pyhea_serve_poll(p.chain_id, p.N) for p in jobs}
        c = srv.pyhea_serve_counters()
    assert c["finished"] == len(jobs) and c["rounds"] > 1
    for p in jobs:
        code, sp, st, _ = results[p.chain_id]
        assert code == pb.OK
        sp_a, st_a = alone(p, p.n_trials)
        np.testing.assert_array_equal(sp, sp_a)
        for f in ["trials", "null_trials", "commits", "steps", "S", "F"]:
            assert st[f] == st_a[f], f
