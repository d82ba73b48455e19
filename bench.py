"""Benchmark of the SRO hot path on one MI355X.

Workload (one "step" = one pass over the whole hot path):
  * full SRO evaluation of a batch of K independent FCC 20x20x20 configurations
    (32,000 sites, 5 species, shells 1-3) in one launch, of one such configuration
    alone (latency), and of 4,096 FCC 40x40x40 configurations (256,000 sites,
    4 species, shells 1-2);
  * the plain single chain of that shape: 5 equiatomic species, target alpha 0,
    unit weights, 10^6 Philox trial swaps, B = 64, disjoint commits;
  * the batched form: 512 chains of uneven FCC/BCC cells (250-16,000 sites,
    3-6 species, 10^5 trials each) in one persistent launch.
Inputs are synthetic, seeded and resident in HBM before the timed region.

After the timed steps the same 512 chains run once more one after another
through the single-chain entry point ("plain"), and their final configurations
must equal the batched ones; then 2,000 jobs are served with Poisson arrivals
at 70 % of the measured batched capacity under a 512 MB HBM budget (p50/p99 of
completion - arrival, and of the wait for admission).

Prints one JSON line: value = trial swaps/s of the single chain; the full
evaluation's GB/s (with the HBM roofline of its kernel) and the batched
chains' trial swaps/s ride along in the same line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The serving leg spreads each round's launch shapes over 16 streams.  The HIP
# runtime serves a process's streams from GPU_MAX_HW_QUEUES hardware queues (4
# by default) and launches that share a queue run one after another, so this
# process asks for at least 16.  The runtime reads it once, when it starts (the
# first torch or library call), so it is set here.
try:
    _queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _queues = 4
if _queues < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

HBM_PEAK_GBPS = 8000.0
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes per clock x clock
METRIC = "MC trial swaps/sec + full-SRO eval GB/s; batched vs plain at equal SRO error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eval-configs", type=int, default=32768)
    ap.add_argument("--chains", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="eval,eval3,lat,chain,chain1,chain3,batch,copy")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain (one after another) chains")
    ap.add_argument("--serve-jobs", type=int, default=2000, help="served jobs (0 = skip serving)")
    ap.add_argument("--serve-budget-mb", type=int, default=512)
    ap.add_argument("--no-global", action="store_true", help="skip the global search leg")
    ap.add_argument("--no-baseline", action="store_true", help="skip the incremental-vs-full leg")
    ap.add_argument("--serve-load", type=float, default=0.7, help="offered load / measured serving capacity")
    ap.add_argument("--no-best", action="store_true", help="skip the DISJOINT vs BEST comparison")
    ap.add_argument("--no-cpu-batch", action="store_true", help="skip the all-core oracle run of the batched chains")
    return ap.parse_args()


def cpu_baseline(p, budget_s: float = 12.0):
    """The oracle, as it stands, on one host core: trial swaps/s of the same
    chain (first trials of the budget) and sites/s of the full evaluation."""
    from oracle import oracle as orc
    t0 = time.perf_counter()
    T = 20000
    orc.mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species, seed=p.seed,
               chain_id=p.chain_id, n_trials=T, B=p.B)
    dt = time.perf_counter() - t0
    # grow the sample to about the budget
    if dt < budget_s / 2:
        T2 = int(T * (budget_s / 2) / max(dt, 1e-3))
        t0 = time.perf_counter()
        orc.mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, p.species, seed=p.seed,
                   chain_id=p.chain_id, n_trials=T2, B=p.B)
        dt, T = time.perf_counter() - t0, T2
    t0 = time.perf_counter()
    n_eval = 0
    while time.perf_counter() - t0 < budget_s / 4 or n_eval == 0:
        orc.counts(p.lattice, p.L, p.M, p.S, p.species)
        n_eval += 1
    de = time.perf_counter() - t0
    return {"value": T / dt, "unit": "trial swaps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {T} trials of the FCC 20^3 5-species chain (B=64); "
                      f"{n_eval} full evaluations of one 32,000-site configuration",
            "full_eval_sites_per_s": n_eval * p.N / de,
            "full_eval_GBps": n_eval * p.N / de / 1e9}


def progress(msg: str):
    """A progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_chain(job):
    """Worker: one oracle chain (the oracle as it stands)."""
    from oracle import oracle as orc
    j = dict(job)
    args = [j.pop(k) for k in ("lattice", "L", "M", "S", "target", "weight", "species")]
    t0 = time.perf_counter()
    orc.mc_run(*args, **j)
    return time.perf_counter() - t0


def cpu_batch_baseline(chains, n_sample: int = 128):
    """The oracle on the batched chains across all host cores: the first
    n_sample chains of the 512 (10^5 trials each), one process per core."""
    import multiprocessing
    import platform
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, os.cpu_count() or 1))   # the box grants a share of 16 CPUs
    sample = chains[:n_sample]
    jobs = [dict(lattice=c.lattice, L=tuple(c.L), M=c.M, S=c.S, target=c.target, weight=c.weight,
                 species=c.species, seed=c.seed, chain_id=c.chain_id, n_trials=c.n_trials, B=c.B)
            for c in sample]
    with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as ex:
        list(ex.map(_oracle_chain, jobs[:cores]))   # warm the workers (imports, library load)
        t0 = time.perf_counter()
        per = list(ex.map(_oracle_chain, jobs))
        wall = time.perf_counter() - t0
    trials = sum(c.n_trials for c in sample)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": trials / wall, "unit": "trial swaps/s", "cores": cores, "kind": "oracle",
            "sample": f"first {len(sample)} of the {len(chains)} batched chains ({trials} trials), "
                      f"one oracle process per core",
            "nproc": os.cpu_count(), "cpu_model": model or platform.processor(),
            "wall_s": wall, "cpu_s": float(sum(per))}


def best_vs_disjoint(pb, p, torch, T=None):
    """Paper-literal BEST commits (one swap per step, Eq. 6) against DISJOINT
    commits on problem p: the DISJOINT chain of T trials sets F; then the
    fewest trials (to 1/16) with which BEST reaches that F, and the time it
    takes.  A chain with a smaller budget is a prefix of one with a larger
    budget (counter-based draws), so F falls monotonically with the budget."""
    T = p.n_trials if T is None else T
    d = torch.empty(p.N, dtype=torch.int8, device="cuda")
    src = torch.from_numpy(p.species).cuda()

    def run_mode(T, mode):
        d.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, d,
                                pb.make_params(p.seed, p.chain_id, T, p.B, mode=mode), None)
        return st, time.perf_counter() - t0

    def run(T):
        return run_mode(T, pb.MODE_BEST)

    run_mode(T, pb.MODE_DISJOINT)   # warm: measured launch shapes, caches
    std, t_disjoint_s = run_mode(T, pb.MODE_DISJOINT)
    F_disjoint = std["F"]
    T_cap = 32 * T
    lo, hi = 0, T
    st, _ = run(hi)
    F_at_T = st["F"]
    while st["F"] > F_disjoint and hi < T_cap:
        lo, hi = hi, min(2 * hi, T_cap)
        st, _ = run(hi)
    reached = st["F"] <= F_disjoint
    if reached:
        step = max(p.B, hi // 16)
        while hi - lo > step:
            mid = (lo + hi) // 2 // p.B * p.B
            if mid <= lo:
                break
            if run(mid)[0]["F"] <= F_disjoint:
                hi = mid
            else:
                lo = mid
    st, t_best = run(hi)
    return {"disjoint_trials": T, "disjoint_s": t_disjoint_s, "disjoint_commits": std["commits"],
            "disjoint_final_F": F_disjoint, "best_F_at_equal_trials": F_at_T,
            "best_reached_disjoint_F": bool(reached), "best_trials": hi, "best_s": t_best,
            "best_commits": st["commits"], "best_final_F": st["F"],
            "disjoint_speedup_at_equal_F": t_best / t_disjoint_s if reached else None,
            "workload": f"FCC {p.L[0]}^3, {p.M} species, shells 1-{p.S}, B = {p.B}; BEST commits the best "
                        f"improving swap of a step, DISJOINT every non-conflicting one"}


def recorded(profile: str, source: str, key: str):
    """A figure recorded in a committed rocprofv3 summary, if that summary was
    taken on the current kernel source (otherwise None)."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2411_18906_amd", "csrc", source), "rb")
                             .read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines() if ":" in l and not l.startswith((" ", "|", "#")))
    if vals.get("kernel_source_sha256_prefix", "").strip() != sha or key not in vals:
        return None
    return float(vals[key])


def recorded_traffic():
    """HBM bytes per launch of the full-evaluation kernel from the committed
    rocprofv3 counter summary, if that summary was taken on the current kernel
    source (otherwise None)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "full_eval_fcc20_5sp_traffic.md")
    src = os.path.join(ROOT, "paper_2411_18906_amd", "csrc", "sro_bits.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines() if l.startswith(("traffic_bytes", "kernel_source")))
    if vals.get("kernel_source_sha256_prefix", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def serve(pb, wl, n_jobs, capacity_trials_per_s, load, budget_mb):
    """Poisson arrivals of jobs (2,000-2,000,000 sites, 10^4-10^7 trials) at
    `load` times the given capacity (load 0: every job arrives at once, which
    measures the capacity itself); latency = completion - arrival."""
    jobs = wl.served_jobs(n_jobs=n_jobs)
    T = np.array([j.n_trials for j in jobs], dtype=np.float64)
    if load > 0:
        rate = load * capacity_trials_per_s / T.mean()
        arrivals = wl.poisson_arrivals(len(jobs), rate)
    else:
        rate = float("inf")
        arrivals = np.zeros(len(jobs))
    res = {}
    with pb.Server(hbm_budget_bytes=budget_mb << 20, max_slots=1024, steps_per_round=256) as srv:
        t0 = time.perf_counter()
        for i, j in enumerate(jobs):
            while True:
                wait = t0 + arrivals[i] - time.perf_counter()
                if wait <= 0:
                    break
                time.sleep(min(wait, 1e-3))
            srv.pyhea_serve_submit(i, j.lattice, j.L, j.M, j.S, j.target, j.weight, j.species,
                                   pb.make_params(j.seed, i, j.n_trials, j.B))
        for i, j in enumerate(jobs):
            res[i] = srv.pyhea_serve_poll(i, j.N)
        c = srv.pyhea_serve_counters()
    bad = [i for i, r in res.items() if r[0] != pb.OK]
    if bad:
        print(f"served jobs failed: {bad[:10]}", file=sys.stderr)
        sys.exit(1)
    sub = np.array([r[3][0] for r in res.values()], dtype=np.float64)
    adm = np.array([r[3][1] for r in res.values()], dtype=np.float64)
    fin = np.array([r[3][2] for r in res.values()], dtype=np.float64)
    lat = (fin - sub) / 1e6
    wait = (adm - sub) / 1e6
    trials = sum(r[2]["trials"] for r in res.values())
    span = (fin.max() - sub.min()) / 1e9
    # where the tail goes: the jobs at or above the 99th latency percentile
    p99 = np.percentile(lat, 99)
    order = [i for i in np.argsort(-lat) if lat[i] >= p99][:20]
    tail = [{"sites": int(jobs[i].N), "trials": int(jobs[i].n_trials),
             "lattice": "FCC" if jobs[i].lattice == 0 else "BCC",
             "wait_ms": float(wait[i]), "service_ms": float((fin[i] - adm[i]) / 1e6),
             "latency_ms": float(lat[i])} for i in order]
    return {"jobs": len(jobs), "offered_jobs_per_s": rate if np.isfinite(rate) else None, "offered_load": load,
            "capacity_trials_per_s": capacity_trials_per_s, "hbm_budget_MB": budget_mb,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max()), "admission_wait_ms_p50": float(np.percentile(wait, 50)),
            "admission_wait_ms_p99": float(np.percentile(wait, 99)), "trials": int(trials), "span_s": span,
            "trials_per_s": trials / span, "rounds": c["rounds"], "sites_total": int(sum(j.N for j in jobs)),
            "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
            "p99_tail_jobs": tail}


def global_search(pb, p, torch):
    """Algorithm 1 with the paper's Performance-Optimized preset (64 solutions,
    6 global iterations, 64 tasks, search depth 8) on the FCC 20^3 problem: the
    32 best solutions of each iteration refined (at most 10^5 trial swaps each),
    half of them kept as seeds.  One warm-up search, then one timed search."""
    comp = np.bincount(p.species, minlength=p.M)
    best = torch.empty(p.N, dtype=torch.int8, device="cuda")
    kw = dict(n_solutions=64, iterations=6, n_refine=32, discard_frac=0.5, seed=p.seed, B=64,
              n_trials=10**5, depth_limit=8)
    pb.pyhea_global_search(p.lattice, p.L, p.M, p.S, p.target, p.weight, comp, best, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, hist = pb.pyhea_global_search(p.lattice, p.L, p.M, p.S, p.target, p.weight, comp, best, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"s": dt, "evaluations": st["evaluations"], "trials": st["trials"], "commits": st["commits"],
            "trials_per_s": st["trials"] / dt, "best_F": st["F"], "best_F_per_iteration": [float(x) for x in hist],
            "preset": "64 solutions, 6 iterations, 32 refined (<= 1e5 trials, depth 8, B = 64), p_a = 0.5"}


def incremental_vs_full(pb, p, torch, out):
    """The paper's incremental-versus-full comparison on the FCC 20^3 problem:
    dS of random swaps from two full evaluations per swap (the baseline) --
    4,096 swaps per call (throughput) and 64 per call (one MC step of B = 64) --
    against the incremental recount of the MC kernel (the FCC 20^3 chain and
    the 512 batched chains of this run) and of the standalone pyhea_trial_eval."""
    rng = np.random.default_rng(17)
    n = 4096
    pairs = torch.from_numpy(rng.integers(0, p.N, size=(n, 2)).astype(np.int32)).cuda()
    sp = torch.from_numpy(p.species).cuda()
    dS_i = torch.zeros(n, dtype=torch.float64, device="cuda")
    dS_f = torch.zeros(n, dtype=torch.float64, device="cuda")

    def timed(fn, reps, per):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps / per * 1e9

    args = (p.lattice, p.L, p.M, p.S, sp, p.target, p.weight)
    full = timed(lambda: pb.pyhea_trial_eval_full(*args, pairs, dS_f), 3, n)
    full64 = timed(lambda: pb.pyhea_trial_eval_full(*args, pairs[:64], dS_f[:64]), 20, 64)
    inc = timed(lambda: pb.pyhea_trial_eval(*args, pairs, dS_i), 3, n)
    res = {"full_ns_per_swap": full, "full_ns_per_swap_64_per_call": full64,
           "trial_eval_ns_per_swap": inc, "max_abs_dS_difference": (dS_i - dS_f).abs().max().item()}
    if out.get("value"):
        res["chain_ns_per_trial"] = 1e9 / out["value"]
        res["chain_reduction_vs_full_64"] = 1.0 - res["chain_ns_per_trial"] / full64
    if "batched" in out:
        res["batched_ns_per_trial"] = 1e9 / out["batched"]["trials_per_s"]
        res["batched_reduction_vs_full"] = 1.0 - res["batched_ns_per_trial"] / full
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(independent chains and batches shard across GPUs with no exchange).",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2411_18906_amd import binding as pb
    from paper_2411_18906_amd import workloads as wl

    torch.cuda.set_device(0)
    pb.lib()
    legs = set(args.legs.split(","))
    stream = torch.cuda.current_stream()

    # ---- inputs, resident in HBM -------------------------------------------------
    p = wl.fcc20_chain()
    N, M, S = p.N, p.M, p.S
    K = args.eval_configs
    eval_in = torch.from_numpy(wl.iid_configs(N, M, min(K, 2048), seed=2)).cuda()
    if K > eval_in.shape[0]:  # tile seeded blocks up to K configurations, each block re-permuted
        reps = (K + eval_in.shape[0] - 1) // eval_in.shape[0]
        blocks = [eval_in]
        g = torch.Generator(device="cuda").manual_seed(3)
        for r in range(1, reps):
            perm = torch.randperm(N, device="cuda", generator=g)
            blocks.append(eval_in[:, perm])
        eval_in = torch.cat(blocks)[:K].contiguous()
    counts = torch.zeros((K, S, M, M), dtype=torch.int32, device="cuda")
    S_F = torch.zeros((K, 2), dtype=torch.float64, device="cuda")
    chain0 = torch.from_numpy(p.species).cuda()
    chain = chain0.clone()
    log = torch.zeros((p.n_trials, 4), dtype=torch.int32, device="cuda")
    par = pb.make_params(p.seed, p.chain_id, p.n_trials, p.B)

    p1 = wl.fcc4_chain()
    chain1_0 = torch.from_numpy(p1.species).cuda()
    chain1 = chain1_0.clone()
    par1 = pb.make_params(p1.seed, p1.chain_id, p1.n_trials, p1.B)
    p3c = wl.fcc40_chain()
    chain3_0 = torch.from_numpy(p3c.species).cuda()
    chain3 = chain3_0.clone()
    par3 = pb.make_params(p3c.seed, p3c.chain_id, p3c.n_trials, p3c.B)

    chains = wl.mixed_chains(n_chains=args.chains)
    bspecies0 = torch.from_numpy(np.concatenate([c.species for c in chains])).cuda()
    bspecies = bspecies0.clone()
    boff = np.concatenate([[0], np.cumsum([c.N for c in chains])])
    bprobs = [(c.lattice, c.L, c.M, c.S, c.target, c.weight) for c in chains]
    bpars = [pb.make_params(c.seed, c.chain_id, c.n_trials, c.B) for c in chains]
    # the chains marshalled into the C structures once, as a caller that repeats a
    # batch does (the marshalling itself is timed and reported beside the leg)
    t_pack = time.perf_counter()
    bpack = pb.pack_batch(bprobs, bpars)
    pack_ms = 1e3 * (time.perf_counter() - t_pack)
    b_trials = sum(c.n_trials for c in chains)

    p3 = wl.fcc40_chain()
    K3 = 4096
    eval3_in = None
    if "eval3" in legs:
        blk = torch.from_numpy(wl.iid_configs(p3.N, p3.M, 256, seed=4)).cuda()
        g3 = torch.Generator(device="cuda").manual_seed(5)
        eval3_in = torch.cat([blk] + [blk[:, torch.randperm(p3.N, device="cuda", generator=g3)]
                                      for _ in range(K3 // 256 - 1)]).contiguous()
        counts3 = torch.zeros((K3, p3.S, p3.M, p3.M), dtype=torch.int32, device="cuda")
        S_F3 = torch.zeros((K3, 2), dtype=torch.float64, device="cuda")
    lat_counts = torch.zeros((1, S, M, M), dtype=torch.int32, device="cuda")
    lat_SF = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    lat_reps = 20

    copy_dst = torch.empty_like(eval_in) if "copy" in legs else None

    def step(ev):
        if "copy" in legs:   # plain copy of the evaluation batch: achievable HBM, counter calibration
            ev["copy0"].record(stream)
            copy_dst.copy_(eval_in)
            ev["copy1"].record(stream)
        if "eval" in legs:
            ev["eval0"].record(stream)
            pb.pyhea_sro_eval_batch(p.lattice, p.L, M, S, eval_in, counts, p.target, p.weight, S_F)
            ev["eval1"].record(stream)
        if "eval3" in legs:
            ev["eval30"].record(stream)
            pb.pyhea_sro_eval_batch(p3.lattice, p3.L, p3.M, p3.S, eval3_in, counts3, p3.target, p3.weight, S_F3)
            ev["eval31"].record(stream)
        if "lat" in legs:
            ev["lat0"].record(stream)
            for _ in range(lat_reps):
                pb.pyhea_sro_eval_batch(p.lattice, p.L, M, S, chain0.view(1, -1), lat_counts, p.target,
                                        p.weight, lat_SF)
            ev["lat1"].record(stream)
        if "chain" in legs:
            chain.copy_(chain0)
            ev["chain0"].record(stream)
            st, _ = pb.pyhea_mc_run(p.lattice, p.L, M, S, p.target, p.weight, chain, par, log)
            ev["chain1"].record(stream)
            ev["chain_stats"] = st
        if "chain1" in legs:
            chain1.copy_(chain1_0)
            ev["c1_0"].record(stream)
            st, _ = pb.pyhea_mc_run(p1.lattice, p1.L, p1.M, p1.S, p1.target, p1.weight, chain1, par1, None)
            ev["c1_1"].record(stream)
            ev["chain1_stats"] = st
        if "chain3" in legs:
            chain3.copy_(chain3_0)
            ev["c3_0"].record(stream)
            st, _ = pb.pyhea_mc_run(p3c.lattice, p3c.L, p3c.M, p3c.S, p3c.target, p3c.weight, chain3, par3, None)
            ev["c3_1"].record(stream)
            ev["chain3_stats"] = st
        if "batch" in legs:
            bspecies.copy_(bspecies0)
            ev["batch0"].record(stream)
            ev["batch_stats"] = pb.pyhea_mc_batch(bpack, bspecies, boff)
            ev["batch1"].record(stream)

    # one-time costs of a structure's first calls -- the single chains' measured
    # launch shapes and the recorded graph that later calls of the structure
    # replay -- paid here, untimed, with 64 trials per chain (the structure does
    # not depend on the trial count when every chain of a call has the same)
    progress("first use: launch shapes and recorded graphs")
    for _ in range(2):
        w = None
        if "chain" in legs:
            w = chain0.clone()
            pb.pyhea_mc_run(p.lattice, p.L, p.M, p.S, p.target, p.weight, w,
                            pb.make_params(p.seed, p.chain_id, 64, p.B), None)
        if "chain1" in legs:
            w = chain1_0.clone()
            pb.pyhea_mc_run(p1.lattice, p1.L, p1.M, p1.S, p1.target, p1.weight, w,
                            pb.make_params(p1.seed, p1.chain_id, 64, p1.B), None)
        if "chain3" in legs:
            w = chain3_0.clone()
            pb.pyhea_mc_run(p3c.lattice, p3c.L, p3c.M, p3c.S, p3c.target, p3c.weight, w,
                            pb.make_params(p3c.seed, p3c.chain_id, 64, p3c.B), None)
        if "batch" in legs:
            w = bspecies0.clone()
            pb.pyhea_mc_batch(bprobs, w, boff, [pb.make_params(c.seed, c.chain_id, 64, c.B) for c in chains])
        del w
    torch.cuda.synchronize()

    progress("inputs resident; warm-up")
    names = ["eval0", "eval1", "eval30", "eval31", "lat0", "lat1", "chain0", "chain1", "batch0", "batch1",
             "c1_0", "c1_1", "c3_0", "c3_1", "copy0", "copy1"]
    for _ in range(args.warmup):
        step({n: torch.cuda.Event(enable_timing=True) for n in names})
    torch.cuda.synchronize()
    evs = [{n: torch.cuda.Event(enable_timing=True) for n in names} for _ in range(args.steps)]
    progress(f"{args.steps} timed steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def leg_ms(a, b):
        return [e[a].elapsed_time(e[b]) for e in evs]

    out = {"metric": METRIC, "unit": "trial swaps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32 counts + f64 objective",
           "data": "synthetic (seeded)",
           "config": {"workload": "FCC 20x20x20 (32,000 sites), 5 species, shells 1-3, target 0, "
                                  "unit weights; chain of 10^6 trial swaps, B=64, disjoint commits",
                      "eval_batch": K, "batched_chains": len(chains),
                      "parallelism": "single GPU"}}
    if "chain" in legs:
        ms = np.array(leg_ms("chain0", "chain1"))
        out["value"] = p.n_trials / (ms.mean() / 1e3)
        st = evs[-1]["chain_stats"]
        out["chain"] = {"ms": float(ms.mean()), "trials": st["trials"], "commits": st["commits"],
                        "final_F": st["F"], "effective_trials_per_s":
                            (st["trials"] - st["null_trials"]) / (ms.mean() / 1e3),
                        "launch_shape": int(st["shape"]), "launch_shape_measured": bool(st["shape_measured"])}
    if "chain" in legs:
        # the chain's own roofline: bytes gathered per trial 2(1 + Z) (Z = 42), and
        # VALU lane operations per trial from the recorded instruction counts
        tps = out["value"]
        lane_ops = recorded("mc_chain_fcc20_counters.md", "mc_kernels.hip", "valu_lane_ops_per_trial")
        out["roofline_chain"] = {
            "bound": "latency", "gathered_bytes_per_trial": 86, "hbm_frac": tps * 86 / (HBM_PEAK_GBPS * 1e9),
            "valu_lane_ops_per_trial": lane_ops,
            "valu_frac_chip": None if lane_ops is None else tps * lane_ops / VALU_LANE_OPS_PEAK,
            "valu_frac_one_cu": None if lane_ops is None else tps * lane_ops / (VALU_LANE_OPS_PEAK / 256)}
    for leg, (a, b), pp, key, lanes_key in (("chain1", ("c1_0", "c1_1"), p1, "chain_fcc4", "fcc4"),
                                             ("chain3", ("c3_0", "c3_1"), p3c, "chain_fcc40", "fcc40")):
        if leg not in legs:
            continue
        ms = np.array(leg_ms(a, b))
        st = evs[-1][leg + "_stats"]
        tps = pp.n_trials / (ms.mean() / 1e3)
        zsum = {0: [12, 6, 24, 12], 1: [8, 6, 12, 24]}[pp.lattice][:pp.S]
        gathered = 2 * (1 + sum(zsum))
        out[key] = {"trials_per_s": tps, "ms": float(ms.mean()), "trials": st["trials"],
                    "commits": st["commits"], "final_F": st["F"],
                    "launch_shape": int(st["shape"]), "launch_shape_measured": bool(st["shape_measured"]),
                    "workload": f"FCC {pp.L[0]}^3 ({pp.N} sites), {pp.M} species, shells 1-{pp.S}, "
                                f"{pp.n_trials} trials, B={pp.B}, disjoint commits",
                    "roofline_chain": {"bound": "latency", "gathered_bytes_per_trial": gathered,
                                       "hbm_frac": tps * gathered / (HBM_PEAK_GBPS * 1e9)}}
    if "copy" in legs:
        ms = np.array(leg_ms("copy0", "copy1"))
        moved = 2 * eval_in.numel()   # read + write
        out["achievable_hbm"] = {"GBps": moved / (ms.mean() / 1e3) / 1e9, "ms": float(ms.mean()),
                                 "bytes_read_plus_written": moved,
                                 "what": "torch copy_ of the 1.05 GB evaluation batch (HIP copy kernel)"}
    if "eval" in legs:
        ms = np.array(leg_ms("eval0", "eval1"))
        alg_bytes = K * (N + S * M * M * 4 + 16)
        gbps = alg_bytes / (ms.mean() / 1e3) / 1e9
        out["sro_eval"] = {"GBps": gbps, "configs_per_s": K / (ms.mean() / 1e3), "ms": float(ms.mean()),
                           "ms_steps": [round(float(x), 4) for x in ms], "frac_hbm": gbps / HBM_PEAK_GBPS}
        tb = recorded_traffic()
        out["roofline"] = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": gbps / HBM_PEAK_GBPS,
                           "traffic": None if tb is None else tb / (ms.mean() / 1e3) / 1e9,
                           "kernel": "full SRO evaluation (pair counts + objective) of the batch"}
        # the same kernel against the VALU issue rate, from its recorded instruction count
        ops = recorded("full_eval_fcc20_5sp_traffic.md", "sro_bits.hip", "valu_lane_ops_per_site")
        if ops is not None:
            cap = VALU_LANE_OPS_PEAK / ops / 1e9   # GB/s at one byte per site
            out["roofline_valu"] = {"bound": "alu", "lane_ops_per_site": ops, "valu_cap_GBps": cap,
                                    "frac": gbps / cap}
    if "eval3" in legs:
        ms = np.array(leg_ms("eval30", "eval31"))
        gbps = K3 * (p3.N + p3.S * p3.M * p3.M * 4 + 16) / (ms.mean() / 1e3) / 1e9
        out["sro_eval_fcc40"] = {"GBps": gbps, "configs_per_s": K3 / (ms.mean() / 1e3), "ms": float(ms.mean()),
                                 "frac_hbm": gbps / HBM_PEAK_GBPS, "configs": K3,
                                 "workload": "FCC 40x40x40 (256,000 sites), 4 species, shells 1-2"}
    if "lat" in legs:
        ms = np.array(leg_ms("lat0", "lat1"))
        out["sro_eval_one_config_us"] = float(ms.mean() * 1e3 / lat_reps)
        # the single-configuration entry point itself, synchronous: counts, alpha,
        # S and F of the FCC 20^3 configuration read back to the host per call
        one = chain0.contiguous()
        for _ in range(5):
            pb.pyhea_sro_eval(p.lattice, p.L, M, S, one, p.target, p.weight)
        t_s = time.perf_counter()
        for _ in range(50):
            pb.pyhea_sro_eval(p.lattice, p.L, M, S, one, p.target, p.weight)
        out["sro_eval_sync_us"] = (time.perf_counter() - t_s) / 50 * 1e6
    if "batch" in legs:
        ms = np.array(leg_ms("batch0", "batch1"))
        bst = evs[-1]["batch_stats"]
        fs = np.array([s["F"] for s in bst])
        out["batched"] = {"trials_per_s": b_trials / (ms.mean() / 1e3), "ms": float(ms.mean()),
                          "chains": len(chains), "trials": b_trials,
                          "mean_final_F": float(fs.mean()),
                          "graph_replayed": bool(bst["graph"].all()),
                          "python_pack_ms": pack_ms,
                          "trials_per_s_with_pack": b_trials / ((ms.mean() + pack_ms) / 1e3)}
        if "chain" in legs:
            out["batched"]["vs_fcc20_chain"] = out["batched"]["trials_per_s"] / out["value"]
        if not args.no_plain:
            progress("plain chains one after another")
            # the same chains one after another through the single-chain entry point;
            # its launch shapes are measured on the first chain of each kind, which
            # happens in a short untimed pass first
            warm = bspecies0.clone()
            for i, c in enumerate(chains):
                pb.pyhea_mc_run(c.lattice, c.L, c.M, c.S, c.target, c.weight, warm[boff[i]:boff[i + 1]],
                                pb.make_params(c.seed, c.chain_id, 64, c.B), None)
            del warm
            batched_final = bspecies.clone()
            bspecies.copy_(bspecies0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i, c in enumerate(chains):
                view = bspecies[boff[i]:boff[i + 1]]
                pb.pyhea_mc_run(c.lattice, c.L, c.M, c.S, c.target, c.weight, view, bpars[i], None)
            e1.record(stream)
            torch.cuda.synchronize()
            pms = e0.elapsed_time(e1)
            same = bool(torch.equal(bspecies, batched_final))
            out["batched"]["plain_ms"] = pms
            out["batched"]["plain_trials_per_s"] = b_trials / (pms / 1e3)
            out["batched"]["vs_plain"] = pms / float(ms.mean())
            out["batched"]["plain_final_equal"] = same
            if not same:
                print("batched and plain chains ended in different configurations", file=sys.stderr)
                sys.exit(1)
    if args.serve_jobs > 0:
        progress("serving: capacity run")
        # capacity of the server on this job mix: every job submitted at once
        probe = serve(pb, wl, args.serve_jobs, 0.0, 0.0, args.serve_budget_mb)
        out["serving_capacity"] = {k: probe[k] for k in ("jobs", "trials", "span_s", "trials_per_s", "rounds")}
        out["serving_capacity"]["what"] = "all jobs submitted at t = 0 (saturated server)"
        progress("serving: Poisson arrivals")
        # Poisson arrivals at a fraction of that capacity: latency of a server that keeps up
        out["serving"] = serve(pb, wl, args.serve_jobs, probe["trials_per_s"], args.serve_load, args.serve_budget_mb)
        out["serving"]["capacity_source"] = "saturated run of the same job mix (serving_capacity)"
    if not args.no_best:
        progress("BEST vs DISJOINT")
        # FCC 20^3 with target 0 starts near its optimum; FCC 40^3 with a nonzero
        # target is far from it (its DISJOINT chain meets the target within ~10^5 trials)
        out["best_vs_disjoint"] = {"fcc20": best_vs_disjoint(pb, p, torch),
                                   "fcc40": best_vs_disjoint(pb, wl.fcc40_chain(), torch, T=200_000)}
    if not args.no_global:
        progress("global search")
        out["global_search"] = global_search(pb, p, torch)
    if not args.no_baseline:
        progress("incremental vs full")
        out["incremental_vs_full"] = incremental_vs_full(pb, p, torch, out)
    if "value" not in out:
        out["value"] = None
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(p)
        if not args.no_cpu_batch and "batch" in legs:
            out["cpu_baseline_batched"] = cpu_batch_baseline(chains)
            out["cpu_baseline_batched"]["gpu_batched_trials_per_s"] = out["batched"]["trials_per_s"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
