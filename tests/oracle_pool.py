"""A process pool that runs oracle chains beside the GPU tests.

Test infrastructure: the full-length parity cases need minutes of oracle CPU
time in total, spread over many independent chains, so they are computed in
worker processes (spawned, never forked from a process that holds the GPU)
while the GPU side runs.  Workers only import the oracle.
"""
from __future__ import annotations

import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

_pool = None


def workers() -> int:
    # at most 16 workers: the process may hold a share of 16 CPUs whatever os.cpu_count() shows
    return max(1, min(16, os.cpu_count() or 1))


def pool() -> ProcessPoolExecutor:
    global _pool
    if _pool is None:
        _pool = ProcessPoolExecutor(max_workers=workers(), mp_context=multiprocessing.get_context("spawn"))
    return _pool


def shutdown():
    global _pool
    if _pool is not None:
        _pool.shutdown(wait=False, cancel_futures=True)
        _pool = None


def chain_job(p, *, n_trials=None, chain_id=None, log_cap=None, mode=0, depth_limit=0, tau=0.0):
    """Arguments of one oracle chain for problem p (a workloads.Problem)."""
    return dict(lattice=p.lattice, L=tuple(p.L), M=p.M, S=p.S, target=p.target, weight=p.weight,
                species=p.species, seed=p.seed, chain_id=p.chain_id if chain_id is None else chain_id,
                n_trials=p.n_trials if n_trials is None else n_trials, B=p.B, mode=mode,
                depth_limit=depth_limit, tau=tau, log_cap=log_cap)


def run_chain(job: dict):
    """Worker side: oracle.mc_run on one job dict."""
    from oracle import oracle as orc
    j = dict(job)
    args = [j.pop(k) for k in ("lattice", "L", "M", "S", "target", "weight", "species")]
    return orc.mc_run(*args, **j)


def submit_chain(job: dict):
    return pool().submit(run_chain, job)
