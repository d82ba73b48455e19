"""Thin ctypes binding of libpyhea (include/pyhea.h).

Functions carry the C names and only marshal arguments: torch tensors become
device pointers, numpy arrays become host pointers, and the current torch
stream is passed as the HIP stream.  Every computation runs in the HIP
library; if the library is missing this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes
import itertools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpyhea.so")

OK, EINVAL, ENOMEM, EDEVICE, EBUSY, ECANCELLED, ENOSYS, ENOENT = 0, -1, -2, -3, -4, -5, -6, -7
FCC, BCC = 0, 1
MODE_DISJOINT, MODE_BEST = 0, 1
STOP_TRIALS, STOP_DEPTH = 0, 1

EXPORTS = [
    "pyhea_version", "pyhea_last_error", "pyhea_sro_eval", "pyhea_sro_eval_batch",
    "pyhea_trial_eval", "pyhea_mc_run", "pyhea_mc_batch", "pyhea_serve_open",
    "pyhea_serve_submit", "pyhea_serve_poll", "pyhea_serve_cancel", "pyhea_serve_counters",
    "pyhea_serve_close", "pyhea_philox4x32_10", "pyhea_tune_force",
    "pyhea_tune_force_eval", "pyhea_tune_force_lookahead", "pyhea_global_search",
    "pyhea_random_configs", "pyhea_trial_eval_full", "pyhea_sro_eval_batch_noalloc",
    "pyhea_tune_force_stream", "pyhea_map_sites", "pyhea_tune_measure", "pyhea_tune_graphs",
]


class PyheaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pyhea error {code}: {msg}")
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("L", ctypes.c_int32 * 3),
                ("n_species", ctypes.c_int32), ("n_shells", ctypes.c_int32)]


class Objective(ctypes.Structure):
    _fields_ = [("target", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class McParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("chain_id", ctypes.c_uint32),
                ("cand_per_step", ctypes.c_int32), ("n_trials", ctypes.c_int64),
                ("commit_mode", ctypes.c_int32), ("depth_limit", ctypes.c_int32),
                ("accept_tol", ctypes.c_double)]


class GlobalParams(ctypes.Structure):
    _fields_ = [("n_solutions", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("n_refine", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("discard_frac", ctypes.c_double), ("local", McParams)]


class GlobalStats(ctypes.Structure):
    _fields_ = [("evaluations", ctypes.c_int64), ("trials", ctypes.c_int64),
                ("commits", ctypes.c_int64), ("S", ctypes.c_double), ("F", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class McStats(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int64), ("null_trials", ctypes.c_int64),
                ("commits", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("stop_reason", ctypes.c_int32), ("status", ctypes.c_int32),
                ("S", ctypes.c_double), ("F", ctypes.c_double), ("log_len", ctypes.c_int64),
                ("shape", ctypes.c_int32), ("shape_measured", ctypes.c_int32), ("graph", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libpyhea.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "pyhea_version": ([], i32),
            "pyhea_last_error": ([], ctypes.c_char_p),
            "pyhea_sro_eval": ([P, P, P, P, P, P, P], i32),
            "pyhea_sro_eval_batch": ([P, i64, P, P, P, P, P], i32),
            "pyhea_sro_eval_batch_noalloc": ([P, i64, P, P, P, P, P], i32),
            "pyhea_trial_eval": ([P, P, P, i64, P, P, P, P], i32),
            "pyhea_mc_run": ([P, P, P, P, P, i64, P, P, P], i32),
            "pyhea_mc_batch": ([i32, P, P, P, P, P, P, P, P, P], i32),
            "pyhea_serve_open": ([i64, i32, i32, P], i32),
            "pyhea_serve_submit": ([P, u64, P, P, P, P], i32),
            "pyhea_serve_poll": ([P, u64, P, P, P, i32], i32),
            "pyhea_serve_cancel": ([P, u64], i32),
            "pyhea_serve_counters": ([P, P], i32),
            "pyhea_serve_close": ([P], i32),
            "pyhea_philox4x32_10": ([P, u64, i64, P, P], i32),
            "pyhea_tune_force": ([i32], i32),
            "pyhea_tune_force_eval": ([i32], i32),
            "pyhea_tune_force_stream": ([i32, i32], i32),
            "pyhea_map_sites": ([P, P, ctypes.c_double, i64, P, P, P, P, P], i32),
            "pyhea_tune_measure": ([i32], i32),
            "pyhea_tune_graphs": ([i32], i32),
            "pyhea_tune_force_lookahead": ([i32], i32),
            "pyhea_global_search": ([P, P, P, P, P, P, P, P], i32),
            "pyhea_random_configs": ([i64, i32, P, u64, ctypes.c_uint32, ctypes.c_uint32, i32, P, P], i32),
            "pyhea_trial_eval_full": ([P, P, P, i64, P, P, P], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(code: int):
    if code != OK:
        raise PyheaError(code, lib().pyhea_last_error().decode())
    return code


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t, dtype=None):
    """Device pointer of a contiguous torch tensor on the GPU."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: np.ndarray | None):
    # the array interface's address (numpy's .ctypes helper object costs ~17 us)
    return None if a is None else ctypes.c_void_p(a.__array_interface__["data"][0])


def make_lattice(lattice: int, L, M: int, S: int) -> Lattice:
    return Lattice(lattice, (ctypes.c_int32 * 3)(*[int(x) for x in L]), M, S)


def n_sites(lattice: int, L) -> int:
    """Sites of the supercell (4 per FCC cell, 2 per BCC cell); the library
    itself rejects a malformed lattice code."""
    a = 4 if lattice == FCC else 2
    return a * int(L[0]) * int(L[1]) * int(L[2])


def _need(t, numel: int, what: str):
    """Raise ValueError unless buffer t holds exactly numel elements."""
    n = int(t.numel()) if hasattr(t, "numel") and callable(t.numel) else int(np.asarray(t).size)
    if n != numel:
        raise ValueError(f"{what}: expected {numel} elements, got {n}")


def _need_shape(t, shape, what: str):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


class _Obj:
    """Objective with its host arrays kept alive."""

    def __init__(self, target, weight, S: int, M: int):
        self.t = np.ascontiguousarray(np.asarray(target, dtype=np.float64).reshape(S, M, M))
        self.w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64).reshape(S))
        self.c = Objective(_hptr(self.t), _hptr(self.w))


def make_params(seed: int, chain_id: int, n_trials: int, B: int = 64, mode: int = MODE_DISJOINT,
                depth_limit: int = 0, tau: float = 0.0) -> McParams:
    return McParams(seed, chain_id, B, n_trials, mode, depth_limit, tau)


# --------------------------------------------------------------------------- API

def pyhea_version() -> int:
    return int(lib().pyhea_version())


def pyhea_sro_eval(lattice: int, L, M: int, S: int, species, target=None, weight=None,
                   stream=None):
    """Full evaluation of one configuration: (counts int64, alpha, S, F)."""
    import torch
    lat = make_lattice(lattice, L, M, S)
    _need(species, n_sites(lattice, L), "species")
    counts = np.zeros((S, M, M), np.int64)
    alpha = np.zeros((S, M, M))
    sf = np.zeros(2)
    obj = _Obj(target, weight, S, M) if target is not None else None
    _check(lib().pyhea_sro_eval(ctypes.byref(lat), _dptr(species, torch.int8),
                                ctypes.byref(obj.c) if obj else None, _hptr(counts), _hptr(alpha),
                                _hptr(sf), _stream(stream)))
    return counts, alpha, (float(sf[0]) if obj else None), (float(sf[1]) if obj else None)


def pyhea_sro_eval_batch(lattice: int, L, M: int, S: int, species, counts, target=None,
                         weight=None, S_F=None, stream=None):
    """Full evaluation of K configurations species[K][N] into counts[K][S][M][M]
    (int32) and optionally S_F[K][2]; asynchronous on the stream."""
    _eval_batch("pyhea_sro_eval_batch", lattice, L, M, S, species, counts, target, weight, S_F, stream)


def pyhea_sro_eval_batch_noalloc(lattice: int, L, M: int, S: int, species, counts, target=None,
                                 weight=None, S_F=None, stream=None):
    """pyhea_sro_eval_batch whose scratch is the library's fixed device array
    (the call allocates no device memory)."""
    _eval_batch("pyhea_sro_eval_batch_noalloc", lattice, L, M, S, species, counts, target, weight, S_F,
                stream)


def _eval_batch(fn, lattice, L, M, S, species, counts, target, weight, S_F, stream):
    import torch
    lat = make_lattice(lattice, L, M, S)
    N = n_sites(lattice, L)
    if species.dim() != 2 or species.shape[1] != N:
        raise ValueError(f"species: expected shape [K][{N}], got {tuple(species.shape)}")
    K = species.shape[0]
    _need(counts, K * S * M * M, "counts")
    if S_F is not None:
        _need(S_F, 2 * K, "S_F")
    obj = _Obj(target, weight, S, M) if target is not None else None
    _check(getattr(lib(), fn)(ctypes.byref(lat), K, _dptr(species, torch.int8),
                              ctypes.byref(obj.c) if obj else None,
                              _dptr(counts, torch.int32),
                              _dptr(S_F, torch.float64) if S_F is not None else None,
                              _stream(stream)))


def pyhea_map_sites(lattice: int, L, M: int, S: int, box, max_disp: float, xyz, types, species,
                    atom_of_site=None, stream=None):
    """Nearest-site assignment of an external structure: xyz [N][3] float64 and
    types [N] int8 (device) onto species [N] int8 (device, written); optional
    atom_of_site [N] int32 (device, written)."""
    import torch
    lat = make_lattice(lattice, L, M, S)
    N = n_sites(lattice, L)
    _need_shape(xyz, (N, 3), "xyz")
    _need(types, N, "types")
    _need(species, N, "species")
    if atom_of_site is not None:
        _need(atom_of_site, N, "atom_of_site")
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
    _check(lib().pyhea_map_sites(ctypes.byref(lat), _hptr(b), float(max_disp), N, _dptr(xyz, torch.float64),
                                 _dptr(types, torch.int8), _dptr(species, torch.int8),
                                 _dptr(atom_of_site, torch.int32) if atom_of_site is not None else None,
                                 _stream(stream)))


def _pairs_check(pairs):
    if pairs.dim() != 2 or pairs.shape[1] != 2:
        raise ValueError(f"pairs: expected shape [n][2], got {tuple(pairs.shape)}")


def pyhea_trial_eval(lattice: int, L, M: int, S: int, species, target, weight, pairs, dS,
                     dN=None, stream=None):
    import torch
    lat = make_lattice(lattice, L, M, S)
    _need(species, n_sites(lattice, L), "species")
    _pairs_check(pairs)
    _need(dS, pairs.shape[0], "dS")
    if dN is not None:
        _need(dN, pairs.shape[0] * S * M * M, "dN")
    obj = _Obj(target, weight, S, M)
    _check(lib().pyhea_trial_eval(ctypes.byref(lat), ctypes.byref(obj.c), _dptr(species, torch.int8),
                                  pairs.shape[0], _dptr(pairs, torch.int32), _dptr(dS, torch.float64),
                                  _dptr(dN, torch.int32) if dN is not None else None,
                                  _stream(stream)))


def pyhea_trial_eval_full(lattice: int, L, M: int, S: int, species, target, weight, pairs, dS, stream=None):
    """dS of each swap from full evaluations before and after (the
    non-incremental baseline)."""
    import torch
    lat = make_lattice(lattice, L, M, S)
    _need(species, n_sites(lattice, L), "species")
    _pairs_check(pairs)
    _need(dS, pairs.shape[0], "dS")
    obj = _Obj(target, weight, S, M)
    _check(lib().pyhea_trial_eval_full(ctypes.byref(lat), ctypes.byref(obj.c), _dptr(species, torch.int8),
                                       pairs.shape[0], _dptr(pairs, torch.int32), _dptr(dS, torch.float64),
                                       _stream(stream)))


def pyhea_mc_run(lattice: int, L, M: int, S: int, target, weight, species, params: McParams,
                 log=None, stream=None):
    """One chain; species (device int8 [N]) is updated in place.  Returns
    (stats dict, final counts int64 [S][M][M])."""
    import torch
    lat = make_lattice(lattice, L, M, S)
    _need(species, n_sites(lattice, L), "species")
    if log is not None and (log.dim() != 2 or log.shape[1] != 4):
        raise ValueError(f"log: expected shape [cap][4], got {tuple(log.shape)}")
    obj = _Obj(target, weight, S, M)
    st = McStats()
    counts = np.zeros((S, M, M), np.int64)
    cap = 0 if log is None else log.shape[0]
    _check(lib().pyhea_mc_run(ctypes.byref(lat), ctypes.byref(obj.c), ctypes.byref(params),
                              _dptr(species, torch.int8),
                              _dptr(log, torch.int32) if log is not None else None, cap,
                              ctypes.byref(st), _hptr(counts), _stream(stream)))
    return st.as_dict(), counts


_LAT_DTYPE = np.dtype([("lattice", "<i4"), ("L", "<i4", (3,)), ("n_species", "<i4"), ("n_shells", "<i4")])


def _batch_descriptors(problems):
    """Lattice array, objective pointer array and the host block they point
    into, for n problems, built with a few numpy calls."""
    n = len(problems)
    lat = np.fromiter(itertools.chain.from_iterable((p[0], *p[1], p[2], p[3]) for p in problems),
                      dtype=np.int32, count=6 * n).view(_LAT_DTYPE)
    try:
        block = np.concatenate([a.ravel() for p in problems for a in (p[4], p[5])]).astype(np.float64, copy=False)
    except AttributeError:   # targets or weights given as sequences
        block = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for p in problems for a in (p[4], p[5])])
    block = np.ascontiguousarray(block)
    S = lat["n_shells"].astype(np.int64)
    E = S * lat["n_species"].astype(np.int64) ** 2
    start = np.concatenate([[0], np.cumsum(E + S)])
    if block.size != start[-1]:
        raise ValueError("target/weight sizes do not match the problems' S and M")
    obj = np.empty((n, 2), np.uint64)
    obj[:, 0] = block.ctypes.data + 8 * start[:-1]
    obj[:, 1] = block.ctypes.data + 8 * (start[:-1] + E)
    return lat, obj, block


_STATS_DTYPE = np.dtype(McStats)


def _params_block(params_list):
    """The McParams array as one host buffer (bytes of each structure)."""
    if all(type(x) is McParams for x in params_list):
        raw = b"".join(map(bytes, params_list))
    else:
        raw = bytes((McParams * len(params_list))(*params_list))
    return np.frombuffer(raw, dtype=np.uint8).copy()   # aligned, owned


class BatchPack:
    """The chains of a batched call marshalled once into the C structures
    (lattices, objectives, parameters), for callers that repeat a batch; pass
    it to pyhea_mc_batch in place of the problem and parameter lists."""

    def __init__(self, problems, params_list):
        self.n = len(problems)
        if len(params_list) != self.n:
            raise ValueError("one parameter set per problem")
        self.lat, self.obj, self.block = _batch_descriptors(problems)
        self.pars = _params_block(params_list)
        a = np.where(self.lat["lattice"] == FCC, 4, 2).astype(np.int64)
        self.sizes = a * self.lat["L"].astype(np.int64).prod(axis=1)


def pack_batch(problems, params_list) -> BatchPack:
    return BatchPack(problems, params_list)


def pyhea_mc_batch(problems, species, offsets, params_list=None, log=None, log_offsets=None,
                   stream=None):
    """Many chains in one call.  problems: list of (lattice, L, M, S, target,
    weight) with params_list, or a BatchPack; species: device int8, chains
    concatenated; offsets: [n+1] int64.  Returns the per-chain stats as a
    numpy structured array (fields of pyhea_mc_stats: stats[i]["F"], ...)."""
    import torch
    if isinstance(problems, BatchPack):
        if params_list is not None:
            raise ValueError("a BatchPack carries its parameters")
        pack = problems
    else:
        if params_list is None:
            raise ValueError("one parameter set per problem")
        pack = BatchPack(problems, params_list)
    n = pack.n
    stats = np.zeros(n, dtype=_STATS_DTYPE)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    loff = None if log_offsets is None else np.ascontiguousarray(np.asarray(log_offsets, np.int64))
    # every chain's slice must hold exactly its sites, and the slices must tile species
    if off.shape != (n + 1,) or off[0] != 0 or not np.array_equal(np.diff(off), pack.sizes):
        raise ValueError("offsets: need n+1 values from 0 whose differences are each chain's site count")
    _need(species, int(off[-1]), "species")
    if log is not None:
        if log.dim() != 2 or log.shape[1] != 4:
            raise ValueError(f"log: expected shape [cap][4], got {tuple(log.shape)}")
        if loff is None or loff.shape != (n + 1,) or loff[0] != 0 or np.any(np.diff(loff) < 0) \
                or loff[-1] > log.shape[0]:
            raise ValueError("log_offsets: need n+1 non-decreasing values from 0 within the log's rows")
    _check(lib().pyhea_mc_batch(n, _hptr(pack.lat), _hptr(pack.obj), _hptr(pack.pars), _dptr(species, torch.int8),
                                _hptr(off), _dptr(log, torch.int32) if log is not None else None,
                                _hptr(loff), _hptr(stats), _stream(stream)))
    return stats


def pyhea_philox4x32_10(ctr, seed: int, out, stream=None):
    import torch
    _need_shape(ctr, (ctr.shape[0], 4), "ctr")
    _need_shape(out, tuple(ctr.shape), "out")
    _check(lib().pyhea_philox4x32_10(_dptr(ctr, torch.int32), seed, ctr.shape[0],
                                     _dptr(out, torch.int32), _stream(stream)))


def pyhea_random_configs(N: int, composition, seed: int, iteration: int, slot0: int, out, stream=None):
    """Random global-search solutions into out[n][N] (device int8)."""
    import torch
    comp = np.ascontiguousarray(np.asarray(composition, dtype=np.int64))
    if out.dim() != 2 or out.shape[1] != N:
        raise ValueError(f"out: expected shape [n][{N}], got {tuple(out.shape)}")
    _check(lib().pyhea_random_configs(N, comp.size, _hptr(comp), seed, iteration, slot0, out.shape[0],
                                      _dptr(out, torch.int8), _stream(stream)))


def pyhea_global_search(lattice: int, L, M: int, S: int, target, weight, composition, best, *,
                        n_solutions: int, iterations: int, n_refine: int, discard_frac: float,
                        seed: int, B: int, n_trials: int, mode: int = MODE_DISJOINT,
                        depth_limit: int = 0, tau: float = 0.0, stream=None):
    """Algorithm 1; best (device int8 [N]) receives the best solution.
    Returns (stats dict, best F after each iteration)."""
    import torch
    lat = make_lattice(lattice, L, M, S)
    _need(best, n_sites(lattice, L), "best")
    obj = _Obj(target, weight, S, M)
    comp = np.ascontiguousarray(np.asarray(composition, dtype=np.int64))
    if comp.size != M:
        raise ValueError(f"composition: expected {M} species counts, got {comp.size}")
    p = GlobalParams(n_solutions, iterations, n_refine, 0, discard_frac,
                     make_params(seed, 0, n_trials, B, mode, depth_limit, tau))
    hist = np.zeros(max(iterations, 1))
    st = GlobalStats()
    _check(lib().pyhea_global_search(ctypes.byref(lat), ctypes.byref(obj.c), _hptr(comp), ctypes.byref(p),
                                     _dptr(best, torch.int8), _hptr(hist), ctypes.byref(st), _stream(stream)))
    return st.as_dict(), hist[:iterations]


def pyhea_tune_force(variant: int):
    _check(lib().pyhea_tune_force(variant))


def pyhea_tune_force_eval(kernel: int):
    _check(lib().pyhea_tune_force_eval(kernel))


def pyhea_tune_measure(on: bool):
    _check(lib().pyhea_tune_measure(1 if on else 0))


def pyhea_tune_graphs(on: bool):
    """Replay recorded graphs for repeated chain calls of one structure (default on)."""
    _check(lib().pyhea_tune_graphs(1 if on else 0))


def pyhea_tune_force_stream(layers_per_group: int, threads: int):
    _check(lib().pyhea_tune_force_stream(int(layers_per_group), int(threads)))


def pyhea_tune_force_lookahead(steps: int):
    _check(lib().pyhea_tune_force_lookahead(steps))


class Server:
    """Serving handle: pyhea_serve_open / submit / poll / cancel / counters / close."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, steps_per_round: int = 0):
        h = ctypes.c_void_p()
        _check(lib().pyhea_serve_open(hbm_budget_bytes, max_slots, steps_per_round, ctypes.byref(h)))
        self.h = h
        self.n_of = {}   # job id -> sites, checked against the poll's output buffer

    def pyhea_serve_submit(self, job_id: int, lattice: int, L, M: int, S: int, target, weight,
                           species: np.ndarray, params: McParams):
        lat = make_lattice(lattice, L, M, S)
        obj = _Obj(target, weight, S, M)
        sp = np.ascontiguousarray(species, dtype=np.int8)
        N = n_sites(lattice, L)
        _need(sp, N, "species")
        _check(lib().pyhea_serve_submit(self.h, job_id, ctypes.byref(lat), ctypes.byref(obj.c),
                                        ctypes.byref(params), _hptr(sp)))
        self.n_of[job_id] = N

    def pyhea_serve_poll(self, job_id: int, N: int, blocking: bool = True):
        """(status, final species or None, stats dict, (submit, admit, finish) ns)."""
        if job_id in self.n_of and self.n_of[job_id] != N:
            raise ValueError(f"job {job_id} has {self.n_of[job_id]} sites, not {N}")
        # a job this handle did not submit gets no output buffer (the library
        # answers ENOENT or its status)
        out = np.zeros(N, np.int8) if job_id in self.n_of else None
        st = McStats()
        times = np.zeros(3, np.int64)
        code = lib().pyhea_serve_poll(self.h, job_id, _hptr(out), ctypes.byref(st), _hptr(times),
                                      1 if blocking else 0)
        if code == EBUSY:
            return code, None, None, None
        self.n_of.pop(job_id, None)   # a polled job is forgotten
        return code, (out if code == OK else None), st.as_dict(), tuple(int(t) for t in times)

    def pyhea_serve_cancel(self, job_id: int) -> int:
        return int(lib().pyhea_serve_cancel(self.h, job_id))

    def pyhea_serve_counters(self) -> dict:
        out = np.zeros(8, np.int64)
        _check(lib().pyhea_serve_counters(self.h, _hptr(out)))
        keys = ["submitted", "admitted", "finished", "rejected", "resident", "queued", "rounds",
                "bytes_resident"]
        return dict(zip(keys, (int(v) for v in out)))

    def pyhea_serve_close(self):
        if self.h:
            _check(lib().pyhea_serve_close(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.pyhea_serve_close()
