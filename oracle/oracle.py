"""ctypes front end of the CPU oracle (``sro_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.

Every function takes and returns numpy arrays.  ``build()`` compiles the C
source with ``-O2 -ffp-contract=off`` (no fused multiply-add, no fast-math), so
all binary64 results are fixed to the bit.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sro_oracle.c")
_LIB = os.path.join(_HERE, "libsro_oracle.so")

FCC, BCC = 0, 1
MODE_DISJOINT, MODE_BEST = 0, 1


class McStats(ctypes.Structure):
    _fields_ = [
        ("trials", ctypes.c_int64),
        ("null_trials", ctypes.c_int64),
        ("commits", ctypes.c_int64),
        ("steps", ctypes.c_int64),
        ("stop_reason", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("S", ctypes.c_double),
        ("F", ctypes.c_double),
        ("log_len", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


def build() -> str:
    """Compile the oracle into a shared library next to its source."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall",
           "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.or_shells.argtypes = [i32, i32, P, P, P]
        L.or_shells.restype = i32
        L.or_n_sites.argtypes = [i32, P]
        L.or_n_sites.restype = i64
        L.or_site_pos.argtypes = [i32, P, i64, P]
        L.or_site_id.argtypes = [i32, P, P]
        L.or_site_id.restype = i64
        L.or_neighbors.argtypes = [i32, P, i32, i64, P]
        L.or_neighbors.restype = i32
        L.or_validate.argtypes = [i32, P, i32, i32, P]
        L.or_validate.restype = i32
        L.or_counts.argtypes = [i32, P, i32, i32, P, P]
        L.or_alpha_objective.argtypes = [i32, P, i32, i32, P, P, P, P, P, P, P]
        L.or_swap_delta.argtypes = [i32, P, i32, i32, P, i64, i64, P]
        L.or_swap_dS.argtypes = [i32, P, i32, i32, P, i64, i64, P, P]
        L.or_swap_dS.restype = ctypes.c_double
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_mc_run.argtypes = [i32, P, i32, i32, P, P, ctypes.c_uint64, ctypes.c_uint32, i64,
                                i32, i32, i32, ctypes.c_double, P, P, i64,
                                ctypes.POINTER(McStats), P]
        L.or_mc_run.restype = i32
        L.or_random_config.argtypes = [i64, i32, P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, P]
        L.or_random_config.restype = i32
        L.or_map_sites.argtypes = [i32, P, i32, P, ctypes.c_double, i64, P, P, P, P]
        L.or_map_sites.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _L(L) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32).reshape(3))


def shells(lattice: int, n_shells: int):
    """(r2[S], z[S], offsets[sum z][3]) in half-lattice units."""
    r2 = np.zeros(4, np.int32)
    z = np.zeros(4, np.int32)
    off = np.zeros((64, 3), np.int32)
    n = lib().or_shells(lattice, n_shells, _p(r2), _p(z), _p(off))
    if n < 0:
        raise ValueError("bad lattice or shell count")
    return r2[:n_shells].copy(), z[:n_shells].copy(), off[:n].copy()


def n_sites(lattice: int, L) -> int:
    return int(lib().or_n_sites(lattice, _p(_L(L))))


def site_pos(lattice: int, L, p: int) -> np.ndarray:
    pos = np.zeros(3, np.int32)
    lib().or_site_pos(lattice, _p(_L(L)), p, _p(pos))
    return pos


def neighbors(lattice: int, L, n_shells: int, p: int) -> np.ndarray:
    out = np.zeros(64, np.int64)
    n = lib().or_neighbors(lattice, _p(_L(L)), n_shells, p, _p(out))
    return out[:n].copy()


def validate(lattice: int, L, M: int, S: int, species: np.ndarray | None) -> int:
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int8)
    return int(lib().or_validate(lattice, _p(_L(L)), M, S, None if sp is None else _p(sp)))


def counts(lattice: int, L, M: int, S: int, species: np.ndarray) -> np.ndarray:
    sp = np.ascontiguousarray(species, dtype=np.int8)
    out = np.zeros((S, M, M), np.int64)
    lib().or_counts(lattice, _p(_L(L)), M, S, _p(sp), _p(out))
    return out


def alpha_objective(lattice: int, L, M: int, S: int, species: np.ndarray, cnt: np.ndarray,
                    target: np.ndarray, weight: np.ndarray):
    """(alpha[S][M][M], sq[S][M][M] = (alpha - target)^2, S, F) by Eq. 2-3."""
    sp = np.ascontiguousarray(species, dtype=np.int8)
    c = np.ascontiguousarray(cnt, dtype=np.int64)
    t = np.ascontiguousarray(target, dtype=np.float64).reshape(S, M, M)
    w = np.ascontiguousarray(weight, dtype=np.float64).reshape(S)
    alpha = np.zeros((S, M, M))
    sq = np.zeros((S, M, M))
    sf = np.zeros(2)
    lib().or_alpha_objective(lattice, _p(_L(L)), M, S, _p(sp), _p(c), _p(t), _p(w), _p(alpha),
                             _p(sq), _p(sf))
    return alpha, sq, float(sf[0]), float(sf[1])


def swap_delta(lattice: int, L, M: int, S: int, species: np.ndarray, p: int, q: int):
    sp = np.ascontiguousarray(species, dtype=np.int8)
    out = np.zeros((S, M, M), np.int64)
    lib().or_swap_delta(lattice, _p(_L(L)), M, S, _p(sp), p, q, _p(out))
    return out


def swap_dS(lattice: int, L, M: int, S: int, species: np.ndarray, p: int, q: int,
            target: np.ndarray, weight: np.ndarray) -> float:
    sp = np.ascontiguousarray(species, dtype=np.int8)
    t = np.ascontiguousarray(target, dtype=np.float64).reshape(S, M, M)
    w = np.ascontiguousarray(weight, dtype=np.float64).reshape(S)
    return float(lib().or_swap_dS(lattice, _p(_L(L)), M, S, _p(sp), p, q, _p(t), _p(w)))


def swap_dS_recount(lattice: int, L, M: int, S: int, species: np.ndarray, p: int, q: int, target,
                    weight) -> float:
    """dS of swapping sites p and q from two full evaluations (Eq. 2-3):
    S(after) - S(before), the recalculation the incremental update replaces."""
    sp = np.array(species, dtype=np.int8, copy=True)
    _, _, S0, _ = alpha_objective(lattice, L, M, S, sp, counts(lattice, L, M, S, sp), target, weight)
    sp[p], sp[q] = sp[q], sp[p]
    _, _, S1, _ = alpha_objective(lattice, L, M, S, sp, counts(lattice, L, M, S, sp), target, weight)
    return S1 - S0


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def mc_run(lattice: int, L, M: int, S: int, target, weight, species: np.ndarray, *, seed: int,
           chain_id: int, n_trials: int, B: int = 64, mode: int = MODE_DISJOINT,
           depth_limit: int = 0, tau: float = 0.0, log_cap: int | None = None):
    """Run one chain.  Returns (final species, log[n][4] uint32, stats dict,
    maintained counts[S][M][M])."""
    sp = np.array(species, dtype=np.int8, copy=True)
    t = np.ascontiguousarray(target, dtype=np.float64).reshape(S, M, M)
    w = np.ascontiguousarray(weight, dtype=np.float64).reshape(S)
    if log_cap is None:
        log_cap = n_trials
    log = np.zeros((max(log_cap, 1), 4), np.uint32)
    st = McStats()
    cnt = np.zeros((S, M, M), np.int64)
    rc = lib().or_mc_run(lattice, _p(_L(L)), M, S, _p(t), _p(w), seed, chain_id, n_trials, B,
                         mode, depth_limit, tau, _p(sp), _p(log), log_cap, ctypes.byref(st),
                         _p(cnt))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return sp, log[: st.log_len].copy(), st.as_dict(), cnt


def random_config(N: int, composition, *, seed: int, iteration: int, slot: int) -> np.ndarray:
    """A new solution of the global search: the composition-sorted species list
    placed through a keyed Feistel permutation of the sites (sro_oracle.c)."""
    comp = np.ascontiguousarray(np.asarray(composition, dtype=np.int64))
    out = np.full(N, -1, np.int8)
    rc = lib().or_random_config(N, comp.size, _p(comp), seed, iteration, slot, _p(out))
    if rc != 0:
        raise ValueError("composition does not add up to N")
    return out


def retained_count(n_refine: int, discard_frac: float) -> int:
    """Solutions kept as seeds after an iteration: the refined ones minus the
    discarded fraction p_a (rounded up), at most half of those refined."""
    return max(0, min(n_refine // 2, n_refine - int(np.ceil(discard_frac * n_refine))))


def global_search(lattice: int, L, M: int, S: int, target, weight, composition, *,
                  n_solutions: int, iterations: int, n_refine: int, discard_frac: float,
                  seed: int, B: int, n_trials: int, mode: int = MODE_DISJOINT,
                  depth_limit: int = 0, tau: float = 0.0, trace: list | None = None):
    """Algorithm 1 (Sec. 4.1), in its order:
      pool: iteration 0 draws every solution at random; later iterations keep
        the seeds retained by the previous one in slots 0..R-1 and draw new
        random solutions into the rest;
      fitness F (Eq. 3) of every solution from a full evaluation;
      the n_refine best (by F, then slot) are refined by Monte Carlo local
        search (mc_run, chain id = iteration * n_solutions + slot);
      refined solutions ranked by final F (then by their rank before the
        refinement); the worst fraction p_a is discarded and the best R =
        retained_count(...) become the next iteration's seeds;
      the best solution so far is kept (a later one replaces it only if its F
        is strictly lower).
    Returns (best species, best S, best F, best F after each iteration, stats)."""
    N = n_sites(lattice, L)
    if not (1 <= n_refine <= n_solutions) or iterations < 1 or not (0.0 <= discard_frac <= 1.0):
        raise ValueError("bad global search parameters")
    R = retained_count(n_refine, discard_frac)
    pool = [None] * n_solutions
    kept = 0
    best_F, best_S, best = np.inf, np.inf, None
    history = []
    st = {"trials": 0, "commits": 0, "evaluations": 0}
    for t in range(iterations):
        for s in range(kept, n_solutions):
            pool[s] = random_config(N, composition, seed=seed, iteration=t, slot=s)
        F = []
        for s in range(n_solutions):
            _, _, _, f = alpha_objective(lattice, L, M, S, pool[s], counts(lattice, L, M, S, pool[s]),
                                         target, weight)
            F.append(f)
        st["evaluations"] += n_solutions
        top = sorted(range(n_solutions), key=lambda s: (F[s], s))[:n_refine]
        refined = []
        for rank, s in enumerate(top):
            sp, _, ms, _ = mc_run(lattice, L, M, S, target, weight, pool[s], seed=seed,
                                  chain_id=t * n_solutions + s, n_trials=n_trials, B=B, mode=mode,
                                  depth_limit=depth_limit, tau=tau, log_cap=0)
            st["trials"] += ms["trials"]
            st["commits"] += ms["commits"]
            refined.append((ms["F"], rank, ms["S"], sp))
        refined.sort(key=lambda r: (r[0], r[1]))
        if refined[0][0] < best_F:
            best_F, best_S, best = refined[0][0], refined[0][2], refined[0][3].copy()
        history.append(best_F)
        if trace is not None:
            trace.append({"F": F, "top": top, "refined_F": [r[0] for r in refined]})
        for s in range(R):
            pool[s] = refined[s][3]
        kept = R
    return best, best_S, best_F, np.array(history), st


MAP_ERRORS = {1: "atom count differs from the number of sites", 2: "an atom lies farther than max_disp from every site",
              3: "two atoms share a site", 4: "a type lies outside [0, M)"}


def map_sites(lattice: int, L, M: int, box, max_disp: float, xyz, types):
    """Nearest-site assignment of an external structure (brute force over all
    sites, periodic minimum image, ties to the lower site id): returns
    (species[N] int8, site_of_atom[n] int64); raises ValueError with the reason
    (1 count, 2 displacement, 3 double occupancy, 4 type) in its args."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    types = np.ascontiguousarray(np.asarray(types, dtype=np.int8))
    box = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3))
    N = n_sites(lattice, L)
    sp = np.zeros(N, np.int8)
    site = np.zeros(xyz.shape[0], np.int64)
    rc = lib().or_map_sites(lattice, _p(_L(L)), M, _p(box), float(max_disp), xyz.shape[0], _p(xyz), _p(types),
                            _p(sp), _p(site))
    if rc:
        raise ValueError(MAP_ERRORS.get(rc, "allocation failed"), rc)
    return sp, site
