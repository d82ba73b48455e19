"""Independent brute-force helpers for pinning the oracle.

Written separately from the oracle (numpy, Cartesian positions, distance
enumeration) so that a mistake in the oracle's index arithmetic cannot hide
behind the same mistake here.  Textbook facts used:
  FCC shells (lattice constant a): r^2 = a^2/2, a^2, 3a^2/2, 2a^2 with
  coordination 12, 6, 24, 12; BCC: r^2 = 3a^2/4, a^2, 2a^2, 11a^2/4 with
  coordination 8, 6, 12, 24.  In half-lattice units (a = 2) the squared
  radii are FCC 2, 4, 6, 8 and BCC 3, 4, 8, 11.
"""
from __future__ import annotations

import itertools

import numpy as np

FCC, BCC = 0, 1
R2 = {FCC: [2, 4, 6, 8], BCC: [3, 4, 8, 11]}
Z = {FCC: [12, 6, 24, 12], BCC: [8, 6, 12, 24]}
# Cartesian positions of the basis atoms in a conventional cubic cell (units a/2)
BASIS = {FCC: np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]]),
         BCC: np.array([[0, 0, 0], [1, 1, 1]])}


def positions(lattice: int, L) -> np.ndarray:
    """[N][3] positions in site-id order: p = ((cz*Ly + cy)*Lx + cx)*A + b."""
    Lx, Ly, Lz = L
    out = []
    for cz in range(Lz):
        for cy in range(Ly):
            for cx in range(Lx):
                for b in BASIS[lattice]:
                    out.append(2 * np.array([cx, cy, cz]) + b)
    return np.array(out, dtype=np.int64)


def min_image_r2(lattice: int, L) -> np.ndarray:
    """[N][N] squared minimum-image distance (half units)."""
    pos = positions(lattice, L)
    box = 2 * np.array(L)
    d = pos[:, None, :] - pos[None, :, :]
    d = (d + box // 2) % box - box // 2
    return (d * d).sum(-1)


def counts_by_distance(lattice: int, L, S: int, M: int, species) -> np.ndarray:
    """N[k][i][j] from the distance matrix: valid when every shell offset is
    shorter than half the box along each axis (no neighbour reached twice)."""
    r2 = min_image_r2(lattice, L)
    s = np.asarray(species, dtype=np.int64)
    out = np.zeros((S, M, M), np.int64)
    for k in range(S):
        P, Q = np.nonzero(r2 == R2[lattice][k])
        np.add.at(out[k], (s[P], s[Q]), 1)
    return out


def offset_vectors(lattice: int, k: int) -> np.ndarray:
    """Lattice vectors of shell k (0-based) in half units, by enumeration."""
    rng = range(-4, 5)
    vs = []
    for v in itertools.product(rng, rng, rng):
        v = np.array(v)
        if int(v @ v) != R2[lattice][k]:
            continue
        if lattice == FCC and v.sum() % 2 == 0:
            vs.append(v)
        if lattice == BCC and len(set(v % 2)) == 1:
            vs.append(v)
    return np.array(vs)


def neighbor_table(lattice: int, L, S: int) -> list:
    """Per shell, [N][z_k] neighbour ids along every offset (a multigraph: on
    tiny cells one site can be reached along several offsets)."""
    pos = positions(lattice, L)
    box = 2 * np.array(L)
    index = {tuple(p): i for i, p in enumerate(pos)}
    tabs = []
    for k in range(S):
        offs = offset_vectors(lattice, k)
        t = np.empty((len(pos), len(offs)), np.int64)
        for i, p in enumerate(pos):
            for m, d in enumerate(offs):
                t[i, m] = index[tuple((p + d) % box)]
        tabs.append(t)
    return tabs


def counts_by_offsets(tabs, M: int, species) -> np.ndarray:
    s = np.asarray(species, dtype=np.int64)
    out = np.zeros((len(tabs), M, M), np.int64)
    for k, t in enumerate(tabs):
        np.add.at(out[k], (np.repeat(s, t.shape[1]), s[t.ravel()]), 1)
    return out


def objective(counts: np.ndarray, species, target, weight, z) -> float:
    """S = sum_k w_k sum_ij (alpha_ij - target_ij)^2 with alpha = 1 - P_ij/c_j,
    P_ij = N_ij/(n_i z_k), c_j = n_j/N (Eq. 2-3), in plain numpy float64."""
    s = np.asarray(species)
    N = len(s)
    M = counts.shape[1]
    n = np.bincount(s, minlength=M).astype(np.float64)
    tot = 0.0
    for k in range(counts.shape[0]):
        P = counts[k] / (n[:, None] * z[k])
        alpha = 1.0 - P / (n[None, :] / N)
        tot += weight[k] * float(((alpha - target[k]) ** 2).sum())
    return tot
