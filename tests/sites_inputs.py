"""Synthetic external structures for the nearest-site tests: lattice positions
of a configuration, thermally perturbed, shifted by periodic images and
shuffled in atom order.  Input generation only; no method arithmetic."""
import numpy as np

FCC_BASIS = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]])
BCC_BASIS = np.array([[0, 0, 0], [1, 1, 1]])


def site_half_units(lattice: int, L) -> np.ndarray:
    """[N][3] half-unit positions in site-id order p = ((cz Ly + cy) Lx + cx) A + b."""
    basis = FCC_BASIS if lattice == 0 else BCC_BASIS
    Lx, Ly, Lz = L
    cz, cy, cx = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    return (2 * cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)


def nn_distance(lattice: int, box, L) -> float:
    """Nearest-neighbour distance of the (possibly stretched) lattice: the
    shortest lattice vector in Cartesian units."""
    a = np.asarray(box, float) / np.asarray(L, float)   # cell edge per axis
    if lattice == 0:
        vecs = [(1, 1, 0), (1, 0, 1), (0, 1, 1), (1, -1, 0), (1, 0, -1), (0, 1, -1)]
    else:
        vecs = [(1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2)]
    return min(float(np.linalg.norm(np.array(v) * a / 2)) for v in vecs)


def structure(lattice: int, L, box, species: np.ndarray, noise: float, seed: int, images: bool = True,
              shuffle: bool = True):
    """(xyz [N][3], types [N], order): atom i sits at site order[i], displaced by
    a random vector of length < noise (Cartesian), optionally moved by a random
    periodic image, atoms listed in a random order."""
    rng = np.random.default_rng(seed)
    h = site_half_units(lattice, L).astype(np.float64)
    N = h.shape[0]
    box = np.asarray(box, float)
    xyz = h * box / (2 * np.asarray(L, float))
    v = rng.normal(size=(N, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    xyz = xyz + v * (noise * rng.uniform(0, 1, size=(N, 1)) ** (1 / 3))
    if images:
        xyz = xyz + rng.integers(-2, 3, size=(N, 3)) * box
    order = rng.permutation(N) if shuffle else np.arange(N)
    return np.ascontiguousarray(xyz[order]), np.ascontiguousarray(species[order]), order
