"""Pins of the oracle's nearest-site assignment (the analysis of structures from
other codes in the application workflow, Sec. 2.3) by properties the geometry
fixes: exact lattice positions and any displacement shorter than half the
nearest-neighbour distance map each atom to its own site (the sites' Voronoi
cells contain those balls), periodic images and atom order do not matter, a
swap of two atoms swaps their sites' species, and each failure mode is
reported."""
import numpy as np
import pytest

from oracle import oracle as orc
import sites_inputs as si

CASES = [(0, (3, 3, 3), (10.8, 10.8, 10.8)), (0, (4, 3, 2), (14.0, 10.9, 7.6)),
         (1, (4, 4, 4), (11.5, 11.5, 11.5)), (1, (3, 5, 2), (8.4, 14.6, 5.9))]


@pytest.mark.parametrize("lattice,L,box", CASES)
@pytest.mark.parametrize("noise_frac", [0.0, 0.45])
def test_positions_within_half_nn_map_to_their_sites(lattice, L, box, noise_frac):
    N = orc.n_sites(lattice, L)
    rng = np.random.default_rng(N)
    sp = rng.integers(0, 4, size=N).astype(np.int8)
    noise = noise_frac * si.nn_distance(lattice, box, L)
    xyz, types, order = si.structure(lattice, L, box, sp, noise, seed=N + 1)
    got_sp, site = orc.map_sites(lattice, L, 4, box, 0.5 * si.nn_distance(lattice, box, L), xyz, types)
    np.testing.assert_array_equal(site, order)
    np.testing.assert_array_equal(got_sp, sp)


def test_same_counts_as_the_configuration_it_came_from():
    lattice, L, box = 0, (4, 4, 4), (14.4, 14.4, 14.4)
    N = orc.n_sites(lattice, L)
    sp = np.random.default_rng(5).integers(0, 3, size=N).astype(np.int8)
    xyz, types, _ = si.structure(lattice, L, box, sp, 0.3 * si.nn_distance(lattice, box, L), seed=6)
    got, _ = orc.map_sites(lattice, L, 3, box, 1.0, xyz, types)
    np.testing.assert_array_equal(orc.counts(lattice, L, 3, 2, got), orc.counts(lattice, L, 3, 2, sp))


def test_swapping_two_atoms_swaps_their_sites():
    lattice, L, box = 1, (3, 3, 3), (8.6, 8.6, 8.6)
    N = orc.n_sites(lattice, L)
    sp = (np.arange(N) % 3).astype(np.int8)
    xyz, types, _ = si.structure(lattice, L, box, sp, 0.0, seed=1, images=False, shuffle=False)
    xyz[[4, 9]] = xyz[[9, 4]]
    got, site = orc.map_sites(lattice, L, 3, box, 0.1, xyz, types)
    assert site[4] == 9 and site[9] == 4
    want = sp.copy()
    want[[4, 9]] = want[[9, 4]]
    np.testing.assert_array_equal(got, want)


def test_failures_are_reported():
    lattice, L, box = 0, (3, 3, 3), (10.8, 10.8, 10.8)
    N = orc.n_sites(lattice, L)
    sp = np.zeros(N, np.int8)
    xyz, types, _ = si.structure(lattice, L, box, sp, 0.0, seed=2, images=False, shuffle=False)
    with pytest.raises(ValueError) as e:              # one atom too few
        orc.map_sites(lattice, L, 2, box, 0.5, xyz[:-1], types[:-1])
    assert e.value.args[1] == 1
    far = xyz.copy()
    far[7] += np.array([0.9, 0.0, 0.0])                # 0.9 from its site, 1.65 from the others
    with pytest.raises(ValueError) as e:
        orc.map_sites(lattice, L, 2, box, 0.5, far, types)
    assert e.value.args[1] == 2
    dbl = xyz.copy()
    dbl[7] = dbl[8]                                    # two atoms on site 8, site 7 vacant
    with pytest.raises(ValueError) as e:
        orc.map_sites(lattice, L, 2, box, 0.5, dbl, types)
    assert e.value.args[1] == 3
    bad = types.copy()
    bad[3] = 2
    with pytest.raises(ValueError) as e:
        orc.map_sites(lattice, L, 2, box, 0.5, xyz, bad)
    assert e.value.args[1] == 4
