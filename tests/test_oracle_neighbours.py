"""Pins of the oracle's neighbour sets: an independent NumPy brute force of the
definition (same rounded operations), cell list vs brute force, symmetry, and
the FCC shell count."""
import itertools

import numpy as np

import workloads as W


def numpy_brute(R, h, rc, m=4):
    """All (j, n) with n in [-m, m]^3 and ((dx*dx + dy*dy) + dz*dz) < rc*rc, where
    d = (R_j - R_i) + ((n0 h0 + n1 h1) + n2 h2); NumPy float64 ops round one by one."""
    n = len(R)
    rc2 = rc * rc
    shifts = np.array(list(itertools.product(range(-m, m + 1), repeat=3)), dtype=np.int64)
    sh = (shifts[:, 0:1] * h[0] + shifts[:, 1:2] * h[1]) + shifts[:, 2:3] * h[2]
    out = []
    for i in range(n):
        ent = []
        for j in range(n):
            d = (R[j] - R[i])[None, :] + sh
            r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            for s in np.nonzero(r2 < rc2)[0]:
                if i == j and not shifts[s].any():
                    continue
                ent.append((j, *shifts[s]))
        out.append(np.array(sorted(ent), dtype=np.int32).reshape(-1, 4))
    return out


def _same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_brute_matches_numpy_definition(orc):
    for seed in range(4):
        R, h = W.random_cell(12, seed, density=0.05)
        rc = 0.9 * np.min(orc.widths(h))
        _same(orc.nlist(R, h, rc, "brute"), numpy_brute(R, h, rc, m=3))


def test_narrow_cell_many_images(orc):
    # cell narrower than the cutoff in every direction: many periodic images per pair
    R, h = W.random_cell(3, 11, density=0.05, skew=0.3)
    rc = 1.7 * np.max(orc.widths(h))
    _same(orc.nlist(R, h, rc, "brute"), numpy_brute(R, h, rc, m=5))
    _same(orc.nlist(R, h, rc, "cells"), numpy_brute(R, h, rc, m=5))


def test_cells_match_brute(orc):
    for seed in range(6):
        n = [20, 60, 150][seed % 3]
        R, h = W.random_cell(n, 100 + seed, density=0.1, skew=0.25)
        for rc in [1.5, 2.1, 3.0]:
            _same(orc.nlist(R, h, rc, "cells"), orc.nlist(R, h, rc, "brute"))


def test_lists_are_symmetric(orc):
    R, h = W.random_cell(80, 5, density=0.1, skew=0.2)
    L = orc.nlist(R, h, 2.5)
    s = {(i, int(e[0]), int(e[1]), int(e[2]), int(e[3])) for i, l in enumerate(L) for e in l}
    for (i, j, a, b, c) in s:
        assert (j, i, -a, -b, -c) in s


def test_fcc_shell_count(orc):
    # FCC at a = 1.5496: shells at a/sqrt2, a, a sqrt(3/2), a sqrt2, a sqrt(5/2)
    # hold 12 + 6 + 24 + 12 + 24 = 78 neighbours inside 2.5
    sites, cell = W.fcc_sites(4, 4, 4, 1.5496)
    L = orc.nlist(sites, cell, 2.5)
    assert all(len(l) == 78 for l in L)
    # 2 x 2 x 2 cells: width 3.0992 is barely above the cutoff, pairs appear through
    # several images and the count is still 78
    sites, cell = W.fcc_sites(2, 2, 2, 1.5496)
    L = orc.nlist(sites, cell, 2.5)
    assert all(len(l) == 78 for l in L)


def test_graphite_coordination(orc):
    g = W.graphite_to_diamond(3, 2, 3, seed=0, sigma=0.0)
    Li = orc.nlist(g["pos_init"], g["cell_init"], 2.1)
    Lf = orc.nlist(g["pos_final"], g["cell_final"], 2.1)
    assert all(len(l) == 3 for l in Li)
    assert all(len(l) == 4 for l in Lf)
