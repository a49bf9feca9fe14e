"""Pins of the oracle's energies, forces and virial: finite differences, closed
forms, lattice sums, invariants and literature values of the Tersoff 1988
carbon parameters."""
import itertools
import math

import numpy as np
import pytest

import workloads as W


def _rot(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def _small_systems():
    out = []
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    rng = np.random.default_rng(3)
    out.append(("lj", w["pos_init"] + rng.normal(0, 0.05, w["pos_init"].shape), w["cell_init"]))
    g = W.graphite_to_diamond(2, 2, 3, seed=4, sigma=0.08)
    mid = 0.5 * (g["pos_init"] + g["pos_final"])
    out.append(("ts", mid, 0.5 * (g["cell_init"] + g["cell_final"])))
    d = W.diamond_vacancy_hop(1, 1, 1)
    out.append(("ts", d["pos_init"] + rng.normal(0, 0.05, d["pos_init"].shape), d["cell_init"]))
    return out


def _params(orc, kind):
    return orc.default_params(orc.LJ if kind == "lj" else orc.TERSOFF)


@pytest.mark.parametrize("case", range(3))
def test_forces_are_minus_energy_gradient(orc, case):
    kind, R, h = _small_systems()[case]
    p = _params(orc, kind)
    E, u, F, V = orc.evaluate(p, R, h)
    assert E == pytest.approx(u.sum(), rel=1e-14)
    delta = 1e-5
    rng = np.random.default_rng(case)
    for i in rng.choice(len(R), 6, replace=False):
        for c in range(3):
            Rp, Rm = R.copy(), R.copy()
            Rp[i, c] += delta
            Rm[i, c] -= delta
            fd = -(orc.evaluate(p, Rp, h)[0] - orc.evaluate(p, Rm, h)[0]) / (2 * delta)
            assert F[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)


@pytest.mark.parametrize("case", range(3))
def test_virial_is_minus_strain_derivative(orc, case):
    # h' = h (I + eps), R' = R (I + eps) at fixed fractional coordinates (Eq. (2)-(3))
    kind, R, h = _small_systems()[case]
    p = _params(orc, kind)
    V = orc.evaluate(p, R, h)[3]
    delta = 1e-6
    for m in range(3):
        for n in range(3):
            eps = np.zeros((3, 3))
            eps[m, n] = delta
            Ep = orc.evaluate(p, R @ (np.eye(3) + eps), h @ (np.eye(3) + eps))[0]
            Em = orc.evaluate(p, R @ (np.eye(3) - eps), h @ (np.eye(3) - eps))[0]
            assert V[m, n] == pytest.approx(-(Ep - Em) / (2 * delta), rel=1e-6, abs=1e-6)


@pytest.mark.parametrize("case", range(3))
def test_translation_and_rotation_invariance(orc, case):
    kind, R, h = _small_systems()[case]
    p = _params(orc, kind)
    E, u, F, V = orc.evaluate(p, R, h)
    np.testing.assert_allclose(F.sum(axis=0), 0.0, atol=1e-10)
    np.testing.assert_allclose(V, V.T, atol=1e-10 * np.abs(V).max())
    Q = _rot(np.random.default_rng(case + 10))
    E2, u2, F2, V2 = orc.evaluate(p, R @ Q, h @ Q)
    assert E2 == pytest.approx(E, rel=1e-12)
    np.testing.assert_allclose(F2, F @ Q, atol=1e-10)
    np.testing.assert_allclose(V2, Q.T @ V @ Q, atol=1e-9)


def _lj(r, eps=1.0, sig=1.0, rc=2.5):
    def phi(x):
        return 4 * eps * ((sig / x) ** 12 - (sig / x) ** 6)
    return np.where(r < rc, phi(r) - phi(rc), 0.0)


def test_lj_fcc_lattice_sum(orc):
    # E/atom of a perfect FCC crystal = 1/2 sum over lattice vectors of phi(|t|)
    a = 1.5496
    basis = W.FCC_BASIS * a
    t = np.array([(np.array(c) * a + b) for c in itertools.product(range(-3, 4), repeat=3)
                  for b in basis])
    r = np.linalg.norm(t, axis=1)
    e_ref = 0.5 * _lj(r[r > 0]).sum()
    sites, cell = W.fcc_sites(4, 4, 4, a)
    E, u, F, V = orc.evaluate(orc.default_params(orc.LJ), sites, cell)
    assert E / len(sites) == pytest.approx(e_ref, rel=1e-13)
    np.testing.assert_allclose(u, e_ref, rtol=1e-12)
    assert np.abs(F).max() < 1e-12
    np.testing.assert_allclose(V, V[0, 0] * np.eye(3), atol=1e-10)


def _tersoff_bond(p, r):
    fc = 1.0 if r < p.ts_R else 0.5 + 0.5 * math.cos(math.pi * (r - p.ts_R) / (p.ts_S - p.ts_R))
    return fc, p.ts_A * math.exp(-p.ts_lambda1 * r), p.ts_B * math.exp(-p.ts_lambda2 * r)


def test_tersoff_dimer_and_trimer_closed_form(orc):
    p = orc.default_params(orc.TERSOFF)
    box = np.eye(3) * 30.0
    # dimer: zeta = 0, b = 1, E = fc (fR - fA)
    for r in [1.3, 1.9, 2.05]:
        R = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        fc, fr, fa = _tersoff_bond(p, r)
        assert orc.evaluate(p, R, box)[0] == pytest.approx(fc * (fr - fa), rel=1e-13)
    # symmetric trimer: atom 0 bonded to 1 and 2 at angle theta, 1-2 beyond the cutoff
    r, th = 1.5, math.radians(110.0)
    R = np.array([[5, 5, 5], [5 + r, 5, 5], [5 + r * math.cos(th), 5 + r * math.sin(th), 5]], float)
    fc, fr, fa = _tersoff_bond(p, r)
    c2, d2 = p.ts_c ** 2, p.ts_d ** 2
    g = 1 + c2 / d2 - c2 / (d2 + (p.ts_h - math.cos(th)) ** 2)
    b_center = (1 + (p.ts_beta * fc * g) ** p.ts_n) ** (-1 / (2 * p.ts_n))
    # atom 0 has two bonds with zeta = fc g; atoms 1, 2 have one bond each with zeta = 0
    e_ref = 0.5 * 2 * fc * (fr - b_center * fa) + 2 * 0.5 * fc * (fr - fa)
    assert orc.evaluate(p, R, box)[0] == pytest.approx(e_ref, rel=1e-13)


def test_tersoff_carbon_literature_values(orc):
    # Tersoff (1988) carbon: diamond about -7.37 eV/atom at a = 3.566 A (equilibrium),
    # graphite about -7.40 eV/atom at a bond length of 1.46 A
    p = orc.default_params(orc.TERSOFF)
    basis = np.concatenate([W.FCC_BASIS, W.FCC_BASIS + 0.25])

    def diamond(a):
        pos = np.array([(np.array(c) + b) * a for c in itertools.product(range(2), repeat=3)
                        for b in basis])
        return orc.evaluate(p, pos, np.eye(3) * 2 * a)

    E, u, F, V = diamond(3.566)
    assert E / 64 == pytest.approx(-7.37, abs=0.005)
    # pressure changes sign across the literature lattice constant
    assert np.trace(diamond(3.556)[3]) > 0 > np.trace(diamond(3.576)[3])

    energies = []
    for d in [1.44, 1.46, 1.48]:
        g = W.graphite_to_diamond(3, 2, 3, seed=0, sigma=0.0, d_graphite=d)
        energies.append(orc.evaluate(p, g["pos_init"], g["cell_init"])[0] / g["n"])
    assert energies[1] == pytest.approx(-7.40, abs=0.01)
    assert energies[1] < energies[0] and energies[1] < energies[2]
    # the diamond-like endpoint of the graphite construction is cubic diamond
    g = W.graphite_to_diamond(3, 2, 3, seed=0, sigma=0.0)
    Ef = orc.evaluate(p, g["pos_final"], g["cell_final"])[0] / g["n"]
    assert Ef == pytest.approx(E / 64, abs=1e-9)


def test_cell_list_and_brute_energies_agree(orc):
    # orc.evaluate switches to the cell list above 64 atoms; a 65-atom system must
    # give the same numbers as 64-atom brute-force pieces of the same definition
    g = W.graphite_to_diamond(3, 2, 3, seed=9, sigma=0.05)
    p = orc.default_params(orc.TERSOFF)
    E, u, F, V = orc.evaluate(p, g["pos_init"], g["cell_init"])
    L = orc.nlist(g["pos_init"], g["cell_init"], 2.1, "brute")
    Lc = orc.nlist(g["pos_init"], g["cell_init"], 2.1, "cells")
    for a, b in zip(L, Lc):
        np.testing.assert_array_equal(a, b)
    assert np.isfinite(E)
