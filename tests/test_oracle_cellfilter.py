"""Pins of the oracle's rotation-free cell filter (Sec. II.C): generalized forces
against finite differences of the enthalpy in generalized coordinates, and the
rotation invariance of R~, B and the generalized forces (Eq. (15))."""
import numpy as np
import pytest

import workloads as W


def _rot(seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    return Q


def _image(orc, kind, pressure=0.0):
    rng = np.random.default_rng(5)
    if kind == "lj":
        w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
        p = orc.default_params(orc.LJ, pressure_GPa=pressure)
    else:
        w = W.graphite_to_diamond(2, 2, 3, seed=4, sigma=0.05)
        p = orc.default_params(orc.TERSOFF, pressure_GPa=pressure)
    XA, XB = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    X = 0.6 * XA + 0.4 * XB
    X[:-3] += rng.normal(0, 0.02, X[:-3].shape)
    return p, w["cell_init"], X


@pytest.mark.parametrize("kind,pressure", [("lj", 0.0), ("ts", 0.0), ("ts", 15.0), ("lj", 40.0)])
def test_generalized_forces_by_finite_differences(orc, kind, pressure):
    p, h0, X = _image(orc, kind, pressure)
    out = orc.cf_eval(p, h0, X)
    n = X.shape[0] - 3
    delta = 1e-6
    # atom rows: F D^T is exactly -dH/dR~
    for i in [0, 3, n // 2]:
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, c] += delta
            Xm[i, c] -= delta
            fd = -(orc.cf_eval(p, h0, Xp)["H"] - orc.cf_eval(p, h0, Xm)["H"]) / (2 * delta)
            assert out["Fg"][i, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    # cell rows hold c_f B; the printed lattice force D^-T V D^-1 / c_f is twice the
    # virtual-work conjugate of B: -dH = 1/2 Fg_cell : d(c_f B)
    dcell = delta * n
    for m in range(3):
        for k in range(m, 3):
            dX = np.zeros((3, 3))
            dX[m, k] += dcell
            dX[k, m] = dX[m, k]
            Xp, Xm = X.copy(), X.copy()
            Xp[n:] += dX
            Xm[n:] -= dX
            fd = -(orc.cf_eval(p, h0, Xp)["H"] - orc.cf_eval(p, h0, Xm)["H"]) / 2.0
            pred = 0.5 * np.sum(out["Fg"][n:] * dX)
            assert pred == pytest.approx(fd, rel=2e-5, abs=1e-9)


def test_enthalpy_adds_p_omega(orc):
    p0, h0, X = _image(orc, "ts", 0.0)
    p1, _, _ = _image(orc, "ts", 15.0)
    a, b = orc.cf_eval(p0, h0, X), orc.cf_eval(p1, h0, X)
    omega = abs(np.linalg.det(a["h"]))
    assert b["H"] - a["H"] == pytest.approx(15.0 / 160.21766208 * omega, rel=1e-12)
    assert b["E"] == a["E"]


def test_identity_deformation_at_reference_cell(orc):
    p, h0, X = _image(orc, "lj")
    XA, _ = orc.build_endpoints(p, X[:-3], h0, X[:-3], h0)
    out = orc.cf_eval(p, h0, XA)
    np.testing.assert_allclose(out["h"], h0, rtol=1e-15)
    np.testing.assert_array_equal(out["R"], XA[:-3])
    E, u, F, V = orc.evaluate(p, XA[:-3], h0)
    assert out["E"] == pytest.approx(E, rel=1e-13)
    np.testing.assert_allclose(out["Fg"][:-3], F, atol=1e-12)


@pytest.mark.parametrize("kind", ["lj", "ts"])
def test_rotation_free_coordinates_and_forces(orc, kind):
    # a rigidly rotated final state (h -> h Q, R -> R Q) has the same B, R~ and
    # generalized forces: the rotational degrees of freedom are gone (Eq. (15))
    if kind == "lj":
        w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
        p = orc.default_params(orc.LJ)
    else:
        w = W.graphite_to_diamond(2, 2, 3, seed=4, sigma=0.05)
        p = orc.default_params(orc.TERSOFF, pressure_GPa=5.0)
    Q = _rot(3)
    XA, XB = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    _, XBr = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"] @ Q,
                                 w["cell_final"] @ Q)
    np.testing.assert_allclose(XBr, XB, rtol=1e-12, atol=1e-10)
    a, b = orc.cf_eval(p, w["cell_init"], XB), orc.cf_eval(p, w["cell_init"], XBr)
    assert b["H"] == pytest.approx(a["H"], rel=1e-12)
    np.testing.assert_allclose(b["Fg"], a["Fg"], atol=1e-8)
    # the final structure itself has the energy of the unrotated input
    E = orc.evaluate(p, w["pos_final"], w["cell_final"])[0]
    assert a["E"] == pytest.approx(E, rel=1e-12)


def test_non_spd_cell_rows_are_rejected(orc):
    p, h0, X = _image(orc, "lj")
    n = X.shape[0] - 3
    X[n:] = -X[n:]
    with pytest.raises(orc.OracleError) as e:
        orc.cf_eval(p, h0, X)
    assert e.value.code == orc.ECELL


def test_default_cell_factor_is_size_consistent(orc):
    # Default c_f = |det h0|^(1/3) n^(1/6) (the generalized solid-state NEB Jacobian):
    # the stiffness of H along a cell coordinate Y = c_f B_xx, and the band-metric
    # length of a uniform strain relative to a uniform per-atom displacement, do not
    # depend on the supercell size.  With c_f = n both would scale as 1/n and n.
    p = orc.default_params(orc.LJ)
    stiff, ratio = [], []
    for m in (2, 3):
        R, h = W.fcc_sites(m, m, m, 1.5496)
        n = len(R)
        XA, _ = orc.build_endpoints(p, R, h, R, h)
        cf = abs(np.linalg.det(h)) ** (1.0 / 3.0) * n ** (1.0 / 6.0)
        np.testing.assert_allclose(XA[-3:], cf * np.eye(3), rtol=1e-15)
        d = 1e-4 * cf
        f = []
        for s in (+1, -1):
            X = XA.copy()
            X[-3, 0] += s * d
            f.append(orc.cf_eval(p, h, X)["Fg"][-3, 0])
        stiff.append(-(f[0] - f[1]) / (2 * d))
        # 1% uniform strain between endpoints against a 0.01 displacement of every atom
        eps = np.diag([1.01, 1.0, 1.0])
        _, XS = orc.build_endpoints(p, R, h, R @ eps, h @ eps)
        _, XU = orc.build_endpoints(p, R, h, R + np.array([0.01, 0.0, 0.0]), h)
        ratio.append(np.sum((XS - XA) ** 2) / np.sum((XU - XA) ** 2))
    assert stiff[0] > 0
    assert stiff[1] == pytest.approx(stiff[0], rel=1e-5)
    assert ratio[1] == pytest.approx(ratio[0], rel=1e-9)


def _image_dvariant(orc, kind, pressure=0.0):
    rng = np.random.default_rng(6)
    if kind == "lj":
        w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
        p = orc.default_params(orc.LJ, pressure_GPa=pressure, cell_filter=1)
    else:
        w = W.graphite_to_diamond(2, 2, 3, seed=4, sigma=0.05)
        p = orc.default_params(orc.TERSOFF, pressure_GPa=pressure, cell_filter=1)
    # a final cell that is strained and rigidly rotated: the D-variant keeps the rotation
    Q = _rot(11)
    XA, XB = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"] @ Q,
                                 (w["cell_final"] @ np.diag([1.02, 0.99, 1.01])) @ Q)
    X = 0.6 * XA + 0.4 * XB
    X[:-3] += rng.normal(0, 0.02, X[:-3].shape)
    return p, w["cell_init"], X


@pytest.mark.parametrize("kind,pressure", [("lj", 0.0), ("ts", 15.0)])
def test_d_variant_forces_by_finite_differences(orc, kind, pressure):
    # D-variant of the filter (Sec. II.C, Eq. (13)): coordinates (R~, c_f D) with the
    # full 3x3 D, forces (F D^T, D^-T V_eff / c_f); the lattice force is the exact
    # conjugate of D, with no factor 1/2 and for all nine entries
    p, h0, X = _image_dvariant(orc, kind, pressure)
    out = orc.cf_eval(p, h0, X)
    n = X.shape[0] - 3
    delta = 1e-6
    for i in [0, n // 2]:
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, c] += delta
            Xm[i, c] -= delta
            fd = -(orc.cf_eval(p, h0, Xp)["H"] - orc.cf_eval(p, h0, Xm)["H"]) / (2 * delta)
            assert out["Fg"][i, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    dcell = delta * n
    for m in range(3):
        for k in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[n + m, k] += dcell
            Xm[n + m, k] -= dcell
            fd = -(orc.cf_eval(p, h0, Xp)["H"] - orc.cf_eval(p, h0, Xm)["H"]) / (2 * dcell)
            assert out["Fg"][n + m, k] == pytest.approx(fd, rel=2e-5, abs=1e-8)


def test_d_variant_keeps_rotations(orc):
    # the rotation-free filter maps a rotated final cell to the same coordinates; the
    # D-variant does not (its three extra coordinates are the rotation), while the
    # enthalpy of the final image is the same either way
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    Q = _rot(12)
    for filt, same in ((2, True), (1, False)):
        p = orc.default_params(orc.LJ, cell_filter=filt)
        _, XB = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
        _, XBr = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"] @ Q, w["cell_final"] @ Q)
        assert np.allclose(XBr, XB, atol=1e-9) == same
        a, b = orc.cf_eval(p, w["cell_init"], XB), orc.cf_eval(p, w["cell_init"], XBr)
        assert b["H"] == pytest.approx(a["H"], rel=1e-12)
    # a relaxation under either filter reaches the same enthalpy and cell metric h h^T
    # from a strained start
    R0, h0 = W.fcc_sites(2, 2, 2, 1.5496)
    strain = np.array([[1.03, 0.01, 0.0], [0.0, 0.98, 0.0], [0.0, 0.0, 1.01]])
    res = []
    for filt in (1, 2):
        p = orc.default_params(orc.LJ, cell_filter=filt, fire_dt0=0.01)
        R, h, steps, fmax = orc.relax(p, R0 @ strain, h0 @ strain, 20000, 1e-7)
        assert fmax < 1e-7
        res.append((orc.evaluate(p, R, h)[0], h @ h.T))
    assert res[0][0] == pytest.approx(res[1][0], abs=1e-9)
    np.testing.assert_allclose(res[0][1], res[1][1], atol=1e-6)


# ------------------------------------------------------------- applied stress
# A constant second Piola-Kirchhoff stress S referred to h0 (the non-hydrostatic
# loading that motivates finite-deformation NEB in Sec. I) adds -Omega0 S : E,
# E = (D D^T - I)/2, to the enthalpy.
STRESS_TS = (6.0, -3.5, 2.0, 4.0, -2.5, 5.0)  # GPa, Voigt xx yy zz yz xz xy
STRESS_LJ = tuple(40.0 * s for s in STRESS_TS)


@pytest.mark.parametrize("kind,filt", [("lj", 2), ("ts", 2), ("lj", 1), ("ts", 1)])
def test_applied_stress_forces_by_finite_differences(orc, kind, filt):
    p, h0, X = (_image if filt == 2 else _image_dvariant)(orc, kind, 5.0)
    p.stress_GPa = STRESS_LJ if kind == "lj" else STRESS_TS
    out = orc.cf_eval(p, h0, X)
    n = X.shape[0] - 3
    delta = 1e-6
    dcell = delta * n
    for m in range(3):
        for k in range(3):
            if filt == 2 and k < m:
                continue
            dX = np.zeros((3, 3))
            dX[m, k] += dcell
            if filt == 2:
                dX[k, m] = dX[m, k]
            Xp, Xm = X.copy(), X.copy()
            Xp[n:] += dX
            Xm[n:] -= dX
            fd = -(orc.cf_eval(p, h0, Xp)["H"] - orc.cf_eval(p, h0, Xm)["H"]) / 2.0
            # rotation-free: the printed B force is twice the conjugate (as without stress)
            pred = (0.5 if filt == 2 else 1.0) * np.sum(out["Fg"][n:] * dX)
            assert pred == pytest.approx(fd, rel=2e-5, abs=1e-9), (m, k)
    # atom rows do not see the stress
    q = orc.default_params(p.potential, pressure_GPa=5.0, cell_filter=filt)
    np.testing.assert_array_equal(out["Fg"][:n], orc.cf_eval(q, h0, X)["Fg"][:n])


def test_applied_stress_work_is_rotation_invariant(orc):
    # the Green-Lagrange strain sees lengths only: rotating the current cell and
    # atoms together (D -> D Q in the D-variant) changes neither U nor the stress work
    p, h0, X = _image_dvariant(orc, "ts", 0.0)
    p.stress_GPa = STRESS_TS
    n = X.shape[0] - 3
    Q = _rot(21)
    Xr = X.copy()
    Xr[n:] = X[n:] @ Q
    a, b = orc.cf_eval(p, h0, X), orc.cf_eval(p, h0, Xr)
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    assert b["H"] == pytest.approx(a["H"], rel=1e-12, abs=1e-12)
    assert abs(a["H"] - a["E"]) > 1e-3  # the work term is not trivially zero here


def test_isotropic_stress_agrees_with_pressure_to_first_order(orc):
    # S = -P I against the pressure P: the stress work P Omega0 tr E equals
    # P (Omega - Omega0) up to O(strain^2)
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    P = 300.0
    ps = orc.default_params(orc.LJ, cell_filter=1, stress_GPa=(-P, -P, -P, 0.0, 0.0, 0.0))
    pp = orc.default_params(orc.LJ, cell_filter=1, pressure_GPa=P)
    XA, _ = orc.build_endpoints(pp, w["pos_init"], w["cell_init"], w["pos_init"], w["cell_init"])
    n = XA.shape[0] - 3
    h0 = w["cell_init"]
    rng = np.random.default_rng(8)
    G = rng.normal(size=(3, 3))
    res = []
    for a in (1e-3, 2e-3, 4e-3):
        X = XA.copy()
        X[n:] = XA[n:] @ (np.eye(3) + a * G)
        hs, hp = orc.cf_eval(ps, h0, X)["H"], orc.cf_eval(pp, h0, X)["H"]
        om0 = abs(np.linalg.det(h0))
        P_ev = P / 160.21766208
        first = P_ev * om0 * a * np.trace(G)  # first-order volume term
        d = hs - (hp - P_ev * om0)  # the pressure's enthalpy carries P Omega0 at the reference
        assert abs(d) < 0.05 * abs(first)
        res.append(d)
    # the difference is second order: doubling the strain multiplies it by four
    assert res[1] / res[0] == pytest.approx(4.0, rel=0.02)
    assert res[2] / res[1] == pytest.approx(4.0, rel=0.02)


def test_relaxed_crystal_carries_the_applied_stress(orc):
    # relaxed under S, the crystal's own Cauchy stress -V/Omega is the push-forward
    # J^-1 F S F^T of S (F = D^T in the row convention); tension lengthens its axis
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    S = (120.0, -40.0, 20.0, 30.0, 0.0, -50.0)  # GPa; LJ in eV and A is stiff (~10^4 GPa)
    for filt in (2, 1):
        p = orc.default_params(orc.LJ, cell_filter=filt, stress_GPa=S)
        R, h, steps, fmax = orc.relax(p, w["pos_init"], w["cell_init"], max_steps=5000, f_tol=1e-7)
        assert fmax < 1e-7
        D = np.linalg.solve(w["cell_init"], h)
        E, u, F, V = orc.evaluate(orc.default_params(orc.LJ), R, h)
        Sm = np.array([[S[0], S[5], S[4]], [S[5], S[1], S[3]], [S[4], S[3], S[2]]]) / 160.21766208
        om, om0 = abs(np.linalg.det(h)), abs(np.linalg.det(w["cell_init"]))
        np.testing.assert_allclose(-V / om, (om0 / om) * D.T @ Sm @ D, rtol=0, atol=2e-5)
        # tension along x gives a positive Green-Lagrange strain there
        assert 0.5 * (D @ D.T - np.eye(3))[0, 0] > 1e-3
