"""Pins of the oracle's energy profile (the enthalpy against the normalized path
coordinate in which the transitions of Sec. III are reported): a cubic along a
straight path is reproduced exactly by the Hermite interpolant with
tangential-force slopes; the slopes are the directional derivative of the real
enthalpy, by central differences; the Hermite basis reduces to smoothstep with
flat slopes; the located maximum agrees with brute-force sampling; a rigid
translation of an image's atoms changes nothing."""
import numpy as np
import pytest

import workloads as W


def _unit_zero_mean(rng, natoms, dim):
    u = rng.standard_normal(dim)
    u[: 3 * natoms].reshape(natoms, 3)[:] -= u[: 3 * natoms].reshape(natoms, 3).mean(axis=0)
    return u / np.linalg.norm(u)


def _straight_cubic_band(rng, natoms=5, s=(0.0, 0.3, 0.5, 1.1, 1.4, 2.0)):
    dim = 3 * (natoms + 3)
    s = np.array(s)
    u = _unit_zero_mean(rng, natoms, dim)
    X0 = rng.standard_normal(dim)
    X = np.array([X0 + sk * u for sk in s])
    # a rigid translation of each image's atoms: removed by the translation-free metric
    for k in range(len(s)):
        X[k, : 3 * natoms].reshape(natoms, 3)[:] += rng.standard_normal(3)
    c = np.array([0.2, 1.5, -0.4, -0.45])  # H(s) = c0 + c1 s + c2 s^2 + c3 s^3
    H = c[0] + c[1] * s + c[2] * s**2 + c[3] * s**3
    dH = c[1] + 2 * c[2] * s + 3 * c[3] * s**2
    Fg = np.empty_like(X)
    for k in range(len(s)):
        w = rng.standard_normal(dim)
        w -= (w @ u) * u  # perpendicular force: no tangential component
        w[: 3 * natoms].reshape(natoms, 3)[:] += rng.standard_normal(3)  # uniform force on the atoms (zero along u)
        Fg[k] = -dH[k] * u + w
    return natoms, s, X, H, dH, Fg, c


def test_straight_path_reproduces_a_cubic(orc):
    rng = np.random.default_rng(11)
    natoms, s, X, H, dH, Fg, c = _straight_cubic_band(rng)
    s_o, sl = orc.profile(X, H, Fg, natoms)
    np.testing.assert_allclose(s_o, s, atol=1e-12)
    np.testing.assert_allclose(sl, dH, atol=1e-11)
    q = np.linspace(0.0, s[-1], 1001)
    np.testing.assert_allclose(orc.spline_eval(s_o, H, sl, q),
                               c[0] + c[1] * q + c[2] * q**2 + c[3] * q**3, atol=1e-11)
    # closed-form maximum of the cubic over [0, S]: ends and roots of its derivative
    roots = np.roots([3 * c[3], 2 * c[2], c[1]])
    cand = [0.0, s[-1]] + [r.real for r in roots if abs(r.imag) < 1e-14 and 0 < r.real < s[-1]]
    vals = [c[0] + c[1] * x + c[2] * x**2 + c[3] * x**3 for x in cand]
    hm, at = orc.spline_max(s_o, H, sl)
    assert hm == pytest.approx(max(vals), abs=1e-11)
    assert at == pytest.approx(cand[int(np.argmax(vals))], abs=1e-7)


def test_flat_slopes_give_smoothstep(orc):
    s = np.array([0.0, 2.0])
    H = np.array([1.0, 3.0])
    t = np.linspace(0, 1, 101)
    out = orc.spline_eval(s, H, np.zeros(2), 2.0 * t)
    np.testing.assert_allclose(out, 1.0 + 2.0 * (3 * t**2 - 2 * t**3), atol=1e-14)
    hm, at = orc.spline_max(s, H, np.zeros(2))
    assert (hm, at) == (3.0, 2.0)


def test_nodes_are_reproduced_and_maximum_matches_brute_force(orc):
    rng = np.random.default_rng(5)
    for trial in range(20):
        M = int(rng.integers(2, 12))
        s = np.concatenate([[0.0], np.cumsum(rng.uniform(0.05, 1.0, M - 1))])
        H = rng.standard_normal(M)
        sl = 3.0 * rng.standard_normal(M)
        np.testing.assert_allclose(orc.spline_eval(s, H, sl, s), H, atol=1e-13)
        dense = orc.spline_eval(s, H, sl, np.linspace(0, s[-1], 200001))
        hm, at = orc.spline_max(s, H, sl)
        assert dense.max() <= hm + 1e-12
        assert hm - dense.max() < 1e-7
        assert orc.spline_eval(s, H, sl, [at])[0] == pytest.approx(hm, abs=1e-12)


def test_slopes_are_directional_derivatives_of_the_enthalpy(orc):
    # three images on a straight line in X (with a rigid translation of the atoms
    # mixed into the line): every tangent is the line's translation-free direction,
    # and dH/ds there is the central difference of the real enthalpy along it
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    p = orc.default_params(orc.LJ, pressure_GPa=1.5)
    XA, XB = orc.build_endpoints(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    n = XA.shape[0] - 3
    h0 = np.asarray(w["cell_init"], float).reshape(3, 3)
    d = 0.3 * (XB - XA)
    d[:n] += np.array([0.02, -0.01, 0.03])
    X = np.array([XA + 0.35 * (XB - XA), XA + 0.35 * (XB - XA) + d, XA + 0.35 * (XB - XA) + 2 * d])
    ev = [orc.cf_eval(p, h0, x) for x in X]
    H = np.array([e["H"] for e in ev])
    Fg = np.array([e["Fg"] for e in ev])
    s, sl = orc.profile(X, H, Fg, n)
    dc = d.copy()
    dc[:n] -= dc[:n].mean(axis=0)
    u = dc / np.linalg.norm(dc)
    assert s[1] == pytest.approx(np.linalg.norm(dc), rel=1e-12)
    eps = 1e-5
    for k in range(3):
        fd = (orc.cf_eval(p, h0, X[k] + eps * u)["H"] - orc.cf_eval(p, h0, X[k] - eps * u)["H"]) / (2 * eps)
        assert sl[k] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_rigid_translation_of_an_image_changes_nothing(orc):
    rng = np.random.default_rng(3)
    natoms, s, X, H, dH, Fg, c = _straight_cubic_band(rng)
    s1, sl1 = orc.profile(X, H, Fg, natoms)
    X2 = X.copy()
    X2[2, : 3 * natoms].reshape(natoms, 3)[:] += np.array([0.7, -0.2, 0.4])
    s2, sl2 = orc.profile(X2, H, Fg, natoms)
    np.testing.assert_allclose(s2, s1, atol=1e-12)
    np.testing.assert_allclose(sl2, sl1, atol=1e-12)


def test_vacancy_hop_profile_peaks_at_the_climbing_image(orc):
    # symmetric hop, converged with a climbing image: the interpolant's maximum is
    # the climbing image (zero force there), at the middle of the path
    from test_oracle_neb import _lj_band
    b = _lj_band(orc, M=7, steps=300, climb_after=30)
    e = b.energies()
    pr = b.profile(n_samples=101)
    np.testing.assert_allclose(pr["H"], pr["H"][::-1], atol=1e-9)
    np.testing.assert_allclose(pr["slope"], -pr["slope"][::-1], atol=1e-7)
    np.testing.assert_allclose(pr["samples"], pr["samples"][::-1], atol=1e-8)
    assert pr["xi_max"] == pytest.approx(0.5, abs=1e-3)
    assert abs(pr["slope"][3]) < 1e-3
    assert pr["barrier"] == pytest.approx(pr["H"][3] - pr["H"][0], abs=1e-6)
    assert pr["barrier"] == pytest.approx(e["barrier"], abs=1e-3)
    assert pr["samples"][0] == pr["H"][0] and pr["samples"][-1] == pr["H"][-1]


def test_coincident_images_give_a_zero_length_interval(orc):
    # two coincident images (same X, so the same H): the interval between them has
    # zero length and carries no curve; the nodes are still reproduced and the maximum
    # agrees with dense sampling
    rng = np.random.default_rng(9)
    s = np.array([0.0, 0.7, 0.7, 1.5, 2.2])
    H = np.array([0.0, 0.8, 0.8, 0.3, -0.2])
    for trial in range(5):
        sl = 2.0 * rng.standard_normal(5)
        np.testing.assert_allclose(orc.spline_eval(s, H, sl, s), H, atol=1e-14)
        # the slopes on the two sides of the zero-length interval differ, so the curve
        # may peak at a kink on a node: the grid includes the nodes
        dense = orc.spline_eval(s, H, sl, np.union1d(np.linspace(0, s[-1], 100001), s))
        assert np.isfinite(dense).all()
        hm, at = orc.spline_max(s, H, sl)
        assert dense.max() <= hm + 1e-12 and hm - dense.max() < 1e-7
    # from coordinates: the coincident pair has zero spacing and one-sided slopes
    natoms, s0, X, H0, dH, Fg, c = _straight_cubic_band(rng)
    X[3] = X[2]
    Fg[3] = Fg[2]
    H0 = H0.copy()
    H0[3] = H0[2]
    s1, sl1 = orc.profile(X, H0, Fg, natoms)
    assert s1[3] == s1[2] and np.isfinite(sl1).all()


def test_profile_of_the_analytic_surface_peaks_at_its_saddle(orc):
    # V(x, y) = (1 - x^2)^2 + kappa (y - x^2)^2 on a curved path: a converged
    # climbing-image band sits on the saddle (0, 0) with V = 1.  With the closed-form
    # gradient as forces (no atoms, no translation to remove), the slopes vanish at
    # the two minima and at the saddle, and the interpolant's maximum is the saddle's
    kappa, M = 2.0, 9
    t = np.linspace(0, 1, M)
    xy = np.stack([-1 + 2 * t, 1.0 + 0.3 * np.sin(np.pi * t)], axis=1)
    xy[0], xy[-1] = [-1, 1], [1, 1]
    out = orc.neb2d(kappa, xy, k_spring=1.0, climb_after=20, dt0=0.01, dtmax=0.05, maxstep=0.05,
                    max_steps=50000, f_tol=1e-9)
    P = out["xy"]
    x, y = P[:, 0], P[:, 1]
    V = (1 - x**2) ** 2 + kappa * (y - x**2) ** 2
    gx = -4 * x * (1 - x**2) - 4 * kappa * x * (y - x**2)
    gy = 2 * kappa * (y - x**2)
    F = -np.stack([gx, gy], axis=1)
    s, sl = orc.profile(P, V, F, 0)
    ci = (M - 1) // 2
    assert abs(sl[0]) < 1e-12 and abs(sl[-1]) < 1e-12 and abs(sl[ci]) < 1e-8
    hm, at = orc.spline_max(s, V, sl)
    assert hm == pytest.approx(1.0, abs=1e-8)
    assert at == pytest.approx(s[ci], abs=1e-6)
    # uphill then downhill along the path
    assert np.all(sl[1:ci] > 0) and np.all(sl[ci + 1:-1] < 0)
