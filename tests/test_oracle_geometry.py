"""Pins of the oracle's 3x3 geometry against library routines and closed forms."""
import numpy as np
import pytest


def _spd(rng):
    A = rng.normal(size=(3, 3))
    return A @ A.T + 0.5 * np.eye(3)


def test_inv_det_match_numpy(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        A = rng.normal(size=(3, 3)) + 2 * np.eye(3)
        assert orc.det3(A) == pytest.approx(np.linalg.det(A), rel=1e-12)
        np.testing.assert_allclose(orc.inv3(A), np.linalg.inv(A), rtol=1e-11, atol=1e-12)


def test_symsqrt_squares_back(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        B = _spd(rng)
        D = orc.symsqrt(B)
        np.testing.assert_allclose(D, D.T, atol=1e-14)
        np.testing.assert_allclose(D @ D, B, rtol=1e-12, atol=1e-13)
        assert np.all(np.linalg.eigvalsh(D) > 0)
        # the positive square root is unique: compare with the eigen-decomposition route
        w, Q = np.linalg.eigh(B)
        np.testing.assert_allclose(D, (Q * np.sqrt(w)) @ Q.T, rtol=1e-11, atol=1e-12)


def test_symsqrt_special_cases(orc):
    np.testing.assert_array_equal(orc.symsqrt(np.eye(3)), np.eye(3))
    np.testing.assert_allclose(orc.symsqrt(np.diag([4.0, 9.0, 0.25])), np.diag([2.0, 3.0, 0.5]),
                               rtol=1e-15)
    with pytest.raises(orc.OracleError) as e:
        orc.symsqrt(np.diag([1.0, -1.0, 1.0]))
    assert e.value.code == orc.ECELL


def test_widths_are_face_distances(orc):
    rng = np.random.default_rng(2)
    for _ in range(20):
        h = np.diag(rng.uniform(3, 8, 3)) + np.tril(rng.normal(0, 1.0, (3, 3)), -1)
        # distance between the faces normal to reciprocal vector k is 1 / |column k of h^-1|
        w_ref = 1.0 / np.linalg.norm(np.linalg.inv(h), axis=0)
        np.testing.assert_allclose(orc.widths(h), w_ref, rtol=1e-12)
    np.testing.assert_allclose(orc.widths(np.diag([2.0, 3.0, 4.0])), [2.0, 3.0, 4.0], rtol=1e-15)
