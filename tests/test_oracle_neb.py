"""Pins of the oracle's NEB pieces: the improved tangent's branches, the
projection's orthogonality (Eq. (1)), a climbing-image band on an analytic
surface with a closed-form saddle, the symmetry of the vacancy-hop band, and
brute-force cases of the adaptive-image decision."""
import numpy as np
import pytest

import workloads as W


def test_tangent_branches(orc):
    # monotonic up: upwind is the next image
    assert orc.tangent_coeffs(0.0, 1.0, 2.0) == (1.0, 0.0)
    # monotonic down: upwind is the previous image
    assert orc.tangent_coeffs(2.0, 1.0, 0.0) == (0.0, 1.0)
    # local maximum, right neighbour higher: weight dmax on tau+
    a, b = orc.tangent_coeffs(0.0, 3.0, 1.0)  # dp = 2, dm = 3, Hp > Hm -> (dmax, dmin)
    assert (a, b) == (3.0, 2.0)
    a, b = orc.tangent_coeffs(1.0, 3.0, 0.0)  # Hp < Hm -> (dmin, dmax)
    assert (a, b) == (2.0, 3.0)
    # local minimum
    a, b = orc.tangent_coeffs(2.0, 0.0, 5.0)
    assert (a, b) == (5.0, 2.0)
    # flat: strict comparisons fall to the weighted branch with zero weights
    assert orc.tangent_coeffs(1.0, 1.0, 1.0) == (0.0, 0.0)


def test_analytic_surface_climbing_image(orc):
    # V(x, y) = (1 - x^2)^2 + kappa (y - x^2)^2: minima (+-1, 1) with V = 0, and the
    # only saddle at (0, 0) with V = 1 (Hessian diag(-4, 2 kappa)); the MEP is curved.
    M = 9
    t = np.linspace(0, 1, M)
    xy = np.stack([-1 + 2 * t, 1.0 + 0.3 * np.sin(np.pi * t)], axis=1)
    xy[0] = [-1, 1]
    xy[-1] = [1, 1]
    out = orc.neb2d(2.0, xy, k_spring=1.0, climb_after=20, dt0=0.01, dtmax=0.05, maxstep=0.05,
                    max_steps=50000, f_tol=1e-9)
    assert out["fmax"] < 1e-9
    ci = out["ci"]
    assert ci == (M - 1) // 2
    np.testing.assert_allclose(out["xy"][ci], [0.0, 0.0], atol=1e-6)
    assert out["E"][ci] - out["E"][0] == pytest.approx(1.0, abs=1e-8)
    # the other images are off the straight line: the band follows the curved path
    assert np.all(out["xy"][1:-1, 1] < 1.0)


def test_analytic_surface_without_climbing(orc):
    # without the climbing image the highest image stays below the saddle
    M = 9
    t = np.linspace(0, 1, M)
    xy = np.stack([-1 + 2 * t, np.ones(M)], axis=1)
    out = orc.neb2d(2.0, xy, climb_after=-1, max_steps=50000, f_tol=1e-9)
    assert out["fmax"] < 1e-9
    assert out["ci"] == -1
    assert out["E"].max() <= 1.0 + 1e-12


def _lj_band(orc, M=7, steps=0, climb_after=50, **kw):
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    p = orc.default_params(orc.LJ, n_images=M, max_images=max(M, kw.pop("max_images", M)),
                           climb_after=climb_after, **kw)
    b = orc.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    if steps:
        b.step(steps)
    return b


def test_projection_invariants_one_step(orc):
    # take the band state, evaluate once (max_steps = 1 with a huge f_tol does not move)
    b = _lj_band(orc, steps=8, climb_after=4, k_spring=2.0)
    sd, fmax, conv = b.step(1, f_tol=1e30)
    assert sd == 0 and conv
    st = b.get_state()
    X = st["X"].reshape(st["X"].shape[0], -1)
    M = len(X)
    H = np.array([b.image(k)["H"] for k in range(M)])
    ci = st["ci"]
    assert 0 < ci < M - 1 and H[ci] == H[1:-1].max()
    n = b.n

    def centred(a):
        # differences and forces are taken modulo a rigid translation of the atoms
        a = a.reshape(-1, 3).copy()
        a[:n] -= a[:n].mean(axis=0)
        return a.ravel()

    for k in range(1, M - 1):
        img = b.image(k)
        Fg, Fn = centred(img["Fg"]), img["Fneb"].ravel()
        np.testing.assert_allclose(Fn.reshape(-1, 3)[:n].sum(axis=0), 0.0, atol=1e-11)
        tp, tm = centred(X[k + 1] - X[k]), centred(X[k] - X[k - 1])
        a, c = orc.tangent_coeffs(H[k - 1], H[k], H[k + 1])
        tau = a * tp + c * tm
        tau /= np.linalg.norm(tau)
        if k == ci:
            # the climbing image inverts the parallel force and keeps the rest
            assert Fn @ tau == pytest.approx(-(Fg @ tau), rel=1e-10, abs=1e-12)
            perp = Fn - (Fn @ tau) * tau
            np.testing.assert_allclose(perp, Fg - (Fg @ tau) * tau, atol=1e-10)
        else:
            spring = 2.0 * (np.linalg.norm(tp) - np.linalg.norm(tm))
            # only the spring acts along the tangent
            assert Fn @ tau == pytest.approx(spring, rel=1e-9, abs=1e-10)
            perp = Fn - (Fn @ tau) * tau
            np.testing.assert_allclose(perp, Fg - (Fg @ tau) * tau, atol=1e-10)


def test_rigid_translation_of_an_endpoint_changes_no_neb_force(orc):
    # a periodic band whose final endpoint is rigidly shifted is the same band: every
    # image moves by a uniform translation, which the NEB forces ignore
    w = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    p = orc.default_params(orc.LJ, n_images=6, max_images=6, climb_after=0, k_spring=3.0)
    shift = np.array([0.31, -0.17, 0.23])
    out = []
    for t in (np.zeros(3), shift):
        b = orc.Band(p, w["pos_init"], w["cell_init"], w["pos_final"] + t, w["cell_final"])
        X = b.get_state()["X"].copy()
        # move the interior images off the straight line, identically in both bands
        X[1:-1, :-3] += 0.05 * np.sin(np.arange(X[1:-1, :-3].size)).reshape(X[1:-1, :-3].shape)
        b.set_state(X, np.zeros_like(X), 0.01, 0.1, 0, 1, 5)
        assert b.step(1, f_tol=1e30)[0] == 0
        out.append([b.image(k)["Fneb"] for k in range(1, 5)])
        H = b.energies()["H"]
    for f0, f1 in zip(*out):
        np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-9)
    assert H[1:-1].max() > H[0]


def test_cell_coordinates_stay_symmetric(orc):
    # the lattice coordinates c_f B of every image stay an exactly symmetric matrix:
    # the force on them has no antisymmetric part, which would be a zero-energy mode
    w = W.graphite_to_diamond(2, 2, 3, seed=4, sigma=0.05)
    p = orc.default_params(orc.TERSOFF, n_images=5, max_images=5, pressure_GPa=5.0)
    b = orc.Band(p, w["pos_init"], w["cell_init"], w["pos_final"], w["cell_final"])
    b.step(40)
    X = b.get_state()["X"]
    for k in range(X.shape[0]):
        C = X[k, -3:]
        np.testing.assert_array_equal(C, C.T)
        Fc = b.image(k)["Fg"][-3:]
        np.testing.assert_array_equal(Fc, Fc.T)


def test_vacancy_hop_band_is_symmetric(orc):
    # inversion through the hop midpoint maps image k onto image M-1-k
    b = _lj_band(orc, M=7, steps=60, climb_after=30)
    e = b.energies()
    np.testing.assert_allclose(e["H"], e["H"][::-1], atol=1e-9)
    assert e["ci"] == 3
    assert e["barrier"] > 0


# ------------------------------------------------------------------ refine
def _band_1d(positions):
    return np.array(positions, float).reshape(-1, 1)


def test_refine_uniform_spacing_does_nothing(orc):
    ins, dele, d2 = orc.refine_decide(_band_1d(np.arange(7.0)), -1, 20, 3)
    assert (ins, dele) == (-1, -1)
    np.testing.assert_array_equal(d2, np.ones(6))


def test_refine_inserts_into_a_long_interval(orc):
    x = [0, 1, 2, 5, 6, 7]  # one gap three times the others
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 20, 3)
    assert (ins, dele) == (3, -1)
    # the same band at the image cap is left alone: no insert, and no image
    # sits between two short intervals below half the RMS spacing
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 6, 3)
    assert (ins, dele) == (-1, -1)


def test_refine_deletes_a_coincident_image(orc):
    x = [0, 1, 2, 2.0001, 2.0002, 3, 4]
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 7, 3)
    assert (ins, dele) == (-1, 3)
    # the climbing image is never deleted; here no other image qualifies
    ins, dele, _ = orc.refine_decide(_band_1d(x), 3, 7, 3)
    assert (ins, dele) == (-1, -1)
    # at the minimum image count nothing is deleted
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 7, 7)
    assert (ins, dele) == (-1, -1)


def test_refine_delete_ties_and_climbing_image(orc):
    # binary-exact spacings: squares 1, 1/256, 1/256, 1/256, 0.66015625, 1
    x = [0, 1, 1.0625, 1.125, 1.1875, 2, 3]
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 7, 3)
    assert (ins, dele) == (-1, 2)  # images 2 and 3 tie: lowest index
    ins, dele, _ = orc.refine_decide(_band_1d(x), 2, 7, 3)
    assert (ins, dele) == (-1, 3)  # the climbing image is skipped


def test_refine_ties_take_the_lowest_index(orc):
    x = [0, 5, 6, 7, 8, 9, 14]  # two equal long intervals (0-1 and 5-6)
    ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 20, 3)
    assert (ins, dele) == (1, -1)


def test_refine_threshold_is_exact(orc):
    # d_k*^2 (M-1) ins_den vs ins_num sum d^2 with ins = 9/4: intervals (a, 1, 1, 1)
    # give 4*4*a^2 > 9 (a^2 + 3)  <=>  a^2 > 27/7; the boundary is decided exactly
    for a2, expect in [(27 / 7 * (1 - 1e-12), -1), (27 / 7 * (1 + 1e-12), 1)]:
        a = np.sqrt(a2)
        x = [0, a, a + 1, a + 2, a + 3]
        ins, dele, _ = orc.refine_decide(_band_1d(x), -1, 20, 5)
        assert ins == expect
