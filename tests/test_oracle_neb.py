"""Pins of the oracle's NEB pieces: the improved tangent's branches, the
projection's orthogonality (Eq. (1)), a climbing-image band on an analytic
surface with a closed-form saddle, the symmetry of the vacancy-hop band,
brute-force cases of the adaptive-image decision, hand-worked FIRE moves, the
path coordinate of known spacings, and a converged vacancy barrier that does not
depend on the number of images."""
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


# ------------------------------------------------------------------ FIRE
# Hand-built states of one FIRE move (Bitzek et al. 2006, the band-global form of
# the band step): every expected value below was worked out by hand from the rules
# (power test, mixing with the old alpha, growth only after more than N_min positive
# steps, reset, v += dt F, X += dt v clamped by the largest row displacement).
def _fire_band(moving_rows, M=3):
    """X, v, F of M images whose moving images have the given rows (lists of 3-vectors)."""
    rows = len(moving_rows[0])
    X = np.zeros((M, rows, 3))
    X[:, :, 0] = 10.0  # endpoints and images sit away from zero
    return X


def _one_image(v_rows, f_rows):
    X = _fire_band([v_rows])
    v = np.zeros_like(X)
    F = np.zeros_like(X)
    v[1] = v_rows
    F[1] = f_rows
    return X, v, F


def test_fire_fresh_step_skips_the_power_test(orc):
    # P = F.v = -2 < 0 would reset; right after creation or a refine it is not tested
    X, v, F = _one_image([[1, 0, 0], [0, 0, 0]], [[-2, 0, 0], [0, 0, 0]])
    X1, v1, dt, alpha, n_pos, fresh = orc.fire_step(X, v, F, 0.1, 0.07, 3, 1, dtmax=1.0, maxstep=1.0)
    assert (dt, alpha, n_pos, fresh) == (0.1, 0.07, 3, 0)
    assert v1[1, 0, 0] == pytest.approx(0.8, abs=1e-15)          # 1 + 0.1 * (-2)
    assert X1[1, 0, 0] - X[1, 0, 0] == pytest.approx(0.08, abs=1e-14)
    # endpoints never move
    np.testing.assert_array_equal(X1[[0, 2]], X[[0, 2]])
    np.testing.assert_array_equal(v1[[0, 2]], 0.0)


@pytest.mark.parametrize("F_row", [[-2, 0, 0], [0, 2, 0]])
def test_fire_non_positive_power_resets(orc, F_row):
    # P < 0 and P = 0 exactly (F perpendicular to v): v = 0, alpha = alpha_start,
    # dt halved, N_P = 0; then v = dt F with the halved dt
    X, v, F = _one_image([[1, 0, 0], [0, 0, 0]], [F_row, [0, 0, 0]])
    X1, v1, dt, alpha, n_pos, fresh = orc.fire_step(X, v, F, 0.1, 0.05, 3, 0, dtmax=1.0, maxstep=1.0,
                                                    astart=0.1, fdec=0.5)
    assert (dt, alpha, n_pos, fresh) == (0.05, 0.1, 0, 0)
    expect_v = 0.05 * np.array(F_row, float)
    np.testing.assert_allclose(v1[1, 0], expect_v, rtol=0, atol=1e-16)
    np.testing.assert_allclose(X1[1, 0] - X[1, 0], 0.05 * expect_v, rtol=0, atol=1e-15)


def test_fire_mixing_without_growth_up_to_nmin(orc):
    # v = (0, 5, 0), F = (3, 4, 0): P = 20, |v| = |F| = 5; alpha 0.1 mixes to
    # 0.9 (0, 5, 0) + 0.1 (3, 4, 0) = (0.3, 4.9, 0).  N_P = 5 = N_min: no growth yet.
    # Then v += 0.1 F = (0.6, 5.3, 0) and X += 0.1 v = (0.06, 0.53, 0).
    X, v, F = _one_image([[0, 5, 0], [0, 0, 0]], [[3, 4, 0], [0, 0, 0]])
    X1, v1, dt, alpha, n_pos, fresh = orc.fire_step(X, v, F, 0.1, 0.1, 5, 0, dtmax=1.0, maxstep=1.0,
                                                    nmin=5)
    assert (dt, alpha, n_pos) == (0.1, 0.1, 6)
    np.testing.assert_allclose(v1[1, 0], [0.6, 5.3, 0.0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(X1[1, 0] - X[1, 0], [0.06, 0.53, 0.0], rtol=0, atol=1e-14)


def test_fire_growth_after_nmin_mixes_with_the_old_alpha(orc):
    # N_P = 6 > N_min = 5: the mix still uses alpha = 0.1, giving (0.3, 4.9, 0); then
    # dt = 0.1 * 1.1 = 0.11 and alpha = 0.1 * 0.99 = 0.099; v = (0.3, 4.9, 0) +
    # 0.11 (3, 4, 0) = (0.63, 5.34, 0); X += 0.11 v = (0.0693, 0.5874, 0)
    X, v, F = _one_image([[0, 5, 0], [0, 0, 0]], [[3, 4, 0], [0, 0, 0]])
    X1, v1, dt, alpha, n_pos, fresh = orc.fire_step(X, v, F, 0.1, 0.1, 6, 0, dtmax=1.0, maxstep=1.0,
                                                    nmin=5, finc=1.1, fa=0.99)
    assert dt == pytest.approx(0.11, abs=1e-16) and alpha == pytest.approx(0.099, abs=1e-16)
    assert n_pos == 7
    np.testing.assert_allclose(v1[1, 0], [0.63, 5.34, 0.0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(X1[1, 0] - X[1, 0], [0.0693, 0.5874, 0.0], rtol=0, atol=1e-14)


def test_fire_dt_is_capped_at_dtmax(orc):
    X, v, F = _one_image([[0, 5, 0], [0, 0, 0]], [[3, 4, 0], [0, 0, 0]])
    _, _, dt, alpha, n_pos, _ = orc.fire_step(X, v, F, 0.95, 0.1, 10, 0, dtmax=1.0, maxstep=10.0)
    assert dt == 1.0 and n_pos == 11


def test_fire_power_and_norms_are_band_global(orc):
    # image 1: v = (3, 0, 0), F = (12, 0, 0), P_1 = 36; image 2: v = (0, 4, 0),
    # F = (0, -5, 0), P_2 = -20.  The band's P = 16 > 0: both images are mixed (none is
    # reset) with |v| = 5 and |F| = 13: v_mix = 0.9 v + 0.1 (5 / 13) F.
    X = _fire_band([[[0, 0, 0]]], M=4)
    v = np.zeros_like(X)
    F = np.zeros_like(X)
    v[1, 0] = [3, 0, 0]
    F[1, 0] = [12, 0, 0]
    v[2, 0] = [0, 4, 0]
    F[2, 0] = [0, -5, 0]
    X1, v1, dt, alpha, n_pos, _ = orc.fire_step(X, v, F, 0.01, 0.1, 0, 0, dtmax=1.0, maxstep=10.0)
    assert (dt, alpha, n_pos) == (0.01, 0.1, 1)
    np.testing.assert_allclose(v1[1, 0], [2.7 + 6.0 / 13.0 + 0.12, 0, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(v1[2, 0], [0, 3.6 - 2.5 / 13.0 - 0.05, 0], rtol=0, atol=1e-14)


def test_fire_step_clamp_uses_the_largest_row(orc):
    # fresh, v = 0, dt = 1: v = F and dr = F with rows of length 0.5, 0.1 and 0.2.
    # maxstep 0.25 scales dr by 0.25 / 0.5 = 1/2 (a global norm, sqrt(0.3), would give
    # 0.456; the largest component, 0.4, would give 0.625); v itself is not scaled.
    rows = np.array([[0.3, 0.4, 0.0], [0.1, 0.0, 0.0], [0.0, 0.0, 0.2]])
    X = _fire_band([rows])
    v = np.zeros_like(X)
    F = np.zeros_like(X)
    F[1] = rows
    X1, v1, dt, *_ = orc.fire_step(X, v, F, 1.0, 0.1, 0, 1, dtmax=1.0, maxstep=0.25)
    np.testing.assert_allclose(X1[1] - X[1], [[0.15, 0.2, 0.0], [0.05, 0.0, 0.0], [0.0, 0.0, 0.1]],
                               rtol=0, atol=1e-15)
    np.testing.assert_array_equal(v1[1], rows)
    # below the limit nothing is scaled
    X1, *_ = orc.fire_step(X, v, F, 1.0, 0.1, 0, 1, dtmax=1.0, maxstep=0.5000001)
    np.testing.assert_allclose(X1[1] - X[1], rows, rtol=0, atol=1e-15)


# ------------------------------------------------------------ path coordinate
def test_path_coordinate_of_known_spacings(orc):
    # four atoms and three cell rows; interval k moves the atoms by (+a, -a, +a, -a)
    # along x (length 2a once the mean is removed) and cell entry (0, 0) by b, with
    # a = 0.3 L_k and b = 0.8 L_k (length L_k), on top of a rigid translation of all
    # atoms that the coordinate ignores.  L = (1, 2, 3): xi = (0, 1/6, 1/2, 1).
    L = [1.0, 2.0, 3.0]
    X = np.zeros((4, 7, 3))
    X[0, :4] = [[0.1, 0.2, 0.3], [1.1, 0.2, 0.3], [0.1, 1.2, 0.3], [0.1, 0.2, 1.3]]
    X[0, 4:] = 5.0 * np.eye(3)
    sign = np.array([1.0, -1.0, 1.0, -1.0])
    for k, Lk in enumerate(L):
        X[k + 1] = X[k]
        X[k + 1, :4, 0] += 0.3 * Lk * sign
        X[k + 1, 4, 0] += 0.8 * Lk
        X[k + 1, :4] += np.array([0.7, -0.4, 0.25]) * [1.0, 0.0, 2.0][k]  # rigid translation
    xi = orc.path_coord(X, 4)
    np.testing.assert_allclose(xi, [0.0, 1.0 / 6.0, 0.5, 1.0], rtol=0, atol=1e-14)
    # the raw differences (translation included) would place the images elsewhere
    raw = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(X.reshape(4, -1), axis=0), axis=1))])
    assert np.abs(raw / raw[-1] - xi).max() > 1e-2
    # without atom rows (natoms = 0) the translation counts
    np.testing.assert_allclose(orc.path_coord(X, 0), raw / raw[-1], rtol=0, atol=1e-14)


def test_band_reports_the_profile_coordinate(orc):
    # the band's readout uses the same coordinate as its energy profile
    b = _lj_band(orc, M=6, steps=20, climb_after=10)
    e = b.energies()
    X = b.get_state()["X"]
    np.testing.assert_array_equal(e["xi"], orc.path_coord(X, b.n))
    prof = b.profile()
    np.testing.assert_allclose(e["xi"], prof["s"] / prof["s"][-1], rtol=0, atol=1e-15)
    assert e["xi"][0] == 0.0 and e["xi"][-1] == 1.0 and np.all(np.diff(e["xi"]) > 0)


# ------------------------------------------- barrier independent of the image count
@pytest.mark.slow
def test_vacancy_barrier_is_independent_of_the_image_count(orc):
    # The 255-atom LJ vacancy hop (4x4x4 FCC cells) from relaxed endpoints: with the
    # climbing image converged (fmax < 1e-3 eV/A) the barrier is the saddle's enthalpy
    # minus the initial minimum's, whatever the number of images.  The climbing image
    # sits on the symmetric midpoint of the hop.
    w = W.lj_fcc_hop_255()
    p0 = orc.default_params(orc.LJ)
    A = orc.relax(p0, w["pos_init"], w["cell_init"], 20000, 1e-6)
    B = orc.relax(p0, w["pos_final"], w["cell_final"], 20000, 1e-6)
    assert A[3] < 1e-6 and B[3] < 1e-6
    # the two relaxed endpoints are images of each other under the hop's symmetry
    assert orc.evaluate(p0, A[0], A[1])[0] == pytest.approx(orc.evaluate(p0, B[0], B[1])[0], abs=1e-9)
    barriers = []
    for M in (7, 9, 11):
        p = orc.default_params(orc.LJ, n_images=M, max_images=M, climb_after=50, k_spring=1.0,
                               fire_dt0=0.005)
        b = orc.Band(p, A[0], A[1], B[0], B[1])
        d, fmax, conv = b.step(20000, 1e-3)
        assert conv
        e = b.energies()
        assert e["ci"] == (M - 1) // 2
        barriers.append(e["barrier"])
    assert max(barriers) - min(barriers) <= 1e-3, barriers
    assert 5.0 < barriers[0] < 6.5
