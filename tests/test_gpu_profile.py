"""Parity of the energy-profile readout (cfneb_profile) with the FP64 oracle.

The oracle takes the device's own coordinates X of every image, evaluates each
image, and forms the arc lengths, slopes dH/ds, the Hermite samples and the
maximum.  Tolerances follow from the force-path bounds: H_k to TOL_E_PER_ATOM * n;
a slope is a force projected on a unit vector, so its error is at most the 2-norm
of the generalized-force error (<= TOL_F per component, two for the FP32 rounding
of D); between nodes the Hermite basis weighs H by at most 1 and d * slope by at
most 4/27 per end.
"""
import numpy as np
import pytest

from gpu_cases import TOL_BARRIER, TOL_E_PER_ATOM, TOL_F, make_pair, oracle_params_like

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)


def _centred(d, n):
    d = d.copy()
    d[:n] -= d[:n].mean(axis=0)
    return d


def _oracle_profile(p, h0, X, n, n_samples):
    import oracle
    ev = [oracle.cf_eval(p, h0, x) for x in X]
    H = np.array([e["H"] for e in ev])
    Fg = np.array([e["Fg"] for e in ev])
    s, sl = oracle.profile(X, H, Fg, n)
    S = s[-1]
    xi = np.arange(n_samples) / (n_samples - 1)
    hm, at = oracle.spline_max(s, H, sl)
    return dict(s=s, H=H, slope=sl, samples=oracle.spline_eval(s, H, sl, xi * S), barrier=hm - H[0],
                s_max=at, H_max=hm)


def _tolerances(n, s):
    tol_h = TOL_E_PER_ATOM * n
    tol_slope = 2.0 * TOL_F * np.sqrt(3.0 * (n + 3))
    dmax = np.diff(s).max()
    tol_samp = tol_h + (8.0 / 27.0) * dmax * tol_slope
    return tol_h, tol_slope, tol_samp


@pytest.mark.parametrize("name,fp64,steps,press", [("lj31", True, 40, 0.0), ("lj_ragged", False, 25, 0.0),
                                                   ("ts_small", False, 15, 2.0), ("ts_diamond", False, 10, 0.0)])
def test_profile_matches_oracle(name, fp64, steps, press):
    import oracle
    kw = dict(n_images=7, max_images=9, climb_after=10, pressure_GPa=press)
    g, _, w, kind = make_pair(name, fp64=fp64, oracle_too=False, **kw)
    g.step(steps)
    ns = 257
    pr = g.profile(n_samples=ns)
    X = g.get_state()["X"]
    n = g.n
    ref = _oracle_profile(oracle_params_like(kind, **kw), w["cell_init"], X, n, ns)
    tol_h, tol_slope, tol_samp = _tolerances(n, ref["s"])
    np.testing.assert_allclose(pr["s"], ref["s"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pr["H"], ref["H"], rtol=0, atol=tol_h)
    np.testing.assert_allclose(pr["slope"], ref["slope"], rtol=0, atol=tol_slope)
    np.testing.assert_allclose(pr["samples"], ref["samples"], rtol=0, atol=tol_samp)
    assert abs(pr["barrier"] - ref["barrier"]) <= 2 * tol_samp
    assert pr["barrier"] >= pr["H"].max() - pr["H"][0] - 1e-12
    # the device's maximum is a maximum of the oracle's interpolant to the same bound
    S = ref["s"][-1]
    at = oracle.spline_eval(ref["s"], ref["H"], ref["slope"], [pr["xi_max"] * S])[0]
    assert at >= ref["H_max"] - 2 * tol_samp
    # the nodes are reproduced and the ends are the endpoint enthalpies
    assert pr["samples"][0] == pr["H"][0] and pr["samples"][-1] == pr["H"][-1]
    # the images' stored enthalpies are those of the current coordinates
    for k in range(len(X)):
        assert g.image(k)["H"] == pr["H"][k]


def test_profile_of_a_converged_band_peaks_at_the_climbing_image():
    kw = dict(n_images=7, max_images=7, climb_after=50, k_spring=1.0, fire_dt0=0.005)
    g, _, w, kind = make_pair("lj31", fp64=True, oracle_too=False, **kw)
    _, fmax, conv = g.step(6000, 1e-3)
    assert conv
    e = g.energies()
    pr = g.profile(n_samples=101)
    assert e["ci"] == 3
    assert abs(pr["slope"][3]) <= 2e-3  # |F . tau| <= |F_CI| < f_tol at the climbing image
    assert abs(pr["barrier"] - e["barrier"]) <= TOL_BARRIER
    assert pr["xi_max"] == pytest.approx(0.5, abs=0.02)
    np.testing.assert_allclose(pr["samples"], pr["samples"][::-1], rtol=0, atol=5e-3)
    # the band still steps after the readout: converged again at once
    sd, fm, c2 = g.step(10, 1e-3)
    assert c2 and sd == 0


def test_profile_arguments_and_edge_cases():
    from paper_2510_16721_amd import cfneb
    g, _, w, kind = make_pair("lj31", fp64=False, oracle_too=False, n_images=3, max_images=3)
    for bad in (-1, 1, 4097):  # at most CFNEB_PROFILE_MAX_SAMPLES = 4096
        with pytest.raises(cfneb.CfnebError):
            g.profile(n_samples=bad)
    pr = g.profile(n_samples=4096)  # the largest sample count, minimal band
    assert len(pr["samples"]) == 4096 and np.isfinite(pr["samples"]).all()
    assert pr["s"][0] == 0.0 and np.all(np.diff(pr["s"]) >= 0)
    pr0 = g.profile()  # no samples
    assert pr0["samples"].size == 0 and pr0["barrier"] == pytest.approx(pr["barrier"], abs=1e-12)


def test_profile_with_the_maximum_image_count():
    import oracle
    kw = dict(n_images=64, max_images=64, climb_after=-1)
    g, _, w, kind = make_pair("lj31", fp64=True, oracle_too=False, **kw)
    g.step(3)
    pr = g.profile(n_samples=640)
    X = g.get_state()["X"]
    ref = _oracle_profile(oracle_params_like(kind, **kw), w["cell_init"], X, g.n, 640)
    tol_h, tol_slope, tol_samp = _tolerances(g.n, ref["s"])
    assert len(pr["H"]) == 64
    np.testing.assert_allclose(pr["s"], ref["s"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pr["slope"], ref["slope"], rtol=0, atol=tol_slope)
    np.testing.assert_allclose(pr["samples"], ref["samples"], rtol=0, atol=tol_samp)


def test_full_size_profile_sampled():
    # 98,304-atom graphite band of 24 images at 15 GPa, as in the benchmark: the arc
    # lengths against the device's coordinates, the slope of the first image and of a
    # middle image against the oracle (the middle image's tangent branch taken from
    # the device's enthalpies, in which the device decides it)
    import oracle
    kw = dict(n_images=24, max_images=40, min_images=5, pressure_GPa=15.0, refine_every=20,
              climb_after=100)
    g, _, w, kind = make_pair("ts98304", oracle_too=False, **kw)
    g.step(2)
    pr = g.profile(n_samples=4096)
    X = g.get_state()["X"]
    n = g.n
    seg = np.array([np.linalg.norm(_centred(X[k + 1] - X[k], n)) for k in range(len(X) - 1)])
    np.testing.assert_allclose(np.diff(pr["s"]), seg, rtol=1e-9)
    p = oracle_params_like(kind, pressure_GPa=15.0)
    tol_h, tol_slope, tol_samp = _tolerances(n, pr["s"])
    k = 11
    ev = [oracle.cf_eval(p, w["cell_init"], X[j]) for j in (k - 1, k, k + 1)]
    for j, e in zip((k - 1, k, k + 1), ev):
        assert abs(e["H"] - pr["H"][j]) <= tol_h
    _, sl = oracle.profile(X[k - 1:k + 2], pr["H"][k - 1:k + 2], np.array([e["Fg"] for e in ev]), n)
    assert abs(sl[1] - pr["slope"][k]) <= tol_slope
    e0 = oracle.cf_eval(p, w["cell_init"], X[0])
    _, sl0 = oracle.profile(X[:2], pr["H"][:2], np.array([e0["Fg"], np.zeros_like(e0["Fg"])]), n)
    assert abs(sl0[0] - pr["slope"][0]) <= tol_slope
    assert np.isfinite(pr["samples"]).all()
    assert pr["barrier"] >= pr["H"].max() - pr["H"][0] - 1e-9


def test_profile_with_coincident_images():
    # two coincident images: a zero-length interval (no curve on it), one-sided
    # tangents beside it; the device and the oracle agree on the whole profile
    import oracle
    kw = dict(n_images=7, max_images=7, climb_after=-1)
    g, _, w, kind = make_pair("lj31", fp64=True, oracle_too=False, **kw)
    g.step(5)
    st = g.get_state()
    X = st["X"].copy()
    X[3] = X[2]
    g.set_state(X, st["v"], st["dt"], st["alpha"], st["n_pos"], st["fresh"], st["step"], st["ci"])
    pr = g.profile(n_samples=301)
    ref = _oracle_profile(oracle_params_like(kind, **kw), w["cell_init"], X, g.n, 301)
    tol_h, tol_slope, tol_samp = _tolerances(g.n, ref["s"])
    assert pr["s"][3] == pr["s"][2] and ref["s"][3] == ref["s"][2]
    assert pr["H"][3] == pr["H"][2]
    np.testing.assert_allclose(pr["s"], ref["s"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pr["slope"], ref["slope"], rtol=0, atol=tol_slope)
    np.testing.assert_allclose(pr["samples"], ref["samples"], rtol=0, atol=tol_samp)
    assert abs(pr["barrier"] - ref["barrier"]) <= 2 * tol_samp


def test_profile_of_a_band_stepped_in_a_batch():
    # a band stepped inside a batch (between batch calls) reads out the same profile
    # as the oracle computes from its coordinates
    from paper_2510_16721_amd import cfneb
    kw = dict(n_images=7, max_images=9, climb_after=10, pressure_GPa=2.0)
    g, _, w, kind = make_pair("ts_small", oracle_too=False, **kw)
    other, _, _, _ = make_pair("lj_ragged", oracle_too=False, n_images=5, max_images=5)
    batch = cfneb.Batch(4)
    batch.attach(g)
    batch.attach(other)
    batch.step(12)
    pr = g.profile(n_samples=129)
    X = g.get_state()["X"]
    ref = _oracle_profile(oracle_params_like(kind, **kw), w["cell_init"], X, g.n, 129)
    tol_h, tol_slope, tol_samp = _tolerances(g.n, ref["s"])
    np.testing.assert_allclose(pr["s"], ref["s"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pr["H"], ref["H"], rtol=0, atol=tol_h)
    np.testing.assert_allclose(pr["samples"], ref["samples"], rtol=0, atol=tol_samp)
    # the batch goes on stepping after the readout
    steps, conv, errs = batch.step(3)
    assert not errs.any()
    batch.close()
