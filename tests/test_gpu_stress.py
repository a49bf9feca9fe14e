"""Applied stress on the device against the oracle: a constant second
Piola-Kirchhoff stress S referred to h0 (enthalpy term -Omega0 S : E with
E = (D D^T - I)/2) in both cell filters.  Generalized forces per image from the
device's own coordinates; converged barriers under stress in both filters (the
stress work depends on lengths only, so both filters share the saddle and the
barrier); relaxation under stress, whose crystal carries the push-forward of S.
"""
import numpy as np
import pytest

from gpu_cases import TOL_BARRIER, TOL_E_PER_ATOM, TOL_F, TOL_V_PER_ATOM, make_pair, oracle_params_like

pytestmark = pytest.mark.gpu

S_TS = (6.0, -3.5, 2.0, 4.0, -2.5, 5.0)  # GPa, Voigt xx yy zz yz xz xy
S_LJ = (120.0, -40.0, 20.0, 30.0, 0.0, -50.0)  # LJ in eV and A is stiff (~10^4 GPa)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("name,fp64,filt", [("lj31", True, 2), ("lj31", True, 1), ("ts_small", False, 2),
                                            ("ts_small", False, 1)])
def test_applied_stress_generalized_forces(name, fp64, filt):
    import oracle
    kind = "lj" if name.startswith("lj") else "ts"
    kw = dict(n_images=5, max_images=5, cell_filter=filt, pressure_GPa=3.0 if kind == "ts" else 0.0,
              stress_GPa=S_LJ if kind == "lj" else S_TS)
    g, _, w, _ = make_pair(name, fp64=fp64, oracle_too=False, **kw)
    g.step(6)  # cells move off the reference under the stress
    assert g.step(1, 1e30)[0] == 0  # evaluate at the current coordinates without moving
    op = oracle_params_like(kind, **kw)
    st = g.get_state()
    n = g.n
    scale = 1e-6 if fp64 else 1.0
    moved = 0.0
    for k in range(5):
        ref = oracle.cf_eval(op, w["cell_init"], st["X"][k])
        img = g.image(k)
        assert abs(img["H"] - ref["H"]) / n <= TOL_E_PER_ATOM * scale
        assert np.abs(img["Fg"][:n] - ref["Fg"][:n]).max() <= 2 * TOL_F * scale
        np.testing.assert_allclose(img["Fg"][n:], ref["Fg"][n:], rtol=0, atol=TOL_V_PER_ATOM * scale * 10)
        moved = max(moved, np.abs(ref["h"] - w["cell_init"]).max())
    assert moved > 1e-4


def test_applied_stress_converged_barrier_in_both_filters():
    # LJ FCC vacancy hop under a general stress, climbing image: the device's
    # rotation-free and D-variant bands and the oracle's band reach one barrier
    import oracle
    kw = dict(n_images=7, max_images=7, climb_after=50, k_spring=1.0, fire_dt0=0.005, stress_GPa=S_LJ)
    g2, o2, w, kind = make_pair("lj31", fp64=True, cell_filter=2, **kw)
    g1, _, _, _ = make_pair("lj31", fp64=True, oracle_too=False, cell_filter=1, **kw)
    for band in (g2, g1, o2):
        steps, fmax, conv = band.step(6000, 1e-3)
        assert conv
    b2, b1, bo = g2.energies(), g1.energies(), o2.energies()
    assert b2["ci"] == b1["ci"] == bo["ci"] == 3
    assert abs(b2["barrier"] - bo["barrier"]) <= TOL_BARRIER
    assert abs(b1["barrier"] - bo["barrier"]) <= TOL_BARRIER
    # the stress matters: the unstressed barrier of the same hop is about 1 eV higher
    p0 = {k: v for k, v in kw.items() if k != "stress_GPa"}
    g0, _, _, _ = make_pair("lj31", fp64=True, oracle_too=False, cell_filter=2, **p0)
    assert g0.step(6000, 1e-3)[2]
    assert g0.energies()["barrier"] - b2["barrier"] > 0.5
    del oracle


def test_relaxation_under_stress():
    # the device and the oracle relax the same crystal under S; the relaxed crystal's
    # own Cauchy stress -V/Omega is the push-forward J^-1 D^T S D of S
    import oracle
    from paper_2510_16721_amd import cfneb
    from gpu_cases import workload
    w, kind = workload("lj_ragged")
    n = w["n"]
    Sm = np.array([[S_LJ[0], S_LJ[5], S_LJ[4]], [S_LJ[5], S_LJ[1], S_LJ[3]],
                   [S_LJ[4], S_LJ[3], S_LJ[2]]]) / 160.21766208
    for filt in (2, 1):
        gp = cfneb.default_params(cfneb.CFNEB_LJ, force_fp64=1, cell_filter=filt, stress_GPa=S_LJ)
        op = oracle_params_like(kind, cell_filter=filt, stress_GPa=S_LJ)
        pos, cell = w["pos_init"], w["cell_init"]
        R, h, steps, fmax, conv = cfneb.relax(gp, pos, cell, 5000, 1e-5)
        Ro, ho, so, fo = oracle.relax(op, pos, cell, 5000, 1e-5)
        assert conv and fmax < 1e-5 and fo < 1e-5
        np.testing.assert_allclose(h, ho, rtol=0, atol=1e-4)
        np.testing.assert_allclose(R, Ro, rtol=0, atol=1e-3)
        E, u, F, V = oracle.evaluate(oracle_params_like(kind), R, h)
        D = np.linalg.solve(cell, h)
        om, om0 = abs(np.linalg.det(h)), abs(np.linalg.det(cell))
        np.testing.assert_allclose(-V / om, (om0 / om) * D.T @ Sm @ D, rtol=0, atol=1e-3 * np.abs(Sm).max())
        assert D[0, 0] > 1.005  # tension along x
