"""Batched execution: many bands of different sizes and potentials stepped by one
persistent launch per phase.  Each band's result must not depend on its
batch-mates: bit-identical to the same band stepped alone."""
import numpy as np
import pytest

from gpu_cases import make_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)


CASES = [("lj31", dict(n_images=5, max_images=5, fp64=True, climb_after=10)),
         ("ts_small", dict(n_images=6, max_images=8, refine_every=5, climb_after=8)),
         ("lj_ragged", dict(n_images=7, max_images=7, climb_after=10)),
         ("ts_diamond", dict(n_images=5, max_images=5, pressure_GPa=5.0))]


def _bands():
    return [make_pair(name, oracle_too=False, **kw)[0] for name, kw in CASES]


def _same_state(a, b):
    sa, sb = a.get_state(), b.get_state()
    assert sa["X"].shape == sb["X"].shape
    np.testing.assert_array_equal(sa["X"], sb["X"])
    np.testing.assert_array_equal(sa["v"], sb["v"])
    for key in ("dt", "alpha", "n_pos", "fresh", "step", "ci", "image_steps"):
        assert sa[key] == sb[key], key
    np.testing.assert_array_equal(a.energies()["H"], b.energies()["H"])


def test_batch_equals_alone_bit_for_bit():
    from paper_2510_16721_amd import cfneb
    alone = _bands()
    for b in alone:
        assert b.step(23)[0] == 23
    mixed = _bands()
    batch = cfneb.Batch(8)
    slots = [batch.attach(b) for b in mixed]
    steps, conv, errs = batch.step(23)
    assert list(steps[slots]) == [23] * len(mixed) and not conv.any() and not errs.any()
    for a, b in zip(alone, mixed):
        _same_state(a, b)
    batch.close()


def test_batch_attach_detach_between_calls():
    from paper_2510_16721_amd import cfneb
    ref = _bands()
    for b in ref:
        b.step(20)
    bands = _bands()
    batch = cfneb.Batch(4)
    s0 = batch.attach(bands[0])
    s1 = batch.attach(bands[1])
    batch.step(10)
    batch.detach(s0)
    s2 = batch.attach(bands[2])
    batch.step(10)
    batch.detach(s1)
    batch.detach(s2)
    bands[0].step(10)  # the detached band goes on alone
    s3 = batch.attach(bands[3])
    batch.step(20)
    bands[2].step(10)
    for r, b in zip(ref, bands):
        _same_state(r, b)
    del s3
    batch.close()


def test_batch_bands_converge_independently():
    from paper_2510_16721_amd import cfneb
    kw = dict(n_images=5, max_images=5, climb_after=20, fp64=True)
    fast = make_pair("lj31", oracle_too=False, **kw)[0]
    slow = make_pair("lj_ragged", oracle_too=False, **kw)[0]
    batch = cfneb.Batch(2)
    sf, ss = batch.attach(fast), batch.attach(slow)
    steps, conv, errs = batch.step(4000, 5e-3)
    assert conv[sf] and not errs.any()
    # the same band alone takes the same number of steps to the same barrier
    ref = make_pair("lj31", oracle_too=False, **kw)[0]
    nref, fref, cref = ref.step(4000, 5e-3)
    assert cref and nref == steps[sf]
    assert ref.energies()["barrier"] == fast.energies()["barrier"]
    batch.close()


def test_batch_capacity_and_errors():
    from paper_2510_16721_amd import cfneb
    bands = _bands()
    batch = cfneb.Batch(2)
    batch.attach(bands[0])
    batch.attach(bands[1])
    with pytest.raises(cfneb.CfnebError) as e:
        batch.attach(bands[2])
    assert e.value.code == -7  # CFNEB_ECAPACITY
    with pytest.raises(cfneb.CfnebError):
        batch.attach(bands[0])  # already attached
    batch.close()


def test_batch_workload_subset_matches_oracle():
    # Two LJ vacancy bands of the 64-band batch workload (seed 3), run exactly as the
    # batched benchmark runs them (FP32 forces, climbing image from step 50, endpoints
    # relaxed with the cell filter), converged in one batch; the oracle relaxes its own
    # endpoints and converges the same bands.  Barriers within 1 meV; the climbing image
    # is the same or its mirror.
    import oracle
    import workloads as W
    from paper_2510_16721_amd import cfneb
    from gpu_cases import TOL_BARRIER
    mix = W.band_mix(3, 64, 256, 32000, 5, 17)
    picks = [q for q in range(0, 64, 2) if mix[q]["n"] <= 500][:2]
    assert len(picks) == 2
    bands, refs = [], []
    for q in picks:
        e = mix[q]
        m, w = e["n_images"], e["endpoints"]
        kw = dict(n_images=m, max_images=m, min_images=3, climb_after=50)
        gp = cfneb.default_params(cfneb.CFNEB_LJ, **kw)
        op = oracle.default_params(oracle.LJ, **kw)
        ge = [cfneb.relax(gp, w["pos_" + s], w["cell_" + s], 20000, 1e-4)[:2] for s in ("init", "final")]
        oe = [oracle.relax(op, w["pos_" + s], w["cell_" + s], 20000, 1e-4)[:2] for s in ("init", "final")]
        bands.append(cfneb.Band(gp, ge[0][0], ge[0][1], ge[1][0], ge[1][1]))
        o = oracle.Band(op, oe[0][0], oe[0][1], oe[1][0], oe[1][1])
        assert o.step(4000, 0.01)[2]
        refs.append(o.energies())
    batch = cfneb.Batch(4)
    slots = [batch.attach(b) for b in bands]
    steps, conv, errs = batch.step(4000, 0.01)
    assert all(conv[s] for s in slots) and not errs.any()
    for b, r in zip(bands, refs):
        g = b.energies()
        # an even image count leaves two mirror images next to the saddle; either may
        # become the climbing image and both climb to the same saddle
        M = len(g["H"])
        assert g["ci"] in (r["ci"], M - 1 - r["ci"])
        assert abs(g["barrier"] - r["barrier"]) <= TOL_BARRIER, (g["barrier"], r["barrier"])
    batch.close()


# Refinement kernels launch only on the steps that can end with a refinement (the
# host predicts them from each band's step count); one call of many steps must equal
# single-step calls, where every call reads the step count afresh.  ins_num = 0 makes
# every due refinement insert an image until max_images.
REFINE_KW = [dict(n_images=5, max_images=9, refine_every=3, ins_num=0, climb_after=8),
             dict(n_images=5, max_images=8, refine_every=4, ins_num=0, climb_after=8)]


def test_refinement_schedule_one_call_equals_single_steps():
    a = make_pair("ts_small", oracle_too=False, **REFINE_KW[0])[0]
    b = make_pair("ts_small", oracle_too=False, **REFINE_KW[0])[0]
    assert a.step(31)[0] == 31
    for _ in range(31):
        assert b.step(1)[0] == 1
    assert a.get_state()["X"].shape[0] == 9  # four insertions at steps 3, 6, 9, 12
    _same_state(a, b)


def test_batch_refinement_schedule_one_call_equals_single_steps():
    from paper_2510_16721_amd import cfneb
    runs = []
    for single in (False, True):
        bands = [make_pair("ts_small", oracle_too=False, **kw)[0] for kw in REFINE_KW]
        batch = cfneb.Batch(4)
        slots = [batch.attach(b) for b in bands]
        if single:
            for _ in range(25):
                steps, conv, errs = batch.step(1)
                assert list(steps[slots]) == [1, 1] and not errs.any()
        else:
            steps, conv, errs = batch.step(25)
            assert list(steps[slots]) == [25, 25] and not errs.any()
        runs.append((bands, batch))
    for x, y in zip(runs[0][0], runs[1][0]):
        assert x.get_state()["X"].shape[0] == y.get_state()["X"].shape[0]
        _same_state(x, y)
    assert [b.get_state()["X"].shape[0] for b in runs[0][0]] == [9, 8]
    for _, batch in runs:
        batch.close()


def test_force_grid_shapes_give_identical_batches(monkeypatch):
    # the tuner chooses between the persistent grid (2,048 blocks) and one block per
    # atom tile (16,384 for a batch) for the force kernels: both give the same bands
    # bit for bit
    from paper_2510_16721_amd import cfneb
    runs = []
    for shape in ("persistent", "tile"):
        monkeypatch.setenv("CFNEB_FORCE_GRID", shape)
        bands = _bands()
        batch = cfneb.Batch(8)
        for b in bands:
            batch.attach(b)
        batch.step(23)
        batch.close()
        runs.append(bands)
    for a, b in zip(*runs):
        _same_state(a, b)


def test_graph_and_direct_launches_give_identical_bands(monkeypatch):
    # CFNEB_NO_GRAPH=1 launches the step kernel by kernel: the same band bit for bit,
    # refinements included
    runs = []
    for no_graph in ("1", "0"):
        monkeypatch.setenv("CFNEB_NO_GRAPH", no_graph)
        g, _, _, _ = make_pair("ts_small", oracle_too=False, n_images=6, max_images=8, refine_every=5,
                               climb_after=8)
        assert g.step(23)[0] == 23
        runs.append(g)
    _same_state(runs[0], runs[1])
