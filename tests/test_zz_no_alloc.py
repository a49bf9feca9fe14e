"""The allocation-free relaxation entry point (cfneb_relax_noalloc) against the
workspace one (cfneb_relax): same kernels, so the same relaxed structure bit for bit,
on two calls in a row (the second smaller, reusing the static array), for both
potentials; sizes beyond the static array are rejected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    torch.cuda.set_device(0)


def _same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[2:] == b[2:]


@pytest.mark.parametrize("kind", ["lj", "ts"])
def test_noalloc_relax_equals_workspace_relax(kind):
    from paper_2510_16721_amd import cfneb
    if kind == "lj":
        pot, big, small = cfneb.CFNEB_LJ, W.fcc_vacancy_hop(10, 10, 10, 1.5496), W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    else:
        pot, big, small = cfneb.CFNEB_TERSOFF_C, W.diamond_vacancy_hop(6, 6, 6), W.diamond_vacancy_hop(2, 2, 2)
    p = cfneb.default_params(pot, pressure_GPa=2.0)
    for w in (big, small):  # the second call is smaller than the first
        for which in ("init", "final"):
            pos, cell = w["pos_" + which], w["cell_" + which]
            print(f"noalloc relax {kind}: {w['n']} atoms ({which})", flush=True)
            ref = cfneb.relax(p, pos, cell, 400, 1e-4)
            got = cfneb.relax_noalloc(p, pos, cell, 400, 1e-4)
            _same(got, ref)
            assert got[2] > 10
            # the inputs are not modified by the binding; a repeat gives the same result
            _same(cfneb.relax_noalloc(p, pos, cell, 400, 1e-4), ref)


def test_noalloc_relax_rejects_sizes_beyond_the_array():
    from paper_2510_16721_amd import cfneb
    p = cfneb.default_params(cfneb.CFNEB_LJ)
    q = cfneb.default_params(cfneb.CFNEB_LJ, n_images=3, max_images=3, min_images=3)
    w = W.fcc_vacancy_hop(16, 16, 16, 1.5496)  # 16,383 atoms
    assert cfneb.band_bytes(q, w["n"], 3) > cfneb.RELAX_SCRATCH_BYTES
    with pytest.raises(cfneb.CfnebError) as e:
        cfneb.relax_noalloc(p, w["pos_init"], w["cell_init"], 10, 1e-4)
    assert e.value.code == -2  # CFNEB_ENOMEM
    # the array is still usable afterwards
    s = W.fcc_vacancy_hop(2, 2, 2, 1.5496)
    _same(cfneb.relax_noalloc(p, s["pos_init"], s["cell_init"], 50, 1e-4),
          cfneb.relax(p, s["pos_init"], s["cell_init"], 50, 1e-4))
