"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/cfneb.h declares; host-only calls work."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cfneb.h")).read()
    return sorted(set(re.findall(r"\b(cfneb_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2510_16721_amd import cfneb
    if not os.path.exists(cfneb.LIB_PATH):
        from paper_2510_16721_amd import build
        build.build()
    return cfneb.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "cfneb_create_band" in names and "cfneb_step" in names
    for name in names:
        assert hasattr(L, name), name


def test_binding_covers_the_header():
    from paper_2510_16721_amd import cfneb
    assert sorted(cfneb.SYMBOLS) == _declared()


def test_params_default_and_struct_layout(L):
    from paper_2510_16721_amd import cfneb
    p = cfneb.default_params(cfneb.CFNEB_TERSOFF_C)
    # the last field lands where the C struct has it only if the layouts agree
    assert p.nbr_cap == 16 and p.del_den == 4 and p.ts_S == 2.1 and p.ts_c == 38049.0
    p = cfneb.default_params(cfneb.CFNEB_LJ)
    assert p.nbr_cap == 128 and p.fire_dt0 == 0.005 and p.fire_dtmax == pytest.approx(0.05)


def test_band_bytes_and_argument_checks(L):
    from paper_2510_16721_amd import cfneb
    p = cfneb.default_params(cfneb.CFNEB_LJ, n_images=7, max_images=7)
    small = cfneb.band_bytes(p, 255)
    big = cfneb.band_bytes(p, 255, 40)
    assert 0 < small < big
    with pytest.raises(cfneb.CfnebError):
        cfneb.band_bytes(p, 0)
    bad = cfneb.default_params(cfneb.CFNEB_LJ, n_images=2)
    with pytest.raises(cfneb.CfnebError):
        cfneb.band_bytes(bad, 10)
    bad = cfneb.default_params(cfneb.CFNEB_LJ, max_images=65, n_images=7)
    with pytest.raises(cfneb.CfnebError):
        cfneb.band_bytes(bad, 10)
    assert L.cfneb_strerror(-5) == b"neighbour list capacity exceeded"


def test_size_limits_are_rejected_on_the_host(L):
    # atom indices are 20-bit: 2^20 - 1 atoms is the largest band, 2^20 is refused;
    # an empty structure and an unknown filter are refused
    from paper_2510_16721_amd import cfneb
    p = cfneb.default_params(cfneb.CFNEB_TERSOFF_C, n_images=3, max_images=3)
    assert cfneb.band_bytes(p, 2**20 - 1) > 0
    for n in (0, -1, 2**20):
        with pytest.raises(cfneb.CfnebError) as e:
            cfneb.band_bytes(p, n)
        assert e.value.code == -1
    for filt in (-1, 3):
        q = cfneb.default_params(cfneb.CFNEB_LJ, cell_filter=filt)
        with pytest.raises(cfneb.CfnebError):
            cfneb.band_bytes(q, 10)
    q = cfneb.default_params(cfneb.CFNEB_LJ, nbr_skin=-0.1)
    with pytest.raises(cfneb.CfnebError):
        cfneb.band_bytes(q, 10)


def test_missing_library_fails_loudly(monkeypatch):
    # no CPU fallback: without the built HIP library every call raises
    from paper_2510_16721_amd import cfneb
    monkeypatch.setattr(cfneb, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libcfneb.so"))
    monkeypatch.setattr(cfneb, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        cfneb.lib()
    with pytest.raises(RuntimeError, match="not built"):
        cfneb.default_params(cfneb.CFNEB_LJ)


def test_product_never_reaches_the_oracle():
    # the package and the HIP sources name no oracle module, header or library
    pkg = os.path.join(ROOT, "paper_2510_16721_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\bimport\s+oracle\b|\bfrom\s+oracle\b|oracle\.h|liborc", text), f


def test_applied_stress_is_validated_on_the_host(L):
    # the six stress components sit at the end of cfneb_params: a non-finite one is
    # refused, finite ones are accepted (and the default is no stress)
    from paper_2510_16721_amd import cfneb
    p = cfneb.default_params(cfneb.CFNEB_TERSOFF_C)
    assert list(p.stress_GPa) == [0.0] * 6
    ok = cfneb.default_params(cfneb.CFNEB_TERSOFF_C, stress_GPa=(1.0, -2.0, 0.5, 0.0, 3.0, -1.0))
    assert cfneb.band_bytes(ok, 100) > 0
    for q in range(6):
        s = [0.0] * 6
        s[q] = float("inf") if q % 2 else float("nan")
        bad = cfneb.default_params(cfneb.CFNEB_TERSOFF_C, stress_GPa=tuple(s))
        with pytest.raises(cfneb.CfnebError):
            cfneb.band_bytes(bad, 100)


def test_lane_table_rows_and_header():
    # the tuner's table: thresholds at the geometric mean of neighbouring sizes whose
    # fastest lane counts differ, runs of equal counts merged, the last row open-ended
    from paper_2510_16721_amd import tune_lanes as T
    res = [(100, {1: 3.0, 2: 2.0, 4: 1.0, 8: 1.5}), (400, {1: 3.0, 2: 2.0, 4: 1.0, 8: 1.5}),
           (1600, {1: 2.0, 2: 1.0, 4: 1.5, 8: 3.0}), (6400, {1: 1.0, 2: 2.0, 4: 3.0, 8: 4.0})]
    assert T.table_rows(res) == [(800, 4), (3200, 2), (None, 1)]
    assert T.table_rows(res[3:]) == [(None, 1)]
    # within 3 % of the fastest, the fewest lanes
    assert T.pick({1: 1.02, 2: 1.0, 4: 1.1, 8: 1.2}) == 1
    assert T.pick({1: 1.04, 2: 1.0, 4: 1.01, 8: 1.2}) == 2
    # the committed table is well formed: increasing thresholds, lane counts 1/2/4/8,
    # and an open-ended last row
    src = open(T.TABLE).read()
    rows = [(int(a), int(b)) for a, b in re.findall(r"\{(\d+)LL, (\d)\}", src)]
    assert rows and rows[-1][0] == 9223372036854775807
    assert all(r[1] in (1, 2, 4, 8) for r in rows)
    assert [r[0] for r in rows] == sorted(r[0] for r in rows)
