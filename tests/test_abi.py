"""Host-side checks of the C ABI: load, exports, validation, analytic coefficients.

No device call is made: plan_check and analytic_coeffs touch no GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbessfm.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cbessfm_[a-z_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2409_14489_amd import _lib
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(_lib.lib, n), f"{n} declared in cbessfm.h but not exported"
    assert sorted(_lib.EXPORTED) == names


def test_strerror_codes():
    from paper_2409_14489_amd import _lib
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert _lib.strerror(code) and _lib.strerror(code) != "unknown error"
    assert _lib.strerror(-99) == "unknown error"


from paper_2409_14489_amd import LinkSpec, analytic_coeffs, plan_check  # noqa: E402

LINK = LinkSpec(n_spans=15, sample_rate_hz=640e9)


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(n_sb=0), -1),
    (dict(n_sb=9), -1),
    (dict(block_sb=4000), -2),
    (dict(block_sb=128), -2),
    (dict(block_sb=16384), 0),        # streaming path
    (dict(block_sb=2 ** 17), 0),
    (dict(block_sb=2 ** 18), -2),
    (dict(block_sb=2 ** 17, overlap=5 * 2 ** 17), -1),
    (dict(overlap=3), -1),
    (dict(overlap=-2), -1),
    (dict(overlap=5 * 4096), -1),
    (dict(steps=0), -1),
    (dict(split_ratio=1.5), -1),
    (dict(split_ratio=-0.1), -1),
    (dict(split_ratio=float("nan")), -1),
    (dict(n_taps=20), -1),
    (dict(n_taps=0), -1),
    (dict(n_taps=257), -2),
    (dict(boundary="zero"), 0),
    (dict(grid_m=22), -1),
    (dict(grid_m=19), -1),
    (dict(grid_m=41), 0),
])
def test_plan_check_codes(kw, code):
    args = dict(n_sb=5, block_sb=4096, overlap=2560, steps=15, split_ratio=0.3, n_taps=21)
    args.update(kw)
    assert plan_check(LINK, **args) == code


def test_plan_check_rejects_bad_link():
    bad = LinkSpec(n_spans=0)
    assert plan_check(bad, 1, 1024, 128, 1, 0.5, 11) == -1
    bad = LinkSpec(sample_rate_hz=0.0)
    assert plan_check(bad, 1, 1024, 128, 1, 0.5, 11) == -1
    assert plan_check(LinkSpec(), 1, 1024, 128, 1, 0.5, 2049) == -1   # taps > N'


@pytest.mark.parametrize("n_sb,steps,rho,taps,spans,rate,grid", [
    (1, 1, 0.5, 11, 1, 64e9, 0),
    (2, 3, 0.3, 7, 3, 128e9, 0),
    (5, 2, 0.12, 21, 2, 640e9, 0),
    (1, 15, 0.5, 11, 1, 64e9, 0),      # fractional-span steps
    (3, 4, 0.8, 9, 2, 192e9, 15),      # finer grid
])
def test_host_analytic_coeffs_match_oracle(n_sb, steps, rho, taps, spans, rate, grid):
    from oracle.coeffs import Link, dbp_coefficients
    lk = LinkSpec(n_spans=spans, sample_rate_hz=rate)
    ours = analytic_coeffs(lk, n_sb, steps, rho, taps, grid)
    ref = dbp_coefficients(Link(n_spans=spans, sample_rate=rate), n_sb, steps, rho, taps,
                           grid_m=grid or None)
    assert np.max(np.abs(ours - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_manakov_flag_scales_gamma():
    a = analytic_coeffs(LinkSpec(), 1, 1, 0.5, 5)
    b = analytic_coeffs(LinkSpec(manakov_8_9=True), 1, 1, 0.5, 5)
    assert np.allclose(b, a * 8 / 9, rtol=1e-13)


def test_fir_mode_validation():
    from paper_2409_14489_amd._lib import EINVAL, EUNSUPPORTED, OK
    assert plan_check(LINK, 5, 4096, 2560, 15, 0.3, 21, fir_mode="freq") == OK
    assert plan_check(LINK, 5, 4096, 2560, 15, 0.3, 21, fir_mode="time") == OK
    assert plan_check(LINK, 5, 2 ** 15, 2560, 15, 0.3, 21, fir_mode="freq") == EUNSUPPORTED
    assert plan_check(LINK, 5, 2 ** 15, 2560, 15, 0.3, 21, fir_mode="auto") == OK
    import ctypes
    from paper_2409_14489_amd._lib import Coeffs, Subbands, lib
    sb = Subbands(2, 1024, 0, 3, 0)
    co = Coeffs(11, None, 0)
    assert lib.cbessfm_plan_check(ctypes.byref(LINK.c()), ctypes.byref(sb), 2, 0.5, ctypes.byref(co)) == EINVAL
