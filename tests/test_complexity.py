"""The complexity model of Sec. III-D: the oracle against the figures the
paper prints (tests/golden/complexity_sec4.txt) and against a recount from
the per-component costs the section states; the library against the oracle."""
import math
import os

import numpy as np
import pytest

from oracle import complexity as ocx
from paper_2409_14489_amd import complexity
from paper_2409_14489_amd._lib import CbessfmError

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "complexity_sec4.txt")


def golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                kind, n, big_n, n_ov, st, sb, nc, rm = line.split()
                rows.append((kind, float(n), int(big_n), int(n_ov), int(st), int(sb), int(nc), int(rm)))
    return rows


@pytest.mark.parametrize("row", golden_rows())
def test_oracle_reproduces_the_printed_figures(row):
    kind, n, big_n, n_ov, st, sb, nc, rm = row
    got = ocx.cb_essfm(n, big_n, n_ov, st, sb)[0] if kind == "freq" else ocx.essfm_time(n, big_n, n_ov, st, nc)[0]
    assert round(got) == rm, (row, got)


def recount(n_sps, big_n, n_ov, n_st, n_sb=None, n_c=None):
    """Per-block counts summed from the components Sec. III-D lists: split-radix
    CFFT (N log2 N - 3N + 4 RM, 3 N log2 N - 3N + 4 RA), dispersion step 6N RM
    and 6N RA, intensity 4N RM 3N RA, output rotation 6N RM 8N RA, and for the
    frequency-domain filter the half-spectrum matrix-vector products (per bin
    N_sb (N_sb - 1) CMs with a fixed multiplier at 3 RM / 3 RA, N_sb real-by-
    complex products at 2 RM, N_sb (N_sb - 1) complex additions), between an
    RFFT and an inverse RFFT per subband (half a CFFT each)."""
    def cfft(m):
        return m * math.log2(m) - 3 * m + 4, 3 * m * math.log2(m) - 3 * m + 4
    rm = ra = 0.0
    if n_sb is not None:                          # CB-ESSFM, Fig. "scheme_OeS" / "scheme_NLPR"
        np_ = big_n // n_sb
        f_rm, f_ra = cfft(big_n)
        s_rm, s_ra = cfft(np_)
        rm += 4 * f_rm + 4 * n_sb * n_st * s_rm + 6 * big_n * (n_st + 1)
        ra += 4 * f_ra + 4 * n_sb * n_st * s_ra + 6 * big_n * (n_st + 1)
        bins = np_ / 2
        mimo_rm = 2 * n_sb * (s_rm / 2) + bins * (3 * n_sb * (n_sb - 1) + 2 * n_sb)
        mimo_ra = 2 * n_sb * (s_ra / 2) + bins * (3 * n_sb * (n_sb - 1) + 2 * n_sb * (n_sb - 1))
        rm += n_st * (4 * big_n + mimo_rm + 6 * big_n)
        ra += n_st * (3 * big_n + mimo_ra + 8 * big_n)
    else:                                         # time-domain NLPR, symmetric real FIR
        f_rm, f_ra = cfft(big_n)
        rm += (n_st + 1) * (4 * f_rm + 6 * big_n) + n_st * big_n * (4 + (n_c + 1) + 6)
        ra += (n_st + 1) * (4 * f_ra + 6 * big_n) + n_st * big_n * (3 + 2 * n_c + 8)
    per = n_sps / 2 / (big_n - n_ov)
    return rm * per, ra * per


@pytest.mark.parametrize("n_st", [1, 4, 15, 60])
@pytest.mark.parametrize("n_sb", [1, 2, 4, 8])
def test_closed_forms_equal_the_component_recount(n_st, n_sb):
    for big_n, n_ov in [(16384, 1800), (8192, 2688), (65536, 0)]:
        want = recount(2.0, big_n, n_ov, n_st, n_sb=n_sb)
        got = ocx.cb_essfm(2.0, big_n, n_ov, n_st, n_sb)
        # the RFFT is "approximately half" a CFFT: the closed form drops the +4 / 2 terms
        assert np.allclose(got, want, rtol=2e-4), (got, want)
        for n_c in (0, 10, 44):
            assert np.allclose(ocx.essfm_time(2.0, big_n, n_ov, n_st, n_c),
                               recount(2.0, big_n, n_ov, n_st, n_c=n_c), rtol=1e-12)


@pytest.mark.parametrize("n_sps,big_n,n_ov", [(1.125, 16384, 1800), (2.0, 8192, 2688), (1.0, 512, 0)])
def test_library_matches_the_oracle(n_sps, big_n, n_ov):
    for st in (0, 1, 7, 15, 300):
        for sb in (1, 2, 4, 8):
            got = complexity("cb-essfm", n_sps, big_n, n_ov, st, n_sb=sb)
            want = ocx.cb_essfm(n_sps, big_n, n_ov, st, sb)
            assert np.allclose((got["rm"], got["ra"]), want, rtol=1e-12)
        for nc in (0, 3, 44):
            got = complexity("time", n_sps, big_n, n_ov, st, n_c=nc)
            assert np.allclose((got["rm"], got["ra"]), ocx.essfm_time(n_sps, big_n, n_ov, st, nc), rtol=1e-12)


def test_bad_arguments():
    for args in [(2.0, 1024, 1024, 1), (2.0, 1024, -2, 1), (0.0, 1024, 0, 1), (2.0, 1024, 0, -1)]:
        with pytest.raises(CbessfmError):
            complexity("time", *args)
    with pytest.raises(CbessfmError):
        complexity("cb-essfm", 2.0, 1000, 0, 1, n_sb=3)      # N_sb must divide N
