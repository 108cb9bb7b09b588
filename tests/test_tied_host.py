"""Host-side tied-coefficient helpers of the library (step weights, the tap
rule, the SSFM start, analytic rows) against the FP64 oracle (no device)."""
import numpy as np
import pytest

import oracle
from oracle.tied import expand
from paper_2409_14489_amd import LinkSpec, analytic_coeffs, analytic_rows, ssfm_start, step_weights, tied_half_taps
from paper_2409_14489_amd._lib import CbessfmError

LINKS = [
    dict(alpha_db_km=0.2, beta2_ps2_km=-21.7, gamma_w_km=1.3, span_km=80.0, n_spans=1, sample_rate_hz=64e9),
    dict(alpha_db_km=0.25, beta2_ps2_km=-21.68, gamma_w_km=1.27, span_km=75.0, n_spans=3, sample_rate_hz=640e9),
    dict(alpha_db_km=0.0, beta2_ps2_km=-5.0, gamma_w_km=2.0, span_km=50.0, n_spans=4, sample_rate_hz=200e9),
]


def o_link(d):
    return oracle.Link(alpha_db_km=d["alpha_db_km"], beta2_ps2_km=d["beta2_ps2_km"], gamma_w_km=d["gamma_w_km"],
                       span_km=d["span_km"], n_spans=d["n_spans"], sample_rate=d["sample_rate_hz"])


@pytest.mark.parametrize("d", LINKS)
@pytest.mark.parametrize("steps", [1, 2, 5, 7, 12])
def test_step_weights_and_tap_rule_match_the_oracle(d, steps):
    w, leff = step_weights(LinkSpec(**d), steps)
    ow = oracle.step_weights(o_link(d), steps)
    assert np.allclose(w, ow, rtol=1e-12, atol=0)
    for n_sb in (1, 3, 5):
        for taps in (1, 21, 255):
            got = tied_half_taps(LinkSpec(**d), n_sb, steps, taps)
            assert np.array_equal(got, oracle.tied_half_taps(o_link(d), n_sb, steps, taps))
    start = ssfm_start(LinkSpec(**d), 3, steps, 9)
    assert np.allclose(start, oracle.ssfm_start(o_link(d), 3, steps, 9), rtol=1e-12, atol=0)


def test_analytic_rows_expand_to_the_analytic_tensor():
    link = LinkSpec(n_spans=2, span_km=60.0, sample_rate_hz=192e9)
    rows = analytic_rows(link, 3, 6, 0.3, 11)
    c = analytic_coeffs(link, 3, 6, 0.3, 11)
    w, _ = step_weights(link, 6)
    assert np.allclose(expand(rows, w), c, rtol=0, atol=1e-10 * np.abs(c).max())


def test_bad_arguments():
    link = LinkSpec()
    with pytest.raises(CbessfmError):
        step_weights(link, 0)
    with pytest.raises(CbessfmError):
        tied_half_taps(link, 9, 1, 11)
    with pytest.raises(CbessfmError):
        tied_half_taps(link, 2, 1, 10)
    with pytest.raises(CbessfmError):
        step_weights(LinkSpec(n_spans=0), 3)
