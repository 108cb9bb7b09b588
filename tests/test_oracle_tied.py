"""Pins of the tied-coefficient oracle (Sec. III-B assumptions (i)-(iii),
eqs. (23)-(25)) against the physics of the analytic coefficients and the
paper's own statements, not against itself."""
import math

import numpy as np
import pytest

from oracle.coeffs import Link, dbp_coefficients, effective_length
from oracle.tied import expand, expand_adjoint, ssfm_start, step_weights, tied_half_taps


def paper_link(n_spans=15):
    """15 x 80 km, D = 17 ps/nm/km at 1550 nm, gamma 1.27, 93 GBd x 1.125 (Sec. IV-A)."""
    b2 = -17.0e-6 * (1550e-9) ** 2 / (2 * math.pi * 299792458.0) * 1e27
    return Link(alpha_db_km=0.2, beta2_ps2_km=b2, gamma_w_km=1.27, span_km=80.0, n_spans=n_spans,
                sample_rate=93e9 * 1.125)


@pytest.mark.parametrize("n_sb,n_taps", [(1, 5), (3, 7), (5, 9)])
def test_expansion_has_the_symmetries_of_eqs_23_to_25(n_sb, n_taps):
    rng = np.random.default_rng(n_sb)
    w = rng.uniform(0.5, 2.0, 4)
    c = expand(rng.standard_normal((n_sb, n_taps)), w)
    for s in range(4):
        assert np.allclose(c[s], c[0] * w[s] / w[0], rtol=1e-14, atol=0)
        for i in range(n_sb):
            assert np.array_equal(c[s, i, i], c[s, i, i, ::-1])                # (25)
            for l in range(n_sb):
                assert np.array_equal(c[s, i, l], c[s, l, i, ::-1])            # (24)
                for k in range(-min(i, l), n_sb - max(i, l)):
                    assert np.array_equal(c[s, i, l], c[s, i + k, l + k])       # (23)


def test_every_parameter_but_the_mirrored_half_of_c0_is_used():
    n_sb, n_taps = 3, 7
    for h in range(n_sb):
        for t in range(n_taps):
            p = np.zeros((n_sb, n_taps))
            p[h, t] = 1.0
            used = np.abs(expand(p, np.ones(2))).sum() > 0
            assert used == (h > 0 or t >= n_taps // 2)


@pytest.mark.parametrize("steps_per_span,n_spans", [(3, 2), (2, 3), (1, 4)])
def test_analytic_coefficients_of_equal_fractional_steps_are_tied(steps_per_span, n_spans):
    """Assumption (i) holds exactly for steps that cover equal parts of a span:
    the kernel of eq. (6) over [z, z + L] is g(z) times the one over [0, L].
    So the analytic tensor is w_s times one tied tensor, and its rows
    C[0][0][h] reproduce it through the expansion."""
    link = Link(alpha_db_km=0.2, beta2_ps2_km=-21.7, gamma_w_km=1.3, span_km=60.0, n_spans=n_spans,
                sample_rate=96e9)
    n_sb, n_taps = 3, 9
    n_steps = steps_per_span * n_spans
    c = dbp_coefficients(link, n_sb, n_steps, 0.3, n_taps)
    w = step_weights(link, n_steps)
    params = c[0, 0] / w[0]                       # row h of subband 0 is c_h
    assert np.allclose(expand(params, w), c, rtol=0, atol=1e-10 * np.abs(c).max())
    if steps_per_span == 1:
        assert np.allclose(w, 1.0, rtol=1e-14)


def test_step_weights_follow_the_power_at_the_step_input():
    """k equal steps per span: backpropagation step s undoes physical step
    N_st - 1 - s, whose input power is exp(-alpha (j mod k) L / k)."""
    link = Link(alpha_db_km=0.25, span_km=75.0, n_spans=2)
    k = 5
    w = step_weights(link, 2 * k)
    j = 2 * k - 1 - np.arange(2 * k)
    g = np.exp(-link.alpha * (j % k) * link.span_km / k)
    assert np.allclose(w, g / g.mean(), rtol=1e-12)
    # steps of three spans: all equal
    assert np.allclose(step_weights(Link(n_spans=15), 5), 1.0, rtol=1e-14)


def test_adjoint_identity():
    rng = np.random.default_rng(3)
    for n_sb, n_taps, half in [(1, 5, None), (4, 11, [5, 3, 2, 0]), (2, 1, None)]:
        w = rng.uniform(0.2, 1.5, 3)
        p = rng.standard_normal((n_sb, n_taps))
        g = rng.standard_normal((3, n_sb, n_sb, n_taps))
        lhs = np.sum(expand(p, w, half) * g)
        rhs = np.sum(p * expand_adjoint(g, w, half))
        assert abs(lhs - rhs) <= 1e-12 * np.abs(g).sum() * np.abs(p).max() * w.max()


def test_half_taps_zero_the_outer_taps_per_distance():
    p = np.ones((3, 9))
    c = expand(p, np.ones(1), [4, 2, 0])
    m = np.arange(9) - 4
    assert np.array_equal(c[0, 0, 0] != 0, np.abs(m) <= 4)
    assert np.array_equal(c[0, 0, 1] != 0, np.abs(m) <= 2)
    assert np.array_equal(c[0, 2, 0] != 0, m == 0)


def test_tap_rule_iii_matches_the_paper_example_and_the_analytic_support():
    """Sec. IV-B, on the 15 x 80 km link with 5 steps of three spans and two
    subbands: the intraband response c_11 is limited to about 50 samples and
    the interband c_12 extends to about 120.  Rule (iii) gives 2 Nc(h) + 1 of
    about pi L beta2 R'^2 (h + 1); the analytic c_11 is nonzero (above 1 % of
    its peak) over exactly that many samples."""
    link = paper_link()
    half = tied_half_taps(link, 2, 5, 401)
    assert 40 <= 2 * half[0] + 1 <= 55
    assert abs((2 * half[1] + 1) / (2 * half[0] + 1) - 2.0) < 0.05
    c = dbp_coefficients(link, 2, 5, 0.5, 161)
    m = np.arange(161) - 80
    sup11 = m[np.abs(c[0, 0, 0]) > 0.01 * np.abs(c[0, 0, 0]).max()]
    sup12 = m[np.abs(c[0, 0, 1]) > 0.01 * np.abs(c[0, 0, 1]).max()]
    assert sup11.max() - sup11.min() + 1 == 2 * half[0] + 1
    assert 100 <= sup12.max() - sup12.min() + 1 <= 140
    assert sup12.max() != -sup12.min()            # asymmetric (walk-off)


def test_ssfm_start_is_the_one_tap_analytic_ssfm():
    """The fit starts from the SSFM (Sec. III-B): one tap per step equal to the
    nonlinear phase per unit power, which is what the analytic coefficients
    give with one tap and a one-point grid (K at b = 0 is gamma L_eff)."""
    link = Link(alpha_db_km=0.2, gamma_w_km=1.3, span_km=80.0, n_spans=2)
    n_steps = 6
    p = ssfm_start(link, 1, n_steps, 1)
    c = dbp_coefficients(link, 1, n_steps, 0.5, 1, grid_m=1)
    assert np.allclose(expand(p, step_weights(link, n_steps)), c, rtol=1e-12, atol=0)
    step = link.length_km / n_steps
    leff = np.mean([effective_length(link, j * step, (j + 1) * step) for j in range(n_steps)])
    # three steps per span: the mean effective length is a third of a span's
    assert abs(p[0, 0] + 1.3 * (1 - math.exp(-link.alpha * 80.0)) / link.alpha / 3) < 1e-12 * abs(p[0, 0])
    assert abs(p[0, 0] + 1.3 * leff) < 1e-12 * abs(p[0, 0])
    wide = ssfm_start(link, 3, n_steps, 7)
    assert np.count_nonzero(wide) == 1 and wide[0, 3] == p[0, 0]
