"""Pins of the analytic-coefficient oracle (Sec. II-D, App. C, Sec. III-B)."""
import numpy as np
import pytest
from scipy import integrate

from oracle.coeffs import (Link, dbp_coefficients, effective_length, kernel, kernel_eq22,
                           physical_coefficients)


def quad_kernel(b, z_lo, z_hi, z0, link):
    """int gamma g(z) exp(-j 2 b (z - z0)) dz by adaptive quadrature (App. C eq. kernel_b)."""
    span = link.span_km
    breaks = [z for z in np.arange(np.ceil(z_lo / span) * span, z_hi, span) if z_lo < z < z_hi]

    def g(z):
        return np.exp(-link.alpha * (z - np.floor(z / span + 1e-12) * span))

    re = integrate.quad(lambda z: g(z) * np.cos(2 * b * (z - z0)), z_lo, z_hi, points=breaks or None,
                        limit=500, epsabs=1e-13, epsrel=1e-12)[0]
    im = integrate.quad(lambda z: -g(z) * np.sin(2 * b * (z - z0)), z_lo, z_hi, points=breaks or None,
                        limit=500, epsabs=1e-13, epsrel=1e-12)[0]
    return link.gamma * (re + 1j * im)


@pytest.mark.parametrize("n_sp", [1, 2, 3, 5])
def test_kernel_equals_eq22_for_symmetric_whole_spans(n_sp):
    link = Link(n_spans=n_sp)
    b = np.linspace(-0.3, 0.3, 41)          # rad/km, spans many sin(bL) zeros
    b = b[np.abs(np.sin(b * 80.0)) > 1e-6]
    L = 80.0 * n_sp
    k = kernel(b, 0.0, L, L / 2.0, link)
    ref = kernel_eq22(b, L, n_sp, link)
    assert np.max(np.abs(k - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("z_lo,z_hi,z0", [
    (0.0, 80.0, 8.0),          # one span, NLPR near the amplifier
    (80.0, 240.0, 100.0),      # two spans
    (53.3, 106.7, 60.0),       # fractional step across an amplifier
    (10.0, 15.3, 14.0),        # short fractional step
])
def test_kernel_equals_quadrature(z_lo, z_hi, z0):
    link = Link(n_spans=3)
    for b in (-0.2, -0.013, 0.0, 0.004, 0.09):
        assert abs(kernel(np.array([b]), z_lo, z_hi, z0, link)[0]
                   - quad_kernel(b, z_lo, z_hi, z0, link)) < 1e-9


def test_coefficients_sum_to_gamma_leff():
    """sum_m c[m] = (1/M) sum_p K(mu_p, mu_p) = gamma L_eff, since b = 0 on the diagonal."""
    link = Link(n_spans=2, sample_rate=160e9)
    c = physical_coefficients(link, 3, 80.0, 160.0, 92.0, 15)
    leff = effective_length(link, 80.0, 160.0)
    assert np.allclose(c.sum(-1), link.gamma * leff, rtol=1e-12)
    assert abs(leff - (1 - np.exp(-link.alpha * 80)) / link.alpha) < 1e-9


def test_zero_dispersion_gives_delta():
    link = Link(beta2_ps2_km=0.0, sample_rate=64e9)
    c = physical_coefficients(link, 2, 0.0, 80.0, 40.0, 9)
    leff = effective_length(link, 0.0, 80.0)
    expect = np.zeros(9)
    expect[4] = link.gamma * leff
    for i in range(2):
        for l in range(2):
            assert np.allclose(c[i, l], expect, atol=1e-13)


def test_symmetries_eq23_to_eq25():
    link = Link(n_spans=1, sample_rate=320e9)
    c = physical_coefficients(link, 5, 0.0, 80.0, 17.0, 21)
    for i in range(5):
        assert np.allclose(c[i, i], c[i, i][::-1], atol=1e-15 * np.abs(c).max())     # (25)
        for l in range(5):
            assert np.allclose(c[i, l], c[l, i][::-1], rtol=1e-10, atol=1e-14)       # (24)
            for k in range(-i, 5 - max(i, l)):
                if 0 <= l + k < 5 and 0 <= i + k < 5:
                    assert np.allclose(c[i, l], c[i + k, l + k], rtol=1e-10)         # (23)


def test_linear_in_gamma():
    a = physical_coefficients(Link(gamma_w_km=1.3), 2, 0.0, 80.0, 40.0, 11)
    b = physical_coefficients(Link(gamma_w_km=2.6), 2, 0.0, 80.0, 40.0, 11)
    assert np.allclose(b, 2 * a, rtol=1e-13)


def test_fractional_steps_scale_with_input_power():
    """A span cut in three equal steps: same kernel, power exp(-alpha L) and
    exp(-2 alpha L) below the first (Sec. II-D)."""
    link = Link(n_spans=1, sample_rate=64e9)
    L = 80.0 / 3
    cs = [physical_coefficients(link, 1, k * L, (k + 1) * L, k * L + 0.4 * L, 11) for k in range(3)]
    assert np.allclose(cs[1], cs[0] * np.exp(-link.alpha * L), rtol=1e-12)
    assert np.allclose(cs[2], cs[0] * np.exp(-2 * link.alpha * L), rtol=1e-12)


def test_dbp_tensor_sign_xpm_factor_and_step_order():
    link = Link(n_spans=3, sample_rate=128e9)
    C = dbp_coefficients(link, 2, 3, 0.3, 7)
    for s in range(3):
        j = 3 - s                                  # physical step undone by DBP step s
        c = physical_coefficients(link, 2, (j - 1) * 80.0, j * 80.0, (j - 1) * 80.0 + 24.0, 7)
        assert np.allclose(C[s, 0, 0], -c[0, 0])
        assert np.allclose(C[s, 0, 1], -1.5 * c[0, 1])
        assert np.allclose(C[s, 1, 0], -1.5 * c[1, 0])
    # whole-span steps of a periodically amplified link share one kernel
    assert np.allclose(C[0], C[2])


def test_tap_extent_matches_fig6_description():
    """N_st = 5 (three spans per step), two bands at n = 1.125 x 93 GBd:
    the intraband response is symmetric and roughly 50 samples long, the
    interband one longer because of walk-off (Sec. IV-B)."""
    link = Link(beta2_ps2_km=-21.68, gamma_w_km=1.27, n_spans=15, sample_rate=1.125 * 93e9)
    c = physical_coefficients(link, 2, 0.0, 240.0, 120.0, 201, grid_m=201)

    def support(v):
        nz = np.nonzero(np.abs(v) > 0.02 * np.abs(v).max())[0] - 100
        return nz.min(), nz.max()
    lo11, hi11 = support(c[0, 0])
    lo12, hi12 = support(c[0, 1])
    assert 35 <= hi11 - lo11 + 1 <= 60 and lo11 == -hi11       # ~50 samples, symmetric
    assert 100 <= hi12 - lo12 + 1 <= 140 and lo12 != -hi12     # ~120 samples, asymmetric
    assert np.allclose(c[0, 0], c[0, 0][::-1])
