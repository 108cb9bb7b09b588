"""Pins of the oracle with free dispersion segments (step sizes and split per
step, Sec. III-C / V) and of its gradient with respect to the segment lengths."""
import copy

import numpy as np

import oracle
from oracle.grad import vjp, vjp_lengths
from synth import random_field


def base(n_sb=2, steps=3, taps=5, coeff_scale=30.0, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps)) * coeff_scale
    return oracle.OraclePlan(-21.7e-24, n_sb * 64e9, 25.0, steps, 0.3, n_sb, n_sb * 256, 64, c)


def test_dispersion_only_depends_on_the_total_length():
    """With zero coefficients the map is dispersion only, which commutes with
    itself: any distribution of the same total gives the same output, and the
    gradient is the same for every segment."""
    p = base()
    p.coeffs = np.zeros_like(p.coeffs)
    x = random_field((2, 1500), 3, power_w=4e-3)
    a = oracle.run(x, p)
    q = copy.copy(p)
    q.gvd_km = np.array([3.0, 40.0, 11.0, 21.0])          # sum 75 = 3 x 25
    b = oracle.run(x, q)
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
    g = random_field((2, 1500), 4, power_w=1.0)
    _, _, gl = vjp_lengths(x, q, g)
    assert np.allclose(gl, gl[0], rtol=1e-9, atol=1e-12 * np.abs(gl).max())


def test_length_gradient_reproduces_the_split_ratio_gradient():
    """(1 - rho) L, L, ..., rho L: dL/drho = L (dL/dd_last - dL/dd_first)."""
    p = base(seed=1)
    x = random_field((2, 1500), 5, power_w=4e-3)
    g = random_field((2, 1500), 6, power_w=1.0)
    _, gc_r, (rf, rl) = vjp(x, p, g, rho_parts=True)
    gi, gc, gl = vjp_lengths(x, p, g)
    L = p.step_km
    assert abs(L * (gl[-1] - gl[0]) - (rf + rl)) <= 1e-9 * (abs(rf) + abs(rl))
    assert np.allclose(gc, gc_r, rtol=1e-12, atol=0)


def test_length_gradient_matches_finite_differences():
    p = base(seed=2)
    p.gvd_km = np.array([14.0, 30.0, 18.0, 13.0])
    x = random_field((2, 1500), 7, power_w=4e-3)
    g = random_field((2, 1500), 8, power_w=1.0)
    _, _, gl = vjp_lengths(x, p, g)

    def loss(lengths):
        q = copy.copy(p)
        q.gvd_km = np.asarray(lengths, dtype=np.float64)
        return float(np.real(np.sum(np.conj(g) * oracle.run(x, q))))
    for j in range(4):
        h = 1e-3
        e = np.zeros(4)
        e[j] = h
        fd = (loss(p.gvd_km + e) - loss(p.gvd_km - e)) / (2 * h)
        assert abs(fd - gl[j]) <= 1e-5 * np.abs(gl).max(), (j, fd, gl[j])
