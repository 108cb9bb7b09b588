"""Pins of the FP64 gradient oracle: finite differences of the numpy forward
oracle, the adjoint identity of the linear case, and agreement of the two
forward implementations."""
import copy

import numpy as np
import pytest
import torch

import oracle
from oracle.cbessfm import OraclePlan
from oracle.grad import forward_torch, vjp
from synth import random_field

BETA2 = -21.7e-24


def make_plan(n_sb=2, n_steps=3, rho=0.3, n_taps=5, scale=40.0, seed=1, boundary="circular"):
    c = np.random.default_rng(seed).standard_normal((n_steps, n_sb, n_sb, n_taps)) * scale
    return OraclePlan(BETA2, 64e9, 25.0, n_steps, rho, n_sb, 64 * n_sb, 16 * n_sb, c,
                      boundary=boundary)


def loss(x, p, g):
    return float(np.real(np.sum(np.conj(g) * oracle.run(x, p))))


@pytest.mark.parametrize("boundary", ["circular", "zero"])
def test_torch_forward_equals_numpy_forward(boundary):
    p = make_plan(boundary=boundary)
    x = random_field((2, 300), 3) * 3
    y = oracle.run(x, p)
    yt = forward_torch(torch.from_numpy(x), torch.from_numpy(p.coeffs),
                       torch.tensor(p.rho, dtype=torch.float64), p).detach().numpy()
    assert np.linalg.norm(yt - y) / np.linalg.norm(y) < 1e-14


def test_coefficient_and_rho_gradients_match_central_differences():
    p = make_plan()
    x = random_field((2, 300), 5) * 3
    g = random_field((2, 300), 6)
    _, gc, gr = vjp(x, p, g)
    rng = np.random.default_rng(0)
    for _ in range(6):
        idx = tuple(rng.integers(0, n) for n in p.coeffs.shape)
        for rel_h in (1e-3, 1e-5):
            h = rel_h * max(abs(p.coeffs[idx]), 1.0)
            pa, pb = copy.copy(p), copy.copy(p)
            pa.coeffs = p.coeffs.copy()
            pb.coeffs = p.coeffs.copy()
            pa.coeffs[idx] += h
            pb.coeffs[idx] -= h
            fd = (loss(x, pa, g) - loss(x, pb, g)) / (2 * h)
            assert abs(fd - gc[idx]) <= 1e-5 * max(abs(gc[idx]), 1e-3 * np.abs(gc).max())
    h = 1e-5
    pa, pb = copy.copy(p), copy.copy(p)
    pa.rho, pb.rho = p.rho + h, p.rho - h
    fd = (loss(x, pa, g) - loss(x, pb, g)) / (2 * h)
    assert abs(fd - gr) < 1e-6 * abs(gr)


def test_input_gradient_matches_directional_difference():
    p = make_plan(n_sb=1, n_taps=3)
    x = random_field((2, 200), 7) * 3
    g = random_field((2, 200), 8)
    gi, _, _ = vjp(x, p, g)
    v = random_field((2, 200), 9)
    h = 1e-4
    fd = (loss(x + h * v, p, g) - loss(x - h * v, p, g)) / (2 * h)
    assert abs(fd - np.real(np.sum(np.conj(gi) * v))) < 1e-7 * abs(fd)


def test_linear_case_adjoint_identity():
    """At C = 0 the map is complex-linear, out = A x, and the input gradient of
    Re<g, A x> is A^H g: <A v, w> = <v, A^H w> for random v, w."""
    p = make_plan(scale=0.0)
    v = random_field((2, 320), 10)
    w = random_field((2, 320), 11)
    av = oracle.run(v, p)
    ahw, gc, _ = vjp(v, p, w)          # input gradient is A^H w, independent of v
    assert abs(np.vdot(w, av) - np.vdot(ahw, v)) < 1e-12 * np.linalg.norm(av) * np.linalg.norm(w)


def test_batch_gradients_sum_over_instances():
    p = make_plan(n_sb=1, n_taps=3, n_steps=2)
    x = random_field((2, 2, 200), 12) * 3
    g = random_field((2, 2, 200), 13)
    gi, gc, gr = vjp(x, p, g)
    parts = [vjp(x[i], p, g[i]) for i in range(2)]
    assert np.allclose(gc, parts[0][1] + parts[1][1], rtol=1e-12)
    assert np.isclose(gr, parts[0][2] + parts[1][2], rtol=1e-12)
    assert np.allclose(gi[1], parts[1][0], rtol=1e-12)
