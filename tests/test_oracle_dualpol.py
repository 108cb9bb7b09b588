"""Pins of the oracle's dual-polarisation NLPR (eqs. (20)-(21)) against what
Sec. II-C states about it, not against its own formula:

* cross-band XPM from a co-polarised subband is twice as strong as from an
  orthogonally polarised one with the same power;
* with equal intensities in the two polarisations it is the averaged NLPR of
  eq. (15), which models the average of the two (Sec. II-C);
* exchanging the polarisations exchanges the phases;
* a single subband has no cross-band term, so both models agree.
"""
import numpy as np
import pytest

import oracle
from oracle.cbessfm import coupled_fir, dual_pol_phases
from synth import random_field


def rand_c(nsb, taps, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nsb, nsb, taps))


def test_copolarised_xpm_is_twice_the_orthogonal():
    rng = np.random.default_rng(1)
    c = rand_c(3, 5, 2)
    inten = rng.uniform(0.0, 1.0, (3, 64))
    zero = np.zeros_like(inten)
    # subband 0 carries nothing; subbands 1, 2 only x (co-polarised with x_0) or only y
    co = dual_pol_phases(np.where(np.arange(3)[:, None] > 0, inten, 0.0), zero, c)
    orth = dual_pol_phases(zero, np.where(np.arange(3)[:, None] > 0, inten, 0.0), c)
    assert np.allclose(co[0, 0], 2.0 * orth[0, 0], rtol=1e-13, atol=1e-13)   # theta^x of subband 0
    assert np.allclose(orth[0, 1], 2.0 * co[0, 1], rtol=1e-13, atol=1e-13)   # theta^y of subband 0
    # and the averaged model, which uses the mean of the two for both polarisations
    avg = coupled_fir(np.where(np.arange(3)[:, None] > 0, inten, 0.0), c)
    assert np.allclose(co[0, 0] + orth[0, 0], 2.0 * avg[0], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nsb", [1, 2, 4])
def test_equal_polarisation_intensities_give_the_averaged_nlpr(nsb):
    rng = np.random.default_rng(nsb)
    c = rand_c(nsb, 7, nsb)
    half = rng.uniform(0.0, 1.0, (nsb, 80))
    th = dual_pol_phases(half, half, c)
    avg = coupled_fir(2.0 * half, c)
    assert np.allclose(th[:, 0], avg, rtol=1e-13, atol=1e-13)
    assert np.allclose(th[:, 1], avg, rtol=1e-13, atol=1e-13)


def test_exchanging_polarisations_exchanges_the_phases():
    rng = np.random.default_rng(5)
    c = rand_c(3, 9, 6)
    px, py = rng.uniform(0, 1, (3, 50)), rng.uniform(0, 1, (3, 50))
    a, b = dual_pol_phases(px, py, c), dual_pol_phases(py, px, c)
    assert np.allclose(a[:, 0], b[:, 1], rtol=1e-14, atol=0) and np.allclose(a[:, 1], b[:, 0], rtol=1e-14, atol=0)


def test_whole_map_single_subband_and_equal_power_fields_match_the_averaged_map():
    c = rand_c(1, 5, 3) * 50.0
    x = random_field((2, 3000), 9, power_w=4e-3)
    kw = dict(beta2_s2_km=-21.7e-24, sample_rate=64e9, step_km=20.0, n_steps=3, rho=0.4, n_sb=1,
              n_block=1024, n_overlap=128)
    c3 = c[None].repeat(3, axis=0)
    a = oracle.run(x, oracle.OraclePlan(coeffs=c3, **kw))
    b = oracle.run(x, oracle.OraclePlan(coeffs=c3, nlpr="dual", **kw))
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
    # two subbands, a field whose y is x delayed by nothing but a phase: equal intensities everywhere
    kw.update(n_sb=2, sample_rate=128e9)
    c2 = rand_c(2, 5, 4)[None].repeat(3, axis=0) * 50.0
    f = random_field((1, 3000), 10, power_w=2e-3)[0]
    xy = np.stack([f, f * np.exp(0.7j)])
    a = oracle.run(xy, oracle.OraclePlan(coeffs=c2, **kw))
    b = oracle.run(xy, oracle.OraclePlan(coeffs=c2, nlpr="dual", **kw))
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())
    # and with unequal intensities the two differ
    b2 = oracle.run(x, oracle.OraclePlan(coeffs=c2, nlpr="dual", **kw))
    a2 = oracle.run(x, oracle.OraclePlan(coeffs=c2, **kw))
    assert np.abs(a2 - b2).max() > 1e-6 * np.abs(a2).max()
