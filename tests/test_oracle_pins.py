"""Pins of the FP64 forward oracle against what the paper and mathematics fix.

Each test names the property and the passage that fixes it.  None of them
retypes the oracle's formula: they check it against closed forms, a textbook
split-step implementation written here independently, exact inverses and
invariants.
"""
import copy

import numpy as np
import pytest

import oracle
from oracle.cbessfm import OraclePlan, dft_bruteforce
from synth import random_field

BETA2 = -21.7e-24  # s^2/km


def plan(**kw):
    base = dict(beta2_s2_km=BETA2, sample_rate=64e9, step_km=40.0, n_steps=2, rho=0.5,
                n_sb=1, n_block=256, n_overlap=0, coeffs=None)
    base.update(kw)
    if base["coeffs"] is None:
        base["coeffs"] = np.zeros((base["n_steps"], base["n_sb"], base["n_sb"], 5))
    return OraclePlan(**base)


def rand_coeffs(n_steps, n_sb, n_taps, scale, seed):
    return np.random.default_rng(seed).standard_normal((n_steps, n_sb, n_sb, n_taps)) * scale


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- P1: brute-force DFT --------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 16, 64])
def test_bruteforce_dft_closed_forms(n):
    """DFT of a unit impulse is all ones; of exp(+j2pi q0 n/N) is N at bin q0."""
    delta = np.zeros(n, complex)
    delta[0] = 1
    assert np.allclose(dft_bruteforce(delta), np.ones(n), atol=1e-13)
    q0 = n // 3
    tone = np.exp(2j * np.pi * q0 * np.arange(n) / n)
    expect = np.zeros(n, complex)
    expect[q0] = n
    assert np.allclose(dft_bruteforce(tone), expect, atol=1e-10)
    # forward then inverse (unnormalised) is N * identity
    x = random_field((n,), 3)
    assert np.allclose(dft_bruteforce(dft_bruteforce(x), inverse=True) / n, x, atol=1e-12)


@pytest.mark.parametrize("n", [4, 16, 32, 64])
def test_bruteforce_dft_equals_fft(n):
    x = random_field((2, n), 7)
    assert np.allclose(dft_bruteforce(x), np.fft.fft(x, axis=-1), atol=1e-12)


def test_oracle_bruteforce_path_matches_fft_path():
    """The whole chain with O(N^2) DFTs equals the numpy FFT chain (tiny sizes)."""
    c = rand_coeffs(2, 2, 3, 30.0, 1)
    p_fft = plan(n_sb=2, n_block=32, n_overlap=8, coeffs=c, rho=0.3)
    p_bf = copy.copy(p_fft)
    p_bf.dft = dft_bruteforce
    x = random_field((2, 80), 2)
    assert relerr(oracle.run(x, p_bf), oracle.run(x, p_fft)) < 1e-12


# --- P2: zero coefficients = dispersion compensation that inverts the link --------

def linear_channel(x, length_km, sample_rate):
    """Fibre GVD over length_km, H(z, f) = exp(-j 2 pi^2 beta2 f^2 z) (eq. (5))."""
    f = np.fft.fftfreq(x.shape[-1], d=1.0 / sample_rate)
    h = np.exp(-1j * 2 * np.pi ** 2 * BETA2 * f * f * length_km)
    return np.fft.ifft(np.fft.fft(x, axis=-1) * h, axis=-1)


@pytest.mark.parametrize("n_sb,n_steps,rho", [(1, 1, 0.5), (2, 3, 0.3), (4, 2, 0.0), (3, 4, 1.0)])
def test_edc_exactly_inverts_linear_link(n_sb, n_steps, rho):
    t = 384  # one block covering the whole (periodic) sequence
    x = random_field((2, t), 11)
    step = 30.0
    y = linear_channel(x, n_steps * step, 64e9)
    p = plan(n_sb=n_sb, n_steps=n_steps, rho=rho, step_km=step, n_block=t, n_overlap=0)
    assert relerr(oracle.run(y, p), x) < 1e-12


def test_edc_with_overlap_save_converges_with_overlap():
    """Blocked EDC approaches the exact inverse as N_ov covers the memory (Sec. III-A)."""
    from synth import WdmSpec, wdm_transmit, rng_for
    spec = WdmSpec(n_symbols=2 ** 11, baud=32e9, sample_rate=64e9, rolloff=0.1)
    x, _ = wdm_transmit(spec, rng_for(5))
    y = linear_channel(x, 160.0, 64e9)   # memory ~ 2 pi |b2| L R^2 ~ 90 samples
    errs = []
    for nov in (16, 64, 256):
        p = plan(n_steps=2, step_km=80.0, n_block=1024, n_overlap=nov)
        errs.append(relerr(oracle.run(y, p), x))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


# --- P3: subband split is exact at zero coefficients --------------------------------

def test_subband_count_invariance_at_zero_coeffs():
    x = random_field((2, 2 * 960), 13)
    outs = []
    for nsb in (1, 2, 3, 4, 5):
        p = plan(n_sb=nsb, n_block=960, n_overlap=120, n_steps=3, rho=0.2)
        outs.append(oracle.run(x, p))
    for o in outs[1:]:
        assert relerr(o, outs[0]) < 1e-13


# --- P4: unitary filters and pure-phase rotation ----------------------------------

def test_energy_conserved_single_block():
    t = 512
    x = random_field((2, t), 17)
    p = plan(n_sb=4, n_block=t, n_overlap=0, n_steps=3, rho=0.3,
             coeffs=rand_coeffs(3, 4, 7, 100.0, 3))
    y = oracle.run(x, p)
    assert abs(np.sum(np.abs(y) ** 2) / np.sum(np.abs(x) ** 2) - 1.0) < 1e-13


def test_rotation_is_pure_phase_driven_by_circular_fir():
    """rho = 1, one step, one band: out = GVD(L)[u exp(-j theta)], theta = C (*) |u|^2.

    After undoing GVD(L) with the link's own transfer function, the field has
    the input's per-sample power and the phase -theta with theta the circular
    convolution (index k - m, eq. (8)) computed here through FFTs.
    """
    t = 256
    x = random_field((2, t), 19)
    c = rand_coeffs(1, 1, 9, 40.0, 4)
    p = plan(n_sb=1, n_block=t, n_overlap=0, n_steps=1, rho=1.0, step_km=50.0, coeffs=c)
    w = linear_channel(oracle.run(x, p), 50.0, 64e9)
    assert np.allclose(np.abs(w), np.abs(x), rtol=1e-12, atol=0)
    inten = np.abs(x[0]) ** 2 + np.abs(x[1]) ** 2
    taps = np.zeros(t)
    for k, cm in enumerate(c[0, 0, 0]):
        taps[(k - 4) % t] = cm                       # c[m] at lag m
    theta = np.real(np.fft.ifft(np.fft.fft(inten) * np.fft.fft(taps)))
    ratio = w / x
    assert np.allclose(ratio, np.exp(-1j * theta)[None], atol=1e-12)


# --- P5: one band with delta coefficients = textbook SSFM ---------------------------

def textbook_ssfm_dbp(x, n_steps, step_km, rho, phis, sample_rate):
    f = np.fft.fftfreq(x.shape[-1], d=1.0 / sample_rate)

    def gvd(u, dz):
        return np.fft.ifft(np.fft.fft(u, axis=-1) * np.exp(1j * 2 * np.pi ** 2 * BETA2 * f * f * dz), axis=-1)
    u = gvd(x, (1 - rho) * step_km)
    for s in range(n_steps):
        if s:
            u = gvd(u, step_km)
        u = u * np.exp(-1j * phis[s] * (np.abs(u[0]) ** 2 + np.abs(u[1]) ** 2))
    return gvd(u, rho * step_km)


def test_single_band_delta_coeffs_is_ssfm():
    t = 512
    x = random_field((2, t), 23) * 3
    phis = np.array([30.0, -12.0, 55.0])
    c = np.zeros((3, 1, 1, 5))
    c[:, 0, 0, 2] = phis
    p = plan(n_sb=1, n_block=t, n_overlap=0, n_steps=3, rho=0.12, step_km=70.0, coeffs=c)
    ref = textbook_ssfm_dbp(x, 3, 70.0, 0.12, phis, 64e9)
    assert relerr(oracle.run(x, p), ref) < 1e-12


# --- P6: the reversed chain undoes the chain -------------------------------------------

@pytest.mark.parametrize("n_sb", [1, 2, 3])
def test_reversed_chain_is_exact_inverse(n_sb):
    t = 480
    x = random_field((2, t), 29) * 4
    c = rand_coeffs(4, n_sb, 7, 80.0, 5)
    p = plan(n_sb=n_sb, n_block=t, n_overlap=0, n_steps=4, rho=0.27, step_km=60.0, coeffs=c)
    y = oracle.run(x, p)
    inv = plan(n_sb=n_sb, n_block=t, n_overlap=0, n_steps=4, rho=1 - 0.27, step_km=60.0,
               coeffs=-c[::-1].copy(), beta2_s2_km=-BETA2)
    assert relerr(oracle.run(y, inv), x) < 1e-12
    assert relerr(y, x) > 1e-2


# --- P8: framing covariance ----------------------------------------------------------

def test_shift_by_hop_shifts_output():
    p = plan(n_sb=2, n_block=128, n_overlap=32, n_steps=2, rho=0.4,
             coeffs=rand_coeffs(2, 2, 5, 60.0, 6))
    x = random_field((2, 96 * 7), 31)
    y = oracle.run(x, p)
    y_shift = oracle.run(np.roll(x, p.hop, axis=-1), p)
    assert relerr(y_shift, np.roll(y, p.hop, axis=-1)) < 1e-13


def test_batch_equals_instances_and_sampled_blocks():
    p = plan(n_sb=2, n_block=128, n_overlap=32, n_steps=2, rho=0.4,
             coeffs=rand_coeffs(2, 2, 5, 60.0, 8))
    x = random_field((3, 2, 300), 37)
    yb = oracle.run(x, p)
    for i in range(3):
        assert np.array_equal(yb[i], oracle.run(x[i], p))
    blocks = oracle.run_blocks(x[1], p, [0, 2, 3])
    for b, v in blocks.items():
        assert np.array_equal(v, yb[1][:, b * p.hop:b * p.hop + v.shape[-1]])


def test_zero_boundary_reads_zeros_outside():
    """With zero boundary the output of a field padded by zeros matches circular."""
    p_zero = plan(n_sb=1, n_block=128, n_overlap=32, n_steps=1, boundary="zero",
                  coeffs=rand_coeffs(1, 1, 3, 10.0, 9))
    p_circ = copy.copy(p_zero)
    p_circ.boundary = "circular"
    x = random_field((2, 96 * 4), 41)
    pad = np.concatenate([x, np.zeros((2, 96 * 4))], axis=-1)
    # interior blocks never read past the padded end, so zero and circular agree
    a = oracle.run(pad, p_zero)[:, 96:96 * 3]
    b = oracle.run(pad, p_circ)[:, 96:96 * 3]
    assert relerr(a, b) < 1e-13


def test_plan_validation():
    with pytest.raises(ValueError):
        plan(n_sb=3, n_block=256)
    with pytest.raises(ValueError):
        plan(n_overlap=3)
    with pytest.raises(ValueError):
        plan(rho=1.5)
    with pytest.raises(ValueError):
        plan(coeffs=np.zeros((2, 1, 1, 4)))
