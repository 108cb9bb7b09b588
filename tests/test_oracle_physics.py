"""Physical pins of the readings that no equation fixes alone.

The DBP sign of the coefficients, the orientation of the cross-band filter
(C[i, l] acting on p_l with index k - m) and the coupling itself are checked by
what they are for (Sec. I, Sec. II-C): undoing a simulated Manakov link.  A
4-channel WDM field is propagated over 2 x 80 km by a fine-step split-step
simulator without noise; backpropagation with the analytic coefficients must
beat dispersion compensation, and every deliberate misreading must do worse.
"""
import numpy as np
import pytest

import oracle
from oracle.coeffs import Link, dbp_coefficients
from synth import ChannelSpec, WdmSpec, received_field, rng_for, wdm_transmit


@pytest.fixture(scope="module")
def link_case():
    spec = WdmSpec(n_symbols=2 ** 12, n_channels=4, baud=32e9, spacing=40e9, rolloff=0.05,
                   qam_order=16, sample_rate=160e9, power_dbm_per_channel=2.0)
    ch = ChannelSpec(n_spans=2, steps_per_span=100, ase=False)
    rx, _ = received_field(spec, ch, 7)
    tx, _ = wdm_transmit(spec, rng_for(7))
    return rx, tx, Link(n_spans=2, sample_rate=160e9)


def dbp_error(rx, tx, link, C, rho=0.2):
    t = rx.shape[-1]
    p = oracle.OraclePlan(link.beta2, link.sample_rate, 80.0, 2, rho, C.shape[1], t, 0, C)
    return np.linalg.norm(oracle.run(rx, p) - tx) / np.linalg.norm(tx)


def test_backpropagation_readings(link_case):
    rx, tx, link = link_case
    C = dbp_coefficients(link, 4, 2, 0.2, 61)
    e_cb = dbp_error(rx, tx, link, C)
    e_edc = dbp_error(rx, tx, link, 0 * C)
    assert e_cb < 0.2 * e_edc                     # the method works at all

    assert dbp_error(rx, tx, link, -C) > e_edc    # DBP sign: C = -c_forward

    flipped = C.copy()                            # cross-band index k + m instead of k - m
    off = ~np.eye(4, dtype=bool)
    flipped[:, off] = C[:, off][..., ::-1]
    assert dbp_error(rx, tx, link, flipped) > 1.03 * e_cb

    no_xpm = C.copy()
    no_xpm[:, off] = 0.0
    assert dbp_error(rx, tx, link, no_xpm) > 5 * e_cb


def test_asymmetric_split_helps_one_step_per_span(link_case):
    """With one step per span the NLPR belongs near the amplifier (rho < 0.5,
    Sec. III-C)."""
    rx, tx, link = link_case
    e = {rho: dbp_error(rx, tx, link, dbp_coefficients(link, 4, 2, rho, 61), rho)
         for rho in (0.2, 0.5)}
    assert e[0.2] < e[0.5]


@pytest.fixture(scope="module")
def one_span_case():
    """One channel, 32 GBd DP-16QAM at 9 dBm over a single 80 km span (fine
    steps, no noise): the signal power falls by 16 dB along the span, so
    fractional DBP steps of the same length carry very different nonlinear
    phases."""
    spec = WdmSpec(n_symbols=2 ** 12, n_channels=1, baud=32e9, spacing=40e9, rolloff=0.1,
                   qam_order=16, sample_rate=64e9, power_dbm_per_channel=9.0)
    ch = ChannelSpec(n_spans=1, steps_per_span=400, ase=False)
    rx, _ = received_field(spec, ch, 11)
    tx, _ = wdm_transmit(spec, rng_for(11))
    return rx, tx, Link(n_spans=1, sample_rate=64e9)


@pytest.mark.parametrize("n_steps", [3, 4, 5])
@pytest.mark.parametrize("rho", [0.5, 0.2])
def test_fractional_step_order(one_span_case, n_steps, rho):
    """DBP step s undoes physical step N_st - s + 1 (the link is traversed
    backwards, Sec. I; per-step kernels of fractional steps, Sec. II-D): with
    the analytic coefficients in that order the link is undone better than
    with the same steps in the reverse order (the reading DBP step s <->
    physical step s) or with their mean in every step."""
    rx, tx, link = one_span_case

    def err(C):
        p = oracle.OraclePlan(link.beta2, link.sample_rate, 80.0 / n_steps, n_steps, rho, 1, rx.shape[-1], 0, C)
        return np.linalg.norm(oracle.run(rx, p) - tx) / np.linalg.norm(tx)

    C = dbp_coefficients(link, 1, n_steps, rho, 21)
    e = err(C)
    assert e < 0.25 * err(0 * C)
    assert 1.3 * e < err(C[::-1].copy())
    assert e < err(np.repeat(C.mean(axis=0, keepdims=True), n_steps, axis=0))
