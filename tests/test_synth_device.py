"""The torch generator of long records (``received_field_torch``) against the
numpy generator of the same recipe: same symbols, same transmitted field and
the same noiseless link output, evaluated on the CPU in FP64."""
import numpy as np
import pytest
import torch

from synth.field import ChannelSpec, WdmSpec, received_field, received_field_torch


@pytest.mark.parametrize("n_ch,spans", [(1, 0), (3, 2)])
def test_torch_generator_matches_numpy(n_ch, spans):
    spec = WdmSpec(n_symbols=2 ** 10, n_channels=n_ch, baud=32e9, spacing=50e9, rolloff=0.1, qam_order=16,
                   sample_rate=64e9 * n_ch, power_dbm_per_channel=4.0)
    ch = ChannelSpec(n_spans=spans, span_km=80.0, steps_per_span=20, ase=False)
    ref, syms = received_field(spec, ch, 77)
    got, syms_t = received_field_torch(spec, ch, 77, device="cpu")
    assert np.array_equal(syms, syms_t)
    got = got.numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def test_torch_generator_noise_power():
    """ASE of the textbook variance n_sp h nu (G - 1) R per EDFA, both polarisations."""
    spec = WdmSpec(n_symbols=2 ** 12, n_channels=1, baud=32e9, rolloff=0.1, sample_rate=64e9,
                   power_dbm_per_channel=-100.0)
    ch = ChannelSpec(n_spans=1, span_km=80.0, steps_per_span=2, nf_db=5.0)
    u, _ = received_field_torch(spec, ch, 5, device="cpu")
    alpha = 0.2 * np.log(10) / 10
    var = (10 ** 0.5 / 2) * 6.62607015e-34 * 193.41e12 * (np.exp(alpha * 80) - 1) * 64e9
    meas = float(torch.mean(torch.abs(u) ** 2))
    assert abs(meas / var - 1.0) < 0.05
