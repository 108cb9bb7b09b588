"""Named workloads: field recipe + DBP shape, after the systems of Sec. IV-A.

Each entry gives the transmitted WDM signal, the forward link used to make the
received field, and the CB-ESSFM shape run on it.  Names state what the
workload is.  ``n_overlap`` is in full-field samples; ``n_sub`` is N' = N/N_sb.
"""
from __future__ import annotations

from .field import ChannelSpec, WdmSpec, received_field, received_field_torch, select_channel

WORKLOADS = {
    # single channel, one span, one DBP step: the small parity case
    "1ch-32GBd-16QAM-2^14sym-1x80km": dict(
        wdm=WdmSpec(n_symbols=2 ** 14, n_channels=1, baud=32e9, spacing=100e9, rolloff=0.1,
                    qam_order=16, sample_rate=64e9, power_dbm_per_channel=2.0),
        ch=ChannelSpec(n_spans=1, span_km=80.0, steps_per_span=200, nf_db=5.0),
        dbp=dict(n_sb=1, n_sub=1024, n_overlap=128, n_steps=1, rho=0.5, n_taps=11),
    ),
    # five 64-GBd channels on a 100-GHz grid, 15 spans, 15 asymmetric steps
    "5ch-64GBd-64QAM-2^16sym-15x80km": dict(
        wdm=WdmSpec(n_symbols=2 ** 16, n_channels=5, baud=64e9, spacing=100e9, rolloff=0.05,
                    qam_order=64, sample_rate=640e9, power_dbm_per_channel=2.0),
        ch=ChannelSpec(n_spans=15, span_km=80.0, steps_per_span=1000, nf_db=5.0),
        dbp=dict(n_sb=5, n_sub=4096, n_overlap=2560, n_steps=15, rho=0.3, n_taps=21),
    ),
    # five 64-GBd channels, 15 spans; only the central channel is selected
    # (decimated to 128 GS/s, 2 samples/symbol) and backpropagated, as in the
    # paper's system of Sec. IV-A: the coefficient-fitting and comparison
    # workload.  The overlap covers the channel's dispersion memory.
    "5ch-64GBd-64QAM-2^13sym-15x80km-central": dict(
        wdm=WdmSpec(n_symbols=2 ** 13, n_channels=5, baud=64e9, spacing=100e9, rolloff=0.05,
                    qam_order=64, sample_rate=640e9, power_dbm_per_channel=3.0),
        ch=ChannelSpec(n_spans=15, span_km=80.0, steps_per_span=50, nf_db=5.0),
        select=dict(offset_hz=0.0, decim=5, channel=2),
        dbp=dict(n_sb=2, n_sub=4096, n_overlap=2688, n_steps=15, rho=0.3, n_taps=45),
    ),
    # five 64-GBd channels over 40 spans: the long link whose dispersion memory
    # (1.8e5 full-field samples) needs blocks of N' = 2^17 per subband; the
    # backpropagation step count is swept over ``step_sweep``.  The record
    # (1.05e7 samples per polarisation) is generated on the device.
    "5ch-64GBd-64QAM-2^20sym-40x80km": dict(
        wdm=WdmSpec(n_symbols=2 ** 20, n_channels=5, baud=64e9, spacing=100e9, rolloff=0.05,
                    qam_order=64, sample_rate=640e9, power_dbm_per_channel=2.0),
        ch=ChannelSpec(n_spans=40, span_km=80.0, steps_per_span=500, nf_db=5.0),
        dbp=dict(n_sb=5, n_sub=2 ** 17, n_overlap=196608, n_steps=10, rho=0.3, n_taps=21,
                 step_sweep=(1, 2, 5, 10, 20, 40, 80)),
        device_generator=True,
    ),
    # single channel, one span, 15 fractional-span DBP steps (gradient workload)
    "1ch-32GBd-16QAM-2^14sym-1x80km-15steps": dict(
        wdm=WdmSpec(n_symbols=2 ** 14, n_channels=1, baud=32e9, spacing=100e9, rolloff=0.1,
                    qam_order=16, sample_rate=64e9, power_dbm_per_channel=2.0),
        ch=ChannelSpec(n_spans=1, span_km=80.0, steps_per_span=200, nf_db=5.0),
        dbp=dict(n_sb=1, n_sub=1024, n_overlap=128, n_steps=15, rho=0.5, n_taps=11),
    ),
}


def workload(name: str, seed: int, steps_per_span: int | None = None, ase: bool = True, device=None):
    """Seeded received field (2, T), symbols and the workload entry.  With a
    channel selection the field is that channel at its reduced rate
    (``dbp_rate``) and the symbols are that channel's, shape (1, 2, n).
    Workloads marked ``device_generator`` (or any, given ``device``) are
    generated with torch on ``device`` (default "cuda") and the field is a
    complex128 tensor there.

    ``steps_per_span`` overrides the forward simulator's step count (the
    received field's fine structure does not change the cost or the parity of
    the backpropagation, only its SNR).
    """
    w = WORKLOADS[name]
    ch = w["ch"]
    if steps_per_span is not None or not ase:
        ch = ChannelSpec(**{**ch.__dict__,
                            "steps_per_span": steps_per_span or ch.steps_per_span,
                            "ase": ase})
    if device is not None or w.get("device_generator"):
        field, syms = received_field_torch(w["wdm"], ch, seed, device or "cuda")
        if w.get("select") is not None:
            raise ValueError("channel selection runs on the CPU generator")
        return field, syms, w
    field, syms = received_field(w["wdm"], ch, seed)
    sel = w.get("select")
    if sel is not None:
        field = select_channel(field, w["wdm"].sample_rate, sel["offset_hz"], sel["decim"])
        syms = syms[sel["channel"]:sel["channel"] + 1]
    return field, syms, w


def dbp_rate(w) -> float:
    """Sampling rate of the field the workload backpropagates."""
    sel = w.get("select")
    return w["wdm"].sample_rate / (sel["decim"] if sel else 1)
