"""Seeded synthetic WDM fields standing in for the simulated links of Sec. IV-A.

This module only produces inputs: transmitted symbols and the received
dual-polarisation field.  It holds none of the backpropagation arithmetic and
is used by the tests, the oracle timing and the benchmark alike.

Recipe (Sec. IV-A, at the sizes of the named workloads in ``workloads.py``):
* uniform i.i.d. square QAM per polarisation and channel, unit mean energy,
  numpy ``Generator(PCG64(seed))``;
* frequency-domain root-raised-cosine pulses;
* channels on a uniform grid centred on 0 Hz;
* per span: symmetric split-step Manakov propagation with attenuation,
  GVD transfer function exp(-j 2 pi^2 beta2 f^2 z) (eq. (5)), Kerr term
  -j gamma |u|^2 u with |u|^2 = |x|^2 + |y|^2 (Sec. II-C), then an EDFA that
  restores the span loss and adds ASE (per polarisation complex AWGN of
  variance n_sp h nu (G - 1) R, NF = 2 n_sp).
The received field is in sqrt(W).
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

try:  # multi-threaded FFT for the generator only
    import scipy.fft as _sfft

    def _fft(x):
        return _sfft.fft(x, axis=-1, workers=-1)

    def _ifft(x):
        return _sfft.ifft(x, axis=-1, workers=-1)
except ImportError:  # pragma: no cover
    _fft, _ifft = np.fft.fft, np.fft.ifft

PLANCK = 6.62607015e-34
NU0 = 193.41e12  # carrier frequency (1550 nm)


@dataclass
class WdmSpec:
    n_symbols: int = 2 ** 14         # per channel
    n_channels: int = 1
    baud: float = 32e9
    spacing: float = 100e9
    rolloff: float = 0.1
    qam_order: int = 16
    sample_rate: float = 64e9        # full-field sampling rate R
    power_dbm_per_channel: float = 2.0


@dataclass
class ChannelSpec:
    n_spans: int = 1
    span_km: float = 80.0
    alpha_db_km: float = 0.2
    beta2_ps2_km: float = -21.7
    gamma_w_km: float = 1.3
    steps_per_span: int = 200
    nf_db: float = 5.0
    ase: bool = True


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def qam_symbols(order: int, shape, rng: np.random.Generator) -> np.ndarray:
    """Uniform i.i.d. square QAM with unit average energy."""
    m = int(round(np.sqrt(order)))
    if m * m != order:
        raise ValueError("square QAM only")
    levels = np.arange(-(m - 1), m, 2, dtype=np.float64)
    i = levels[rng.integers(0, m, size=shape)]
    q = levels[rng.integers(0, m, size=shape)]
    energy = 2.0 * (m * m - 1) / 3.0
    return (i + 1j * q) / np.sqrt(energy)


def rrc_amplitude(f: np.ndarray, baud: float, rolloff: float) -> np.ndarray:
    """Root-raised-cosine amplitude response, unit height in the flat part."""
    af = np.abs(f)
    f1 = (1.0 - rolloff) * baud / 2.0
    f2 = (1.0 + rolloff) * baud / 2.0
    out = np.zeros_like(af)
    out[af <= f1] = 1.0
    mid = (af > f1) & (af <= f2)
    if rolloff > 0:
        out[mid] = np.sqrt(0.5 * (1.0 + np.cos(np.pi / (rolloff * baud) * (af[mid] - f1))))
    return out


def wdm_transmit(spec: WdmSpec, rng: np.random.Generator):
    """Transmitted field (2, T) in sqrt(W) and symbols (n_ch, 2, n_symbols)."""
    sps = spec.sample_rate / spec.baud
    if abs(sps - round(sps)) > 1e-9:
        raise ValueError("sample_rate must be an integer multiple of the baud rate")
    sps = int(round(sps))
    t_len = spec.n_symbols * sps
    f = np.fft.fftfreq(t_len, d=1.0 / spec.sample_rate)
    df = spec.sample_rate / t_len
    syms = qam_symbols(spec.qam_order, (spec.n_channels, 2, spec.n_symbols), rng)
    field = np.zeros((2, t_len), dtype=np.complex128)
    p_ch = 1e-3 * 10.0 ** (spec.power_dbm_per_channel / 10.0)
    offsets = (np.arange(spec.n_channels) - (spec.n_channels - 1) / 2.0) * spec.spacing
    for c in range(spec.n_channels):
        shift = offsets[c] / df
        if abs(shift - round(shift)) > 1e-6:
            raise ValueError("channel offset must fall on a DFT bin")
        shift = int(round(shift))
        # zero-stuffed symbols have spectrum A[q mod n_symbols]; shape with RRC
        a_spec = np.fft.fft(syms[c], axis=-1)
        q = np.arange(t_len)
        base = a_spec[:, q % spec.n_symbols] * rrc_amplitude(f, spec.baud, spec.rolloff)[None]
        chan = np.roll(base, shift, axis=-1)          # move to its carrier
        x = np.fft.ifft(chan, axis=-1)
        x *= np.sqrt(p_ch / np.mean(np.sum(np.abs(x) ** 2, axis=0)))
        field += x
    return field, syms


def manakov_link(field: np.ndarray, ch: ChannelSpec, sample_rate: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Forward propagation over ch.n_spans spans with EDFA + ASE."""
    t_len = field.shape[-1]
    f = np.fft.fftfreq(t_len, d=1.0 / sample_rate)
    alpha = ch.alpha_db_km * np.log(10.0) / 10.0
    beta2 = ch.beta2_ps2_km * 1e-24
    gamma = ch.gamma_w_km
    dz = ch.span_km / ch.steps_per_span
    half_lin = np.exp(-1j * 2.0 * np.pi ** 2 * beta2 * f * f * (dz / 2.0) - alpha * dz / 4.0)
    gain = np.exp(alpha * ch.span_km)
    nf = 10.0 ** (ch.nf_db / 10.0)
    ase_var = (nf / 2.0) * PLANCK * NU0 * (gain - 1.0) * sample_rate
    u = field.astype(np.complex128).copy()
    for _ in range(ch.n_spans):
        spec = _fft(u)
        for _ in range(ch.steps_per_span):
            spec *= half_lin
            u = _ifft(spec)
            pw = np.abs(u[0]) ** 2 + np.abs(u[1]) ** 2
            u *= np.exp(-1j * gamma * pw * dz)[None]
            spec = _fft(u)
            spec *= half_lin
        u = _ifft(spec) * np.sqrt(gain)
        if ch.ase:
            u += np.sqrt(ase_var / 2.0) * (rng.standard_normal(u.shape)
                                           + 1j * rng.standard_normal(u.shape))
    return u


def received_field(spec: WdmSpec, ch: ChannelSpec, seed: int):
    """Seeded (received field (2, T), transmitted symbols)."""
    rng = rng_for(seed)
    tx, syms = wdm_transmit(spec, rng)
    rx = manakov_link(tx, ch, spec.sample_rate, rng) if ch.n_spans > 0 else tx
    return rx, syms


def random_field(shape, seed: int, power_w: float = 1.6e-3) -> np.ndarray:
    """Complex Gaussian field of the given shape (..., 2, T), mean |x|^2+|y|^2 = power_w.

    For shape-only tests (edge cases, framing) where no link is needed.
    """
    rng = rng_for(seed)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return z * np.sqrt(power_w / 4.0)


def select_channel(field: np.ndarray, sample_rate: float, offset_hz: float, decim: int) -> np.ndarray:
    """The band of width sample_rate / decim around offset_hz, shifted to
    baseband and decimated by ``decim`` (ideal brick-wall selection in the
    frequency domain): the single-channel input of a receiver that
    backpropagates one WDM channel (Sec. IV-A).  T must be a multiple of decim."""
    t_len = field.shape[-1]
    if t_len % decim:
        raise ValueError("record length must be a multiple of decim")
    t_out = t_len // decim
    shift = offset_hz * t_len / sample_rate
    if abs(shift - round(shift)) > 1e-6:
        raise ValueError("channel offset must fall on a DFT bin")
    spec = np.fft.fft(field, axis=-1)
    k = np.fft.fftfreq(t_out, d=1.0 / t_out).astype(np.int64)       # -t_out/2 .. t_out/2 - 1
    # a T-point DFT over a t_out-point inverse: the sample values need 1 / decim
    return np.fft.ifft(spec[..., (k + int(round(shift))) % t_len], axis=-1) / decim


def received_field_torch(spec: WdmSpec, ch: ChannelSpec, seed: int, device="cuda"):
    """The same recipe as ``received_field`` evaluated with torch on ``device``
    in complex128, for records too long for the CPU generator (tens of
    millions of samples over thousands of link steps).  Symbols come from the
    same numpy generator; the ASE noise from a torch generator seeded with
    ``seed`` on the device.  Returns (field (2, T) complex128 on the device,
    symbols (n_ch, 2, n) numpy)."""
    import torch
    rng = rng_for(seed)
    sps = spec.sample_rate / spec.baud
    if abs(sps - round(sps)) > 1e-9:
        raise ValueError("sample_rate must be an integer multiple of the baud rate")
    sps = int(round(sps))
    t_len = spec.n_symbols * sps
    df = spec.sample_rate / t_len
    syms = qam_symbols(spec.qam_order, (spec.n_channels, 2, spec.n_symbols), rng)
    f = torch.fft.fftfreq(t_len, d=1.0 / spec.sample_rate, dtype=torch.float64, device=device)
    af = f.abs()
    f1, f2 = (1.0 - spec.rolloff) * spec.baud / 2.0, (1.0 + spec.rolloff) * spec.baud / 2.0
    rrc = (af <= f1).to(torch.float64)
    if spec.rolloff > 0:
        mid = (af > f1) & (af <= f2)
        rrc = torch.where(mid, torch.sqrt(0.5 * (1.0 + torch.cos(math.pi / (spec.rolloff * spec.baud) * (af - f1)))),
                          rrc)
    p_ch = 1e-3 * 10.0 ** (spec.power_dbm_per_channel / 10.0)
    offsets = (np.arange(spec.n_channels) - (spec.n_channels - 1) / 2.0) * spec.spacing
    q = torch.arange(t_len, device=device) % spec.n_symbols
    field = torch.zeros((2, t_len), dtype=torch.complex128, device=device)
    for c in range(spec.n_channels):
        shift = offsets[c] / df
        if abs(shift - round(shift)) > 1e-6:
            raise ValueError("channel offset must fall on a DFT bin")
        a_spec = torch.fft.fft(torch.from_numpy(syms[c]).to(device), dim=-1)
        x = torch.fft.ifft(torch.roll(a_spec[:, q] * rrc, int(round(shift)), dims=-1), dim=-1)
        x *= math.sqrt(p_ch / float(torch.mean(torch.sum(x.abs() ** 2, dim=0))))
        field += x
        del a_spec, x
    if ch.n_spans < 1:
        return field, syms
    alpha = ch.alpha_db_km * np.log(10.0) / 10.0
    beta2 = ch.beta2_ps2_km * 1e-24
    dz = ch.span_km / ch.steps_per_span
    half_lin = torch.exp(torch.complex(-alpha * dz / 4.0 * torch.ones_like(f), -2.0 * np.pi ** 2 * beta2 * f * f * (dz / 2.0)))
    gain = np.exp(alpha * ch.span_km)
    ase_var = (10.0 ** (ch.nf_db / 10.0) / 2.0) * PLANCK * NU0 * (gain - 1.0) * spec.sample_rate
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    u = field
    for _ in range(ch.n_spans):
        sp = torch.fft.fft(u, dim=-1)
        for _ in range(ch.steps_per_span):
            sp *= half_lin
            u = torch.fft.ifft(sp, dim=-1)
            pw = u.real ** 2 + u.imag ** 2
            u *= torch.exp(-1j * ch.gamma_w_km * dz * pw.sum(dim=0))[None]
            sp = torch.fft.fft(u, dim=-1)
            sp *= half_lin
        u = torch.fft.ifft(sp, dim=-1) * math.sqrt(gain)
        del sp
        if ch.ase:
            noise = torch.randn(u.shape, dtype=torch.complex128, device=device, generator=gen)
            u += math.sqrt(ase_var / 2.0) * math.sqrt(2.0) * noise   # randn complex has E|z|^2 = 1
    return u, syms
