"""On-device fitting of the CB-ESSFM coefficients and split ratio (Sec. III-B).

The paper fits the coefficients by minimising the mean square error between
the transmitted symbols and the received ones after backpropagation, matched
filtering and sampling, and picks the split ratio by sweeping it.  Here the
backpropagation and its adjoint are the library's kernels (through
``cbessfm``); the receiver -- channel selection, root-raised-cosine matched
filter, decimation, a common phase estimate -- is a few PyTorch operations on
the device, differentiated by autograd; Adam updates C and rho on the device.
"""
from __future__ import annotations

import math

import torch

from ._lib import CbessfmError
from .autograd import cbessfm, cbessfm_steps


def rrc_amplitude(f: torch.Tensor, baud: float, rolloff: float) -> torch.Tensor:
    """Root-raised-cosine amplitude response, unit height in the flat band."""
    af = f.abs()
    f1 = (1.0 - rolloff) * baud / 2.0
    f2 = (1.0 + rolloff) * baud / 2.0
    out = torch.zeros_like(af)
    out[af <= f1] = 1.0
    if rolloff > 0:
        mid = (af > f1) & (af <= f2)
        out[mid] = torch.sqrt(0.5 * (1.0 + torch.cos(math.pi / (rolloff * baud) * (af[mid] - f1))))
    return out


class SymbolReceiver:
    """Matched filter and symbol sampler of one WDM channel.

    The channel sits at ``offset_hz`` (a whole number of DFT bins of the
    length-T record) and carries symbols at ``baud`` with sample k * sps at
    symbol k, sps = sample_rate / baud.  A transmitter of unit-energy symbols
    normalised to ``power_w`` over both polarisations has a pulse amplitude of
    sps sqrt(power_w / 2); after the matched filter (a raised-cosine overall
    response, Nyquist at the symbol rate) the sample at symbol k is the
    symbol times sqrt(power_w / 2), which the output is divided by.
    """

    def __init__(self, t_len: int, sample_rate: float, baud: float, rolloff: float, power_w: float,
                 offset_hz: float = 0.0, device="cuda"):
        sps = sample_rate / baud
        if abs(sps - round(sps)) > 1e-9:
            raise ValueError("sample_rate must be a whole multiple of baud")
        self.sps = int(round(sps))
        df = sample_rate / t_len
        shift = offset_hz / df
        if abs(shift - round(shift)) > 1e-6:
            raise ValueError("channel offset must fall on a DFT bin")
        self.shift = int(round(shift))
        f = torch.fft.fftfreq(t_len, d=1.0 / sample_rate, device=device, dtype=torch.float64)
        h = rrc_amplitude(f, baud, rolloff) / math.sqrt(power_w / 2.0)
        self.h = h.to(torch.complex64)

    def __call__(self, y: torch.Tensor) -> torch.Tensor:
        spec = torch.fft.fft(y, dim=-1)
        if self.shift:
            spec = torch.roll(spec, -self.shift, dims=-1)
        z = torch.fft.ifft(spec * self.h, dim=-1)
        return z[..., :: self.sps]


def phase_aligned_mse(z: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    """Mean |z exp(-j phi) - s|^2 with phi = arg sum z conj(s) per realisation
    (the common phase is estimated, not learned, so it is held constant)."""
    with torch.no_grad():
        corr = (z * s.conj()).sum(dim=(-2, -1), keepdim=True)
        rot = torch.exp(-1j * torch.angle(corr)).to(z.dtype)
    return (z * rot - s).abs().pow(2).mean()


def adam_loop(params, loss_fn, iters: int, lr: float, graph: bool = False, warmup: int = 3,
              after_step=None, device=None, check=None):
    """Adam on ``params`` for ``iters`` iterations of ``loss_fn()`` (which
    returns a scalar tensor).  With ``graph`` the iteration (forward, loss,
    backward, update) is recorded in a HIP graph after ``warmup`` eager
    iterations on a side stream and replayed for the rest; ``iters`` counts
    all of them.  ``after_step`` runs under no_grad after every update.
    ``check`` (if given) runs after the eager iterations and at the end,
    outside any capture: it raises if the device reported an error.
    Returns the losses as a tensor."""
    opt = torch.optim.Adam(params, lr=lr, capturable=graph)

    def step():
        opt.zero_grad(set_to_none=not graph)
        loss = loss_fn()
        loss.backward()
        opt.step()
        if after_step is not None:
            with torch.no_grad():
                after_step()
        return loss.detach()

    losses = []
    if not graph:
        for _ in range(iters):
            losses.append(step())
        if check is not None:
            check()
        return torch.stack(losses)
    side = torch.cuda.Stream(device=device)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(min(warmup, iters)):
            losses.append(step())
    torch.cuda.current_stream().wait_stream(side)
    if check is not None:
        check()
    if iters > warmup:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            static_loss = step()
        for _ in range(iters - warmup):
            g.replay()
            losses.append(static_loss.clone())
        del g
        if check is not None:
            check()
    return torch.stack(losses)


def plan_check_fn(plan):
    """A ``check`` for adam_loop: raises CbessfmError if a device-side
    exchange wait of the plan gave up (its gradients are then invalid)."""
    def check():
        code = plan.status()
        if code != 0:
            raise CbessfmError(code, "device error during the fit")
    return check


def fit(plan, fields: torch.Tensor, symbols: torch.Tensor, receiver: SymbolReceiver, coeffs0, rho0: float,
        iters: int = 200, lr: float = 1e-2, checkpoint_every: int = 1, fit_rho: bool = True,
        graph: bool = False, warmup: int = 3):
    """Adam on (C, rho) for ``iters`` iterations; returns (coeffs, rho, losses).

    fields: complex64 (B, 2, T) on the device; symbols: complex64 (B, 2, n)
    transmitted symbols of the channel the receiver selects (or sequences of
    receivers and symbol tensors, one per channel: the loss is then the mean
    of the channels' MSEs).  The update of C
    is taken in units of the initial coefficients' scale so that one learning
    rate suits every tap.  With ``graph`` the whole iteration (forward,
    loss, adjoint, Adam update) is recorded once in a HIP graph after
    ``warmup`` eager iterations and replayed for the rest; ``iters`` counts
    all of them.
    """
    c0 = torch.as_tensor(coeffs0, dtype=torch.float32, device=fields.device)
    scale = c0.abs().max().clamp_min(1e-12)
    u = (c0 / scale).clone().requires_grad_(True)
    rho = torch.tensor(float(rho0), dtype=torch.float32, device=fields.device, requires_grad=fit_rho)
    params = [u, rho] if fit_rho else [u]

    def loss_fn():
        y = cbessfm(fields, (u * scale).contiguous(), rho, plan, checkpoint_every)
        return receiver_mse(y, receiver, symbols)

    losses = adam_loop(params, loss_fn, iters, lr, graph=graph, warmup=warmup,
                       after_step=lambda: rho.clamp_(0.0, 1.0), device=fields.device, check=plan_check_fn(plan))
    return (u * scale).detach(), rho.detach(), losses


def receiver_mse(y: torch.Tensor, receiver, symbols) -> torch.Tensor:
    """Phase-aligned MSE of one channel, or the mean over channels when
    ``receiver`` and ``symbols`` are sequences (one receiver and one symbol
    tensor per WDM channel)."""
    if isinstance(receiver, (list, tuple)):
        return sum(phase_aligned_mse(r(y), s) for r, s in zip(receiver, symbols)) / len(receiver)
    return phase_aligned_mse(receiver(y), symbols)


def snr_db(plan, coeffs: torch.Tensor, rho, fields: torch.Tensor, symbols: torch.Tensor,
           receiver: SymbolReceiver) -> float:
    """Effective SNR of the received symbols after backpropagation with the
    given coefficients, matched filtering, sampling and common-phase removal:
    -10 log10 of the phase-aligned mean square error (unit-energy symbols)."""
    rho_t = torch.as_tensor(rho, dtype=torch.float32, device=fields.device).reshape(())
    with torch.no_grad():
        mse = receiver_mse(cbessfm(fields, coeffs.contiguous(), rho_t, plan), receiver, symbols)
    return -10.0 * math.log10(float(mse))


def fit_steps(plan, fields: torch.Tensor, symbols: torch.Tensor, receiver: SymbolReceiver, coeffs0, lengths0,
              iters: int = 150, lr: float = 2e-3, lr_lengths: float | None = None, fit_lengths: bool = True,
              checkpoint_every: int = 1, graph: bool = False, warmup: int = 3):
    """Joint fit of per-step coefficients and the N_st + 1 dispersion segment
    lengths (the step-size distribution and split per step that Sec. V leaves
    to future work).  The lengths are total * softmax(z), so they stay
    positive and keep their sum; Adam on (C / scale) at ``lr`` and on z at
    ``lr_lengths`` (default ``lr``).  The fit starts from a solution that is
    already fitted, so it is kept only where it lowers the training loss:
    if the final loss exceeds the starting one the start is returned.
    Returns (coeffs, lengths (float64), losses)."""
    dev = fields.device
    c0 = torch.as_tensor(coeffs0, dtype=torch.float32, device=dev)
    scale = c0.abs().max().clamp_min(1e-12)
    u = (c0 / scale).clone().requires_grad_(True)
    l0 = torch.as_tensor(lengths0, dtype=torch.float64, device=dev)
    total = float(l0.sum())
    z = torch.log(l0 / total).clone().requires_grad_(fit_lengths)

    def loss_fn():
        lengths = total * torch.softmax(z, 0)
        y = cbessfm_steps(fields, (u * scale).contiguous(), lengths, plan, checkpoint_every)
        return phase_aligned_mse(receiver(y), symbols)

    groups = [{"params": [u], "lr": lr}]
    if fit_lengths:
        groups.append({"params": [z], "lr": lr if lr_lengths is None else lr_lengths})
    losses = adam_loop(groups, loss_fn, iters, lr, graph=graph, warmup=warmup, device=dev,
                       check=plan_check_fn(plan))
    c_fit, l_fit = (u * scale).detach(), (total * torch.softmax(z, 0)).detach()
    with torch.no_grad():
        start = phase_aligned_mse(receiver(cbessfm_steps(fields, c0.contiguous(), l0.contiguous(), plan)), symbols)
        end = phase_aligned_mse(receiver(cbessfm_steps(fields, c_fit.contiguous(), l_fit.contiguous(), plan)),
                                symbols)
    if float(end) > float(start):
        return c0.clone(), l0.clone(), losses
    return c_fit, l_fit, losses


def snr_db_steps(plan, coeffs: torch.Tensor, lengths: torch.Tensor, fields: torch.Tensor, symbols: torch.Tensor,
                 receiver: SymbolReceiver) -> float:
    """``snr_db`` with free dispersion segment lengths."""
    with torch.no_grad():
        mse = phase_aligned_mse(receiver(cbessfm_steps(fields, coeffs.contiguous(), lengths.contiguous(), plan)),
                                symbols)
    return -10.0 * math.log10(float(mse))
