"""FP64 oracle of the CB-ESSFM gradients (reverse-mode through the forward map).

TEST INFRASTRUCTURE ONLY (see ``oracle/cbessfm.py``).

The forward map of Sec. III-A / III-C is rewritten here with plain PyTorch CPU
complex128 ops, step for step as in ``oracle/cbessfm.py``, and differentiated
by torch's autograd.  Given a cotangent G for the output (PyTorch's
convention for a real loss of a complex tensor: G = dL/dRe + j dL/dIm) it
returns dL/dfield_in, dL/dC and dL/drho for L = Re <G, out>.  The paper fits
coefficients offline with finite differences (Sec. III-B) and names automatic
differentiation as future work; this is that derivative, computed exactly.
"""
from __future__ import annotations

import numpy as np
import torch

from .cbessfm import OraclePlan, bin_frequencies


def _demux_index(plan: OraclePlan) -> np.ndarray:
    n, nsub = plan.n_block, plan.n_sub
    delta = np.fft.fftfreq(nsub, d=1.0 / nsub).astype(np.int64)
    return np.stack([(-n // 2 + i * nsub + nsub // 2 + delta) % n for i in range(plan.n_sb)])


def forward_torch(field_in: torch.Tensor, coeffs: torch.Tensor, rho, plan: OraclePlan,
                  lengths: torch.Tensor | None = None) -> torch.Tensor:
    """Same map as ``oracle.cbessfm.run`` for one instance (2, T), in torch FP64.

    ``rho`` is a scalar tensor, or a pair (rho of the first GVD, rho of the
    last GVD) so that the two places where the split ratio enters
    (Sec. III-C) can be differentiated separately.  ``lengths``, if given,
    are the N_st + 1 dispersion segment lengths (km) and replace rho.
    """
    if plan.nlpr != "averaged":
        raise NotImplementedError("the gradient oracle covers the averaged NLPR of eq. (15)")
    rho_first, rho_last = (rho, rho) if not isinstance(rho, (tuple, list)) else rho
    t_len = field_in.shape[-1]
    n, nsub, nsb = plan.n_block, plan.n_sub, plan.n_sb
    L = plan.step_km
    f = torch.from_numpy(bin_frequencies(plan))                       # (N_sb, N')
    ph = 2.0 * np.pi ** 2 * plan.beta2_s2_km * f * f                  # per km
    if lengths is None:
        seg = [(1.0 - rho_first) * L] + [L] * (plan.n_steps - 1) + [rho_last * L]
    else:
        seg = [lengths[j] for j in range(plan.n_steps + 1)]
    hs = [torch.exp(1j * ph * g) for g in seg]
    qidx = torch.from_numpy(_demux_index(plan))
    ntap = coeffs.shape[-1]
    nc = ntap // 2
    keep_lo = plan.n_overlap // 2
    pieces = []
    for b in range(plan.n_blocks(t_len)):
        pos = b * plan.hop - plan.n_overlap // 2 + np.arange(n)
        if plan.boundary == "circular":
            u = field_in[:, torch.from_numpy(pos % t_len)]
        else:
            ok = (pos >= 0) & (pos < t_len)
            u = torch.zeros((2, n), dtype=torch.complex128)
            u[:, torch.from_numpy(np.nonzero(ok)[0])] = field_in[:, torch.from_numpy(pos[ok])]
        spec = torch.fft.fft(u, dim=-1)
        v_spec = spec[:, qidx].permute(1, 0, 2)                        # (N_sb, 2, N')
        for s in range(plan.n_steps):
            v_spec = v_spec * hs[s][:, None, :]
            v = torch.fft.ifft(v_spec, dim=-1) * (nsub / n)
            p = v[:, 0].abs() ** 2 + v[:, 1].abs() ** 2                # (N_sb, N')
            theta = torch.zeros((nsb, nsub), dtype=torch.float64)
            for i in range(nsb):
                for l in range(nsb):
                    for t in range(ntap):
                        theta[i] = theta[i] + coeffs[s, i, l, t] * torch.roll(p[l], t - nc)
            v = v * torch.exp(-1j * theta)[:, None, :]
            v_spec = nsb * torch.fft.fft(v, dim=-1)
        v_spec = v_spec * hs[-1][:, None, :]
        full = torch.zeros((2, n), dtype=torch.complex128)
        full[:, qidx.reshape(-1)] = v_spec.permute(1, 0, 2).reshape(2, -1)
        y = torch.fft.ifft(full, dim=-1)
        n_keep = min(plan.hop, t_len - b * plan.hop)
        pieces.append(y[:, keep_lo:keep_lo + n_keep])
    return torch.cat(pieces, dim=-1)


def vjp(field_in: np.ndarray, plan: OraclePlan, grad_out: np.ndarray, rho_parts: bool = False):
    """(dL/dfield_in, dL/dC, dL/drho) for L = Re sum conj(G) * out.

    field_in / grad_out: (2, T) or (B, 2, T); C and rho gradients are summed
    over the batch.  With ``rho_parts`` the split-ratio derivative is returned
    as the pair (through the first GVD, through the last GVD), whose sum is
    dL/drho.
    """
    x = np.asarray(field_in, dtype=np.complex128)
    g = np.asarray(grad_out, dtype=np.complex128)
    squeeze = x.ndim == 2
    if squeeze:
        x, g = x[None], g[None]
    coeffs = torch.tensor(plan.coeffs, dtype=torch.float64, requires_grad=True)
    rho_f = torch.tensor(float(plan.rho), dtype=torch.float64, requires_grad=True)
    rho_l = torch.tensor(float(plan.rho), dtype=torch.float64, requires_grad=True)
    gin = []
    for bi in range(x.shape[0]):
        xi = torch.tensor(x[bi], requires_grad=True)
        out = forward_torch(xi, coeffs, (rho_f, rho_l), plan)
        loss = (torch.conj(torch.from_numpy(g[bi])) * out).real.sum()
        loss.backward()
        gin.append(xi.grad.numpy().copy())
    grad_in = np.stack(gin)
    g_rho = (float(rho_f.grad), float(rho_l.grad)) if rho_parts else float(rho_f.grad) + float(rho_l.grad)
    return (grad_in[0] if squeeze else grad_in), coeffs.grad.numpy().copy(), g_rho


def vjp_lengths(field_in: np.ndarray, plan: OraclePlan, grad_out: np.ndarray):
    """(dL/dfield_in, dL/dC, dL/d(segment lengths)) for L = Re sum conj(G) * out,
    with the plan's N_st + 1 dispersion segment lengths as free parameters
    (``OraclePlan.gvd_lengths``)."""
    x = np.asarray(field_in, dtype=np.complex128)
    g = np.asarray(grad_out, dtype=np.complex128)
    squeeze = x.ndim == 2
    if squeeze:
        x, g = x[None], g[None]
    coeffs = torch.tensor(plan.coeffs, dtype=torch.float64, requires_grad=True)
    lengths = torch.tensor(plan.gvd_lengths(), dtype=torch.float64, requires_grad=True)
    gin = []
    for bi in range(x.shape[0]):
        xi = torch.tensor(x[bi], requires_grad=True)
        out = forward_torch(xi, coeffs, None, plan, lengths=lengths)
        loss = (torch.conj(torch.from_numpy(g[bi])) * out).real.sum()
        loss.backward()
        gin.append(xi.grad.numpy().copy())
    grad_in = np.stack(gin)
    return (grad_in[0] if squeeze else grad_in), coeffs.grad.numpy().copy(), lengths.grad.numpy().copy()
