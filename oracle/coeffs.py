"""FP64 oracle of the analytic CB-ESSFM coefficients (Sec. II-D, App. C).

TEST INFRASTRUCTURE ONLY (see ``oracle/cbessfm.py``).

Definitions followed:

* kernel, eq. (6) / App. C eq. ``kernel_b``:
  K(mu, nu) = int gamma g(z) exp(-j 2 b (z - z0)) dz over the step, with
  b = 2 pi^2 beta2 nu (mu - nu) and g(z) the power profile relative to the
  launch power (exp(-alpha * distance from the last amplifier)).
  z0 is the position of the nonlinear phase rotation inside the step.  For a
  symmetric step of whole spans this is eq. (22); the asymmetric split of
  Sec. III-C moves z0 to rho L from the physical start of the step.
* coefficients, eq. (13) evaluated on an M x M midpoint grid over
  [f_il - R'/2, f_il + R'/2]^2 (Sec. II-D: diagonal of the 2-D DFT of K):
  c_il[m] = Re{ (1/M^2) sum_{p,q} K(mu_p, nu_q) exp(j 2 pi m (p - q) / M) }.
  The real part is taken because the phase rotation must be real (Sec. III-D
  states that the coefficients are real).
* applied tensor of the backpropagation (reversed link, Sec. I): step s of the
  DBP undoes physical step j = N_st - s + 1, so
  C_s[i, i] = -c_ii^(j) and C_s[i, l != i] = -(3/2) c_il^(j) (eq. (15)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Link:
    alpha_db_km: float = 0.2
    beta2_ps2_km: float = -21.7
    gamma_w_km: float = 1.3
    span_km: float = 80.0
    n_spans: int = 1
    sample_rate: float = 64e9
    manakov_8_9: bool = False

    @property
    def alpha(self) -> float:
        """Power attenuation coefficient in 1/km."""
        return self.alpha_db_km * np.log(10.0) / 10.0

    @property
    def beta2(self) -> float:
        """beta2 in s^2/km."""
        return self.beta2_ps2_km * 1e-24

    @property
    def gamma(self) -> float:
        return self.gamma_w_km * (8.0 / 9.0 if self.manakov_8_9 else 1.0)

    @property
    def length_km(self) -> float:
        return self.span_km * self.n_spans


def _one_minus_exp_over(kappa: np.ndarray, length: float) -> np.ndarray:
    """(1 - exp(-kappa * length)) / kappa, stable as kappa -> 0."""
    x = kappa * length
    small = np.abs(x) < 1e-6
    safe = np.where(small, 1.0, kappa)
    out = -np.expm1(-x) / safe
    series = length * (1.0 - x / 2.0 + x * x / 6.0)
    return np.where(small, series, out)


def kernel(b: np.ndarray, z_lo: float, z_hi: float, z0: float, link: Link) -> np.ndarray:
    """K = int_{z_lo}^{z_hi} gamma g(z) exp(-j 2 b (z - z0)) dz, in 1/W.

    Integrated exactly piece by piece between amplifiers (App. C does the
    same sum over spans); g(z) = exp(-alpha (z - last amplifier position)).
    """
    b = np.asarray(b, dtype=np.float64)
    alpha, span = link.alpha, link.span_km
    kappa = alpha + 2j * b
    total = np.zeros(b.shape, dtype=np.complex128)
    a = z_lo
    while a < z_hi - 1e-12 * max(1.0, z_hi):
        span_start = np.floor(a / span + 1e-12) * span
        c = min(z_hi, span_start + span)
        total += (np.exp(-alpha * (a - span_start)) * np.exp(-2j * b * (a - z0))
                  * _one_minus_exp_over(kappa, c - a))
        a = c
    return link.gamma * total


def kernel_eq22(b: np.ndarray, step_km: float, n_sp: int, link: Link) -> np.ndarray:
    """Eq. (22): symmetric step of n_sp whole spans, NLPR in the middle."""
    a = link.alpha / 2.0
    b = np.asarray(b, dtype=np.float64)
    lsp = step_km / n_sp
    ab = a + 1j * b
    # sin(bL) / sin(bL/n_sp), whose b -> 0 limit is n_sp
    small = np.abs(b * lsp) < 1e-12
    ratio = np.where(small, float(n_sp),
                     np.sin(b * step_km) / np.where(small, 1.0, np.sin(b * lsp)))
    return link.gamma * np.exp(-a * lsp) * np.sinh(ab * lsp) / ab * ratio


def subband_centres(n_sb: int, sample_rate: float) -> np.ndarray:
    """f_i = -R/2 + (i + 1/2) R', R' = R / N_sb (equal contiguous partition)."""
    rp = sample_rate / n_sb
    return -sample_rate / 2.0 + (np.arange(n_sb) + 0.5) * rp


def physical_coefficients(link: Link, n_sb: int, z_lo: float, z_hi: float, z0: float,
                          n_taps: int, grid_m: int | None = None) -> np.ndarray:
    """c_il[m] for one physical step [z_lo, z_hi] with NLPR at z0.

    Returns shape (N_sb, N_sb, n_taps); tap t <-> m = t - (n_taps - 1) / 2.
    """
    if n_taps % 2 != 1:
        raise ValueError("n_taps must be odd")
    grid_m = n_taps if grid_m is None else grid_m
    if grid_m % 2 != 1 or grid_m < n_taps:
        raise ValueError("grid must be odd and >= n_taps")
    nc = n_taps // 2
    rp = link.sample_rate / n_sb
    fc = subband_centres(n_sb, link.sample_rate)
    half = grid_m // 2
    pidx = np.arange(-half, half + 1)
    m = np.arange(-nc, nc + 1)
    # exp(j 2 pi m (p - q) / M), shape (taps, M, M)
    phase = np.exp(2j * np.pi * m[:, None, None] * (pidx[None, :, None] - pidx[None, None, :]) / grid_m)
    out = np.empty((n_sb, n_sb, n_taps))
    for i in range(n_sb):
        for l in range(n_sb):
            f_il = fc[l] - fc[i]
            mu = f_il + pidx * rp / grid_m
            nu = mu
            mu_g, nu_g = np.meshgrid(mu, nu, indexing="ij")   # K(mu_p, nu_q)
            b = 2.0 * np.pi ** 2 * link.beta2 * nu_g * (mu_g - nu_g)
            k = kernel(b, z_lo, z_hi, z0, link)
            c = (phase * k[None]).sum(axis=(1, 2)) / grid_m ** 2
            out[i, l] = c.real
    return out


def dbp_coefficients(link: Link, n_sb: int, n_steps: int, rho: float, n_taps: int,
                     grid_m: int | None = None) -> np.ndarray:
    """Applied DBP tensor C[s][i][l][tap], shape (N_st, N_sb, N_sb, n_taps)."""
    step = link.length_km / n_steps
    out = np.empty((n_steps, n_sb, n_sb, n_taps))
    for s in range(n_steps):
        j = n_steps - s                       # physical step (1-based)
        z_lo = (j - 1) * step
        c = physical_coefficients(link, n_sb, z_lo, z_lo + step, z_lo + rho * step,
                                  n_taps, grid_m)
        xpm = np.full((n_sb, n_sb), 1.5)
        np.fill_diagonal(xpm, 1.0)
        out[s] = -xpm[:, :, None] * c
    return out


def effective_length(link: Link, z_lo: float, z_hi: float) -> float:
    """int g(z) dz over [z_lo, z_hi] (K at b = 0, divided by gamma)."""
    return float(kernel(np.zeros(1), z_lo, z_hi, 0.0, link)[0].real / link.gamma)
