"""FP64 CPU oracle of the CB-ESSFM digital-backpropagation forward map.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path and must never be used as a fallback for it.

What it computes (Sec. III-A, Figs. "scheme_OeS", "scheme_CB-ESSFM",
"scheme_NLPR"; Sec. III-C for the asymmetric split; eqs. (2)-(5) and (15)):

For every batch instance and every overlap-and-save block b:

1. gather ``u_p[k] = field[p][(b*(N-N_ov) - N_ov/2 + k) mod T]`` (Sec. III-A,
   overlap-and-save framing; circular boundary, or zeros outside [0, T)).
2. ``U_p = DFT_N(u_p)`` with kernel exp(-j 2 pi q n / N) (Fourier convention of
   the footnote to eq. (2)); bin q in [-N/2, N/2) has frequency q R / N.  The
   N bins, in increasing frequency, are cut into N_sb contiguous subbands of
   N' = N / N_sb bins (the DEMUX of Fig. "scheme_CB-ESSFM").
3. for s = 1..N_st:
     a. GVD compensation h = exp(+j 2 pi^2 beta2 dz f^2) at the absolute bin
        frequency f (Sec. III-A); dz = (1 - rho) L for s = 1, else L (Sec. III-C).
     b. subband time samples v = (1/N) sum_delta V[delta] exp(+j 2 pi delta k / N'),
        i.e. the lowpass-equivalent samples at rate R' = R / N_sb (App. B).
     c. intensity p_i = |x_i|^2 + |y_i|^2 (Sec. II-C).
     d. theta_i[k] = sum_l sum_{m=-Nc}^{Nc} C_s[i, l, m] p_l[(k - m) mod N']
        (eq. (15); the 3/2 cross-band factor and the backpropagation sign are
        part of C; the filter is circular over the N' samples of the block).
     e. v *= exp(-j theta_i)  (eq. (3)).
     f. V = N_sb * DFT_N'(v).
4. final GVD with dz = rho L (Sec. III-C).
5. MUX, ``u_p = IDFT_N(U_p) / N``, keep samples [N_ov/2, N - N_ov/2).

Readings of points the paper leaves open are documented with the design (subband
placement and scaling, DBP sign, circular FIR, framing, boundary).
"""
from __future__ import annotations

from dataclasses import dataclass, field as dc_field
from typing import Callable, Optional

import numpy as np


# ---------------------------------------------------------------------------
# transforms
# ---------------------------------------------------------------------------

def dft_bruteforce(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Plain O(N^2) DFT: X[q] = sum_n x[n] exp(-+ j 2 pi q n / N), unnormalised.

    The sign follows the Fourier convention of the footnote to eq. (2);
    ``inverse`` flips it (no 1/N factor).
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    idx = np.arange(n)
    sign = 1.0 if inverse else -1.0
    w = np.exp(sign * 2j * np.pi * np.outer(idx, idx) / n)
    return x @ w.T


def _dft_numpy(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    if inverse:
        return np.fft.ifft(x, axis=-1) * x.shape[-1]
    return np.fft.fft(x, axis=-1)


# ---------------------------------------------------------------------------
# plan
# ---------------------------------------------------------------------------

@dataclass
class OraclePlan:
    """Parameters of one CB-ESSFM instance.

    beta2_s2_km   : fibre dispersion beta2 in s^2/km (negative for SMF)
    sample_rate   : full-field sampling rate R in Hz
    step_km       : step length L in km (uniform steps, Sec. IV-A)
    n_steps       : N_st >= 1
    rho           : splitting ratio in [0, 1] (Sec. III-C)
    n_sb          : number of subbands N_sb
    n_block       : block length N (full-field samples), divisible by n_sb
    n_overlap     : overlap N_ov (even, < N)
    coeffs        : applied coefficients C[s][i][l][tap], shape
                    (N_st, N_sb, N_sb, 2 Nc + 1), tap index t <-> m = t - Nc
    boundary      : "circular" (default) or "zero"
    nlpr          : "averaged" (default): one phase per subband from the total
                    intensity, eq. (15); "dual": separate phases for the two
                    polarisations, eqs. (20)-(21)
    gvd_km        : optional lengths (km) of the N_st + 1 dispersion segments
                    (before the first NLPR, between consecutive NLPRs, after
                    the last one): a free step-size distribution and split
                    ratio per step (Sec. III-C, V).  Default: (1 - rho) L,
                    L, ..., L, rho L.
    """

    beta2_s2_km: float
    sample_rate: float
    step_km: float
    n_steps: int
    rho: float
    n_sb: int
    n_block: int
    n_overlap: int
    coeffs: np.ndarray
    boundary: str = "circular"
    nlpr: str = "averaged"
    gvd_km: Optional[np.ndarray] = None
    dft: Callable[..., np.ndarray] = dc_field(default=_dft_numpy, repr=False)

    def __post_init__(self) -> None:
        c = np.asarray(self.coeffs, dtype=np.float64)
        if c.ndim != 4 or c.shape[0] != self.n_steps or c.shape[1] != self.n_sb \
                or c.shape[2] != self.n_sb or c.shape[3] % 2 != 1:
            raise ValueError(f"coeffs shape {c.shape} does not match plan")
        if self.n_block % self.n_sb:
            raise ValueError("N must be divisible by N_sb")
        if self.n_overlap % 2 or not (0 <= self.n_overlap < self.n_block):
            raise ValueError("N_ov must be even and in [0, N)")
        if not (0.0 <= self.rho <= 1.0):
            raise ValueError("rho must lie in [0, 1]")
        if self.boundary not in ("circular", "zero"):
            raise ValueError("boundary must be 'circular' or 'zero'")
        if self.nlpr not in ("averaged", "dual"):
            raise ValueError("nlpr must be 'averaged' or 'dual'")
        if self.gvd_km is not None:
            g = np.asarray(self.gvd_km, dtype=np.float64)
            if g.shape != (self.n_steps + 1,) or np.any(g < 0):
                raise ValueError("gvd_km must hold N_st + 1 non-negative lengths")
            self.gvd_km = g
        self.coeffs = c

    @property
    def n_sub(self) -> int:
        """N' = N / N_sb samples per subband."""
        return self.n_block // self.n_sb

    @property
    def hop(self) -> int:
        return self.n_block - self.n_overlap

    def n_blocks(self, t_len: int) -> int:
        return -(-t_len // self.hop)

    def gvd_lengths(self) -> np.ndarray:
        """Lengths of the N_st + 1 dispersion segments in km."""
        if self.gvd_km is not None:
            return self.gvd_km
        g = np.full(self.n_steps + 1, self.step_km)
        g[0] = (1.0 - self.rho) * self.step_km
        g[-1] = self.rho * self.step_km
        return g


# ---------------------------------------------------------------------------
# building blocks (each one a step of Sec. III-A)
# ---------------------------------------------------------------------------

def bin_frequencies(plan: OraclePlan) -> np.ndarray:
    """Absolute frequency (Hz) of every bin of every subband, shape (N_sb, N').

    Subband i holds bins q_i + delta, q_i = -N/2 + i N' + N'/2,
    delta in [-N'/2, N'/2), stored in natural DFT order (delta mod N').
    """
    n, nsub = plan.n_block, plan.n_sub
    delta = np.fft.fftfreq(nsub, d=1.0 / nsub)  # 0..N'/2-1, -N'/2..-1
    q = np.empty((plan.n_sb, nsub))
    for i in range(plan.n_sb):
        q_i = -n // 2 + i * nsub + nsub // 2
        q[i] = q_i + delta
    return q * plan.sample_rate / n


def gvd_filter(plan: OraclePlan, dz_km: float) -> np.ndarray:
    """h = exp(+j 2 pi^2 beta2 dz f^2) for every subband bin (Sec. III-A)."""
    f = bin_frequencies(plan)
    return np.exp(1j * 2.0 * np.pi ** 2 * plan.beta2_s2_km * dz_km * f * f)


def demux(u_spec: np.ndarray, plan: OraclePlan) -> np.ndarray:
    """Full-field spectrum (2, N) in DFT order -> subband spectra (N_sb, 2, N')."""
    n, nsub = plan.n_block, plan.n_sub
    delta = np.fft.fftfreq(nsub, d=1.0 / nsub).astype(np.int64)
    out = np.empty((plan.n_sb, 2, nsub), dtype=np.complex128)
    for i in range(plan.n_sb):
        q = (-n // 2 + i * nsub + nsub // 2 + delta) % n
        out[i] = u_spec[:, q]
    return out


def mux(v_spec: np.ndarray, plan: OraclePlan) -> np.ndarray:
    """Inverse of :func:`demux`: subband spectra -> full-field spectrum (2, N)."""
    n, nsub = plan.n_block, plan.n_sub
    delta = np.fft.fftfreq(nsub, d=1.0 / nsub).astype(np.int64)
    out = np.zeros((2, n), dtype=np.complex128)
    for i in range(plan.n_sb):
        q = (-n // 2 + i * nsub + nsub // 2 + delta) % n
        out[:, q] = v_spec[i]
    return out


def coupled_fir(p: np.ndarray, c_step: np.ndarray) -> np.ndarray:
    """theta_i[k] = sum_l sum_m C[i, l, m] p_l[(k - m) mod N'] (eq. (15)).

    p: (N_sb, N') intensities; c_step: (N_sb, N_sb, 2 Nc + 1).
    Written as the literal double sum over l and m with circular shifts.
    """
    nsb, nsub = p.shape
    ntap = c_step.shape[-1]
    nc = ntap // 2
    theta = np.zeros((nsb, nsub))
    for i in range(nsb):
        for l in range(nsb):
            for t in range(ntap):
                m = t - nc
                # p_l[(k - m) mod N'] for all k  ==  roll p_l right by m
                theta[i] += c_step[i, l, t] * np.roll(p[l], m)
    return theta


def dual_pol_phases(px: np.ndarray, py: np.ndarray, c_step: np.ndarray) -> np.ndarray:
    """theta^x and theta^y of eqs. (20)-(21), shape (N_sb, 2, N').

    px, py: (N_sb, N') intensities |x_l|^2, |y_l|^2.  The applied tensor C
    carries the 3/2 cross-band factor of eq. (15) (C_il = (3/2) c_il for
    l != i), so the paper's c_il is (2/3) C_il: the same subband acts through
    c_ii on |x_i|^2 + |y_i|^2, another subband through c_il on 2 |x_l|^2 +
    |y_l|^2 (co-polarised twice the orthogonal) for theta^x and on
    |x_l|^2 + 2 |y_l|^2 for theta^y.  Same tap convention as ``coupled_fir``.
    """
    nsb = px.shape[0]
    own = np.zeros_like(c_step)
    cross = np.zeros_like(c_step)
    for i in range(nsb):
        for l in range(nsb):
            if i == l:
                own[i, l] = c_step[i, l]
            else:
                cross[i, l] = c_step[i, l] * (2.0 / 3.0)
    spm = coupled_fir(px + py, own)
    th_x = spm + coupled_fir(2.0 * px + py, cross)
    th_y = spm + coupled_fir(px + 2.0 * py, cross)
    return np.stack([th_x, th_y], axis=1)


def process_block(u: np.ndarray, plan: OraclePlan) -> np.ndarray:
    """Run steps 2-5 on one block u of shape (2, N); returns (2, N)."""
    dft = plan.dft
    n, nsb = plan.n_block, plan.n_sb
    seg = plan.gvd_lengths()                          # (1 - rho) L, L, ..., rho L by default
    spec = dft(u)                                     # 2.  U_p = DFT_N(u_p)
    v_spec = demux(spec, plan)                        #     DEMUX
    for s in range(plan.n_steps):                     # 3.
        h = gvd_filter(plan, seg[s])
        v_spec = v_spec * h[:, None, :]               # 3a. GVD
        v = dft(v_spec, inverse=True) / n             # 3b. subband samples
        if plan.nlpr == "dual":                       # 3c-3e, eqs. (20)-(21)
            theta = dual_pol_phases(np.abs(v[:, 0]) ** 2, np.abs(v[:, 1]) ** 2, plan.coeffs[s])
            v = v * np.exp(-1j * theta)
        else:
            p = np.abs(v[:, 0]) ** 2 + np.abs(v[:, 1]) ** 2   # 3c. intensity
            theta = coupled_fir(p, plan.coeffs[s])        # 3d. coupled FIR
            v = v * np.exp(-1j * theta)[:, None, :]       # 3e. rotation
        v_spec = nsb * dft(v)                         # 3f. back to frequency
    v_spec = v_spec * gvd_filter(plan, seg[-1])[:, None, :]   # 4.  final GVD
    return dft(mux(v_spec, plan), inverse=True) / n   # 5.  MUX + IDFT_N


def gather_block(field: np.ndarray, plan: OraclePlan, b: int) -> np.ndarray:
    """Input samples of block b: field[:, (b hop - N_ov/2 + k)], k < N."""
    t_len = field.shape[-1]
    pos = b * plan.hop - plan.n_overlap // 2 + np.arange(plan.n_block)
    if plan.boundary == "circular":
        return field[:, pos % t_len]
    out = np.zeros((2, plan.n_block), dtype=np.complex128)
    ok = (pos >= 0) & (pos < t_len)
    out[:, ok] = field[:, pos[ok]]
    return out


def run(field_in: np.ndarray, plan: OraclePlan) -> np.ndarray:
    """CB-ESSFM over a field of shape (2, T) or (B, 2, T); returns same shape."""
    x = np.asarray(field_in, dtype=np.complex128)
    squeeze = x.ndim == 2
    if squeeze:
        x = x[None]
    if x.ndim != 3 or x.shape[1] != 2:
        raise ValueError("field must have shape (2, T) or (B, 2, T)")
    bsz, _, t_len = x.shape
    out = np.zeros_like(x)
    keep_lo, keep_hi = plan.n_overlap // 2, plan.n_block - plan.n_overlap // 2
    for bi in range(bsz):
        for b in range(plan.n_blocks(t_len)):
            y = process_block(gather_block(x[bi], plan, b), plan)
            start = b * plan.hop                      # output of sample keep_lo
            n_keep = min(keep_hi - keep_lo, t_len - start)
            out[bi, :, start:start + n_keep] = y[:, keep_lo:keep_lo + n_keep]
    return out[0] if squeeze else out


def run_blocks(field_in: np.ndarray, plan: OraclePlan, blocks) -> dict:
    """Outputs of selected blocks only: {b: (2, hop) kept samples}.

    Used for sampled parity at sizes where the whole field would take too
    long on the CPU; identical arithmetic to :func:`run`.
    """
    x = np.asarray(field_in, dtype=np.complex128)
    t_len = x.shape[-1]
    keep_lo = plan.n_overlap // 2
    res = {}
    for b in blocks:
        y = process_block(gather_block(x, plan, b), plan)
        start = b * plan.hop
        n_keep = min(plan.hop, t_len - start)
        res[b] = y[:, keep_lo:keep_lo + n_keep]
    return res


def zero_coeffs(n_steps: int, n_sb: int, n_taps: int) -> np.ndarray:
    return np.zeros((n_steps, n_sb, n_sb, n_taps))
