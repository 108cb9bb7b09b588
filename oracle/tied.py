"""FP64 oracle of the tied coefficient parametrisation used by the paper's
coefficient fitting (Sec. III-B, assumptions (i)-(iii); eqs. (23)-(25)).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path.

Parameters: one row c_h of n_taps applied coefficients (rad/W, DBP sign and
3/2 cross-band factor included, tap t <-> m = t - Nc) per subband distance
h = 0 .. N_sb - 1, and one weight w_s per step s.  The applied tensor is

    C_s[i][l][m] = w_s c_{l-i}[m]     for l >= i   (eq. (23): only l - i matters)
    C_s[i][l][m] = w_s c_{i-l}[-m]    for l <  i   (eq. (24))
    c_0[m] = c_0[-m]                                (eq. (25))

so of row 0 only the taps m >= 0 are parameters (the others are ignored and
get a zero gradient).  With per-distance half lengths Nc(h) (assumption
(iii)), taps with |m| > Nc(h) are zero.

Step weights (assumption (i)): the same coefficients in every step, rescaled
in proportion to the signal power at the step input.  For steps that cover
equal parts of a span that power is proportional to the power integrated over
the step (the effective length), which also covers steps spanning several
amplifiers; w_s = L_eff(step s) / mean over steps.  Backpropagation step s
(0-based) undoes physical step N_st - 1 - s.
"""
from __future__ import annotations

import math

import numpy as np

from .coeffs import Link, effective_length


def step_weights(link: Link, n_steps: int) -> np.ndarray:
    """w_s for s = 0 .. n_steps - 1 in backpropagation order, mean 1."""
    step = link.length_km / n_steps
    leff = np.empty(n_steps)
    for s in range(n_steps):
        j = n_steps - 1 - s                      # physical step, 0-based
        leff[s] = effective_length(link, j * step, (j + 1) * step)
    return leff / leff.mean()


def tied_half_taps(link: Link, n_sb: int, n_steps: int, n_taps: int) -> np.ndarray:
    """Nc(h) of assumption (iii): 2 Nc(h) + 1 is the odd integer nearest to
    pi L |beta2| R'^2 (h + 1), L the step length and R' = R / N_sb the
    subband sampling rate (n R in the paper's notation), capped at n_taps."""
    step = link.length_km / n_steps
    rp = link.sample_rate / n_sb
    out = np.empty(n_sb, dtype=np.int64)
    for h in range(n_sb):
        x = math.pi * step * abs(link.beta2) * rp * rp * (h + 1)
        out[h] = min(n_taps // 2, max(0, int(math.floor((x - 1.0) / 2.0 + 0.5))))
    return out


def _source(i: int, l: int, t: int, nc: int, half: np.ndarray):
    """(h, tap) of the parameter that C[.][i][l][t] reads, or None for a zero."""
    h = abs(l - i)
    m = t - nc
    if l < i:
        m = -m
    if h == 0:
        m = abs(m)
    if abs(m) > half[h]:
        return None
    return h, m + nc


def expand(params: np.ndarray, weights: np.ndarray, half_taps=None) -> np.ndarray:
    """C[s][i][l][t] from params [n_sb][n_taps] and weights [n_steps]."""
    params = np.asarray(params, dtype=np.float64)
    n_sb, n_taps = params.shape
    nc = n_taps // 2
    half = np.full(n_sb, nc) if half_taps is None else np.asarray(half_taps)
    out = np.zeros((len(weights), n_sb, n_sb, n_taps))
    for s, w in enumerate(weights):
        for i in range(n_sb):
            for l in range(n_sb):
                for t in range(n_taps):
                    src = _source(i, l, t, nc, half)
                    if src is not None:
                        out[s, i, l, t] = w * params[src]
    return out


def expand_adjoint(grad_c: np.ndarray, weights: np.ndarray, half_taps=None) -> np.ndarray:
    """dL/dparams from dL/dC: every entry of C adds w_s dL/dC to the
    parameter it reads."""
    grad_c = np.asarray(grad_c, dtype=np.float64)
    n_steps, n_sb, _, n_taps = grad_c.shape
    nc = n_taps // 2
    half = np.full(n_sb, nc) if half_taps is None else np.asarray(half_taps)
    out = np.zeros((n_sb, n_taps))
    for s in range(n_steps):
        for i in range(n_sb):
            for l in range(n_sb):
                for t in range(n_taps):
                    src = _source(i, l, t, nc, half)
                    if src is not None:
                        out[src] += weights[s] * grad_c[s, i, l, t]
    return out


def ssfm_start(link: Link, n_sb: int, n_steps: int, n_taps: int) -> np.ndarray:
    """Starting point of the fit (Sec. III-B): all zeros except the central
    coefficient of c_0, the mean nonlinear phase rotation per unit power of a
    step, gamma L_eff, with the backpropagation sign."""
    step = link.length_km / n_steps
    leff = np.mean([effective_length(link, j * step, (j + 1) * step) for j in range(n_steps)])
    p = np.zeros((n_sb, n_taps))
    p[0, n_taps // 2] = -link.gamma * leff
    return p
