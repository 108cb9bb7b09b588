"""Complexity model of Sec. III-D: real multiplications (RM) and real
additions (RA) per 2D symbol.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.

* CB-ESSFM (frequency-domain NLPR), eqs. (28)-(29):
  the FFT, GVD and NLPR counts of a block of N 4D samples, per output 2D
  symbol (n samples per symbol, N - N_ov kept samples, two polarisations).
* Single-band ESSFM with a time-domain NLPR of 2 Nc + 1 coefficients,
  eqs. (30)-(31); the SSFM and the OSSFM are Nc = 0; EDC is one dispersion
  step (no NLPR): N_st = 0.
"""
from __future__ import annotations

import math


def cb_essfm(n_sps: float, n: int, n_ov: int, n_st: int, n_sb: int):
    """(RM, RA) per 2D symbol of the CB-ESSFM, eqs. (28)-(29)."""
    lead = n_sps / 2.0 * n / (n - n_ov)
    lg = math.log2(n / n_sb)
    tail = (20.0 * n_sb * n_st + 16.0) / n
    rm = (5 * n_st + 4) * lg + n_st * (3 * n_sb + 1) / 2.0 + 4 * math.log2(n_sb) - 6 + tail
    ra = (15 * n_st + 12) * lg + n_st * (5 * n_sb - 1) / 2.0 + 12 * math.log2(n_sb) - 6 + tail
    return lead * rm, lead * ra


def essfm_time(n_sps: float, n: int, n_ov: int, n_st: int, n_c: int):
    """(RM, RA) per 2D symbol of the time-domain single-band ESSFM, eqs.
    (30)-(31); SSFM / OSSFM with n_c = 0, EDC with n_st = 0."""
    lead = n_sps / 2.0 * n / (n - n_ov)
    lg = math.log2(n)
    rm = (n_st + 1) * (4 * lg - 6 + 16.0 / n) + n_st * (11 + n_c)
    ra = (n_st + 1) * (12 * lg - 6 + 16.0 / n) + n_st * (11 + 2 * n_c)
    return lead * rm, lead * ra
