"""Comparison methods on the same kernels (Sec. IV-B) and the complexity model
(Sec. III-D).

Every method is a configuration of the CB-ESSFM plan:

* EDC: dispersion only, one step with zero coefficients;
* SSFM: one subband, one coefficient per step, the nonlinear phase per watt
  of the step (gamma L_eff, with the backpropagation sign), rho = 0.5;
* OSSFM: the SSFM with that one coefficient fitted (Nc = 0);
* ESSFM: one subband, rho = 0.5, 2 Nc + 1 taps from rule (iii), fitted;
* CB-ESSFM: N_sb subbands, fitted rows, optimised rho;
* CB-ESSFM with free steps: the tied fit, then every step's coefficients and
  all dispersion segment lengths fitted jointly on the adjoint (Sec. V);
* ideal DBP: the SSFM with many steps per span.

Fits follow the tied protocol of Sec. III-B (``tied.fit_tied``) on training
fields; SNRs are measured on other fields.  Complexity (real multiplications
per 2D symbol) is the paper's model, ``complexity``: eqs. (28)-(29) for the
CB-ESSFM and eqs. (30)-(31) for the time-domain ESSFM, SSFM/OSSFM (Nc = 0)
and EDC (no step).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib
from .plan import LinkSpec, Plan, analytic_coeffs
from .tied import fit_tied, ssfm_start, tied_coeffs, tied_half_taps
from .train import SymbolReceiver, fit_steps, snr_db, snr_db_steps

CX_FREQ, CX_TIME = 0, 1


def complexity(kind: str, n_sps: float, block: int, overlap: int, steps: int, n_sb: int = 1, n_c: int = 0) -> dict:
    """{'rm', 'ra'} per 2D symbol.  kind: 'cb-essfm' (frequency-domain NLPR,
    eqs. (28)-(29)) or 'time' (time-domain single-band NLPR with 2 n_c + 1
    coefficients, eqs. (30)-(31); SSFM/OSSFM n_c = 0, EDC steps = 0)."""
    code = {"cb-essfm": CX_FREQ, "time": CX_TIME}[kind]
    rm, ra = ctypes.c_double(), ctypes.c_double()
    check(lib.cbessfm_complexity(code, float(n_sps), int(block), int(overlap), int(steps), int(n_sb), int(n_c),
                                 ctypes.byref(rm), ctypes.byref(ra)), "cbessfm_complexity")
    return {"rm": rm.value, "ra": ra.value}


def _zeros(steps, n_sb, n_taps):
    return np.zeros((steps, n_sb, n_sb, n_taps), dtype=np.float32)


def _plan(link, n_sb, block_sb, overlap, steps, rho, n_taps):
    return Plan(link, n_sb, block_sb, overlap, steps, rho, coeffs=_zeros(steps, n_sb, n_taps))


def run_method(method: str, link: LinkSpec, train, test, receiver: SymbolReceiver, *, steps: int = 1,
               n_sb: int = 1, block: int = 8192, overlap: int = 0, n_sps: float = 2.0, rho: float = 0.5,
               n_taps: int = 1, iters_per_row: int = 60, lr: float = 2e-2, graph: bool = True,
               free_iters: int = 150, free_lr: float = 2e-3) -> dict:
    """SNR (on ``test``) and complexity of one method; ``train`` / ``test`` are
    (fields (B, 2, T), symbols (B, 2, n)) device tensors.  ``block`` is the
    full-field block N."""
    block_sb = block // n_sb
    res = {"method": method, "steps": steps, "n_sb": n_sb, "rho": rho, "block": block, "overlap": overlap}
    if method == "edc":
        plan = _plan(link, 1, block, overlap, 1, 0.5, 1)
        c = torch.zeros((1, 1, 1, 1), device=test[0].device)
        res.update(snr_test_db=snr_db(plan, c, 0.5, test[0], test[1], receiver),
                   **complexity("time", n_sps, block, overlap, 0), steps=0)
        plan.close()
        return res
    if method in ("ssfm", "ideal"):
        plan = _plan(link, 1, block, overlap, steps, 0.5, 1)
        c = torch.tensor(analytic_coeffs(link, 1, steps, 0.5, 1, 1), dtype=torch.float32, device=test[0].device)
        res.update(snr_test_db=snr_db(plan, c, 0.5, test[0], test[1], receiver),
                   **complexity("time", n_sps, block, overlap, steps))
        plan.close()
        return res
    if method == "ossfm":
        n_sb, n_taps, half = 1, 1, None
        kind = ("time", 0)
    elif method == "essfm":
        n_sb, rho = 1, 0.5
        half = tied_half_taps(link, 1, steps, n_taps)
        kind = ("time", int(half[0]))
    elif method in ("cb-essfm", "cb-essfm-free"):
        half = tied_half_taps(link, n_sb, steps, n_taps)
        kind = ("cb-essfm", 0)
    else:
        raise ValueError(f"unknown method {method!r}")
    plan = _plan(link, n_sb, block // n_sb, overlap, steps, rho, n_taps)
    try:
        rows, losses = fit_tied(plan, link, train[0], train[1], receiver, rho, iters_per_row=iters_per_row,
                                lr=lr, half_taps=half, graph=graph)
        c = tied_coeffs(rows, link, steps, half)
        start = tied_coeffs(torch.tensor(ssfm_start(link, n_sb, steps, n_taps), dtype=torch.float32,
                                         device=rows.device), link, steps, None)
        res.update(snr_train_db=snr_db(plan, c, rho, train[0], train[1], receiver),
                   snr_test_db=snr_db(plan, c, rho, test[0], test[1], receiver),
                   snr_start_test_db=snr_db(plan, start, rho, test[0], test[1], receiver),
                   half_taps=[int(v) for v in (half if half is not None else [0])],
                   final_loss=[float(losses[h][-1]) for h in sorted(losses)])
        if kind[0] == "time":
            res.update(complexity("time", n_sps, block, overlap, steps, n_c=kind[1]))
        else:
            res.update(complexity("cb-essfm", n_sps, block, overlap, steps, n_sb=n_sb))
        if method == "cb-essfm-free":
            # then every step's coefficients and all dispersion segment lengths, jointly
            step_km = link.length_km / steps
            l0 = np.full(steps + 1, step_km)
            l0[0], l0[-1] = (1.0 - rho) * step_km, rho * step_km
            c_free, lengths, _ = fit_steps(plan, train[0], train[1], receiver, c, l0, iters=free_iters,
                                           lr=free_lr, graph=graph)
            res.update(snr_tied_test_db=res["snr_test_db"], snr_tied_train_db=res["snr_train_db"],
                       snr_train_db=snr_db_steps(plan, c_free, lengths, train[0], train[1], receiver),
                       snr_test_db=snr_db_steps(plan, c_free, lengths, test[0], test[1], receiver),
                       gvd_km=[float(v) for v in lengths.cpu().numpy()])
    finally:
        plan.close()
    return res
