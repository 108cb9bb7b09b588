"""Tied coefficients and the paper's sequential coefficient fit (Sec. III-B).

The paper fits a reduced set of coefficients:

(i)   the same coefficients in every step, rescaled by the step's signal
      power (weights w_s, ``step_weights``);
(ii)  the symmetries of eqs. (23)-(25): one row c_h per subband distance h,
      mirrored below the diagonal, c_0 even;
(iii) 2 Nc(h) + 1 taps for distance h, about pi L beta2 R'^2 (h + 1)
      (``tied_half_taps``).

``tie`` maps the rows [n_sb][n_taps] to the applied tensor
[steps][n_sb][n_sb][n_taps] with the library's ``cbessfm_tie_expand`` kernel;
its gradient is ``cbessfm_tie_reduce``.  ``fit_tied`` runs the paper's
protocol: start from the SSFM (only the central tap of c_0, the mean
nonlinear phase per watt of a step), then fit c_0, c_1, ... one at a time,
each with the earlier rows fixed and the later ones zero.  The paper uses a
trust-region least-squares solver with finite-difference gradients; here each
row is fitted by Adam on the exact gradient (the library's adjoint followed
by ``cbessfm_tie_reduce``).  ``sweep_split_ratio`` and ``sweep_subbands`` give
the SNR-versus-rho and SNR-versus-N_sb curves of Sec. IV-B on held-out data.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import check, lib
from .autograd import cbessfm
from .plan import LinkSpec, Plan, _stream_ptr, analytic_coeffs
from .train import SymbolReceiver, adam_loop, phase_aligned_mse, plan_check_fn, snr_db

def step_weights(link: LinkSpec, steps: int):
    """(w [steps] float64 with mean 1, mean effective step length in km)."""
    w = np.empty(int(steps), dtype=np.float64)
    mean = ctypes.c_double()
    lk = link.c()
    check(lib.cbessfm_step_weights(ctypes.byref(lk), int(steps), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(mean)), "cbessfm_step_weights")
    return w, mean.value


def tied_half_taps(link: LinkSpec, n_sb: int, steps: int, n_taps: int) -> np.ndarray:
    """Nc(h) for h = 0 .. n_sb - 1 (assumption (iii)), capped at n_taps // 2."""
    out = np.empty(int(n_sb), dtype=np.int32)
    lk = link.c()
    check(lib.cbessfm_tied_half_taps(ctypes.byref(lk), int(n_sb), int(steps), int(n_taps),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "cbessfm_tied_half_taps")
    return out


def ssfm_start(link: LinkSpec, n_sb: int, steps: int, n_taps: int) -> np.ndarray:
    """Rows [n_sb][n_taps] of the SSFM starting point: zeros but the central
    tap of c_0, minus gamma times the mean effective step length."""
    _, leff = step_weights(link, steps)
    gamma = link.gamma_w_km * (8.0 / 9.0 if link.manakov_8_9 else 1.0)
    p = np.zeros((int(n_sb), int(n_taps)), dtype=np.float64)
    p[0, int(n_taps) // 2] = -gamma * leff
    return p


def analytic_rows(link: LinkSpec, n_sb: int, steps: int, rho: float, n_taps: int) -> np.ndarray:
    """Rows c_h of the analytic coefficients (Sec. II-D), for starting the fit
    there instead of at the SSFM: row h is the analytic C[0][0][h] of the
    first step divided by its weight.  For steps that cover equal parts of a
    span the analytic tensor is exactly the expansion of these rows."""
    c = analytic_coeffs(link, n_sb, steps, rho, n_taps)
    w, _ = step_weights(link, steps)
    return c[0, 0] / w[0]


def _half_array(half_taps, n_sb):
    if half_taps is None:
        return None
    h = np.ascontiguousarray(np.asarray(half_taps, dtype=np.int32))
    if h.shape != (n_sb,):
        raise ValueError("half_taps must have one entry per subband distance")
    return h


def _half_ptr(h):
    return None if h is None else h.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def tie_expand(params: torch.Tensor, weights: torch.Tensor, half_taps=None, stream=None) -> torch.Tensor:
    """Applied tensor [steps][n_sb][n_sb][n_taps] from rows [n_sb][n_taps] (no autograd)."""
    _check_dev(params, weights)
    n_sb, n_taps = params.shape
    steps = weights.numel()
    h = _half_array(half_taps, n_sb)
    out = torch.empty((steps, n_sb, n_sb, n_taps), dtype=torch.float32, device=params.device)
    check(lib.cbessfm_tie_expand(ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(weights.data_ptr()), steps,
                                 n_sb, n_taps, _half_ptr(h), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
          "cbessfm_tie_expand")
    return out


def tie_reduce(grad_c: torch.Tensor, weights: torch.Tensor, half_taps=None, stream=None) -> torch.Tensor:
    """Gradient with respect to the rows from the gradient with respect to the
    applied tensor (the transpose of ``tie_expand``)."""
    _check_dev(grad_c, weights)
    steps, n_sb, _, n_taps = grad_c.shape
    if weights.numel() != steps:
        raise ValueError("one weight per step")
    h = _half_array(half_taps, n_sb)
    out = torch.empty((n_sb, n_taps), dtype=torch.float32, device=grad_c.device)
    check(lib.cbessfm_tie_reduce(ctypes.c_void_p(grad_c.data_ptr()), ctypes.c_void_p(weights.data_ptr()), steps,
                                 n_sb, n_taps, _half_ptr(h), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
          "cbessfm_tie_reduce")
    return out


def _check_dev(*ts):
    for t in ts:
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("tied coefficients take contiguous float32 CUDA tensors")


class TieFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, weights, half_taps):
        ctx.half_taps = half_taps
        ctx.save_for_backward(weights)
        return tie_expand(params.detach().contiguous(), weights.detach().contiguous(), half_taps)

    @staticmethod
    def backward(ctx, grad_c):
        (weights,) = ctx.saved_tensors
        return tie_reduce(grad_c.contiguous(), weights, ctx.half_taps), None, None


def tie(params: torch.Tensor, weights: torch.Tensor, half_taps=None) -> torch.Tensor:
    """Differentiable map rows [n_sb][n_taps] -> applied tensor [steps][n_sb][n_sb][n_taps]."""
    return TieFunction.apply(params, weights, half_taps)


def fit_tied(plan: Plan, link: LinkSpec, fields: torch.Tensor, symbols: torch.Tensor, receiver: SymbolReceiver,
             rho: float, iters_per_row: int = 100, lr: float = 2e-2, params0=None, half_taps="rule",
             rows=None, checkpoint_every: int = 1, graph: bool = False, warmup: int = 3):
    """The sequential fit of Sec. III-B.  Returns (rows [n_sb][n_taps] float32
    on the device, {h: losses of row h's iterations}).

    params0: starting rows (default: ``ssfm_start``); while row h is fitted,
    the rows fitted before it keep their fitted values and the rows still to
    be fitted are held at zero (each then starts from params0).  half_taps:
    "rule" for assumption (iii), None for the plan's full length, or Nc(h)
    per distance.  rows: which distances to fit, in order (default all)."""
    n_sb, steps, n_taps = plan.n_sb, plan.steps, plan.n_taps
    dev = fields.device
    w_np, _ = step_weights(link, steps)
    weights = torch.tensor(w_np, dtype=torch.float32, device=dev)
    if isinstance(half_taps, str):
        if half_taps != "rule":
            raise ValueError("half_taps must be 'rule', None or one entry per distance")
        half_taps = tied_half_taps(link, n_sb, steps, n_taps)
    half = _half_array(half_taps, n_sb)
    start = ssfm_start(link, n_sb, steps, n_taps) if params0 is None else np.asarray(params0, dtype=np.float64)
    if start.shape != (n_sb, n_taps):
        raise ValueError("params0 must be [n_sb][n_taps]")
    rows = list(range(n_sb)) if rows is None else [int(h) for h in rows]
    fitted = torch.tensor(start, dtype=torch.float32, device=dev)
    scale = float(max(abs(start).max(), 1e-12))
    rho_t = torch.tensor(float(rho), dtype=torch.float32, device=dev)
    losses = {}
    for k, h in enumerate(rows):
        base = fitted.clone()
        for later in rows[k + 1:]:
            base[later] = 0.0           # rows not fitted yet are held at zero
        u = (base[h] / scale).clone().requires_grad_(True)
        head, tail = base[:h].clone(), base[h + 1:].clone()

        def loss_fn(u=u, head=head, tail=tail):
            rows_t = torch.cat([head, (u * scale)[None], tail])
            c = tie(rows_t, weights, half)
            return phase_aligned_mse(receiver(cbessfm(fields, c, rho_t, plan, checkpoint_every)), symbols)

        losses[h] = adam_loop([u], loss_fn, iters_per_row, lr, graph=graph, warmup=warmup, device=dev,
                              check=plan_check_fn(plan))
        with torch.no_grad():
            fitted[h] = u.detach() * scale
    return fitted, losses


def tied_coeffs(rows: torch.Tensor, link: LinkSpec, steps: int, half_taps="rule") -> torch.Tensor:
    """Applied tensor of fitted rows (as ``fit_tied`` built it)."""
    n_sb, n_taps = rows.shape
    w_np, _ = step_weights(link, steps)
    if isinstance(half_taps, str):
        half_taps = tied_half_taps(link, n_sb, steps, n_taps)
    return tie_expand(rows.contiguous(), torch.tensor(w_np, dtype=torch.float32, device=rows.device), half_taps)


def sweep_split_ratio(plan: Plan, link: LinkSpec, train, test, receiver: SymbolReceiver, rhos,
                      **fit_args):
    """SNR versus rho (Sec. III-C, IV-B): for each rho the full sequential fit on
    ``train`` = (fields, symbols), the SNR on ``test``.  Returns a list of
    dicts (rho, snr_train_db, snr_test_db, ssfm_test_db)."""
    out = []
    for r in rhos:
        rows, _ = fit_tied(plan, link, train[0], train[1], receiver, float(r), **fit_args)
        c = tied_coeffs(rows, link, plan.steps, fit_args.get("half_taps", "rule"))
        c0 = tied_coeffs(torch.tensor(ssfm_start(link, plan.n_sb, plan.steps, plan.n_taps), dtype=torch.float32,
                                      device=rows.device), link, plan.steps, None)
        out.append(dict(rho=float(r), snr_train_db=snr_db(plan, c, r, train[0], train[1], receiver),
                        snr_test_db=snr_db(plan, c, r, test[0], test[1], receiver),
                        ssfm_test_db=snr_db(plan, c0, r, test[0], test[1], receiver)))
    return out


def sweep_subbands(make_plan, link: LinkSpec, train, test, receiver: SymbolReceiver, n_sbs, rho: float,
                   **fit_args):
    """SNR versus N_sb (Sec. IV-B, Fig. "SNR_vs_Nbands"): ``make_plan(n_sb)``
    returns a plan for each subband count; the full sequential fit on
    ``train``, the SNR on ``test``.  Returns a list of dicts."""
    out = []
    for n in n_sbs:
        plan = make_plan(int(n))
        try:
            rows, _ = fit_tied(plan, link, train[0], train[1], receiver, rho, **fit_args)
            c = tied_coeffs(rows, link, plan.steps, fit_args.get("half_taps", "rule"))
            out.append(dict(n_sb=int(n), block_sb=plan.block_sb, n_taps=plan.n_taps,
                            snr_train_db=snr_db(plan, c, rho, train[0], train[1], receiver),
                            snr_test_db=snr_db(plan, c, rho, test[0], test[1], receiver)))
        finally:
            plan.close()
    return out
