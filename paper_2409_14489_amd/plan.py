"""Python face of libcbessfm: a CB-ESSFM plan bound to device tensors.

PyTorch supplies device memory and the current stream; every step of the
backpropagation runs in the library's HIP kernels (see ``include/cbessfm.h``
for the operation, Sec. III-A / III-C of the paper).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import FIR_MODES, Coeffs, Info, Link, Subbands, check, lib


@dataclass
class LinkSpec:
    """Fibre link (Sec. IV-A); fields follow ``cbessfm_link``."""
    alpha_db_km: float = 0.2
    beta2_ps2_km: float = -21.7
    gamma_w_km: float = 1.3
    span_km: float = 80.0
    n_spans: int = 1
    sample_rate_hz: float = 64e9
    manakov_8_9: bool = False

    def c(self) -> Link:
        return Link(self.alpha_db_km, self.beta2_ps2_km, self.gamma_w_km, self.span_km,
                    int(self.n_spans), self.sample_rate_hz, int(bool(self.manakov_8_9)))

    @property
    def length_km(self) -> float:
        return self.span_km * self.n_spans


_BOUNDARY = {"circular": 0, "zero": 1}


def _subbands(n_sb: int, block_sb: int, overlap: int, boundary: str, fir_mode: str = "auto") -> Subbands:
    if boundary not in _BOUNDARY:
        raise ValueError("boundary must be 'circular' or 'zero'")
    if fir_mode not in FIR_MODES:
        raise ValueError("fir_mode must be 'auto', 'time' or 'freq'")
    return Subbands(int(n_sb), int(block_sb), int(overlap), FIR_MODES[fir_mode], _BOUNDARY[boundary])


def _coeff_struct(coeffs, n_taps, grid_m):
    if coeffs is None:
        return Coeffs(int(n_taps), None, int(grid_m)), None
    host = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float32))
    ptr = host.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    return Coeffs(int(host.shape[-1]), ptr, int(grid_m)), host


def plan_check(link: LinkSpec, n_sb: int, block_sb: int, overlap: int, steps: int, split_ratio: float,
               n_taps: int, boundary: str = "circular", grid_m: int = 0, fir_mode: str = "auto") -> int:
    """Host-only validation (``cbessfm_plan_check``); returns the C error code."""
    lk, sb = link.c(), _subbands(n_sb, block_sb, overlap, boundary, fir_mode)
    co = Coeffs(int(n_taps), None, int(grid_m))
    return lib.cbessfm_plan_check(ctypes.byref(lk), ctypes.byref(sb), int(steps), float(split_ratio),
                                  ctypes.byref(co))


def analytic_coeffs(link: LinkSpec, n_sb: int, steps: int, split_ratio: float, n_taps: int,
                    grid_m: int = 0) -> np.ndarray:
    """Applied analytic coefficients [steps][n_sb][n_sb][n_taps] in FP64 (host)."""
    out = np.empty((steps, n_sb, n_sb, n_taps), dtype=np.float64)
    lk = link.c()
    sb = Subbands(int(n_sb), 256, 0, 0, 0)
    check(lib.cbessfm_analytic_coeffs(ctypes.byref(lk), ctypes.byref(sb), int(steps), float(split_ratio),
                                      int(n_taps), int(grid_m),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
          "cbessfm_analytic_coeffs")
    return out


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A CB-ESSFM plan on the current HIP device.

    coeffs: applied coefficients [steps][n_sb][n_sb][n_taps] (rad/W, 3/2 and
    DBP sign included), or None for the analytic ones (then ``n_taps`` is
    required).  fir_mode: "auto", "time" or "freq", how the forward evaluates
    the coupled filter (``cbessfm_subbands.fir_mode``).
    """

    def __init__(self, link: LinkSpec, n_sb: int, block_sb: int, overlap: int, steps: int,
                 split_ratio: float, coeffs=None, n_taps: int | None = None, grid_m: int = 0,
                 boundary: str = "circular", fir_mode: str = "auto"):
        if coeffs is None and n_taps is None:
            raise ValueError("give coeffs or n_taps")
        self.link = link
        self.n_sb, self.block_sb, self.overlap, self.steps = int(n_sb), int(block_sb), int(overlap), int(steps)
        self.boundary = boundary
        self.fir_mode = fir_mode
        lk, sb = link.c(), _subbands(n_sb, block_sb, overlap, boundary, fir_mode)
        co, keep = _coeff_struct(coeffs, n_taps, grid_m)
        self.n_taps = co.n_taps
        self.nlpr = "averaged"
        handle = ctypes.c_void_p()
        rc = lib.cbessfm_plan(ctypes.byref(handle), ctypes.byref(lk), ctypes.byref(sb), int(steps),
                              float(split_ratio), ctypes.byref(co))
        del keep
        check(rc, "cbessfm_plan")
        self._h = handle

    # -------------------------------------------------------------- geometry
    def info(self) -> Info:
        out = Info()
        check(lib.cbessfm_plan_info(self._h, ctypes.byref(out)), "cbessfm_plan_info")
        return out

    @property
    def block(self) -> int:
        return self.n_sb * self.block_sb

    @property
    def hop(self) -> int:
        return self.block - self.overlap

    def n_blocks(self, t_len: int) -> int:
        return -(-t_len // self.hop)

    # -------------------------------------------------------------- calls
    @staticmethod
    def _field(x: torch.Tensor) -> torch.Tensor:
        if not (x.is_cuda and x.dtype == torch.complex64):
            raise TypeError("field must be a complex64 CUDA tensor")
        if x.dim() not in (2, 3) or x.shape[-2] != 2:
            raise ValueError("field must have shape (2, T) or (B, 2, T)")
        return x.contiguous()

    def run(self, field_in: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        x = self._field(field_in)
        bsz = 1 if x.dim() == 2 else x.shape[0]
        t_len = x.shape[-1]
        if out is None:
            out = torch.empty_like(x)
        elif out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous():
            raise ValueError("out must be a contiguous complex64 tensor shaped like field_in")
        check(lib.cbessfm_run(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(t_len), int(bsz), _stream_ptr(stream)), "cbessfm_run")
        return out

    def set_coeffs(self, coeffs: torch.Tensor | None = None, rho: torch.Tensor | None = None, stream=None):
        """Device-side update of coefficients (float32 [steps][n_sb][n_sb][n_taps]) and/or rho (float32 scalar)."""
        cp = ctypes.c_void_p(0)
        rp = ctypes.c_void_p(0)
        if coeffs is not None:
            if not (coeffs.is_cuda and coeffs.dtype == torch.float32 and coeffs.is_contiguous()):
                raise TypeError("coeffs must be a contiguous float32 CUDA tensor")
            if tuple(coeffs.shape) != (self.steps, self.n_sb, self.n_sb, self.n_taps):
                raise ValueError("coeffs shape does not match the plan")
            cp = ctypes.c_void_p(coeffs.data_ptr())
        if rho is not None:
            if not (rho.is_cuda and rho.dtype == torch.float32 and rho.numel() == 1):
                raise TypeError("rho must be a one-element float32 CUDA tensor")
            rp = ctypes.c_void_p(rho.data_ptr())
        check(lib.cbessfm_set_coeffs(self._h, cp, rp, _stream_ptr(stream)), "cbessfm_set_coeffs")

    def set_nlpr(self, mode: str):
        """'averaged' (eq. (15), the default) or 'dual' (separate phases for the
        two polarisations, eqs. (20)-(21); forward only)."""
        codes = {"averaged": 0, "dual": 1}
        if mode not in codes:
            raise ValueError("mode must be 'averaged' or 'dual'")
        check(lib.cbessfm_set_nlpr(self._h, codes[mode]), "cbessfm_set_nlpr")
        self.nlpr = mode

    def set_gvd_lengths(self, lengths: torch.Tensor | None, stream=None):
        """Free dispersion segments: float64 CUDA tensor of steps + 1 lengths
        (km) before, between and after the NLPRs; None returns to the uniform
        steps with the current split ratio."""
        if lengths is None:
            check(lib.cbessfm_set_gvd_lengths(self._h, None, _stream_ptr(stream)), "cbessfm_set_gvd_lengths")
            return
        if not (lengths.is_cuda and lengths.dtype == torch.float64 and lengths.is_contiguous()
                and lengths.numel() == self.steps + 1):
            raise ValueError("lengths must be a contiguous float64 CUDA tensor of steps + 1 entries")
        check(lib.cbessfm_set_gvd_lengths(self._h, ctypes.c_void_p(lengths.data_ptr()), _stream_ptr(stream)),
              "cbessfm_set_gvd_lengths")

    def set_split_ratio(self, rho: float, stream=None):
        check(lib.cbessfm_set_split_ratio(self._h, float(rho), _stream_ptr(stream)), "cbessfm_set_split_ratio")

    def backward_workspace(self, t_len: int, batch: int = 1, checkpoint_every: int = 1) -> int:
        """Device workspace bytes of :meth:`backward` (``cbessfm_backward_workspace``)."""
        out = ctypes.c_size_t()
        check(lib.cbessfm_backward_workspace(self._h, int(t_len), int(batch), int(checkpoint_every),
                                             ctypes.byref(out)), "cbessfm_backward_workspace")
        return out.value

    def backward_gvd(self, field_in: torch.Tensor, grad_out: torch.Tensor, need_grad_in: bool = True,
                     checkpoint_every: int = 1, workspace: torch.Tensor | None = None, stream=None):
        """:meth:`backward` plus dL/d(dispersion segment lengths) [steps + 1]."""
        return self.backward(field_in, grad_out, need_grad_in, checkpoint_every, workspace, stream, _gvd=True)

    def backward(self, field_in: torch.Tensor, grad_out: torch.Tensor, need_grad_in: bool = True,
                 checkpoint_every: int = 1, workspace: torch.Tensor | None = None, stream=None, _gvd=False):
        """(grad_in or None, grad_c [steps][n_sb][n_sb][n_taps], grad_rho [1]) for the current
        coefficients and split ratio, given grad_out = dL/dRe(out) + j dL/dIm(out).

        ``checkpoint_every`` <= 1 stores every step's intermediate field and
        phase (no recompute); 1 < k < steps stores a spectrum every k steps
        and recomputes each k-step segment once (less workspace)."""
        x = self._field(field_in)
        g = self._field(grad_out)
        if g.shape != x.shape:
            raise ValueError("grad_out must be shaped like field_in")
        bsz = 1 if x.dim() == 2 else x.shape[0]
        t_len = x.shape[-1]
        need = self.backward_workspace(t_len, bsz, checkpoint_every)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
        elif workspace.numel() * workspace.element_size() < need or not workspace.is_cuda:
            raise ValueError(f"workspace must be a CUDA tensor of at least {need} bytes")
        grad_in = torch.empty_like(x) if need_grad_in else None
        grad_c = torch.empty((self.steps, self.n_sb, self.n_sb, self.n_taps), dtype=torch.float32,
                             device=x.device)
        grad_rho = torch.empty(1, dtype=torch.float32, device=x.device)
        gi_ptr = ctypes.c_void_p(grad_in.data_ptr()) if grad_in is not None else ctypes.c_void_p(0)
        grad_gvd = torch.empty(self.steps + 1, dtype=torch.float64, device=x.device) if _gvd else None
        gl_ptr = ctypes.c_void_p(grad_gvd.data_ptr()) if _gvd else ctypes.c_void_p(0)
        check(lib.cbessfm_backward_gvd(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                       gi_ptr, ctypes.c_void_p(grad_c.data_ptr()),
                                       ctypes.c_void_p(grad_rho.data_ptr()), gl_ptr, int(t_len), int(bsz),
                                       int(checkpoint_every), ctypes.c_void_p(workspace.data_ptr()),
                                       ctypes.c_size_t(workspace.numel() * workspace.element_size()),
                                       _stream_ptr(stream)), "cbessfm_backward")
        if _gvd:
            return grad_in, grad_c, grad_rho, grad_gvd
        return grad_in, grad_c, grad_rho

    def status(self) -> int:
        return lib.cbessfm_status(self._h)

    def set_wait_limit(self, polls: int) -> None:
        """Polls before a device-side exchange wait gives up (0: the default);
        a launch that gives up ends normally and cbessfm_status reports it."""
        check(lib.cbessfm_set_wait_limit(self._h, int(polls)), "cbessfm_set_wait_limit")

    def close(self):
        if getattr(self, "_h", None):
            lib.cbessfm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
