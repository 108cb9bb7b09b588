"""Batched CB-ESSFM execution, its scheduler and the block-length autotuner.

``Batch`` binds many instances -- each a :class:`Plan` with its own fields --
to one persistent launch per distinct N' up to 8192, and runs instances of
streamed blocks (N' >= 2^14) on the streaming kernels in the same run
(``cbessfm_batch_*`` in ``include/cbessfm.h``).  ``schedule`` exposes the host-only team scheduler and
``autotune`` the N' / N_ov choice.  Argument marshalling only.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import BatchInfo, Instance, SchedJob, SchedStats, TUNE_MEASURE, Tuning, check, lib
from .plan import LinkSpec, Plan, _stream_ptr


class Batch:
    """Instances ``[(plan, field_in, field_out), ...]``: complex64 device tensors
    of shape (2, T) or (B, 2, T); the tensors stay bound to the batch."""

    def __init__(self, instances):
        self._keep = []
        arr = (Instance * len(instances))()
        for k, (plan, x, y) in enumerate(instances):
            x = Plan._field(x)
            if y.shape != x.shape or y.dtype != x.dtype or not y.is_contiguous() or not y.is_cuda:
                raise ValueError("field_out must be a contiguous complex64 CUDA tensor shaped like field_in")
            bsz = 1 if x.dim() == 2 else x.shape[0]
            arr[k] = Instance(plan._h, x.data_ptr(), y.data_ptr(), int(x.shape[-1]), int(bsz))
            self._keep.append((plan, x, y))
        handle = ctypes.c_void_p()
        check(lib.cbessfm_batch_create(ctypes.byref(handle), arr, len(instances)), "cbessfm_batch_create")
        self._h = handle

    def run(self, stream=None):
        check(lib.cbessfm_batch_run(self._h, _stream_ptr(stream)), "cbessfm_batch_run")

    def info(self) -> dict:
        out = BatchInfo()
        check(lib.cbessfm_batch_describe(self._h, ctypes.byref(out)), "cbessfm_batch_describe")
        return {k: getattr(out, k) for k, _ in BatchInfo._fields_}

    def status(self) -> int:
        return lib.cbessfm_batch_status(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib.cbessfm_batch_destroy(self._h)
            self._h = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def schedule(jobs, slots_per_xcd: int, max_wg: int | None = None) -> dict:
    """Team schedule for jobs ``[(width, n_items, cost), ...]`` (``cbessfm_schedule``)."""
    n = len(jobs)
    arr = (SchedJob * n)(*[SchedJob(int(w), int(m), float(c)) for w, m, c in jobs])
    total = int(sum(int(m) for _, m, _ in jobs))
    max_wg = int(max_wg if max_wg is not None else 8 * slots_per_xcd)
    wg_team = np.empty(max_wg, np.int32)
    wg_member = np.empty(max_wg, np.int32)
    item_team = np.empty(max(total, 1), np.int32)
    item_rank = np.empty(max(total, 1), np.int32)
    st = SchedStats()
    ip = ctypes.POINTER(ctypes.c_int32)
    check(lib.cbessfm_schedule(arr, n, int(slots_per_xcd), max_wg, wg_team.ctypes.data_as(ip),
                               wg_member.ctypes.data_as(ip), item_team.ctypes.data_as(ip),
                               item_rank.ctypes.data_as(ip), ctypes.byref(st)), "cbessfm_schedule")
    g = st.grid
    return dict(grid=g, n_teams=st.n_teams, makespan=st.makespan, lower_bound=st.lower_bound,
                wg_team=wg_team[:g].copy(), wg_member=wg_member[:g].copy(),
                item_team=item_team[:total].copy(), item_rank=item_rank[:total].copy())


def autotune(link: LinkSpec, n_sb: int, steps: int, n_taps: int, t_len: int, batch: int = 1,
             measure: bool = True) -> dict:
    """N' and N_ov for one instance (``cbessfm_autotune``); ``measure`` times candidates on the device."""
    out = Tuning()
    lk = link.c()
    check(lib.cbessfm_autotune(ctypes.byref(lk), int(n_sb), int(steps), int(n_taps), int(t_len), int(batch),
                               TUNE_MEASURE if measure else 0, ctypes.byref(out)), "cbessfm_autotune")
    return {k: getattr(out, k) for k, _ in Tuning._fields_}


__all__ = ["Batch", "schedule", "autotune"]
