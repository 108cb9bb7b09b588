"""All-core timing of the oracle (test infrastructure, like the rest of
``oracle/``): the blocks of one field are split into contiguous ranges, one per
worker process, each running :func:`oracle.run_blocks` unchanged.

Usage: ``python -m oracle.timing CASE.npz WORKERS`` prints one JSON line
{"wall_s", "cpu_s", "blocks", "workers"}.  CASE.npz holds ``x`` (complex, 2 x T),
``coeffs`` and the scalar fields of :class:`oracle.OraclePlan`.  The timing
process never touches a GPU; a caller that has one starts this as a child
program.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import sys
import time

import numpy as np

from .cbessfm import OraclePlan, run_blocks

_X = None
_PLAN = None


def _init(x, plan):
    global _X, _PLAN
    _X, _PLAN = x, plan


def _work(blocks):
    p0 = time.process_time()
    run_blocks(_X, _PLAN, blocks)
    return time.process_time() - p0


def main(argv) -> int:
    case = np.load(argv[0], allow_pickle=False)
    workers = max(1, int(argv[1]))
    x = np.asarray(case["x"], dtype=np.complex128)
    plan = OraclePlan(float(case["beta2_s2_km"]), float(case["sample_rate"]), float(case["step_km"]),
                      int(case["n_steps"]), float(case["rho"]), int(case["n_sb"]), int(case["n_block"]),
                      int(case["n_overlap"]), np.asarray(case["coeffs"], np.float64))
    nblk = -(-x.shape[-1] // plan.hop)
    chunks = [list(r) for r in np.array_split(np.arange(nblk), min(workers, nblk))]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks), initializer=_init, initargs=(x, plan)) as pool:
        cpu = pool.map(_work, [[int(b) for b in c] for c in chunks])
    wall = time.perf_counter() - t0
    print(json.dumps({"wall_s": wall, "cpu_s": float(sum(cpu)), "blocks": nblk, "workers": len(chunks)}))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
