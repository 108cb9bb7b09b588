"""Throughput of the CB-ESSFM forward on one MI355X.

Workload: 5 WDM channels x 64 GBd DP-64QAM on a 100 GHz grid, 2^16 symbols per
channel sampled at 640 GS/s (T = 655360 per polarisation), 15 x 80 km SMF;
backpropagation with 5 subbands, N' = 4096, N_ov = 2560, 15 asymmetric steps
(rho = 0.3) and 21 analytic taps, one persistent launch per step.

A "step" of this benchmark is one full pass of the hot path over the field.
Prints one JSON line.  Options:
  --gpus N      only 1 is supported (one GPU per process and per box)
  --steps K     timed passes (default 200)
  --warmup W    untimed passes (default 20)
  --no-cpu      skip the oracle timing
  --copy-mib M  after timing, run one plain device copy of M MiB (counter calibration)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "5ch-64GBd-64QAM-2^16sym-15x80km"
METRIC = "DBP 2D-symbols/s (all channels) + % HBM roofline; coeff-gradient steps/s at ≤1e-5 rel err"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (published)
GEN_STEPS_PER_SPAN = 4         # forward-link simulator steps per span for the synthetic field


def algorithmic_flops_per_block(n_sb, n_sub, steps, n_taps):
    """Flops of one overlap-and-save block (convention in the design doc):
    5 n log2 n per complex DFT of size n, 6 per complex multiply, 7 per
    dual-polarisation intensity, 2 per tap of the direct-form filter of
    eq. (15); the sine/cosine of the rotation is not counted."""
    n = n_sb * n_sub
    dft_n = 5.0 * n * math.log2(n)
    dft_sub = 5.0 * n_sub * math.log2(n_sub)
    per_step = (2 * 6 * n            # GVD filter, both polarisations
                + 4 * n_sb * dft_sub  # inverse + forward DFT per subband and polarisation
                + 7 * n              # intensity
                + 2 * n_taps * n_sb * n  # coupled FIR
                + 2 * 6 * n)         # rotation, both polarisations
    return 4 * dft_n + steps * per_step + 2 * 6 * n


def cpu_baseline(x, coeffs, d, link_rate, step_km):
    """The FP64 oracle, as it stands, on the whole workload (one pass)."""
    import numpy as np
    import oracle
    plan = oracle.OraclePlan(-21.7e-24, link_rate, step_km, d["n_steps"], d["rho"], d["n_sb"],
                             d["n_sb"] * d["n_sub"], d["n_overlap"], np.asarray(coeffs, np.float64))
    t0 = time.perf_counter()
    oracle.run(x, plan)
    return time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(the multi-GPU sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_14489_amd import LinkSpec, Plan, analytic_coeffs
    from synth import workload

    torch.cuda.set_device(0)
    x, _, w = workload(WORKLOAD, 2001, steps_per_span=GEN_STEPS_PER_SPAN)
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = LinkSpec(alpha_db_km=ch.alpha_db_km, beta2_ps2_km=ch.beta2_ps2_km, gamma_w_km=ch.gamma_w_km,
                    span_km=ch.span_km, n_spans=ch.n_spans, sample_rate_hz=wdm.sample_rate)
    coeffs = analytic_coeffs(link, d["n_sb"], d["n_steps"], d["rho"], d["n_taps"]).astype(np.float32)
    plan = Plan(link, d["n_sb"], d["n_sub"], d["n_overlap"], d["n_steps"], d["rho"], coeffs=coeffs)
    t_len = x.shape[-1]
    xin = torch.from_numpy(x.astype(np.complex64)).cuda()
    yout = torch.empty_like(xin)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        plan.run(xin, out=yout)
    torch.cuda.synchronize()
    if plan.status() != 0:
        raise RuntimeError("device error flag set during warm-up")

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        plan.run(xin, out=yout)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if plan.status() != 0:
        raise RuntimeError("device error flag set during the timed region")
    kernel_s = ev0.elapsed_time(ev1) / 1e3 / args.steps   # one launch per step

    n2d = wdm.n_channels * 2 * wdm.n_symbols                # 2D symbols per pass
    ms_per_step = wall / args.steps * 1e3
    value = n2d / (wall / args.steps)
    nblk = plan.n_blocks(t_len)
    flops = algorithmic_flops_per_block(d["n_sb"], d["n_sub"], d["n_steps"], d["n_taps"]) * nblk
    achieved = flops / kernel_s / 1e12
    alg_bytes = 2 * (2 * t_len * 8)                          # read + write complex64, both pols
    hbm_gbs = alg_bytes / kernel_s / 1e9

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "2D-symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic: seeded WDM field, {ch.n_spans}x{ch.span_km:g} km Manakov link "
                f"simulated at {GEN_STEPS_PER_SPAN} steps/span, ASE at NF {ch.nf_db:g} dB",
        "config": {"workload": WORKLOAD, "T": t_len, "batch": 1, "n_sb": d["n_sb"], "block_sb": d["n_sub"],
                   "overlap": d["n_overlap"], "steps": d["n_steps"], "split_ratio": d["rho"],
                   "n_taps": d["n_taps"], "blocks": nblk, "kernel": "cbessfm::fwd_kernel<12>",
                   "threads_per_group": plan.info().threads_per_group},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "flops_per_launch": flops, "kernel_ms": kernel_s * 1e3},
        "hbm_roofline": {"achieved": hbm_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": hbm_gbs / PEAK_HBM_GBS, "bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu:
        secs = cpu_baseline(x, coeffs, d, wdm.sample_rate, ch.span_km * ch.n_spans / d["n_steps"])
        result["cpu_baseline"] = {"value": n2d / secs, "unit": "2D-symbols/s", "cores": 1, "kind": "oracle",
                                  "sample": f"whole workload, one pass ({nblk} blocks), numpy FP64, "
                                            f"{secs:.2f} s"}
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 4 * n
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
