"""Throughput of CB-ESSFM digital backpropagation on one MI355X.

Primary workload (the JSON line's value): 5 WDM channels x 64 GBd DP-64QAM on a
100 GHz grid, 2^16 symbols per channel sampled at 640 GS/s (T = 655360 per
polarisation), 15 x 80 km SMF; backpropagation with 5 subbands, N' = 4096,
N_ov = 2560, 15 asymmetric steps (rho = 0.3) and 21 analytic taps, one
persistent launch per pass.  A "step" of this benchmark is one pass of the
hot path over that field; the timed passes are replayed from a HIP graph
(the eager, cooperative-launch time per pass is reported beside it).

Two more legs are reported in the same line:
  grad     1 ch 32 GBd DP-16QAM, 2^14 symbols, 1 x 80 km, 16 realisations,
           15 steps x 11 taps: forward + adjoint + Adam iterations per second
           (checkpointing on and off), peak device memory, 200 Adam iterations
           of the matched-filter MSE, and the adjoint's error against the FP64
           oracle on one realisation;
  batched  64 uneven instances (1-5 channels, 5-40 spans, 1-40 steps, 2^12 -
           2^18 symbols per channel), N' / N_ov from the measured autotuner,
           one graph-replayed batch against 64 separate launches;
  protocol the paper's tied coefficient fits and method comparison on the
           central channel of a five-channel link;
  longlink 5 channels, 2^20 symbols per channel, 40 x 80 km: the streaming
           path (N' = 2^17, N_ov = 196608) over a sweep of 1 - 80 steps,
           throughput, device-memory roofline, SNR against dispersion-only
           compensation with analytic coefficients and with coefficients and
           split ratio fitted on the device (streaming adjoint, checkpoints
           every 8 steps) on a second realisation, sampled oracle parity;
  streamgrad the streaming forward and adjoint at the long-link block shape
           (10 steps, 23 blocks, random field): times and workspace.

Options:
  --gpus N      only 1 is supported (one GPU per process and per box)
  --steps K     timed passes of the primary workload (default 200)
  --warmup W    untimed passes (default 20)
  --legs L      comma list of grad,batched,protocol,longlink,streamgrad
                (default all; the primary forward always runs)
  --no-cpu      skip the oracle timing (and the full-size parity check)
  --copy-mib M  after timing, one plain device copy of M MiB (counter calibration)
  --fit-iters F Adam iterations per step count of the long-link fit (default 20;
                8 / steps times as many below 8 steps)
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "5ch-64GBd-64QAM-2^16sym-15x80km"
GRAD_WORKLOAD = "1ch-32GBd-16QAM-2^14sym-1x80km-15steps"
CFG1_WORKLOAD = "1ch-32GBd-16QAM-2^14sym-1x80km"
METRIC = "DBP 2D-symbols/s (all channels) + % HBM roofline; coeff-gradient steps/s at ≤1e-5 rel err"
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (published)
GEN_STEPS_PER_SPAN = 4         # forward-link simulator steps per span, 5-channel field
GRAD_GEN_STEPS_PER_SPAN = 50   # the same for the single-channel gradient fields
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fwd_kernel_5ch_64GBd_2p16sym_15x80km_traffic.md")
KERNEL_SOURCES = ["paper_2409_14489_amd/csrc/*.hip", "paper_2409_14489_amd/csrc/*.hpp",
                  "paper_2409_14489_amd/csrc/*.cpp", "include/cbessfm.h",
                  "paper_2409_14489_amd/build.py"]
# the translation unit of the forward kernel the counters were taken on
FWD_KERNEL_SOURCES = ["paper_2409_14489_amd/csrc/forward.hip", "paper_2409_14489_amd/csrc/fft_lds.hpp",
                      "paper_2409_14489_amd/csrc/stages.hpp", "paper_2409_14489_amd/csrc/team.hpp",
                      "paper_2409_14489_amd/csrc/sincos.hpp", "paper_2409_14489_amd/csrc/internal.hpp",
                      "include/cbessfm.h", "paper_2409_14489_amd/build.py"]


def kernel_source_digest(patterns=None) -> str:
    h = hashlib.sha256()
    for pat in patterns or KERNEL_SOURCES:
        for f in sorted(glob.glob(os.path.join(ROOT, pat))):
            h.update(os.path.relpath(f, ROOT).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the forward kernel's sources as they are now; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("fwd_kernel_source_sha256") != kernel_source_digest(FWD_KERNEL_SOURCES):
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Algorithmic FP32 flops per 2D symbol of the named workloads, the per-unit
# figures of the method's operation count (5 n log2 n per complex DFT of size
# n plus the pointwise stages, with the coupled filter in its frequency-domain
# form): the roofline's `achieved` is this times the 2D symbols of one launch.
FLOPS_PER_2D_SYMBOL = {
    "5ch-64GBd-64QAM-2^16sym-15x80km": 7.0e3,
    "1ch-32GBd-16QAM-2^14sym-1x80km": 614.0,
    "1ch-32GBd-16QAM-2^14sym-1x80km-15steps": 5.8e3,
}


def long_link_flops_per_2d_symbol(steps):
    """The operation count per 2D symbol of the long-link workload (5 subbands,
    N' = 2^17, the same convention as FLOPS_PER_2D_SYMBOL): 1.3e3 at one step
    to 6.0e4 at 80, linear in the step count in between."""
    return 1.3e3 + (6.0e4 - 1.3e3) * (steps - 1) / 79.0


def algorithmic_flops_per_block(n_sb, n_sub, steps, n_taps):
    """Flops of one overlap-and-save block, by this convention:
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


def link_of(ch, rate):
    from paper_2409_14489_amd import LinkSpec
    return LinkSpec(alpha_db_km=ch.alpha_db_km, beta2_ps2_km=ch.beta2_ps2_km, gamma_w_km=ch.gamma_w_km,
                    span_km=ch.span_km, n_spans=ch.n_spans, sample_rate_hz=rate)


def oracle_plan(d, rate, step_km, coeffs, beta2_ps2_km):
    import numpy as np
    import oracle
    return oracle.OraclePlan(beta2_ps2_km * 1e-24, rate, step_km, d["n_steps"], d["rho"], d["n_sb"],
                             d["n_sb"] * d["n_sub"], d["n_overlap"], np.asarray(coeffs, np.float64))


def oracle_all_cores(x, oplan, n2d, workers=None):
    """The oracle with the blocks of the field split over worker processes
    (oracle.timing, started as a child program: no process is forked from
    this one, which holds the GPU).  None if the child fails."""
    import subprocess
    import tempfile
    import numpy as np
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="cbessfm_oracle_") as tmp:
        case = os.path.join(tmp, "case.npz")
        np.savez(case, x=np.asarray(x, np.complex128), coeffs=np.asarray(oplan.coeffs, np.float64),
                 beta2_s2_km=oplan.beta2_s2_km, sample_rate=oplan.sample_rate, step_km=oplan.step_km,
                 n_steps=oplan.n_steps, rho=oplan.rho, n_sb=oplan.n_sb, n_block=oplan.n_block,
                 n_overlap=oplan.n_overlap)
        res = subprocess.run([sys.executable, "-m", "oracle.timing", case, str(workers)], cwd=ROOT,
                             capture_output=True, text=True, timeout=600)
    if res.returncode != 0 or not res.stdout.strip():
        return None
    t = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": n2d / t["wall_s"], "unit": "2D-symbols/s", "cores": max(1, round(t["cpu_s"] / t["wall_s"])),
            "workers": t["workers"], "kind": "oracle",
            "sample": f"the whole workload, one pass, {t['blocks']} blocks split over {t['workers']} processes, "
                      f"{t['wall_s']:.1f} s"}


def timed_events(stream, fn, reps):
    """Average seconds per call of fn() on `stream`, HIP events around the loop."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def host_identity():
    """nproc and CPU model of the host the oracle is timed on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model}


def time_oracle(run, min_s=10.0, max_passes=12):
    """Runs run() until about min_s seconds of wall time have passed (at least
    once); returns (passes, wall seconds, process seconds, first result)."""
    passes, wall, proc, first = 0, 0.0, 0.0, None
    while passes < 1 or (wall < min_s and passes < max_passes):
        t0, p0 = time.perf_counter(), time.process_time()
        out = run()
        wall += time.perf_counter() - t0
        proc += time.process_time() - p0
        first = out if first is None else first
        passes += 1
    return passes, wall, proc, first


def worst_block_err(got, ref, hop, block, n_ov):
    """Largest relative L2 error over the kept output segments of the
    overlap-and-save blocks (both polarisations)."""
    import numpy as np
    t_len = got.shape[-1]
    worst = 0.0
    for s in range(0, t_len, hop):
        e = min(s + hop, t_len)
        r = ref[..., s:e]
        den = float(np.sum(np.abs(r) ** 2))
        if den > 0:
            worst = max(worst, (float(np.sum(np.abs(got[..., s:e] - r) ** 2)) / den) ** 0.5)
    return worst


# ------------------------------------------------------------------ primary: 5-channel forward
def leg_forward(args):
    import numpy as np
    import torch
    from paper_2409_14489_amd import Plan, analytic_coeffs
    from synth import workload

    x, _, w = workload(WORKLOAD, 2001, steps_per_span=GEN_STEPS_PER_SPAN)
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = link_of(ch, wdm.sample_rate)
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
    # eager launches (cooperative), for reference
    eager_s = timed_events(stream, lambda: plan.run(xin, out=yout), max(1, args.steps // 4))

    # timed passes: the launches are replayed from a HIP graph (ordinary
    # kernel nodes of the resident-sized persistent grid), `per_graph` per replay
    per_graph = 10 if args.steps % 10 == 0 else 1
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            plan.run(xin, out=yout)
    graph.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps // per_graph):
        graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if plan.status() != 0:
        raise RuntimeError("device error flag set during the timed region")
    kernel_s = ev0.elapsed_time(ev1) / 1e3 / args.steps   # one launch per pass
    del graph

    n2d = wdm.n_channels * 2 * wdm.n_symbols                # 2D symbols per pass
    nblk = plan.n_blocks(t_len)
    flops = FLOPS_PER_2D_SYMBOL[WORKLOAD] * n2d
    flops_own = algorithmic_flops_per_block(d["n_sb"], d["n_sub"], d["n_steps"], d["n_taps"]) * nblk
    achieved = flops / kernel_s / 1e12
    alg_bytes = 2 * (2 * t_len * 8)                          # read + write complex64, both pols
    hbm_gbs = alg_bytes / kernel_s / 1e9
    traffic = measured_traffic()

    result = {
        "metric": METRIC,
        "value": n2d / (wall / args.steps),
        "unit": "2D-symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic: seeded WDM field, {ch.n_spans}x{ch.span_km:g} km Manakov link "
                f"simulated at {GEN_STEPS_PER_SPAN} steps/span, ASE at NF {ch.nf_db:g} dB",
        "config": {"workload": WORKLOAD, "T": t_len, "batch": 1, "n_sb": d["n_sb"], "block_sb": d["n_sub"],
                   "overlap": d["n_overlap"], "steps": d["n_steps"], "split_ratio": d["rho"],
                   "n_taps": d["n_taps"], "blocks": nblk, "kernel": "cbessfm::fwd_kernel<12>",
                   "threads_per_group": plan.info().threads_per_group,
                   "kernel_source_sha256": kernel_source_digest(),
                   "fwd_kernel_source_sha256": kernel_source_digest(FWD_KERNEL_SOURCES)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops, "flops_per_2d_symbol": FLOPS_PER_2D_SYMBOL[WORKLOAD],
                     "kernel_ms": kernel_s * 1e3,
                     "flops_per_launch_direct_filter": flops_own,
                     "frac_direct_filter": flops_own / kernel_s / 1e12 / PEAK_FP32_TFLOPS},
        "launch": {"timed": f"HIP graph replays, {per_graph} launch(es) per replay",
                   "eager_cooperative_ms_per_step": eager_s * 1e3},
        "hbm_roofline": {"achieved": hbm_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": hbm_gbs / PEAK_HBM_GBS, "bytes_per_launch": alg_bytes},
    }
    # the dual-polarisation NLPR (eqs. (20)-(21)) on the same workload, graph-replayed the same way
    plan.set_nlpr("dual")
    ydual = torch.empty_like(xin)
    for _ in range(3):
        plan.run(xin, out=ydual)
    gdual = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gdual):
        for _ in range(per_graph):
            plan.run(xin, out=ydual)
    gdual.replay()
    dual_s = timed_events(stream, gdual.replay, max(1, args.steps // per_graph // 2)) / per_graph
    if plan.status() != 0:
        raise RuntimeError("device error flag set in the dual-polarisation run")
    del gdual
    plan.set_nlpr("averaged")
    result["dual_pol_nlpr"] = {
        "value": n2d / dual_s, "unit": "2D-symbols/s", "kernel_ms": dual_s * 1e3,
        "time_vs_averaged": dual_s / kernel_s,
        "rel_l2_vs_averaged": float(torch.linalg.vector_norm(ydual - yout) / torch.linalg.vector_norm(yout))}
    if not args.no_cpu:
        import oracle
        oplan = oracle_plan(d, wdm.sample_rate, ch.span_km * ch.n_spans / d["n_steps"], coeffs, ch.beta2_ps2_km)
        # sampled parity of the dual-polarisation run: first, middle and last blocks
        import copy
        odual = copy.copy(oplan)
        odual.nlpr = "dual"
        pick = [0, nblk // 2, nblk - 1]
        got_d = ydual.cpu().numpy().astype(np.complex128)
        ref_d = oracle.run_blocks(x, odual, pick)
        num = den = 0.0
        for b, r in ref_d.items():
            seg = got_d[:, b * plan.hop:b * plan.hop + r.shape[-1]]
            num += float(np.sum(np.abs(seg - r) ** 2))
            den += float(np.sum(np.abs(r) ** 2))
        result["dual_pol_nlpr"]["parity_rel_l2_sampled"] = (num / den) ** 0.5
        result["dual_pol_nlpr"]["parity_blocks"] = pick
        passes, cpu_s, proc_s, ref = time_oracle(lambda: oracle.run(x, oplan))
        got = yout.cpu().numpy().astype(np.complex128)
        result["parity_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["parity_rel_l2_worst_block"] = worst_block_err(got, ref, plan.hop, plan.block, d["n_overlap"])
        result["cpu_baseline"] = {"value": n2d * passes / cpu_s, "unit": "2D-symbols/s",
                                  "cores": max(1, round(proc_s / cpu_s)), "kind": "oracle",
                                  "sample": f"the whole workload ({nblk} blocks), {passes} passes of the FP64 "
                                            f"numpy oracle, {cpu_s:.1f} s",
                                  **host_identity()}
        all_cores = oracle_all_cores(x, oplan, n2d)
        if all_cores is not None:
            result["cpu_baseline_all_cores"] = all_cores
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 4 * n
    plan.close()
    return result


# ------------------------------------------------------------------ gradient leg
def leg_grad(args):
    import numpy as np
    import torch
    from paper_2409_14489_amd import Plan, analytic_coeffs, cbessfm
    from paper_2409_14489_amd.train import SymbolReceiver, fit, phase_aligned_mse
    from synth import workload

    n_real, iters = 16, 200
    fields, syms = [], []
    for r in range(n_real):
        x, s, w = workload(GRAD_WORKLOAD, 3000 + r, steps_per_span=GRAD_GEN_STEPS_PER_SPAN)
        fields.append(x)
        syms.append(s[0])                              # channel 0: (2, n_symbols)
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = link_of(ch, wdm.sample_rate)
    x = torch.from_numpy(np.stack(fields).astype(np.complex64)).cuda()
    s = torch.from_numpy(np.stack(syms).astype(np.complex64)).cuda()
    t_len = x.shape[-1]
    c0 = analytic_coeffs(link, d["n_sb"], d["n_steps"], d["rho"], d["n_taps"]).astype(np.float32)
    plan = Plan(link, d["n_sb"], d["n_sub"], d["n_overlap"], d["n_steps"], d["rho"], coeffs=c0)
    p_w = 1e-3 * 10 ** (wdm.power_dbm_per_channel / 10)
    rx = SymbolReceiver(t_len, wdm.sample_rate, wdm.baud, wdm.rolloff, p_w)

    def mse(coeffs, rho):
        with torch.no_grad():
            return float(phase_aligned_mse(rx(cbessfm(x, coeffs, rho, plan)), s))

    c0_t = torch.from_numpy(c0).cuda()
    rho0 = torch.tensor(d["rho"], dtype=torch.float32, device="cuda")
    zero = torch.zeros_like(c0_t)
    mse_edc = mse(zero, rho0)
    mse_analytic = mse(c0_t, rho0)

    out = {"workload": GRAD_WORKLOAD, "realisations": n_real, "T": t_len, "steps": d["n_steps"],
           "n_taps": d["n_taps"], "parameters": int(c0.size) + 1, "unit": "steps/s",
           "step": "forward + matched-filter MSE + adjoint + Adam update, 16 realisations"}
    stream = torch.cuda.current_stream()
    for ck, graph in ((1, True), (5, True), (1, False)):
        fit(plan, x, s, rx, c0, d["rho"], iters=3, checkpoint_every=ck)   # warm-up
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        base_mem = torch.cuda.memory_allocated()
        t0 = time.perf_counter()
        c_fit, rho_fit, losses = fit(plan, x, s, rx, c0, d["rho"], iters=iters, checkpoint_every=ck, graph=graph)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if plan.status() != 0:
            raise RuntimeError("device error flag set in the gradient leg")
        peak = torch.cuda.max_memory_allocated() - base_mem
        key = ("store_every_step" if ck == 1 else f"checkpoint_every_{ck}") + ("" if graph else "_eager")
        out[key] = {"steps_per_s": iters / wall, "ms_per_step": wall / iters * 1e3,
                    "peak_extra_mib": peak / 2 ** 20,
                    "adjoint_workspace_mib": plan.backward_workspace(t_len, n_real, ck) / 2 ** 20,
                    "launch": "HIP graph of the whole iteration (3 eager warm-up iterations included)"
                              if graph else "eager"}
        if ck == 1 and graph:
            mse_fit = mse(c_fit, rho_fit)
            out["adam_iterations"] = iters
            out["snr_db"] = {"edc": -10 * math.log10(mse_edc), "analytic": -10 * math.log10(mse_analytic),
                             "fitted": -10 * math.log10(mse_fit)}
            out["rho_fitted"] = float(rho_fit)
    # adjoint kernel alone (both sweeps + reductions), timed on its stream
    g = torch.from_numpy(((np.random.default_rng(5).standard_normal(x.shape)
                           + 1j * np.random.default_rng(6).standard_normal(x.shape)) * 1e-2)
                         .astype(np.complex64)).cuda()
    plan.set_coeffs(c0_t, rho0)
    ws = torch.empty(plan.backward_workspace(t_len, n_real, 1), dtype=torch.uint8, device="cuda")
    gi, gc, gr = plan.backward(x, g, need_grad_in=False, workspace=ws)
    out["adjoint_ms"] = timed_events(stream, lambda: plan.backward(x, g, need_grad_in=False, workspace=ws),
                                     20) * 1e3
    out["forward_ms"] = timed_events(stream, lambda: plan.run(x), 20) * 1e3
    if not args.no_cpu:
        from oracle.grad import vjp
        oplan = oracle_plan(d, wdm.sample_rate, ch.span_km * ch.n_spans / d["n_steps"], c0, ch.beta2_ps2_km)
        # the gradient the fit uses: cotangent of the phase-aligned symbol MSE
        # (matched filter, symbol sampling) at the analytic coefficients, all
        # 16 realisations
        y = plan.run(x).detach().requires_grad_(True)
        gmse, = torch.autograd.grad(phase_aligned_mse(rx(y), s), y)
        gmse = gmse.contiguous()
        gi, gc, gr = plan.backward(x, gmse)
        torch.cuda.synchronize()
        xs64 = np.stack(fields).astype(np.complex64).astype(np.complex128)
        ogi, ogc, ogr = vjp(xs64, oplan, gmse.cpu().numpy().astype(np.complex128))
        out["parity_rel_l2"] = {
            "grad_c": float(np.linalg.norm(gc.cpu().numpy() - ogc) / np.linalg.norm(ogc)),
            "grad_in": float(np.linalg.norm(gi.cpu().numpy() - ogi) / np.linalg.norm(ogi)),
            "grad_rho_vs_oracle": float(abs(float(gr) - ogr) / abs(ogr)),
            "cotangent": "phase-aligned symbol MSE, 16 realisations",
        }
        # stress case: a white random cotangent on one realisation, whose
        # out-of-band part the FP32 state resolves least well
        gi, gc, gr = plan.backward(x[:1], g[:1])
        torch.cuda.synchronize()
        ogi, ogc, ogr = vjp(fields[0].astype(np.complex64).astype(np.complex128), oplan,
                            g[0].cpu().numpy().astype(np.complex128))
        out["parity_rel_l2_white_cotangent"] = {
            "grad_c": float(np.linalg.norm(gc.cpu().numpy() - ogc) / np.linalg.norm(ogc)),
            "grad_in": float(np.linalg.norm(gi[0].cpu().numpy() - ogi) / np.linalg.norm(ogi)),
            "grad_rho_vs_oracle": float(abs(float(gr) - ogr) / abs(ogr)),
            "cotangent": "white Gaussian, std 1e-2, realisation 0",
        }
    out["value"] = out["store_every_step"]["steps_per_s"]
    plan.close()
    return out


# ------------------------------------------------------------------ batched leg
def batch_instances(seed=4000, n=64):
    """The uneven 64-instance workload: per instance, channels, spans, steps and
    log-uniform symbol counts drawn from PCG64(seed)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        n_ch = int(rng.integers(1, 6))
        spans = int(rng.integers(5, 41))
        steps = int(rng.integers(1, 41))
        n_sym = int(round(2 ** rng.uniform(12, 18)))
        qam = int(rng.choice([16, 64]))
        out.append(dict(n_ch=n_ch, spans=spans, steps=steps, n_sym=n_sym, qam=qam, rate=n_ch * 128e9,
                        T=n_sym * 2 * n_ch, taps=11 if n_ch == 1 else 21))
    return out


def leg_batched(args):
    import numpy as np
    import torch
    from paper_2409_14489_amd import Batch, LinkSpec, Plan, autotune
    from synth import random_field

    specs = batch_instances()
    plans, xs, ys, tuned = [], [], [], []
    t_tune = time.perf_counter()
    for k, sp in enumerate(specs):
        link = LinkSpec(n_spans=sp["spans"], sample_rate_hz=sp["rate"])
        tun = autotune(link, sp["n_ch"], sp["steps"], sp["taps"], sp["T"], measure=True)
        tuned.append(tun)
        plans.append(Plan(link, sp["n_ch"], tun["block_sb"], tun["overlap"], sp["steps"], 0.5,
                          n_taps=sp["taps"]))
        p_w = sp["n_ch"] * 1e-3 * 10 ** 0.2
        xs.append(torch.from_numpy(random_field((2, sp["T"]), 4100 + k, power_w=p_w).astype(np.complex64)).cuda())
        ys.append(torch.empty_like(xs[-1]))
    t_tune = time.perf_counter() - t_tune
    n2d = sum(sp["n_ch"] * 2 * sp["n_sym"] for sp in specs)
    stream = torch.cuda.current_stream()

    b = Batch(list(zip(plans, xs, ys)))
    info = b.info()
    b.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run()
    for _ in range(3):
        graph.replay()
    reps = 10
    t_batch = timed_events(stream, graph.replay, reps)
    if b.status() != 0:
        raise RuntimeError("device error flag set in the batched leg")
    batched_out = [y.clone() for y in ys]

    def separate():
        for p, x, y in zip(plans, xs, ys):
            p.run(x, out=y)
    for _ in range(2):
        separate()
    t_sep = timed_events(stream, separate, reps)
    same = max(float((a - y).abs().max() / y.abs().max()) for a, y in zip(batched_out, ys))
    out = {"workload": "64 uneven instances: 1-5 ch x 64 GBd, 5-40 x 80 km, 1-40 steps, 2^12-2^18 symbols/ch",
           "unit": "2D-symbols/s", "value": n2d / t_batch, "ms_per_run": t_batch * 1e3,
           "separate_launches": {"value": n2d / t_sep, "ms_per_run": t_sep * 1e3, "launches": len(specs)},
           "speedup_vs_separate": t_sep / t_batch, "graph_replayed": True,
           "persistent_launches_per_run": info["launches"], "streamed_instances": info["streamed"],
           "streamed_blocks": info["streamed_items"], "stream_classes": info["stream_classes"],
           "stream_lone": info["stream_lone"], "kernel_launches_per_run": info["kernel_launches"],
           "teams": info["teams"], "workgroups": info["workgroups"],
           "blocks": info["items"], "predicted_ms": info["makespan_s"] * 1e3,
           "lower_bound_ms": info["lower_bound_s"] * 1e3,
           "block_sb_chosen": sorted({t["block_sb"] for t in tuned}),
           "instances_overlap_covers_memory": sum(t["covered"] for t in tuned),
           "max_rel_diff_vs_separate": same, "autotune_s": t_tune, "symbols_2d": n2d}
    b.close()
    for p in plans:
        p.close()
    return out


# ------------------------------------------------------------------ protocol leg
PROTO_WORKLOAD = "5ch-64GBd-64QAM-2^13sym-15x80km-central"


def leg_protocol(args):
    """The paper's coefficient fitting and method comparison (Sec. III-B,
    IV-B) on the central channel of a five-channel link: tied sequential fits
    on two training realisations, SNR on two other realisations, complexity
    from the paper's model."""
    import numpy as np
    import torch
    from paper_2409_14489_amd import run_method
    from paper_2409_14489_amd.train import SymbolReceiver
    from synth import dbp_rate, workload

    def data(seeds):
        xs, ss = [], []
        for sd in seeds:
            x, s, w = workload(PROTO_WORKLOAD, sd)
            xs.append(x)
            ss.append(s[0])
        return (torch.from_numpy(np.stack(xs).astype(np.complex64)).cuda(),
                torch.from_numpy(np.stack(ss).astype(np.complex64)).cuda()), w

    t0 = time.perf_counter()
    train, w = data([6000, 6001])
    test, _ = data([6100, 6101])
    t_gen = time.perf_counter() - t0
    wdm, ch, d = w["wdm"], w["ch"], w["dbp"]
    rate = dbp_rate(w)
    link = link_of(ch, rate)
    p_w = 1e-3 * 10 ** (wdm.power_dbm_per_channel / 10)
    rx = SymbolReceiver(train[0].shape[-1], rate, wdm.baud, wdm.rolloff, p_w)
    block = d["n_sb"] * d["n_sub"]
    common = dict(block=block, overlap=d["n_overlap"], n_sps=rate / wdm.baud, iters_per_row=args.proto_iters)
    taps = 255
    t0 = time.perf_counter()
    methods = [run_method("edc", link, train, test, rx, **common),
               run_method("ideal", link, train, test, rx, steps=20 * ch.n_spans, **common)]
    for st in (1, 3, 5, 15):
        methods.append(run_method("ssfm", link, train, test, rx, steps=st, **common))
        methods.append(run_method("ossfm", link, train, test, rx, steps=st, **common))
        methods.append(run_method("essfm", link, train, test, rx, steps=st, n_taps=taps, **common))
        cands = [run_method("cb-essfm", link, train, test, rx, steps=st, n_sb=2, rho=r, n_taps=taps, **common)
                 for r in (0.1, 0.3, 0.5)]
        methods.append(max(cands, key=lambda m: m["snr_train_db"]))   # rho chosen on the training set
    best15 = methods[-1]["rho"]
    free = [run_method("cb-essfm-free", link, train, test, rx, steps=st, n_sb=2, rho=best15, n_taps=taps, **common)
            for st in (15, 30)]
    vs_nsb = [run_method("cb-essfm", link, train, test, rx, steps=15, n_sb=n, rho=0.5, n_taps=min(taps, block // n),
                         **common) for n in (1, 2, 4, 8)]
    vs_rho = [run_method("cb-essfm", link, train, test, rx, steps=15, n_sb=2, rho=r, n_taps=taps, **common)
              for r in (0.0, 0.1, 0.2, 0.3, 0.4, 0.5)]
    t_fit = time.perf_counter() - t0
    keep = ("method", "steps", "n_sb", "rho", "snr_test_db", "snr_train_db", "snr_start_test_db", "rm", "half_taps",
            "snr_tied_test_db", "snr_tied_train_db", "gvd_km")
    trim = lambda rs: [{k: r[k] for k in keep if k in r} for r in rs]   # noqa: E731
    return {"workload": PROTO_WORKLOAD, "dbp_rate_hz": rate, "block": block, "overlap": d["n_overlap"],
            "train": "2 realisations (seeds 6000-6001)", "test": "2 realisations (seeds 6100-6101)",
            "fit": f"tied sequential protocol, Adam on the adjoint gradient, {args.proto_iters} iterations per row",
            "methods_vs_steps": trim(methods), "snr_vs_n_sb": trim(vs_nsb), "snr_vs_rho": trim(vs_rho),
            "free_steps": trim(free),
            "data_generation_s": t_gen, "fits_s": t_fit}


# ------------------------------------------------------------------ long link: streaming path, step sweep
LONG_WORKLOAD = "5ch-64GBd-64QAM-2^20sym-40x80km"
LONG_GEN_STEPS_PER_SPAN = 20   # forward-link simulator steps per span for the long-link field


def stream_bytes_per_block(n_sb, n_sub, n_ov, steps, n_taps):
    """Device-memory bytes one block moves through the streaming kernels, each
    kernel reading and writing its operands once: per (subband, sample) cell
    of 16 B (both polarisations) the row kernel reads and writes the cell,
    the intensity kernel reads it and writes 4 B, the filter reads the
    intensities (with its halo) and writes 4 B, the rotation kernel reads the
    cell and 4 B and writes the cell; the block's input read and kept output
    write, the forward/inverse block transforms and the two MUX/DEMUX passes
    add the rest."""
    n = n_sb * n_sub
    nc = n_taps // 2
    per_step = 32 + (16 + 4) + (4 * (1 + 2 * nc / 256) + 4) + (16 + 4 + 16)
    head = 16 + 16 + 32 + (32 if n_sb > 1 else 0)                  # read input, column pass, row pass, DEMUX
    tail = 32 + (32 + 32 if n_sb > 1 else 0) + 16 + 16 * (n - n_ov) / n
    return n * (head + steps * per_step + tail)


def leg_longlink(args):
    """Five channels over 40 x 80 km (N' = 2^17 per subband, N_ov = 196608):
    throughput, device-memory roofline and SNR against dispersion-only
    compensation for each step count of the sweep, with analytic coefficients
    and with coefficients and split ratio fitted on the device; sampled
    parity with the FP64 oracle at 5 and 80 steps.

    The fit (Sec. III-B: minimum MSE of the matched-filtered symbols of all
    five channels) runs on a training realisation and every SNR is measured
    on a second, independent one.  It starts from the analytic coefficients
    scaled by the best of a few factors (one forward pass each; the analytic
    taps of a very long step overshoot) and takes ``--fit-iters`` Adam
    iterations of forward + streaming adjoint with recomputation every 8
    steps (8 / steps times as many below 8 steps, where they are cheap)."""
    import numpy as np
    import torch
    from paper_2409_14489_amd import Plan, analytic_coeffs
    from paper_2409_14489_amd.autograd import cbessfm
    from paper_2409_14489_amd.train import SymbolReceiver, fit, receiver_mse
    from synth import workload

    t0 = time.perf_counter()
    x128, syms, w = workload(LONG_WORKLOAD, 5001, steps_per_span=LONG_GEN_STEPS_PER_SPAN)
    xin = x128.to(torch.complex64).contiguous()
    del x128
    x128, syms_tr, _ = workload(LONG_WORKLOAD, 5002, steps_per_span=LONG_GEN_STEPS_PER_SPAN)
    x_tr = x128.to(torch.complex64).contiguous()
    del x128
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = link_of(ch, wdm.sample_rate)
    t_len = xin.shape[-1]
    yout = torch.empty_like(xin)
    p_w = 1e-3 * 10 ** (wdm.power_dbm_per_channel / 10)
    offsets = (np.arange(wdm.n_channels) - (wdm.n_channels - 1) / 2.0) * wdm.spacing
    rxs = [SymbolReceiver(t_len, wdm.sample_rate, wdm.baud, wdm.rolloff, p_w, offset_hz=float(off))
           for off in offsets]
    sym_te = [torch.from_numpy(syms[c].astype(np.complex64)).cuda() for c in range(wdm.n_channels)]
    sym_tr = [torch.from_numpy(syms_tr[c].astype(np.complex64)).cuda() for c in range(wdm.n_channels)]

    def snr_per_channel(y):
        return [-10 * math.log10(float(receiver_mse(y, rx, s))) for rx, s in zip(rxs, sym_te)]

    fit_ck = 8
    n2d = wdm.n_channels * 2 * wdm.n_symbols
    stream = torch.cuda.current_stream()
    reps = max(3, min(20, args.steps // 10))
    rows = []
    parity = None
    memory = None
    for steps in (0,) + tuple(d["step_sweep"]):
        edc = steps == 0
        st = 1 if edc else steps
        coeffs = (np.zeros((1, d["n_sb"], d["n_sb"], 1), np.float32) if edc else
                  analytic_coeffs(link, d["n_sb"], st, d["rho"], d["n_taps"]).astype(np.float32))
        plan = Plan(link, d["n_sb"], d["n_sub"], d["n_overlap"], st, d["rho"], coeffs=coeffs)
        for _ in range(2):
            plan.run(xin, out=yout)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run(xin, out=yout)
        graph.replay()
        run_s = timed_events(stream, graph.replay, reps)
        if plan.status() != 0:
            raise RuntimeError("device error flag set in the long-link run")
        del graph
        nblk = plan.n_blocks(t_len)
        moved = stream_bytes_per_block(d["n_sb"], d["n_sub"], d["n_overlap"], st, coeffs.shape[-1]) * nblk
        snr = snr_per_channel(yout)
        row = {"steps": st, "method": "edc" if edc else "cb-essfm", "ms_per_run": run_s * 1e3,
               "value": n2d / run_s, "unit": "2D-symbols/s",
               "hbm_roofline": {"bound": "hbm", "achieved": moved / run_s / 1e9, "peak": PEAK_HBM_GBS,
                                "unit": "GB/s", "frac": moved / run_s / 1e9 / PEAK_HBM_GBS,
                                "bytes_per_run": moved},
               "min_bytes_frac": 2 * 2 * t_len * 8 / run_s / 1e9 / PEAK_HBM_GBS,
               "snr_db_per_channel": snr, "snr_db_central": snr[len(snr) // 2]}
        if not edc:  # the method's operation count against the FP32 vector peak
            fl = long_link_flops_per_2d_symbol(st) * n2d
            row["flop_roofline"] = {"bound": "alu", "achieved": fl / run_s / 1e12, "peak": PEAK_FP32_TFLOPS,
                                    "unit": "TFLOP/s", "frac": fl / run_s / 1e12 / PEAK_FP32_TFLOPS,
                                    "flops_per_2d_symbol": long_link_flops_per_2d_symbol(st)}
        if not edc:
            row["snr_db_central_analytic"] = row.pop("snr_db_central")
            row["snr_db_per_channel_analytic"] = row.pop("snr_db_per_channel")
        if not edc and args.fit_iters > 0:
            c_an = torch.from_numpy(coeffs).cuda()
            rho_t = torch.tensor(d["rho"], dtype=torch.float32, device="cuda")
            with torch.no_grad():
                trial = {a: float(receiver_mse(cbessfm(x_tr, (a * c_an).contiguous(), rho_t, plan), rxs, sym_tr))
                         for a in (1 / 32, 1 / 16, 0.125, 0.25, 0.5, 1.0)}
            alpha = min(trial, key=trial.get)
            iters = max(args.fit_iters, (8 * args.fit_iters) // st)   # short runs are cheap: more iterations
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            c_fit, rho_fit, losses = fit(plan, x_tr, sym_tr, rxs, alpha * c_an, d["rho"], iters=iters,
                                         lr=1e-2, checkpoint_every=fit_ck)
            ev1.record(stream)
            torch.cuda.synchronize()
            fit_ms = ev0.elapsed_time(ev1) / iters
            with torch.no_grad():
                y_fit = cbessfm(xin, c_fit.contiguous(), rho_fit.reshape(()), plan)
            snr_fit = snr_per_channel(y_fit)
            del y_fit
            ls = losses.cpu().numpy()
            row["fit"] = {"iters": iters, "lr": 1e-2, "checkpoint_every": fit_ck, "alpha": alpha,
                          "alpha_trial_mse": trial, "mse_first": float(ls[0]), "mse_last": float(ls[-1]),
                          "rho": float(rho_fit), "ms_per_iter": fit_ms,
                          "grad_steps_per_s": 1e3 / fit_ms,
                          "snr_db_per_channel": snr_fit, "snr_db_central": snr_fit[len(snr_fit) // 2]}
            if st == max(d["step_sweep"]):
                memory = {"steps": st, "workspace_bytes_ck8": plan.backward_workspace(t_len, 1, fit_ck),
                          "workspace_bytes_every_step": plan.backward_workspace(t_len, 1, 1),
                          "peak_allocated_bytes": torch.cuda.max_memory_allocated()}
            del c_an
        rows.append(row)
        if not args.no_cpu and st in (5, 80) and not edc:
            import oracle
            x_host = xin.cpu().numpy().astype(np.complex128)
            oplan = oracle_plan({**d, "n_steps": st}, wdm.sample_rate, ch.span_km * ch.n_spans / st, coeffs,
                                ch.beta2_ps2_km)
            pick = [0, nblk - 1] if st == 5 else [nblk // 2]
            c0 = time.perf_counter()
            p0 = time.process_time()
            ref = oracle.run_blocks(x_host, oplan, pick)
            cpu_s = time.perf_counter() - c0
            proc_s = time.process_time() - p0
            got = yout.cpu().numpy().astype(np.complex128)
            num = den = 0.0
            for b, r in ref.items():
                seg = got[:, b * plan.hop:b * plan.hop + r.shape[-1]]
                r = r[:, :seg.shape[-1]]
                num += float(np.sum(np.abs(seg - r) ** 2))
                den += float(np.sum(np.abs(r) ** 2))
            per_blk_2d = plan.hop / (wdm.sample_rate / wdm.baud) * 2   # 2D symbols per kept hop
            parity = parity or {}
            parity[f"steps_{st}"] = {"blocks": pick, "rel_l2": (num / den) ** 0.5,
                      "cpu_baseline": {"value": per_blk_2d * len(pick) / cpu_s, "unit": "2D-symbols/s",
                                       "cores": max(1, round(proc_s / cpu_s)), "kind": "oracle",
                                       "sample": f"{len(pick)} blocks of N = {plan.block}, {st} steps, "
                                                 f"{cpu_s:.1f} s"}}
        plan.close()
        print(f"longlink {st} steps done", file=sys.stderr, flush=True)
    return {"workload": LONG_WORKLOAD, "T": t_len, "n_sb": d["n_sb"], "block_sb": d["n_sub"],
            "overlap": d["n_overlap"], "n_taps": d["n_taps"], "split_ratio": d["rho"],
            "kernels": "streaming forward and adjoint (stream.hip); timed runs graph-replayed",
            "data": f"two seeded 5-channel fields (fit on one, SNR on the other), 40 x 80 km Manakov link "
                    f"simulated on the device at {LONG_GEN_STEPS_PER_SPAN} steps/span, ASE at NF {ch.nf_db:g} dB",
            "coefficients": "analytic, and fitted on the device (mean MSE of the five channels)",
            "sweep": rows, "fit_memory": memory, "parity_sampled": parity, "data_generation_s": t_gen}


def leg_streamgrad(args):
    """Streaming forward and adjoint at the long-link block shape (5 subbands
    of N' = 2^17, N_ov = 196608, 21 analytic taps, 40 x 80 km in 10 steps) on
    a seeded complex Gaussian field of 23 blocks: HIP-event times of the
    forward and of the adjoint with recomputation every 8 steps (which also
    runs the forward sweep), and the adjoint's workspace."""
    import numpy as np
    import torch
    from paper_2409_14489_amd import LinkSpec, Plan, analytic_coeffs

    steps, ck = 10, 8
    link = LinkSpec(beta2_ps2_km=-21.7, n_spans=40, span_km=80.0, sample_rate_hz=640e9)
    c = analytic_coeffs(link, 5, steps, 0.3, 21).astype(np.float32)
    plan = Plan(link, 5, 2 ** 17, 196608, steps, 0.3, coeffs=c)
    t_len = 5 * 2 ** 21
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    x = (torch.randn((2, t_len), dtype=torch.complex64, device="cuda", generator=gen) * 0.05).contiguous()
    go = torch.randn((2, t_len), dtype=torch.complex64, device="cuda", generator=gen).contiguous()
    y = plan.run(x)
    ws = torch.empty(plan.backward_workspace(t_len, 1, ck), dtype=torch.uint8, device="cuda")
    plan.backward(x, go, need_grad_in=False, checkpoint_every=ck, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    fwd_s = timed_events(stream, lambda: plan.run(x, out=y), 5)
    bwd_s = timed_events(stream, lambda: plan.backward(x, go, need_grad_in=False, checkpoint_every=ck,
                                                        workspace=ws), 2)
    if plan.status() != 0:
        raise RuntimeError("device error flag set in the streaming adjoint run")
    out = {"shape": "5 subbands x N' = 2^17, N_ov = 196608, 21 taps, 10 steps, T = 5 x 2^21 (23 blocks)",
           "forward_ms": fwd_s * 1e3, "adjoint_ms": bwd_s * 1e3, "checkpoint_every": ck,
           "workspace_bytes": plan.backward_workspace(t_len, 1, ck)}
    plan.close()
    return out


def leg_cfg1(args):
    """The single-channel workload (1 ch 32 GBd DP-16QAM, 2^14 symbols, 1 x 80 km,
    1 step, 11 taps, N' = 1024, N_ov = 128): forward throughput from graph
    replays, full-field parity and the oracle timed on the same field."""
    import numpy as np
    import torch
    from paper_2409_14489_amd import Plan, analytic_coeffs
    from synth import workload

    x, _, w = workload(CFG1_WORKLOAD, 1001)
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = link_of(ch, wdm.sample_rate)
    coeffs = analytic_coeffs(link, d["n_sb"], d["n_steps"], d["rho"], d["n_taps"]).astype(np.float32)
    plan = Plan(link, d["n_sb"], d["n_sub"], d["n_overlap"], d["n_steps"], d["rho"], coeffs=coeffs)
    xin = torch.from_numpy(x.astype(np.complex64)).cuda()
    yout = torch.empty_like(xin)
    for _ in range(5):
        plan.run(xin, out=yout)
    per_graph = 20
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(per_graph):
            plan.run(xin, out=yout)
    graph.replay()
    stream = torch.cuda.current_stream()
    run_s = timed_events(stream, graph.replay, 20) / per_graph
    if plan.status() != 0:
        raise RuntimeError("device error flag set in the single-channel leg")
    del graph
    n2d = wdm.n_channels * 2 * wdm.n_symbols
    t_len = x.shape[-1]
    nblk = plan.n_blocks(t_len)
    flops = FLOPS_PER_2D_SYMBOL[CFG1_WORKLOAD] * n2d
    out = {"workload": CFG1_WORKLOAD, "T": t_len, "blocks": nblk, "value": n2d / run_s, "unit": "2D-symbols/s",
           "ms_per_run": run_s * 1e3, "flops_per_run": flops, "tflops": flops / run_s / 1e12,
           "hbm_gbs_algorithmic": 2 * 2 * t_len * 8 / run_s / 1e9,
           "launch": f"HIP graph replays, {per_graph} launches per replay"}
    if not args.no_cpu:
        import oracle
        oplan = oracle_plan(d, wdm.sample_rate, ch.span_km * ch.n_spans / d["n_steps"], coeffs, ch.beta2_ps2_km)
        passes, cpu_s, proc_s, ref = time_oracle(lambda: oracle.run(x, oplan), min_s=5.0)
        got = yout.cpu().numpy().astype(np.complex128)
        out["parity_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["parity_rel_l2_worst_block"] = worst_block_err(got, ref, plan.hop, plan.block, d["n_overlap"])
        out["cpu_baseline"] = {"value": n2d * passes / cpu_s, "unit": "2D-symbols/s",
                               "cores": max(1, round(proc_s / cpu_s)), "kind": "oracle",
                               "sample": f"the whole field, {passes} passes, {cpu_s:.1f} s", **host_identity()}
    plan.close()
    return out


def leg_cover(args):
    """The five-channel 15 x 80 km field backpropagated with an overlap that
    covers the link's group-delay spread 2 pi |beta2| L R^2 (6.7e4 samples at
    640 GS/s, Sec. III-A): 5 subbands of N' = 2^15 (N = 163840, streaming
    path), N_ov = 67584, 15 steps, 21 analytic taps.  The primary line keeps
    the workload's literal N' = 4096 / N_ov = 2560 framing; this leg gives the
    throughput of a framing that undoes the whole dispersion memory, its SNR
    beside the literal framing's, and sampled oracle parity."""
    import numpy as np
    import torch
    from paper_2409_14489_amd import Plan, analytic_coeffs
    from paper_2409_14489_amd.train import SymbolReceiver, receiver_mse
    from synth import workload

    x, syms, w = workload(WORKLOAD, 2001, steps_per_span=GEN_STEPS_PER_SPAN)
    d, wdm, ch = w["dbp"], w["wdm"], w["ch"]
    link = link_of(ch, wdm.sample_rate)
    spread = 2 * math.pi * abs(ch.beta2_ps2_km) * 1e-24 * ch.span_km * ch.n_spans * wdm.sample_rate ** 2
    n_sub, n_ov = 2 ** 15, 2 * int(math.ceil(spread / 2 / 512.0)) * 512
    coeffs = analytic_coeffs(link, d["n_sb"], d["n_steps"], d["rho"], d["n_taps"]).astype(np.float32)
    xin = torch.from_numpy(x.astype(np.complex64)).cuda()
    t_len = x.shape[-1]
    n2d = wdm.n_channels * 2 * wdm.n_symbols
    p_w = 1e-3 * 10 ** (wdm.power_dbm_per_channel / 10)
    offsets = (np.arange(wdm.n_channels) - (wdm.n_channels - 1) / 2.0) * wdm.spacing
    rxs = [SymbolReceiver(t_len, wdm.sample_rate, wdm.baud, wdm.rolloff, p_w, offset_hz=float(off))
           for off in offsets]
    sym = [torch.from_numpy(syms[c].astype(np.complex64)).cuda() for c in range(wdm.n_channels)]
    stream = torch.cuda.current_stream()
    out = {"workload": WORKLOAD, "group_delay_spread_samples": spread, "unit": "2D-symbols/s"}
    for name, nsub, nov in (("covering", n_sub, n_ov), ("literal", d["n_sub"], d["n_overlap"])):
        plan = Plan(link, d["n_sb"], nsub, nov, d["n_steps"], d["rho"], coeffs=coeffs)
        y = torch.empty_like(xin)
        for _ in range(2):
            plan.run(xin, out=y)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.run(xin, out=y)
        graph.replay()
        run_s = timed_events(stream, graph.replay, 10)
        if plan.status() != 0:
            raise RuntimeError("device error flag set in the covering-overlap leg")
        del graph
        snr = [-10 * math.log10(float(receiver_mse(y, rx, s))) for rx, s in zip(rxs, sym)]
        row = {"block_sb": nsub, "overlap": nov, "blocks": plan.n_blocks(t_len), "ms_per_run": run_s * 1e3,
               "value": n2d / run_s, "snr_db_central": snr[len(snr) // 2], "snr_db_per_channel": snr}
        if name == "covering" and not args.no_cpu:
            import oracle
            oplan = oracle.OraclePlan(ch.beta2_ps2_km * 1e-24, wdm.sample_rate, ch.span_km * ch.n_spans /
                                      d["n_steps"], d["n_steps"], d["rho"], d["n_sb"], d["n_sb"] * nsub, nov,
                                      np.asarray(coeffs, np.float64))
            pick = [plan.n_blocks(t_len) // 2]
            ref = oracle.run_blocks(x, oplan, pick)
            got = y.cpu().numpy().astype(np.complex128)
            num = den = 0.0
            for b, r in ref.items():
                seg = got[:, b * plan.hop:b * plan.hop + r.shape[-1]]
                r = r[:, :seg.shape[-1]]
                num += float(np.sum(np.abs(seg - r) ** 2))
                den += float(np.sum(np.abs(r) ** 2))
            row["parity_rel_l2_sampled"] = (num / den) ** 0.5
            row["parity_blocks"] = pick
        out[name] = row
        plan.close()
    out["value"] = out["covering"]["value"]
    out["ms_per_run"] = out["covering"]["ms_per_run"]
    return out


HEADLINE_KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                 "scaling", "vs_baseline", "dtype", "data")


def headline(result):
    """The compact record of the primary workload (the bench's last line)."""
    line = {k: result[k] for k in HEADLINE_KEYS if k in result}
    cfg = result["config"]
    line["config"] = {k: cfg[k] for k in ("workload", "T", "batch", "n_sb", "block_sb", "overlap", "steps",
                                          "split_ratio", "n_taps", "fir_mode", "blocks", "kernel") if k in cfg}
    line["config"]["fwd_kernel_source_sha256"] = cfg.get("fwd_kernel_source_sha256", "")[:16]
    rf = result["roofline"]
    line["roofline"] = {k: rf.get(k) for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                               "flops_per_launch", "kernel_ms")}
    line["hbm_roofline"] = {k: result["hbm_roofline"][k] for k in ("achieved", "peak", "unit", "frac")}
    if "cpu_baseline" in result:
        line["cpu_baseline"] = result["cpu_baseline"]
    for k in ("parity_rel_l2", "parity_rel_l2_worst_block"):
        if k in result:
            line[k] = result[k]
    g = result.get("grad")
    if g:
        line["grad"] = {"steps_per_s": g.get("value"), "unit": "steps/s", "workload": g.get("workload"),
                        "parity_rel_l2": g.get("parity_rel_l2")}
    c1 = result.get("cfg1")
    if c1:
        line["cfg1"] = {"value": c1["value"], "ms_per_run": c1["ms_per_run"],
                        "parity_rel_l2": c1.get("parity_rel_l2"),
                        "cpu_baseline": (c1.get("cpu_baseline") or {}).get("value")}
    cv = result.get("cover")
    if cv:
        line["cover"] = {"value": cv["value"], "ms_per_run": cv["ms_per_run"], "block_sb": cv["covering"]["block_sb"],
                         "overlap": cv["covering"]["overlap"]}
    b = result.get("batched")
    if b:
        line["batched"] = {"value": b["value"], "speedup_vs_separate": b["speedup_vs_separate"],
                           "persistent_launches_per_run": b["persistent_launches_per_run"],
                           "streamed": b.get("streamed_instances"),
                           "stream_classes": b.get("stream_classes"),
                           "kernel_launches_per_run": b.get("kernel_launches_per_run"),
                           "instances_overlap_covers_memory": b["instances_overlap_covers_memory"]}
    line["legs_file"] = result.get("legs_file")
    return rounded(line)


def rounded(obj, digits=5):
    """Floats of a record to `digits` significant digits (the full values are in
    the legs file)."""
    if isinstance(obj, float):
        return float(f"{obj:.{digits}g}")
    if isinstance(obj, dict):
        return {k: rounded(v, digits) for k, v in obj.items()}
    if isinstance(obj, list):
        return [rounded(v, digits) for v in obj]
    return obj


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--legs", default="cfg1,grad,cover,batched,protocol,longlink,streamgrad")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--proto-iters", type=int, default=60)
    ap.add_argument("--fit-iters", type=int, default=20)
    ap.add_argument("--out", default=os.path.join("gpurun_out", "bench_legs.json"),
                    help="file that receives every leg's full record")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(the path would shard over blocks and batch instances, one process per GPU)", file=sys.stderr)
        sys.exit(2)
    legs = [leg for leg in args.legs.split(",") if leg]

    import torch
    torch.cuda.set_device(0)
    result = leg_forward(args)
    print(json.dumps({"leg": "fwd", "value": result["value"], "ms_per_step": result["ms_per_step"],
                      "roofline_frac": result["roofline"]["frac"]}), flush=True)
    runners = {"cfg1": leg_cfg1, "grad": leg_grad, "batched": leg_batched, "protocol": leg_protocol,
               "longlink": leg_longlink, "streamgrad": leg_streamgrad, "cover": leg_cover}
    for leg in legs:
        if leg not in runners:
            raise SystemExit(f"unknown leg {leg!r}")
        result[leg] = runners[leg](args)
        # one short line per leg as it ends (the full record goes to --out)
        rec = result[leg]
        brief = {"leg": leg, **{k: rec[k] for k in ("value", "unit", "ms_per_run", "parity_rel_l2") if k in rec}}
        print(json.dumps(brief)[:1500], flush=True)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as fh:
            json.dump(result, fh, indent=1)
        result["legs_file"] = args.out
    print(json.dumps(headline(result)), flush=True)


if __name__ == "__main__":
    main()
