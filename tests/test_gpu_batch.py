"""Batched execution, graph replay and the measured autotuner on the GPU.

Every instance of a batch must give what the FP64 oracle gives for it alone
(relative L2 <= 1e-5 over its output and over every block's kept samples),
and what cbessfm_run gives for it; launches recorded in
a HIP graph must give the eager result on every replay, with eager work and
changed inputs between replays.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import random_field
from test_gpu_forward import worst_block_rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
BETA2_PS2 = -21.7


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rand_coeffs(steps, n_sb, taps, phase_rad, power_w, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps))
    c *= phase_rad / (power_w * np.abs(c).sum(axis=(2, 3), keepdims=True))
    return c.astype(np.float32)


# (n_sb, N', overlap, steps, rho, taps, T, batch, boundary, spans)
SHAPES = [
    (1, 1024, 128, 3, 0.5, 11, 9000, 1, "circular", 1),
    (2, 1024, 256, 2, 0.3, 7, 20000, 2, "circular", 2),
    (3, 1024, 384, 4, 0.2, 9, 7000, 1, "zero", 3),
    (5, 1024, 640, 1, 0.5, 21, 30000, 1, "circular", 5),
    (2, 1024, 256, 5, 0.7, 5, 1500, 1, "circular", 1),     # T < N: a block wraps
    (2, 512, 128, 3, 0.4, 5, 6000, 1, "circular", 2),      # second N' class
    (1, 512, 64, 2, 0.5, 3, 4000, 3, "zero", 1),
    (2, 8192, 2048, 3, 0.3, 9, 70000, 1, "circular", 3),   # third class: one workgroup per polarisation
    (1, 8192, 1024, 2, 0.5, 5, 20000, 2, "zero", 2),
    (5, 8192, 10240, 2, 0.3, 21, 70000, 1, "circular", 4),  # a team of 10 workgroups
]


def make_instances(shapes, seed0=0):
    from paper_2409_14489_amd import LinkSpec, Plan
    power = 4e-3
    out = []
    for k, (nsb, np_, ov, steps, rho, taps, t_len, batch, bnd, spans) in enumerate(shapes):
        rate = nsb * 64e9
        c = rand_coeffs(steps, nsb, taps, 0.5, power, seed0 + k)
        link = LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=spans, sample_rate_hz=rate)
        plan = Plan(link, nsb, np_, ov, steps, rho, coeffs=c, boundary=bnd)
        o = oracle.OraclePlan(BETA2_PS2 * 1e-24, rate, 80.0 * spans / steps, steps, rho, nsb, nsb * np_, ov,
                              c.astype(np.float64), boundary=bnd)
        shape = (batch, 2, t_len) if batch > 1 else (2, t_len)
        x = random_field(shape, 500 + seed0 + k, power_w=power)
        xt = torch.from_numpy(x.astype(np.complex64)).cuda()
        out.append(dict(plan=plan, oracle=o, x=x, xt=xt, yt=torch.empty_like(xt)))
    return out


def test_batch_matches_oracle_and_single_runs():
    from paper_2409_14489_amd import Batch
    insts = make_instances(SHAPES)
    b = Batch([(d["plan"], d["xt"], d["yt"]) for d in insts])
    info = b.info()
    print(info)
    assert info["launches"] == 3 and info["items"] > 0
    b.run()
    torch.cuda.synchronize()
    assert b.status() == 0
    for k, d in enumerate(insts):
        got = d["yt"].cpu().numpy().astype(np.complex128)
        ref = oracle.run(d["x"], d["oracle"])
        single = d["plan"].run(d["xt"])
        torch.cuda.synchronize()
        e_or = rel_l2(got, ref)
        e_blk = worst_block_rel_l2(got, ref, d["plan"].hop)
        e_single = rel_l2(got, single.cpu().numpy().astype(np.complex128))
        print(k, SHAPES[k][:4], "vs oracle", e_or, "worst block", e_blk, "vs single run", e_single)
        assert e_or < TOL and e_blk < TOL
        assert e_single < 1e-6
    # a second run of the same batch (device-side round counters) gives the same bytes
    first = [d["yt"].clone() for d in insts]
    b.run()
    torch.cuda.synchronize()
    assert b.status() == 0
    for f, d in zip(first, insts):
        assert torch.equal(f, d["yt"])
    b.close()
    for d in insts:
        d["plan"].close()


def test_batch_of_many_uneven_instances():
    """Forty instances of 1-5 subbands, 1-12 steps and log-uniform lengths in one launch."""
    from paper_2409_14489_amd import Batch
    rng = np.random.default_rng(77)
    shapes = []
    for _ in range(40):
        nsb = int(rng.integers(1, 6))
        steps = int(rng.integers(1, 13))
        t_len = int(2 ** rng.uniform(11, 15)) * nsb
        taps = int(rng.choice([3, 9, 17]))
        shapes.append((nsb, 1024, 128 * nsb, steps, float(rng.uniform(0.1, 0.9)), taps, t_len, 1, "circular",
                       int(rng.integers(1, 6))))
    insts = make_instances(shapes, seed0=1000)
    b = Batch([(d["plan"], d["xt"], d["yt"]) for d in insts])
    info = b.info()
    print(info)
    assert info["launches"] == 1
    b.run()
    torch.cuda.synchronize()
    assert b.status() == 0
    worst = 0.0
    for d in insts:
        got = d["yt"].cpu().numpy().astype(np.complex128)
        ref = oracle.run(d["x"], d["oracle"])
        worst = max(worst, rel_l2(got, ref), worst_block_rel_l2(got, ref, d["plan"].hop))
    print("worst rel L2 (whole outputs and single blocks)", worst)
    assert worst < TOL
    b.close()


def test_batch_graph_replays_match_eager():
    from paper_2409_14489_amd import Batch
    insts = make_instances(SHAPES[:4], seed0=50)
    b = Batch([(d["plan"], d["xt"], d["yt"]) for d in insts])
    b.run()  # eager warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        # new inputs in place, eager work in between, then a replay
        for k, d in enumerate(insts):
            new = random_field(tuple(d["xt"].shape), 900 + 10 * rep + k, power_w=4e-3)
            d["xt"].copy_(torch.from_numpy(new.astype(np.complex64)))
            d["x"] = new
        eager = [d["plan"].run(d["xt"]) for d in insts]
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert b.status() == 0
        for d, e in zip(insts, eager):
            err = rel_l2(d["yt"].cpu().numpy().astype(np.complex128), e.cpu().numpy().astype(np.complex128))
            assert err < 1e-6, (rep, err)
        ref = oracle.run(insts[0]["x"], insts[0]["oracle"])
        assert rel_l2(insts[0]["yt"].cpu().numpy().astype(np.complex128), ref) < TOL
    del g
    b.close()


def test_single_plan_graph_replays_forward_and_adjoint():
    from paper_2409_14489_amd import LinkSpec, Plan
    power = 4e-3
    c = rand_coeffs(3, 2, 7, 0.5, power, 5)
    plan = Plan(LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=2, sample_rate_hz=128e9), 2, 1024, 256, 3, 0.3,
                coeffs=c)
    x = torch.from_numpy(random_field((2, 12000), 61, power_w=power).astype(np.complex64)).cuda()
    gout = torch.from_numpy(random_field((2, 12000), 62, power_w=1.0).astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    ws = torch.empty(plan.backward_workspace(12000, 1, 2), dtype=torch.uint8, device="cuda")
    plan.run(x, out=y)
    plan.backward(x, gout, checkpoint_every=2, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(x, out=y)
        gi, gc, gr = plan.backward(x, gout, checkpoint_every=2, workspace=ws)
    for rep in range(3):
        x.copy_(torch.from_numpy(random_field((2, 12000), 70 + rep, power_w=power).astype(np.complex64)))
        y_e = plan.run(x)
        gi_e, gc_e, gr_e = plan.backward(x, gout, checkpoint_every=2)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert plan.status() == 0
        assert rel_l2(y.cpu().numpy(), y_e.cpu().numpy()) < 1e-6
        assert rel_l2(gi.cpu().numpy(), gi_e.cpu().numpy()) < 1e-6
        assert rel_l2(gc.cpu().numpy(), gc_e.cpu().numpy()) < 1e-6
        assert abs(float(gr) - float(gr_e)) <= 1e-6 * max(1.0, abs(float(gr_e)))
    del g
    plan.close()


def test_many_launches_keep_exchange_consistent():
    """200 launches of one plan: the per-team round counters advance on the
    device and the last result equals the first, byte for byte."""
    from paper_2409_14489_amd import LinkSpec, Plan
    power = 4e-3
    c = rand_coeffs(2, 3, 5, 0.5, power, 8)
    plan = Plan(LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=1, sample_rate_hz=192e9), 3, 512, 192, 2, 0.5, coeffs=c)
    x = torch.from_numpy(random_field((2, 40000), 63, power_w=power).astype(np.complex64)).cuda()
    first = plan.run(x)
    y = torch.empty_like(x)
    for _ in range(200):
        plan.run(x, out=y)
    torch.cuda.synchronize()
    assert plan.status() == 0
    assert torch.equal(first, y)
    plan.close()


def test_measured_autotune_gives_a_working_plan():
    from paper_2409_14489_amd import LinkSpec, Plan, autotune
    link = LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=3, sample_rate_hz=128e9)
    t_len = 50000
    tun = autotune(link, 2, 4, 9, t_len, measure=True)
    print(tun)
    assert tun["measured"] == 1 and tun["covered"] == 1
    assert tun["overlap"] >= tun["memory"] and tun["overlap"] % 2 == 0
    assert 2 * tun["block_sb"] > tun["overlap"] and tun["predicted_s"] > 0
    power = 4e-3
    c = rand_coeffs(4, 2, 9, 0.5, power, 9)
    plan = Plan(link, 2, tun["block_sb"], tun["overlap"], 4, 0.5, coeffs=c)
    x = random_field((2, t_len), 64, power_w=power)
    y = plan.run(torch.from_numpy(x.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    assert plan.status() == 0
    o = oracle.OraclePlan(BETA2_PS2 * 1e-24, 128e9, 240.0 / 4, 4, 0.5, 2, 2 * tun["block_sb"], tun["overlap"],
                          c.astype(np.float64))
    assert rel_l2(y.cpu().numpy().astype(np.complex128), oracle.run(x, o)) < TOL
    plan.close()


def test_batch_with_streamed_instances_matches_oracle_block_by_block():
    """Instances whose blocks are streamed (N' = 2^14 and 2^15) in one batch
    with persistent ones: every instance equals the FP64 oracle over its whole
    output and over every block, equals its own cbessfm_run, and a HIP graph
    of the run replays to the same bytes."""
    from paper_2409_14489_amd import Batch
    shapes = [
        (2, 2 ** 14, 4096, 3, 0.3, 7, 40000, 1, "circular", 2),
        (1, 1024, 128, 2, 0.5, 11, 9000, 1, "circular", 1),
        (1, 2 ** 15, 8192, 2, 0.5, 9, 70001, 1, "zero", 3),
        (3, 512, 192, 2, 0.4, 5, 6000, 2, "circular", 2),
    ]
    insts = make_instances(shapes, seed0=2000)
    b = Batch([(d["plan"], d["xt"], d["yt"]) for d in insts])
    info = b.info()
    print(info)
    assert info["streamed"] == 2 and info["launches"] == 2
    b.run()
    torch.cuda.synchronize()
    assert b.status() == 0
    eager = [d["yt"].clone() for d in insts]
    for k, d in enumerate(insts):
        got = d["yt"].cpu().numpy().astype(np.complex128)
        ref = oracle.run(d["x"], d["oracle"])
        e_or, e_blk = rel_l2(got, ref), worst_block_rel_l2(got, ref, d["plan"].hop)
        single = d["plan"].run(d["xt"])
        torch.cuda.synchronize()
        print(k, shapes[k][:4], "vs oracle", e_or, "worst block", e_blk)
        assert e_or < TOL and e_blk < TOL
        assert torch.equal(single, eager[k])
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run()
    for _ in range(2):
        for d in insts:
            d["yt"].zero_()
        graph.replay()
        torch.cuda.synchronize()
        _ = float(insts[0]["xt"].abs().sum())      # eager work between replays
        for d, e in zip(insts, eager):
            assert torch.equal(d["yt"], e)
    del graph
    assert b.status() == 0
    b.close()
    for d in insts:
        d["plan"].close()


def test_batch_streamed_classes_match_single_runs():
    """Streamed instances of one class (N' = 2^14, two subbands, 7 taps) with
    4, 2 and 3 steps run their steps as shared launches over all their blocks
    (the blocks of the instances still stepping); two instances that share a
    plan run one by one.  Every output equals the instance's own cbessfm_run
    bit for bit, and the FP64 oracle to the parity bar, also after a graph
    replay."""
    from paper_2409_14489_amd import Batch
    shapes = [
        (2, 2 ** 14, 4096, 4, 0.3, 7, 40000, 1, "circular", 2),
        (2, 2 ** 14, 2048, 2, 0.5, 7, 30000, 2, "zero", 1),
        (2, 2 ** 14, 4096, 3, 0.4, 7, 25000, 1, "circular", 2),
        (1, 1024, 128, 2, 0.5, 11, 9000, 1, "circular", 1),
    ]
    insts = make_instances(shapes, seed0=2100)
    # a second field on the plan of instance 2: both of its instances run alone
    x_extra = random_field((2, 25000), 777, power_w=4e-3)
    extra = dict(plan=insts[2]["plan"], oracle=insts[2]["oracle"], x=x_extra,
                 xt=torch.from_numpy(x_extra.astype(np.complex64)).cuda())
    extra["yt"] = torch.empty_like(extra["xt"])
    insts.append(extra)
    b = Batch([(d["plan"], d["xt"], d["yt"]) for d in insts])
    info = b.info()
    print(info)
    assert info["streamed"] == 4 and info["launches"] == 1
    assert info["stream_classes"] == 1 and info["stream_lone"] == 2
    # one persistent launch; the class: 3 input + 4 output kernels + 4 steps x 4
    # stages; each lone instance: 3 + 4 + 3 steps x 4
    assert info["kernel_launches"] == 1 + (7 + 16) + 2 * 19
    b.run()
    torch.cuda.synchronize()
    assert b.status() == 0
    eager = [d["yt"].clone() for d in insts]
    for k, d in enumerate(insts):
        single = d["plan"].run(d["xt"])
        torch.cuda.synchronize()
        assert torch.equal(single, eager[k]), k
    for k in (0, 1, 4):
        d = insts[k]
        got = eager[k].cpu().numpy().astype(np.complex128)
        ref = oracle.run(d["x"], d["oracle"])
        e_or, e_blk = rel_l2(got, ref), worst_block_rel_l2(got, ref, d["plan"].hop)
        print(k, "vs oracle", e_or, "worst block", e_blk)
        assert e_or < TOL and e_blk < TOL
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.run()
    for _ in range(2):
        for d in insts:
            d["yt"].zero_()
        graph.replay()
        torch.cuda.synchronize()
        _ = float(insts[0]["xt"].abs().sum())      # eager work between replays
        for d, e in zip(insts, eager):
            assert torch.equal(d["yt"], e)
    del graph
    assert b.status() == 0
    b.close()
    for d in insts[:4]:
        d["plan"].close()
