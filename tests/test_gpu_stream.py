"""Parity of the streaming forward (blocks of N' = 2^14 .. 2^17 per subband,
larger than one CU holds) with the FP64 oracle, through the C ABI.

Bar: relative L2 error <= 1e-5, complex FP32 against FP64, as for the
persistent kernel.  Where the oracle cannot run every block of a long record
it runs a sample of blocks (``oracle.run_blocks``), compared block by block.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import random_field

from test_gpu_forward import (TOL, assert_parity, case, gpu_plan, oracle_plan, rand_coeffs, rel_l2, run_gpu,
                              worst_block_rel_l2)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("block_sb", [2 ** 14, 2 ** 15, 2 ** 16, 2 ** 17])
def test_stream_parity_every_block_size_single_band(block_sb):
    """Three blocks and a ragged tail, 3 steps, 9 taps."""
    y, ref, hop = case(1, block_sb, block_sb // 4, 3, 0.3, 9, 2 * block_sb + 77, seed=block_sb)
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, hop)
    print(f"N'={block_sb}: rel L2 {err:.3e}, worst block {worst:.3e}")
    assert err < TOL and worst < TOL


@pytest.mark.parametrize("n_sb,block_sb", [(2, 2 ** 14), (3, 2 ** 15), (5, 2 ** 16), (8, 2 ** 14)])
def test_stream_parity_multiband(n_sb, block_sb):
    n = n_sb * block_sb
    y, ref, hop = case(n_sb, block_sb, n // 8, 3, 0.27, 7, 2 * n + 101, seed=n_sb, rate=n_sb * 64e9)
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, hop)
    print(f"n_sb={n_sb} N'={block_sb}: rel L2 {err:.3e}, worst block {worst:.3e}")
    assert err < TOL and worst < TOL


@pytest.mark.parametrize("n_sb,taps", [(1, 31), (2, 23), (3, 31), (4, 15), (5, 31), (6, 7), (7, 31), (8, 23)])
def test_stream_parity_matrix_core_filter(n_sb, taps):
    """The coupled filter on the matrix cores (up to 32 taps) packs 16 / n_sb
    outputs of every subband into a tile's rows: every subband count, with
    7 to 31 taps (padded windows of 8 to 32), two steps, a ragged tail."""
    n = n_sb * 2 ** 14
    y, ref, hop = case(n_sb, 2 ** 14, n // 8, 2, 0.4, taps, n + 3001, seed=100 + n_sb, rate=n_sb * 64e9)
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, hop)
    print(f"n_sb={n_sb} taps={taps}: rel L2 {err:.3e}, worst block {worst:.3e}")
    assert err < TOL and worst < TOL


@pytest.mark.parametrize("taps", [1, 21, 255])
def test_stream_parity_tap_counts(taps):
    y, ref, hop = case(2, 2 ** 14, 4096, 2, 0.5, taps, 50000, seed=taps, rate=128e9)
    assert_parity(y, ref, hop)


def test_stream_parity_zero_boundary_batch_and_short_sequence():
    y, ref, hop = case(2, 2 ** 14, 1024, 2, 0.4, 5, 40000, batch=3, boundary="zero", seed=9, rate=128e9)
    assert_parity(y, ref, hop)
    y, ref, hop = case(3, 2 ** 14, 512, 2, 0.3, 5, 1001, seed=11, rate=192e9)   # T < N: one block, wrapped
    assert_parity(y, ref, hop)


def test_stream_parity_split_extremes_and_many_steps():
    for rho in (0.0, 1.0):
        y, ref, hop = case(2, 2 ** 14, 2048, 3, rho, 5, 40000, seed=13, rate=128e9)
        assert_parity(y, ref, hop)
    y, ref, hop = case(1, 2 ** 15, 8192, 40, 0.5, 11, 70000, seed=14, spans=40, phase=0.05)
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, hop)
    print(f"40 steps: rel L2 {err:.3e}, worst block {worst:.3e}")
    assert err < TOL and worst < TOL


def test_stream_more_blocks_than_one_wave():
    """More blocks than the plan keeps state for: several waves per call;
    sampled blocks of each wave against the oracle, and a second run equal
    bit for bit."""
    power = 4e-3
    n_sb, block_sb, n_ov = 8, 2 ** 17, 2 ** 17
    c = rand_coeffs(2, n_sb, 5, 0.3, power, 21)
    g = gpu_plan(n_sb, block_sb, n_ov, 2, 0.3, c, rate=n_sb * 64e9)
    cap = g.info().team_capacity
    nblk = cap + 3
    t_len = nblk * g.hop - 1000
    assert g.n_blocks(t_len) > cap
    x = random_field((2, t_len), 31, power_w=power)
    y = run_gpu(g, x)
    o = oracle_plan(n_sb, block_sb, n_ov, 2, 0.3, c, rate=n_sb * 64e9)
    blocks = [0, cap - 1, cap, g.n_blocks(t_len) - 1]
    for b, v in oracle.run_blocks(x, o, blocks).items():
        seg = y[:, b * g.hop:b * g.hop + v.shape[-1]]
        assert rel_l2(seg, v[:, :seg.shape[-1]]) < TOL, b
    assert np.array_equal(y, run_gpu(g, x))
    g.close()


def test_stream_set_coeffs_and_split_ratio():
    power = 4e-3
    x = random_field((2, 50000), 55, power_w=power)
    c1 = rand_coeffs(2, 2, 5, 0.5, power, 1)
    c2 = rand_coeffs(2, 2, 5, 0.5, power, 2)
    g = gpu_plan(2, 2 ** 14, 4096, 2, 0.5, c1, rate=128e9)
    g.set_coeffs(torch.from_numpy(c2.astype(np.float32)).cuda(), torch.tensor([0.2], dtype=torch.float32).cuda())
    rho32 = float(np.float32(0.2))
    y = run_gpu(g, x)
    assert rel_l2(y, oracle.run(x, oracle_plan(2, 2 ** 14, 4096, 2, rho32, c2, rate=128e9))) < TOL
    g.set_split_ratio(0.7)
    y = run_gpu(g, x)
    assert rel_l2(y, oracle.run(x, oracle_plan(2, 2 ** 14, 4096, 2, 0.7, c2, rate=128e9))) < TOL
    g.close()


def test_stream_graph_replay():
    """The streaming call recorded in a HIP graph and replayed with new inputs
    gives the eager result on every replay."""
    power = 4e-3
    c = rand_coeffs(3, 2, 7, 0.5, power, 3)
    g = gpu_plan(2, 2 ** 14, 4096, 3, 0.4, c, rate=128e9)
    xs = [torch.from_numpy(random_field((2, 60000), 70 + k, power_w=power).astype(np.complex64)).cuda()
          for k in range(3)]
    ref = [g.run(x).clone() for x in xs]
    x_in = xs[0].clone()
    out = torch.empty_like(x_in)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        g.run(x_in, out=out)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.run(x_in, out=out)
    for k in (1, 2, 0, 1):
        x_in.copy_(xs[k])
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref[k]), k
        _ = (xs[k] * 2).sum().item()   # eager work between replays
    g.close()


def test_stream_rejects_what_it_does_not_cover():
    from paper_2409_14489_amd import CbessfmError
    g = gpu_plan(2, 2 ** 14, 0, 1, 0.5, np.zeros((1, 2, 2, 1)), rate=128e9)
    with pytest.raises(CbessfmError):
        g.set_nlpr("dual")
    g.close()


def test_stream_long_link_full_size_sampled():
    """The long-link shape at full size: 5 subbands of N' = 2^17, N_ov = 196608,
    T = 5 x 2^21 per polarisation (23 blocks), 21 taps, 80 steps over
    40 x 80 km; one block (the last, ragged) against the oracle at 80 steps and
    two blocks at 10 steps."""
    power = 8e-3
    n_sb, block_sb, n_ov, t_len = 5, 2 ** 17, 196608, 5 * 2 ** 21
    x = random_field((2, t_len), 41, power_w=power)
    for steps, blocks in ((10, [0, 11]), (80, [22])):
        c = rand_coeffs(steps, n_sb, 21, 0.02, power, steps)
        g = gpu_plan(n_sb, block_sb, n_ov, steps, 0.3, c, spans=40, rate=640e9)
        assert g.n_blocks(t_len) == 23
        y = run_gpu(g, x)
        o = oracle_plan(n_sb, block_sb, n_ov, steps, 0.3, c, spans=40, rate=640e9)
        for b, v in oracle.run_blocks(x, o, blocks).items():
            seg = y[:, b * g.hop:b * g.hop + v.shape[-1]]
            err = rel_l2(seg, v[:, :seg.shape[-1]])
            print(f"{steps} steps, block {b}: rel L2 {err:.3e}")
            assert err < TOL
        g.close()
