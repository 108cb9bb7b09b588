"""Parity of the HIP forward path (through the C ABI) with the FP64 oracle.

Bar: relative L2 error <= 1e-5 over the whole output and over the kept
samples of every overlap-and-save block on its own, complex FP32 against
FP64.  Coefficients are rounded to FP32 once and both sides use those values.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.coeffs import Link, dbp_coefficients
from synth import random_field, workload

pytestmark = pytest.mark.gpu

TOL = 1e-5
BETA2_PS2 = -21.7


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst_block_rel_l2(y, ref, hop):
    """Largest relative L2 error over the output samples of one block
    ([b hop, (b + 1) hop) of every batch entry, both polarisations)."""
    y = y.reshape(-1, 2, y.shape[-1])
    ref = ref.reshape(-1, 2, ref.shape[-1])
    t_len = y.shape[-1]
    worst = 0.0
    for bi in range(y.shape[0]):
        for lo in range(0, t_len, hop):
            r = ref[bi, :, lo:lo + hop]
            if np.linalg.norm(r) > 0:
                worst = max(worst, rel_l2(y[bi, :, lo:lo + hop], r))
    return worst


def assert_parity(y, ref, hop):
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, hop)
    assert err < TOL and worst < TOL, (err, worst)


def gpu_plan(n_sb, block_sb, overlap, steps, rho, coeffs, spans=1, rate=64e9, boundary="circular",
             span_km=80.0):
    from paper_2409_14489_amd import LinkSpec, Plan
    link = LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=spans, span_km=span_km, sample_rate_hz=rate)
    return Plan(link, n_sb, block_sb, overlap, steps, rho, coeffs=np.asarray(coeffs, np.float32),
                boundary=boundary)


def oracle_plan(n_sb, block_sb, overlap, steps, rho, coeffs, spans=1, rate=64e9, boundary="circular",
                span_km=80.0):
    c64 = np.asarray(np.asarray(coeffs, np.float32), np.float64)
    return oracle.OraclePlan(BETA2_PS2 * 1e-24, rate, span_km * spans / steps, steps, rho, n_sb,
                             n_sb * block_sb, overlap, c64, boundary=boundary)


def run_gpu(plan, x):
    xt = torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).cuda()
    y = plan.run(xt)
    torch.cuda.synchronize()
    assert plan.status() == 0
    return y.cpu().numpy().astype(np.complex128)


def rand_coeffs(steps, n_sb, taps, phase_rad, power_w, seed):
    """Random applied coefficients giving phases of about phase_rad."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps))
    c *= phase_rad / (power_w * np.abs(c).sum(axis=(2, 3), keepdims=True))
    return c


def case(n_sb, block_sb, overlap, steps, rho, taps, t_len, batch=1, boundary="circular", seed=0,
         phase=0.5, spans=1, rate=64e9):
    power = 4e-3
    shape = (batch, 2, t_len) if batch > 1 else (2, t_len)
    x = random_field(shape, 100 + seed, power_w=power)
    c = rand_coeffs(steps, n_sb, taps, phase, power, seed)
    g = gpu_plan(n_sb, block_sb, overlap, steps, rho, c, spans=spans, rate=rate, boundary=boundary)
    o = oracle_plan(n_sb, block_sb, overlap, steps, rho, c, spans=spans, rate=rate, boundary=boundary)
    y = run_gpu(g, x)
    ref = oracle.run(x, o)
    hop = g.hop
    g.close()
    return y, ref, hop


# ------------------------------------------------------------------ the named workloads

def test_parity_single_channel_one_step_analytic():
    """1 ch 32 GBd DP-16QAM, 2^14 symbols, 1 x 80 km, 1 step, 11 analytic taps,
    N = 1024, N_ov = 128."""
    from paper_2409_14489_amd import LinkSpec, analytic_coeffs
    x, _, w = workload("1ch-32GBd-16QAM-2^14sym-1x80km", 1001)
    d = w["dbp"]
    c = analytic_coeffs(LinkSpec(beta2_ps2_km=BETA2_PS2, sample_rate_hz=64e9), 1, 1, 0.5, 11)
    g = gpu_plan(1, 1024, 128, 1, 0.5, c)
    o = oracle_plan(1, 1024, 128, 1, 0.5, c)
    y = run_gpu(g, x)
    assert_parity(y, oracle.run(x, o), g.hop)
    assert d["n_sub"] == 1024 and d["n_overlap"] == 128


@pytest.fixture(scope="module")
def wdm5():
    x, _, w = workload("5ch-64GBd-64QAM-2^16sym-15x80km", 2001, steps_per_span=2)
    c = dbp_coefficients(Link(n_spans=15, sample_rate=640e9), 5, 15, 0.3, 21)
    return x, c


def test_parity_five_channel_fifteen_steps(wdm5):
    """5 x 64 GBd DP-64QAM at 100 GHz, 2^16 symbols/ch at 640 GS/s, 15 x 80 km,
    5 subbands, N' = 4096, N_ov = 2560, 15 steps, rho = 0.3, 21 taps."""
    x, c = wdm5
    g = gpu_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    o = oracle_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    y = run_gpu(g, x)
    ref = oracle.run(x, o)
    err, worst = rel_l2(y, ref), worst_block_rel_l2(y, ref, g.hop)
    print("rel L2 five-channel:", err, "worst of the 37 blocks:", worst)
    assert err < TOL and worst < TOL
    # bitwise determinism of a second run
    y2 = run_gpu(g, x)
    assert np.array_equal(y, y2)


def test_parity_five_channel_batch_beyond_resident_teams(wdm5):
    """Two instances: 74 blocks, more than one wave of persistent teams."""
    x, c = wdm5
    g = gpu_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    assert g.info().team_capacity < 2 * g.n_blocks(x.shape[-1])
    xb = np.stack([x, np.roll(x, 12345, axis=-1) * 0.9])
    y = run_gpu(g, xb)
    o = oracle_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    blocks = [0, 17, 36]
    for bi in range(2):
        ref = oracle.run_blocks(xb[bi], o, blocks)
        for b, v in ref.items():
            seg = y[bi][:, b * g.hop:b * g.hop + v.shape[-1]]
            assert rel_l2(seg, v) < TOL


# ------------------------------------------------------------------ shapes and edges

@pytest.mark.parametrize("block_sb", [256, 512, 1024, 2048, 4096, 8192])
def test_parity_every_block_size_single_band(block_sb):
    y, ref, hop = case(1, block_sb, block_sb // 4, 3, 0.3, 9, 3 * block_sb + 77, seed=block_sb)
    assert_parity(y, ref, hop)


@pytest.mark.parametrize("n_sb,block_sb", [(2, 1024), (3, 512), (4, 256), (5, 2048), (8, 256), (2, 8192)])
def test_parity_multiband(n_sb, block_sb):
    n = n_sb * block_sb
    y, ref, hop = case(n_sb, block_sb, n // 8, 4, 0.27, 7, 3 * n + 101, seed=n_sb, rate=n_sb * 64e9)
    assert_parity(y, ref, hop)


@pytest.mark.parametrize("taps", [1, 3, 8 * 4 + 1, 101, 255])
def test_parity_tap_counts(taps):
    y, ref, hop = case(2, 512, 256, 2, 0.5, taps, 4000, seed=taps, rate=128e9)
    assert_parity(y, ref, hop)


@pytest.mark.parametrize("rho", [0.0, 1.0])
def test_parity_split_extremes(rho):
    y, ref, hop = case(3, 256, 96, 3, rho, 5, 2000, seed=7, rate=192e9)
    assert_parity(y, ref, hop)


def test_parity_zero_boundary_and_batch():
    y, ref, hop = case(2, 256, 64, 2, 0.4, 5, 1500, batch=3, boundary="zero", seed=9, rate=128e9)
    assert_parity(y, ref, hop)


def test_parity_no_overlap():
    y, ref, hop = case(1, 1024, 0, 2, 0.5, 11, 5000, seed=10)
    assert_parity(y, ref, hop)


@pytest.mark.parametrize("t_len", [1, 7, 300, 1023])
def test_parity_sequence_shorter_than_block(t_len):
    y, ref, hop = case(2, 512, 128, 2, 0.3, 5, t_len, seed=t_len, rate=128e9)
    assert_parity(y, ref, hop)


def test_set_coeffs_and_split_ratio_on_device():
    power = 4e-3
    x = random_field((2, 3000), 55, power_w=power)
    c1 = rand_coeffs(2, 2, 5, 0.5, power, 1)
    c2 = rand_coeffs(2, 2, 5, 0.5, power, 2)
    g = gpu_plan(2, 512, 128, 2, 0.5, c1, rate=128e9)
    g.set_coeffs(torch.from_numpy(c2.astype(np.float32)).cuda(), torch.tensor([0.2], dtype=torch.float32).cuda())
    rho32 = float(np.float32(0.2))
    y = run_gpu(g, x)
    assert rel_l2(y, oracle.run(x, oracle_plan(2, 512, 128, 2, rho32, c2, rate=128e9))) < TOL
    g.set_split_ratio(0.7)
    y = run_gpu(g, x)
    assert rel_l2(y, oracle.run(x, oracle_plan(2, 512, 128, 2, 0.7, c2, rate=128e9))) < TOL


def test_run_rejects_overlapping_buffers():
    from paper_2409_14489_amd import CbessfmError
    g = gpu_plan(1, 256, 0, 1, 0.5, np.zeros((1, 1, 1, 1)))
    x = torch.zeros((2, 512), dtype=torch.complex64, device="cuda")
    with pytest.raises(CbessfmError):
        g.run(x, out=x)


def test_exchange_wait_give_up_is_reported_and_recovers(wdm5):
    """The team exchange's bounded wait, forced to give up from the host by a
    limit of one poll: the launch still ends, cbessfm_status reports
    CBESSFM_ESYNC once and resets the exchange state, and the next run with
    the default limit is parity-green and equal to a run before the fault.
    The same for the adjoint."""
    from paper_2409_14489_amd._lib import ESYNC
    x, c = wdm5
    g = gpu_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    o = oracle_plan(5, 4096, 2560, 15, 0.3, c, spans=15, rate=640e9)
    before = run_gpu(g, x)
    xt = torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).cuda()
    g.set_wait_limit(1)
    codes = []
    for _ in range(3):                 # each launch ends normally; stop at the first give-up
        g.run(xt)
        codes.append(g.status())
        if codes[-1] == ESYNC:
            break
    print("status after runs with a one-poll wait limit:", codes)
    assert codes[-1] == ESYNC and all(cd in (0, ESYNC) for cd in codes)
    assert g.status() == 0             # reported once, state reset
    g.set_wait_limit(0)
    after = run_gpu(g, x)
    assert np.array_equal(after, before)
    blocks = [0, 18, 36]
    for b, v in oracle.run_blocks(x, o, blocks).items():
        assert rel_l2(after[:, b * g.hop:b * g.hop + v.shape[-1]], v) < TOL

    gout = torch.from_numpy(random_field(x.shape, 77, power_w=1.0).astype(np.complex64)).cuda()
    ref = g.backward(xt, gout, need_grad_in=False)
    torch.cuda.synchronize()
    assert g.status() == 0
    g.set_wait_limit(1)
    codes = []
    for _ in range(3):
        g.backward(xt, gout, need_grad_in=False)
        codes.append(g.status())
        if codes[-1] == ESYNC:
            break
    print("adjoint status with a one-poll wait limit:", codes)
    assert codes[-1] == ESYNC
    g.set_wait_limit(0)
    again = g.backward(xt, gout, need_grad_in=False)
    torch.cuda.synchronize()
    assert g.status() == 0
    assert torch.equal(again[1], ref[1]) and torch.equal(again[2], ref[2])
    g.close()


@pytest.mark.parametrize("n_sb,block_sb,taps", [(1, 1024, 1), (2, 512, 21), (5, 1024, 45), (3, 256, 101),
                                                (2, 4096, 255), (8, 256, 33), (2, 8192, 65)])
def test_frequency_domain_filter_matches_oracle(n_sb, block_sb, taps):
    """fir_mode 'freq' (the paper's RFFT / MIMO / IRFFT form of eq. (15),
    Sec. III-A) against the oracle's literal double sum, whole output and every
    block, and against the time-domain mode of the same plan shape."""
    power = 4e-3
    n = n_sb * block_sb
    x = random_field((2, 3 * n + 33), 700 + taps, power_w=power)
    c = rand_coeffs(3, n_sb, taps, 0.5, power, taps)
    from paper_2409_14489_amd import LinkSpec, Plan
    link = LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=2, sample_rate_hz=n_sb * 64e9)
    outs = {}
    for mode in ("freq", "time"):
        g = Plan(link, n_sb, block_sb, n // 8, 3, 0.3, coeffs=c.astype(np.float32), fir_mode=mode)
        outs[mode] = run_gpu(g, x)
        hop = g.hop
        g.close()
    ref = oracle.run(x, oracle_plan(n_sb, block_sb, n // 8, 3, 0.3, c, spans=2, rate=n_sb * 64e9))
    assert_parity(outs["freq"], ref, hop)
    assert rel_l2(outs["freq"], outs["time"]) < 2e-6


def test_auto_filter_mode_and_set_coeffs_in_frequency_mode():
    """Above 64 taps 'auto' takes the frequency domain; a coefficient update on
    the device re-derives the row DFTs."""
    from paper_2409_14489_amd import LinkSpec, Plan
    power = 4e-3
    x = random_field((2, 9000), 71, power_w=power)
    c1 = rand_coeffs(2, 2, 81, 0.5, power, 1)
    c2 = rand_coeffs(2, 2, 81, 0.5, power, 2)
    link = LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=1, sample_rate_hz=128e9)
    g = Plan(link, 2, 1024, 256, 2, 0.4, coeffs=c1.astype(np.float32))
    g.set_coeffs(torch.from_numpy(c2.astype(np.float32)).cuda())
    y = run_gpu(g, x)
    ref = oracle.run(x, oracle_plan(2, 1024, 256, 2, 0.4, c2, rate=128e9))
    assert_parity(y, ref, g.hop)
    g.close()
