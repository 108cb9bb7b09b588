"""Parity of the HIP adjoint (through the C ABI) with the FP64 gradient oracle.

The oracle differentiates a plain PyTorch complex128 CPU rewrite of the
forward map (itself pinned to the numpy oracle and to finite differences on
the CPU).  Bar: relative L2 error <= 1e-5 for dL/dC and dL/dfield_in, and
relative error <= 1e-5 for dL/drho.

dL/drho is the difference of the derivatives through the first and the last
GVD (Sec. III-C), each up to hundreds of times larger than the result; the
adjoint forms it step by step from terms that scale with the nonlinear phase
(a dispersion/rotation commutator), so it reaches the same relative bar.
Finite differences of the FP64 oracle are checked as a second reference.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
from oracle.grad import vjp
from synth import random_field, workload

pytestmark = pytest.mark.gpu

TOL = 1e-5
BETA2_PS2 = -21.7


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def plans(n_sb, block_sb, overlap, steps, rho, coeffs, spans=1, rate=64e9, boundary="circular", span_km=80.0):
    from paper_2409_14489_amd import LinkSpec, Plan
    c32 = np.asarray(coeffs, np.float32)
    g = Plan(LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=spans, span_km=span_km, sample_rate_hz=rate),
             n_sb, block_sb, overlap, steps, rho, coeffs=c32, boundary=boundary)
    o = oracle.OraclePlan(BETA2_PS2 * 1e-24, rate, span_km * spans / steps, steps, rho, n_sb, n_sb * block_sb,
                          overlap, c32.astype(np.float64), boundary=boundary)
    return g, o


def rand_coeffs(steps, n_sb, taps, phase_rad, power_w, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps))
    c *= phase_rad / (power_w * np.abs(c).sum(axis=(2, 3), keepdims=True))
    return c


def gpu_grads(g, x, gout, need_in=True, ck=1):
    xt = torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).cuda()
    gt = torch.from_numpy(np.ascontiguousarray(gout.astype(np.complex64))).cuda()
    gi, gc, gr = g.backward(xt, gt, need_grad_in=need_in, checkpoint_every=ck)
    torch.cuda.synchronize()
    assert g.status() == 0
    return (gi.cpu().numpy() if gi is not None else None), gc.cpu().numpy(), float(gr.cpu().numpy()[0])


def check_case(n_sb, block_sb, overlap, steps, rho, taps, t_len, batch=1, ck=1, boundary="circular", seed=0,
               rate=None, need_in=True, phase=0.5):
    power = 4e-3
    rate = rate or n_sb * 64e9
    shape = (batch, 2, t_len) if batch > 1 else (2, t_len)
    x = random_field(shape, 300 + seed, power_w=power)
    gout = random_field(shape, 400 + seed, power_w=1.0)
    c = rand_coeffs(steps, n_sb, taps, phase, power, seed)
    g, o = plans(n_sb, block_sb, overlap, steps, rho, c, rate=rate, boundary=boundary)
    gi, gc, gr = gpu_grads(g, x, gout, need_in=need_in, ck=ck)
    ogi, ogc, ogr = vjp(x, o, gout)
    errs = dict(c=rel(gc, ogc), rho=abs(gr - ogr) / abs(ogr))
    if need_in:
        errs["in"] = rel(gi, ogi)
    print(n_sb, block_sb, steps, taps, ck, errs)
    g.close()
    return errs


@pytest.mark.parametrize("n_sb,block_sb,steps,taps", [
    (1, 256, 3, 5), (1, 1024, 4, 11), (2, 512, 3, 7), (3, 256, 2, 9), (5, 512, 3, 21), (2, 2048, 2, 3),
])
def test_gradients_match_fp64_oracle(n_sb, block_sb, steps, taps):
    n = n_sb * block_sb
    errs = check_case(n_sb, block_sb, n // 8, steps, 0.3, taps, 3 * n + 55, seed=n_sb * 7 + steps)
    assert max(errs.values()) < TOL, errs


@pytest.mark.parametrize("ck", [1, 2, 3, 5, 7])
def test_checkpointing_and_determinism(ck):
    """Any checkpoint spacing meets the bar, is deterministic run to run, and
    needs less workspace than storing every step."""
    power = 4e-3
    x = random_field((2, 2500), 21, power_w=power)
    gout = random_field((2, 2500), 22, power_w=1.0)
    c = rand_coeffs(5, 2, 5, 0.5, power, 3)
    g, o = plans(2, 512, 128, 5, 0.4, c, rate=128e9)
    got = gpu_grads(g, x, gout, ck=ck)
    again = gpu_grads(g, x, gout, ck=ck)
    assert np.array_equal(got[0], again[0]) and np.array_equal(got[1], again[1]) and got[2] == again[2]
    ogi, ogc, ogr = vjp(x, o, gout)
    assert rel(got[0], ogi) < TOL and rel(got[1], ogc) < TOL
    assert abs(got[2] - ogr) < TOL * abs(ogr)
    if 1 < ck < 5:
        assert g.backward_workspace(2500, 1, ck) < g.backward_workspace(2500, 1, 1)


def test_gradients_zero_boundary_batch_and_short_sequence():
    errs = check_case(2, 256, 64, 2, 0.6, 5, 1500, batch=3, boundary="zero", seed=5)
    assert max(errs.values()) < TOL, errs
    errs = check_case(2, 512, 128, 2, 0.2, 5, 700, seed=6)        # T < N: blocks wrap
    assert max(errs.values()) < TOL, errs


def test_gradients_without_input_gradient():
    errs = check_case(3, 512, 192, 3, 0.5, 7, 4000, seed=8, need_in=False)
    assert max(errs.values()) < TOL, errs


def test_gradient_workload_sixteen_realisations_and_finite_differences():
    """1 ch 32 GBd DP-16QAM, 2^14 symbols, 1 x 80 km, 15 fractional-span steps,
    11 taps per step, N = 1024, N_ov = 128; 16 seeded realisations."""
    from paper_2409_14489_amd import LinkSpec, analytic_coeffs
    xs = np.stack([workload("1ch-32GBd-16QAM-2^14sym-1x80km-15steps", 3000 + r, steps_per_span=20)[0]
                   for r in range(16)])
    rng = np.random.default_rng(9)
    gout = (rng.standard_normal(xs.shape) + 1j * rng.standard_normal(xs.shape)) * 1e-2
    c = analytic_coeffs(LinkSpec(beta2_ps2_km=BETA2_PS2, sample_rate_hz=64e9), 1, 15, 0.5, 11)
    g, o = plans(1, 1024, 128, 15, 0.5, c)
    ogi, ogc, ogr = vjp(xs, o, gout)
    for ck in (1, 8):
        gi, gc, gr = gpu_grads(g, xs, gout, ck=ck)
        errs = dict(c=rel(gc, ogc), rho=abs(gr - ogr) / abs(ogr), inp=rel(gi, ogi))
        print("16 realisations, checkpoint every", ck, errs)
        assert max(errs.values()) < TOL, errs

    # central differences of the FP64 oracle, h = 1e-3 relative
    def loss(p):
        return float(np.real(np.sum(np.conj(gout) * oracle.run(xs, p))))
    for idx in [(0, 0, 0, 5), (7, 0, 0, 2), (14, 0, 0, 9)]:
        h = 1e-3 * abs(o.coeffs[idx])
        pa, pb = copy.copy(o), copy.copy(o)
        pa.coeffs = o.coeffs.copy()
        pb.coeffs = o.coeffs.copy()
        pa.coeffs[idx] += h
        pb.coeffs[idx] -= h
        fd = (loss(pa) - loss(pb)) / (2 * h)
        assert abs(gc[idx] - fd) < 1e-4 * abs(fd) + 1e-6 * np.abs(gc).max()
    h = 1e-3 * o.rho
    pa, pb = copy.copy(o), copy.copy(o)
    pa.rho, pb.rho = o.rho + h, o.rho - h
    fd = (loss(pa) - loss(pb)) / (2 * h)
    assert abs(gr - fd) < 1e-4 * abs(fd)


def test_autograd_function_and_adam_step():
    from paper_2409_14489_amd import cbessfm
    power = 4e-3
    x = torch.from_numpy(random_field((2, 3000), 31, power_w=power).astype(np.complex64)).cuda()
    target = torch.from_numpy(random_field((2, 3000), 32, power_w=power).astype(np.complex64)).cuda()
    c0 = rand_coeffs(3, 2, 5, 0.3, power, 4)
    g, o = plans(2, 512, 128, 3, 0.3, c0, rate=128e9)
    coeffs = torch.tensor(c0, dtype=torch.float32, device="cuda", requires_grad=True)
    rho = torch.tensor(0.3, dtype=torch.float32, device="cuda", requires_grad=True)
    y = cbessfm(x, coeffs, rho, g)
    loss = (y - target).abs().pow(2).sum()
    loss.backward()
    gout = 2 * (y - target).detach().cpu().numpy().astype(np.complex128)
    xn = x.cpu().numpy().astype(np.complex128)
    _, ogc, ogr = vjp(xn, o, gout)
    assert rel(coeffs.grad.cpu().numpy(), ogc) < TOL
    assert abs(float(rho.grad) - ogr) < TOL * abs(ogr)
    opt = torch.optim.Adam([coeffs, rho], lr=1e-3)
    before = float(loss)
    for _ in range(20):
        opt.zero_grad()
        loss = (cbessfm(x, coeffs, rho, g) - target).abs().pow(2).sum()
        loss.backward()
        opt.step()
    assert float(loss) < before
