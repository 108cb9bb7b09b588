"""Free dispersion segments (step sizes and split per step) on the GPU: the
forward map and dL/d(segment lengths) from the adjoint against the FP64
oracle (Sec. III-C, V)."""
import numpy as np
import pytest
import torch

import oracle
from oracle.grad import vjp_lengths
from synth import random_field

pytestmark = pytest.mark.gpu

TOL = 1e-5
BETA2_PS2 = -21.7


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def setup(n_sb, block_sb, steps, taps, seed, spans=1):
    from paper_2409_14489_amd import LinkSpec, Plan
    power = 4e-3
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps))
    c = (c * 0.5 / (power * np.abs(c).sum(axis=(2, 3), keepdims=True))).astype(np.float32)
    rate = n_sb * 64e9
    total = 80.0 * spans
    w = rng.uniform(0.2, 1.0, steps + 1)
    lengths = total * w / w.sum()
    g = Plan(LinkSpec(beta2_ps2_km=BETA2_PS2, n_spans=spans, sample_rate_hz=rate), n_sb, block_sb,
             n_sb * block_sb // 8, steps, 0.5, coeffs=c)
    g.set_gvd_lengths(torch.tensor(lengths, dtype=torch.float64, device="cuda"))
    o = oracle.OraclePlan(BETA2_PS2 * 1e-24, rate, total / steps, steps, 0.5, n_sb, n_sb * block_sb,
                          n_sb * block_sb // 8, c.astype(np.float64), gvd_km=lengths)
    return g, o


@pytest.mark.parametrize("n_sb,block_sb,steps,taps", [(1, 1024, 4, 11), (2, 512, 3, 7), (3, 256, 5, 9),
                                                      (5, 2048, 2, 21), (2, 8192, 2, 5)])
def test_forward_with_free_segments_matches_the_oracle(n_sb, block_sb, steps, taps):
    g, o = setup(n_sb, block_sb, steps, taps, seed=n_sb + steps)
    n = n_sb * block_sb
    x = random_field((2, 3 * n + 41), 50 + n_sb, power_w=4e-3)
    y = g.run(torch.from_numpy(x.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    assert g.status() == 0
    ref = oracle.run(x.astype(np.complex64).astype(np.complex128), o)
    err = rel_l2(y.cpu().numpy().astype(np.complex128), ref)
    print(n_sb, block_sb, steps, "forward rel L2", err)
    assert err < TOL
    g.close()


@pytest.mark.parametrize("n_sb,block_sb,steps,taps,ck", [(1, 1024, 4, 11, 1), (2, 512, 3, 7, 1),
                                                         (3, 256, 5, 9, 2), (2, 2048, 6, 5, 4)])
def test_segment_length_gradient_matches_the_oracle(n_sb, block_sb, steps, taps, ck):
    g, o = setup(n_sb, block_sb, steps, taps, seed=10 * n_sb + steps)
    n = n_sb * block_sb
    x = random_field((2, 3 * n + 41), 60 + n_sb, power_w=4e-3)
    gout = random_field((2, 3 * n + 41), 70 + n_sb, power_w=1.0)
    xt = torch.from_numpy(x.astype(np.complex64)).cuda()
    gt = torch.from_numpy(gout.astype(np.complex64)).cuda()
    gi, gc, _, gl = g.backward_gvd(xt, gt, checkpoint_every=ck)
    torch.cuda.synchronize()
    assert g.status() == 0
    ogi, ogc, ogl = vjp_lengths(x.astype(np.complex64).astype(np.complex128), o,
                                gout.astype(np.complex64).astype(np.complex128))
    errs = dict(c=rel_l2(gc.cpu().numpy(), ogc), inp=rel_l2(gi.cpu().numpy(), ogi),
                gvd=rel_l2(gl.cpu().numpy(), ogl))
    print(n_sb, block_sb, steps, ck, errs, gl.cpu().numpy(), ogl)
    assert max(errs.values()) < TOL, errs
    g.close()


def test_uniform_segments_and_mode_switches():
    """Explicit segments equal to (1 - rho) L, L, ..., rho L reproduce the
    uniform plan; None and a split-ratio update return to uniform steps; the
    gradient along the uniform layout gives dL/drho."""
    g, o = setup(2, 512, 4, 7, seed=3)
    x = torch.from_numpy(random_field((2, 5000), 90, power_w=4e-3).astype(np.complex64)).cuda()
    gout = torch.from_numpy(random_field((2, 5000), 91, power_w=1.0).astype(np.complex64)).cuda()
    free = g.run(x)
    g.set_gvd_lengths(None)
    uni = g.run(x)
    L = 80.0 / 4
    g.set_gvd_lengths(torch.tensor([0.5 * L, L, L, L, 0.5 * L], dtype=torch.float64, device="cuda"))
    same = g.run(x)
    _, _, gr, gl = g.backward_gvd(x, gout)
    torch.cuda.synchronize()
    assert g.status() == 0
    assert not torch.equal(free, uni)
    assert rel_l2(same.cpu().numpy(), uni.cpu().numpy()) < 1e-6
    gl = gl.cpu().numpy()
    assert abs(L * (gl[-1] - gl[0]) - float(gr)) <= 1e-4 * L * (abs(gl[0]) + abs(gl[-1]))
    g.set_split_ratio(0.5)
    again = g.run(x)
    torch.cuda.synchronize()
    assert torch.equal(again, uni)
    g.close()


def test_autograd_through_segment_lengths():
    from paper_2409_14489_amd import cbessfm_steps
    g, o = setup(2, 512, 3, 5, seed=4)
    x = torch.from_numpy(random_field((2, 4000), 95, power_w=4e-3).astype(np.complex64)).cuda()
    gout = random_field((2, 4000), 96, power_w=1.0)
    c = torch.tensor(o.coeffs, dtype=torch.float32, device="cuda", requires_grad=True)
    lengths = torch.tensor(o.gvd_km, dtype=torch.float64, device="cuda", requires_grad=True)
    y = cbessfm_steps(x, c, lengths, g)
    gt = torch.from_numpy(gout.astype(np.complex64)).cuda()
    (torch.view_as_real(y) * torch.view_as_real(gt)).sum().backward()
    _, ogc, ogl = vjp_lengths(x.cpu().numpy().astype(np.complex128), o, gout.astype(np.complex64).astype(np.complex128))
    assert rel_l2(c.grad.cpu().numpy(), ogc) < TOL
    assert rel_l2(lengths.grad.cpu().numpy(), ogl) < TOL
    g.close()
