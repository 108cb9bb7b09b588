"""cbessfm_backward_static (the adjoint on the library's fixed device scratch,
for callers that cannot allocate) through the C ABI: the same results as
cbessfm_backward with a caller workspace, bit for bit, on two calls in a row
(the second with a smaller input) for a persistent and a streaming plan, and
CBESSFM_EWORKSPACE for a call whose workspace would exceed the scratch."""
import ctypes

import numpy as np
import pytest
import torch

from synth import random_field

pytestmark = pytest.mark.gpu


def _plan(n_sb, block_sb, overlap, steps, taps, rate, seed):
    from paper_2409_14489_amd import LinkSpec, Plan
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((steps, n_sb, n_sb, taps))
    c *= 0.4 / (4e-3 * np.abs(c).sum(axis=(2, 3), keepdims=True))
    return Plan(LinkSpec(beta2_ps2_km=-21.7, n_spans=2, sample_rate_hz=rate), n_sb, block_sb, overlap, steps, 0.3,
                coeffs=c.astype(np.float32))


def _static(plan, x, g, need_in, ck):
    from paper_2409_14489_amd._lib import lib
    bsz = 1 if x.dim() == 2 else x.shape[0]
    gi = torch.full_like(x, float("nan")) if need_in else None
    gc = torch.full((plan.steps, plan.n_sb, plan.n_sb, plan.n_taps), float("nan"), dtype=torch.float32,
                    device=x.device)
    gr = torch.full((1,), float("nan"), dtype=torch.float32, device=x.device)
    rc = lib.cbessfm_backward_static(plan._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                     ctypes.c_void_p(gi.data_ptr()) if need_in else None,
                                     ctypes.c_void_p(gc.data_ptr()), ctypes.c_void_p(gr.data_ptr()),
                                     int(x.shape[-1]), int(bsz), int(ck), None)
    torch.cuda.synchronize()
    return rc, gi, gc, gr


def _field(shape, seed, power):
    return torch.from_numpy(random_field(shape, seed, power_w=power).astype(np.complex64)).cuda()


@pytest.mark.parametrize("shape,calls", [
    ((2, 512, 128, 3, 5, 128e9), [((2, 2, 6000), True, 1), ((2, 1700), False, 2)]),
    ((1, 2 ** 14, 4096, 2, 7, 64e9), [((2, 30000), True, 1), ((2, 9000), True, 2)]),
])
def test_static_scratch_matches_caller_workspace(shape, calls):
    plan = _plan(*shape, seed=3)
    for k, (fshape, need_in, ck) in enumerate(calls):
        print("static-scratch adjoint", shape, fshape, "grad_in" if need_in else "", "ck", ck, flush=True)
        x = _field(fshape, 40 + k, 4e-3)
        g = _field(fshape, 50 + k, 1.0)
        assert plan.backward_workspace(fshape[-1], 1 if len(fshape) == 2 else fshape[0], ck) <= 64 << 20
        rc, gi, gc, gr = _static(plan, x, g, need_in, ck)
        assert rc == 0
        ri, rcf, rr = plan.backward(x, g, need_grad_in=need_in, checkpoint_every=ck)
        torch.cuda.synchronize()
        assert plan.status() == 0
        assert torch.equal(gc, rcf) and torch.equal(gr, rr)
        if need_in:
            assert torch.equal(gi, ri)
    plan.close()


def test_static_scratch_rejects_a_call_beyond_its_size():
    from paper_2409_14489_amd._lib import EWORKSPACE
    plan = _plan(5, 4096, 2560, 15, 21, 640e9, seed=4)
    t_len = 655360
    assert plan.backward_workspace(t_len, 1, 1) > 64 << 20
    x = torch.zeros((2, t_len), dtype=torch.complex64, device="cuda")
    rc, _, gc, _ = _static(plan, x, x, False, 1)
    assert rc == EWORKSPACE
    assert torch.isnan(gc).all()      # nothing was launched
    plan.close()
