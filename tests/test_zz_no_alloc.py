"""gsp_loss_l1_noalloc, the L1 loss for callers that cannot allocate device
memory, against gsp_loss_l1 (which takes caller scratch), through the C ABI:
the same kernels, so losses and gradients agree bit for bit, on two calls
in a row (the second on smaller views), and sizes beyond the fixed scratch
are rejected before anything is launched."""
import numpy as np
import pytest
import torch

from paper_2410_08743_amd import _native as N
from paper_2410_08743_amd import render as R
from paper_2410_08743_amd.synthetic import Camera

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _noalloc(cams, pred, target, grad, loss):
    return N.lib().gsp_loss_l1_noalloc(R.context(0), len(cams), N.view_array(cams),
                                       R.view_ptrs(pred, cams, 3), R.view_ptrs(target, cams, 3),
                                       R.view_ptrs(grad, cams, 3), R._ptr(loss), R._stream())


def _inputs(rng, cams):
    pred, target = [], []
    for c in cams:
        a = rng.standard_normal(3 * c.width * c.height).astype(np.float32)
        b = a.copy()
        b[::3] = rng.standard_normal(len(b[::3])).astype(np.float32)
        pred.append(torch.tensor(a, device=DEV))
        target.append(torch.tensor(b, device=DEV))
    return pred, target


def test_noalloc_l1_equals_scratch_l1_on_two_calls():
    rng = np.random.default_rng(7)
    calls = [
        [Camera(1008, 756, 815.0, 815.0, 504.0, 378.0), Camera(320, 240, 259.0, 259.0, 160.0, 120.0),
         Camera(640, 480, 517.0, 517.0, 320.0, 240.0)],
        [Camera(101, 37, 90.0, 90.0, 50.0, 18.0)],     # second call: smaller
    ]
    for cams in calls:
        pred, target = _inputs(rng, cams)
        ref_loss, ref_grad = R.loss_l1(cams, pred, target)
        loss = torch.full((len(cams),), float("nan"), device=DEV)
        grad = [torch.full_like(p, float("nan")) for p in pred]
        N.check(_noalloc(cams, pred, target, grad, loss), "gsp_loss_l1_noalloc")
        torch.cuda.synchronize()
        assert torch.equal(loss, ref_loss), (loss, ref_loss)
        for g, r in zip(grad, ref_grad):
            assert torch.equal(g, r)
    # gradient only (no loss): no partial sums are written
    grad = [torch.zeros_like(p) for p in pred]
    N.check(_noalloc(cams, pred, target, grad, None), "gsp_loss_l1_noalloc")
    torch.cuda.synchronize()
    assert all(torch.equal(g, r) for g, r in zip(grad, ref_grad))


def test_noalloc_l1_rejects_sizes_beyond_its_scratch():
    # 3 x (3 x 4096 x 4096) values need 36864 blocks of partial sums, more
    # than the 32768 the fixed 256 KiB scratch holds: rejected before any
    # launch, so the (tiny) buffers are never touched
    cams = [Camera(4096, 4096, 3000.0, 3000.0, 2048.0, 2048.0)] * 3
    dummy = [torch.zeros(1, device=DEV) for _ in cams]
    ptrs = lambda ts: N.ptr_array([t.data_ptr() for t in ts])
    L = N.lib()
    loss = torch.zeros(3, device=DEV)
    st = L.gsp_loss_l1_noalloc(R.context(0), 3, N.view_array(cams), ptrs(dummy), ptrs(dummy), ptrs(dummy),
            R._ptr(loss), R._stream())
    assert st == N.GSP_EINVAL
    assert b"fixed scratch" in L.gsp_last_error()
    torch.cuda.synchronize()
    assert float(loss.abs().sum()) == 0.0
