"""GPU parity of the learned estimator's FP32 training step against the
float64 reference in tests/train_ref.py (which its own CPU pins check
against finite differences and Adam's closed forms).

* Sample records from rdl_train_samples equal the reference's byte for byte
  (border pixels included).
* Three rdl_train_step calls from the same float32 parameters: after each,
  the GPU's Adam moments equal b1 m + (1 - b1) g and b2 v + (1 - b2) g^2
  with the reference gradient g at the GPU's previous parameters, the new
  parameters equal the float64 Adam update (bias correction of that step)
  from the GPU's own moments, and the loss equals the summed squared error.

Tolerances.  Every gradient is a float32 sum over the batch of products
along the chain of the backward pass; in any summation order its rounding
error is at most a few hundred unit roundoffs (2^-24) times the same sum
taken over absolute values, which the reference returns beside each
gradient.  The test allows 2e-5 times that bound (about 340 roundoffs).
Samples whose hidden pre-activations lie within 1e-4 of their magnitude bound
of zero are left out of each step's batch, so that float32 and float64 take
the same ReLU branches.  The test checks that a sign error in any layer's
gradient would exceed the tolerance on most of that layer's parameters.
"""
import numpy as np
import pytest
import torch

import train_ref as T
from paper_2309_11072_amd import synth, train

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
GTOL = 2e-5


@pytest.fixture(scope="module")
def codec():
    from paper_2309_11072_amd import rdl
    c = rdl.Codec(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


def _image(H, W, seed):
    from oracle import oracle as O
    x = synth.generate(H, W, 4.0, seed=seed, spec_frac=0.05)
    ref = O.encode_enh(x, 75)
    return x, ref["sdr"], ref["k_img"]


def test_train_samples_match_reference(codec):
    H, W = 37, 53
    _say("train samples", H, W)
    x, sdr, k_img = _image(H, W, 4301)
    rng = np.random.default_rng(1)
    corners = [0, W - 1, (H - 1) * W, H * W - 1, W, 2 * W - 1]
    idx = np.concatenate([corners, rng.choice(H * W, 500, replace=False)]).astype(np.int64)
    got = codec.train_samples(torch.from_numpy(x).cuda(), torch.from_numpy(sdr).cuda(), k_img,
                              torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    exp = T.samples(x, sdr, k_img, idx)
    assert got.shape == exp.shape
    assert np.array_equal(got.cpu().numpy(), exp)


def test_train_steps_match_float64_reference(codec):
    H, W = 64, 80
    _say("train steps", H, W)
    x, sdr, k_img = _image(H, W, 4302)
    rng = np.random.default_rng(2)
    pool = T.samples(x, sdr, k_img, rng.choice(H * W, 3 * 400, replace=False))
    p = train.init_params(11).astype(np.float32)
    m = np.zeros(T.NPARAM, np.float32)
    v = np.zeros(T.NPARAM, np.float32)
    dp, dm, dv = (torch.from_numpy(a.copy()).cuda() for a in (p, m, v))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr = 2e-3
    for step in (1, 2, 3):
        batch = pool[(step - 1) * 400: step * 400]
        g, _, bound, margin = T.grad(p.astype(np.float64), batch)
        batch = batch[margin > 1e-4]          # same ReLU branches in float32
        assert len(batch) >= 360
        if len(batch) % 64 == 0:
            batch = batch[:-1]                # keep a ragged last workgroup
        g, lref, bound, _ = T.grad(p.astype(np.float64), batch)
        _say("step", step, "batch", len(batch))
        codec.train_step(dp, dm, dv, torch.from_numpy(batch).cuda(), 0, len(batch), lr, step, loss_out=loss)
        torch.cuda.synchronize()
        pn, mn, vn = (t.cpu().numpy() for t in (dp, dm, dv))
        m64, v64, g64 = m.astype(np.float64), v.astype(np.float64), g
        # first moment: b1 m + (1 - b1) g
        m_exp = 0.9 * m64 + 0.1 * g64
        m_tol = 0.1 * GTOL * bound + 4 * U32 * (0.9 * np.abs(m64) + 0.1 * np.abs(g64)) + 1e-30
        bad = np.abs(mn - m_exp) > m_tol
        assert not bad.any(), ("m", step, np.nonzero(bad)[0][:10])
        # second moment: b2 v + (1 - b2) g^2
        v_exp = 0.999 * v64 + 0.001 * g64 * g64
        v_tol = 0.001 * (2 * np.abs(g64) * GTOL * bound + (GTOL * bound) ** 2) + 4 * U32 * (
            0.999 * v64 + 0.001 * g64 * g64) + 1e-38
        bad = np.abs(vn - v_exp) > v_tol
        assert not bad.any(), ("v", step, np.nonzero(bad)[0][:10])
        # parameters: Adam from the GPU's own moments, bias correction of this step
        mh = mn.astype(np.float64) / (1 - 0.9 ** step)
        vh = vn.astype(np.float64) / (1 - 0.999 ** step)
        upd = lr * mh / (np.sqrt(vh) + 1e-8)
        p_exp = p.astype(np.float64) - upd
        p_tol = 8 * U32 * (np.abs(p) + np.abs(upd)) + 1e-30
        bad = np.abs(pn - p_exp) > p_tol
        assert not bad.any(), ("params", step, np.nonzero(bad)[0][:10])
        # loss: summed squared error of the batch
        assert abs(float(loss.item()) - lref) <= 1e-5 * lref
        if step == 1:
            # a sign error in any block's gradient moves m by 0.2 |g|: it
            # would exceed the tolerance on most of each block's parameters
            # (B1: of the bins in the batch)
            bins = np.unique(batch[:, 27]).astype(int)
            for name, (lo, hi) in T.BLOCKS.items():
                sl = np.arange(lo, hi)
                if name == "B1":
                    sl = np.array([lo + 32 * b + j for b in bins for j in range(32)])
                caught = 0.2 * np.abs(g64[sl]) > m_tol[sl]
                assert caught.mean() >= 0.5, (name, caught.mean())
        p, m, v = pn, mn, vn
