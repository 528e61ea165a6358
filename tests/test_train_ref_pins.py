"""Pins for the float64 training reference (tests/train_ref.py), against
things other than itself: central finite differences of the loss for the
gradient, closed forms for the loss and for Adam's bias correction, and
records written out by hand for the sample builder.  CPU only."""
import numpy as np

import train_ref as T
from paper_2309_11072_amd import train


def _records(seed, n):
    rng = np.random.default_rng(seed)
    rec = np.zeros((n, 32), np.uint8)
    rec[:, :27] = rng.integers(-128, 128, (n, 27)).astype(np.int8).view(np.uint8)
    rec[:, 27] = rng.integers(0, 32, n)
    rec[:, 28:31] = rng.integers(0, 256, (n, 3))
    return rec


def _mean_loss(p, rec):
    x, b, t = T.unpack(rec)
    o = T.forward(p, x, b)["o"]
    return float(((o - t) ** 2).sum()) / (3 * len(rec))


def test_gradient_vs_central_differences():
    """Every block's gradient (W1, B1 of the bins present, W2, B2, W3, B3)
    equals the central difference of the mean squared error to 1e-6
    relative, on parameters whose step does not cross a ReLU kink."""
    p = train.init_params(5).astype(np.float64)
    rec = _records(6, 40)
    g, loss, s, margin = T.grad(p, rec)
    rng = np.random.default_rng(7)
    bins = np.unique(rec[:, 27]).astype(int)
    checked = {k: 0 for k in T.BLOCKS}
    for name, (lo, hi) in T.BLOCKS.items():
        cand = np.arange(lo, hi)
        if name == "B1":
            cand = np.array([lo + 32 * b + j for b in bins for j in range(32)])
        for i in rng.choice(cand, size=min(40, len(cand)), replace=False):
            h = 1e-6
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (_mean_loss(pp, rec) - _mean_loss(pm, rec)) / (2 * h)
            # the kink test: the branch pattern is the same at both ends
            xx, bb, _ = T.unpack(rec)
            fa, fb = T.forward(pp, xx, bb), T.forward(pm, xx, bb)
            if ((fa["h1"] > 0) != (fb["h1"] > 0)).any() or ((fa["h2"] > 0) != (fb["h2"] > 0)).any():
                continue
            assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (name, i, fd, g[i])
            checked[name] += 1
    assert all(v >= min(20, T.BLOCKS[k][1] - T.BLOCKS[k][0]) for k, v in checked.items()), checked
    # the summed squared error is 3n times the mean
    assert abs(loss - 3 * len(rec) * _mean_loss(p, rec)) <= 1e-9 * loss


def test_gradient_zero_for_absent_bins_and_loss_closed_form():
    """All weights zero and B3 = c: o = c, so the loss is sum (c - M/256)^2,
    dL/dB3 = 2 mean over samples of (c - t) / 3 per channel, every other
    gradient is zero; bins absent from the batch get no gradient."""
    p = np.zeros(T.NPARAM)
    p[T.P_B3:] = [0.25, 0.5, 0.75]
    rec = _records(8, 17)
    rec[:, 27] = 3
    g, loss, _, _ = T.grad(p, rec)
    t = rec[:, 28:31].astype(np.float64) / 256
    assert abs(loss - float(((p[T.P_B3:] - t) ** 2).sum())) <= 1e-12
    assert np.allclose(g[T.P_B3:], 2 * (p[T.P_B3:] - t).sum(0) / (3 * 17), rtol=0, atol=1e-15)
    assert not g[:T.P_B3].any()
    p2 = train.init_params(9).astype(np.float64)
    g2 = T.grad(p2, rec)[0]
    b1 = g2[T.P_B1:T.P_W2].reshape(32, 32)
    assert not np.delete(b1, 3, axis=0).any() and b1[3].any()


def test_adam_closed_forms():
    """Step 1 from zero moments moves each parameter by lr g / (|g| + eps)
    (the bias-corrected moments are g and g^2 exactly); a constant gradient
    keeps doing so at every later step (bias correction cancels the moments'
    warm-up exactly); a gradient that flips sign at step 2 gives the closed
    form of the corrected moments."""
    rng = np.random.default_rng(10)
    g = rng.normal(0, 1e-3, 50)
    g[0] = 0.0
    p0 = rng.normal(0, 1, 50)
    lr = 1e-3
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        pn, m, v = T.adam(p, m, v, g, lr, step)
        assert np.allclose(pn - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-18), step
        p = pn
    # g then -g: m2 = 0.9 * 0.1 g - 0.1 g = -0.01 g, corrected by 1 - 0.81;
    # v2 = (0.999 * 0.001 + 0.001) g^2, corrected by 1 - 0.999^2
    p1, m1, v1 = T.adam(p0, np.zeros(50), np.zeros(50), g, lr, 1)
    p2, _, _ = T.adam(p1, m1, v1, -g, lr, 2)
    mh = -0.01 * g / (1 - 0.81)
    vh = (0.999 * 0.001 + 0.001) * g * g / (1 - 0.999 ** 2)
    assert np.allclose(p2 - p1, -lr * mh / (np.sqrt(vh) + 1e-8), rtol=1e-9, atol=1e-18)


def test_sample_records_by_hand():
    """A 2 x 3 image: the record of pixel (0, 0) replicates the top row and
    left column for its out-of-image neighbours; bytes are S - 128 as int8,
    then the clamped bin, then the mantissas."""
    sdr = np.arange(18, dtype=np.uint8).reshape(2, 3, 3) * 13
    rgbe = np.zeros((2, 3, 4), np.uint8)
    rgbe[..., :3] = 200
    rgbe[0, 0] = (11, 22, 33, 140)
    rgbe[1, 2] = (1, 2, 3, 0)
    rec = T.samples(rgbe, sdr, -2, np.array([0, 5]))
    nb = [(0, 0), (0, 0), (0, 1), (0, 0), (0, 0), (0, 1), (1, 0), (1, 0), (1, 1)]
    exp = [int(sdr[y, x, c]) - 128 for (y, x) in nb for c in range(3)]
    assert list(rec[0, :27].view(np.int8)) == exp
    assert list(rec[0, 27:]) == [140 - 136 - 2 + 24, 11, 22, 33, 0]
    assert list(rec[1, 27:]) == [0, 1, 2, 3, 0]   # E = 0: bin clamped at 0
    nb = [(0, 1), (0, 2), (0, 2), (1, 1), (1, 2), (1, 2), (1, 1), (1, 2), (1, 2)]
    assert list(rec[1, :27].view(np.int8)) == [int(sdr[y, x, c]) - 128 for (y, x) in nb for c in range(3)]
