"""Float64 reference of the learned estimator's training step (test
infrastructure: only tests import it).

The float model, as the library's training interface defines it: features
x = (S - 128) / 128 over the 3x3 x 3-channel neighbourhood of the decoded
SDRI (border replicated, feature 3k + c for neighbour k = 3(dy+1) + (dx+1)),
a bias row B1[bin] per exponent bin bin = clamp(E - 136 + k_img + 24, 0, 31),
h1 = W1 x + B1[bin], a1 = ReLU(h1), h2 = W2 a1 + B2, a2 = ReLU(h2),
o = W3 a2 + B3 predicting M / 256.  The loss is the squared error summed over
the batch's samples and channels; the gradient is that of its mean over
3 x (samples in the batch).  Adam with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 and bias correction.  The learned estimator is an extension: the
paper's regression needs no learning (Sec. I).

Written from those definitions in plain numpy float64 (matrix products for
the layers, the chain rule written out for the backward pass).  Beside each
gradient it returns a magnitude bound: the same backward pass run on absolute
values (|W|, |x|, and the magnitudes of every intermediate), which bounds the
rounding error of any float32 evaluation of the same sums, in any order, to a
small multiple of the unit roundoff times that bound.
"""
from __future__ import annotations

import numpy as np

P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, NPARAM = 0, 864, 1888, 2912, 2944, 3040, 3043
BLOCKS = {"W1": (P_W1, P_B1), "B1": (P_B1, P_W2), "W2": (P_W2, P_B2), "B2": (P_B2, P_W3), "W3": (P_W3, P_B3),
          "B3": (P_B3, NPARAM)}
SAMPLE_BYTES = 32


def samples(rgbe: np.ndarray, sdr: np.ndarray, k_img: int, idx: np.ndarray) -> np.ndarray:
    """Sample records [n][32] uint8: 27 feature bytes S - 128 (as int8), the
    exponent bin, the three mantissas, one zero pad byte."""
    H, W = rgbe.shape[:2]
    idx = np.asarray(idx, np.int64)
    y, x = idx // W, idx % W
    out = np.zeros((len(idx), SAMPLE_BYTES), np.uint8)
    for k in range(9):
        yy = np.clip(y + k // 3 - 1, 0, H - 1)
        xx = np.clip(x + k % 3 - 1, 0, W - 1)
        for c in range(3):
            out[:, 3 * k + c] = ((sdr[yy, xx, c].astype(np.int64) - 128) & 255).astype(np.uint8)
    E = rgbe[y, x, 3].astype(np.int64)
    out[:, 27] = np.clip(E - 136 + k_img + 24, 0, 31)
    out[:, 28:31] = rgbe[y, x, :3]
    return out


def unpack(rec: np.ndarray):
    """Features (float64 [n][27]), bins [n], targets M/256 (float64 [n][3])."""
    rec = np.asarray(rec, np.uint8)
    x = rec[:, :27].view(np.int8).astype(np.float64) / 128.0
    b = rec[:, 27].astype(np.int64)
    t = rec[:, 28:31].astype(np.float64) / 256.0
    return x, b, t


def split(p: np.ndarray) -> dict:
    p = np.asarray(p, np.float64)
    return {"W1": p[P_W1:P_B1].reshape(32, 27), "B1": p[P_B1:P_W2].reshape(32, 32),
            "W2": p[P_W2:P_B2].reshape(32, 32), "B2": p[P_B2:P_W3], "W3": p[P_W3:P_B3].reshape(3, 32),
            "B3": p[P_B3:NPARAM]}


def flat(g: dict) -> np.ndarray:
    return np.concatenate([np.asarray(g[k], np.float64).reshape(-1) for k in BLOCKS])


def forward(params: np.ndarray, x: np.ndarray, b: np.ndarray) -> dict:
    P = split(params)
    h1 = x @ P["W1"].T + P["B1"][b]
    a1 = np.maximum(h1, 0.0)
    h2 = a1 @ P["W2"].T + P["B2"]
    a2 = np.maximum(h2, 0.0)
    o = a2 @ P["W3"].T + P["B3"]
    # magnitudes: the same sums over absolute values (a ReLU passes the
    # magnitude of what it lets through)
    A = {k: np.abs(v) for k, v in P.items()}
    h1s = np.abs(x) @ A["W1"].T + A["B1"][b]
    a1s = h1s * (h1 > 0)
    h2s = a1s @ A["W2"].T + A["B2"]
    a2s = h2s * (h2 > 0)
    os_ = a2s @ A["W3"].T + A["B3"]
    return {"h1": h1, "a1": a1, "h2": h2, "a2": a2, "o": o, "h1s": h1s, "a1s": a1s, "h2s": h2s, "a2s": a2s,
            "os": os_}


def grad(params: np.ndarray, rec: np.ndarray):
    """(gradient, summed squared error, magnitude bound of the gradient,
    ReLU margin) for one batch of sample records.  The margin is the smallest
    |h| / magnitude(h) over every hidden pre-activation: a float32 evaluation
    takes the same ReLU branches when it is well above the unit roundoff."""
    x, b, t = unpack(rec)
    n = len(rec)
    f = forward(params, x, b)
    P = split(params)
    A = {k: np.abs(v) for k, v in P.items()}
    e = f["o"] - t
    loss = float((e * e).sum())
    d = 2.0 * e / (3.0 * max(n, 1))
    ds = 2.0 * (f["os"] + t) / (3.0 * max(n, 1))
    m1, m2 = f["h1"] > 0, f["h2"] > 0
    g2 = (d @ P["W3"]) * m2          # dL/dh2
    g2s = (ds @ A["W3"]) * m2
    d1 = (g2 @ P["W2"]) * m1         # dL/dh1
    d1s = (g2s @ A["W2"]) * m1
    g = {"W1": d1.T @ x, "B1": np.zeros((32, 32)), "W2": g2.T @ f["a1"], "B2": g2.sum(0), "W3": d.T @ f["a2"],
         "B3": d.sum(0)}
    s = {"W1": d1s.T @ np.abs(x), "B1": np.zeros((32, 32)), "W2": g2s.T @ f["a1s"], "B2": g2s.sum(0),
         "W3": ds.T @ f["a2s"], "B3": ds.sum(0)}
    np.add.at(g["B1"], b, d1)
    np.add.at(s["B1"], b, d1s)
    with np.errstate(divide="ignore", invalid="ignore"):
        r1 = np.where(f["h1s"] > 0, np.abs(f["h1"]) / f["h1s"], np.inf)
        r2 = np.where(f["h2s"] > 0, np.abs(f["h2"]) / f["h2s"], np.inf)
    margin = np.minimum(r1.min(axis=1), r2.min(axis=1)) if n else np.zeros(0)
    return flat(g), loss, flat(s), margin


def adam(p, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step with bias correction, in float64."""
    p, m, v, g = (np.asarray(a, np.float64) for a in (p, m, v, g))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
