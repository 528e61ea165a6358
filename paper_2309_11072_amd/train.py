"""Training and int8 quantisation of the learned mantissa estimator.

The estimator is an extension beyond the paper (whose regression needs no
learning).  Its training pairs are (decoded SDRI neighbourhood, mantissa) pixel
pairs produced by the plain encoder on synthetic images; the FP32 training
steps run in the library's HIP kernels (``rdl_train_samples``,
``rdl_train_step``); this module only orchestrates them and turns the float
parameters into the int8 model blob (``model_format``) with per-channel
requantisation multipliers.

    python -m paper_2309_11072_amd.train --out model.bin
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

from . import model_format, rdl, synth

P_W1, P_B1, P_W2, P_B2, P_W3, P_B3, NPARAM = 0, 864, 1888, 2912, 2944, 3040, 3043


def init_params(seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(NPARAM, np.float32)
    p[P_W1:P_B1] = rng.normal(0, math.sqrt(2 / 27), 864)
    p[P_W2:P_B2] = rng.normal(0, math.sqrt(2 / 32), 1024)
    p[P_W3:P_B3] = rng.normal(0, math.sqrt(1 / 32), 96)
    p[P_B1:P_W2] = 0.1
    p[P_B2:P_W3] = 0.1
    p[P_B3:] = 0.5
    return p


def unflatten(p: np.ndarray) -> dict:
    return {"W1": p[P_W1:P_B1].reshape(32, 27), "B1": p[P_B1:P_W2].reshape(32, 32),
            "W2": p[P_W2:P_B2].reshape(32, 32), "B2": p[P_B2:P_W3], "W3": p[P_W3:P_B3].reshape(3, 32),
            "B3": p[P_B3:NPARAM]}


def _mult_shift(ratio: np.ndarray, rmax: int = 28):
    """m / 2^r ~= ratio with m in [1, M_LIMIT), r in [1, rmax]."""
    mlim = model_format.M_LIMIT
    m = np.zeros(ratio.shape, np.int64)
    r = np.zeros(ratio.shape, np.int64)
    for i, rho in enumerate(ratio.reshape(-1)):
        rho = max(float(rho), 1e-12)
        rr = int(np.clip(math.floor(math.log2((mlim - 1) / rho)), 1, rmax))
        mm = int(round(rho * 2 ** rr))
        while mm >= mlim and rr > 1:
            rr -= 1
            mm = int(round(rho * 2 ** rr))
        m.reshape(-1)[i] = min(max(mm, 1), mlim - 1)
        r.reshape(-1)[i] = rr
    return m, r


def _pow2_shift(ratio: np.ndarray, rmax: int, pair: str):
    """Shift r in [1, rmax] with 2^r >= ratio, the smallest such: a hidden
    activation step of sw 2^r is at least the calibrated step, so no more
    values clip at 255 than the calibration allows.  pair "max" / "min": the
    neurons (2k, 2k + 1) share the larger / smaller of their two shifts (the
    library's fastest path); "" leaves every neuron its own."""
    r = np.clip(np.ceil(np.log2(np.maximum(ratio, 1e-30))), 1, rmax).astype(np.int64)
    if pair:
        f = np.maximum if pair == "max" else np.minimum
        r[0::2] = r[1::2] = f(r[0::2], r[1::2])
    return r


def _hidden_layer(We, B, s, pow2: bool, rmax: int, pair: str):
    """Quantise one hidden layer whose float weights We (already scaled by
    the input step) and biases B produce pre-activations with calibrated
    activation step s: int8 weights, biases, multipliers, shifts and the
    actual activation step."""
    lim = 1 << 18
    sw = np.maximum(np.abs(We).max(axis=1), 1e-12) / 127.0
    if pow2:
        # a row whose calibrated step needs a shift beyond rmax (or beyond the
        # shift it shares with its pair neuron) takes a coarser weight step,
        # keeping its activation step
        sw = np.maximum(sw, s / 2.0 ** rmax)
        r = _pow2_shift(s / sw, rmax, pair)
        sw = np.maximum(sw, s / 2.0 ** r)
        m = np.ones(len(s), np.int64)
        t = sw * 2.0 ** r  # the actual activation step
    else:
        m, r = _mult_shift(sw / s)
        t = s
    Wq = np.clip(np.round(We / sw[:, None]), -127, 127)
    Bq = np.clip(np.round(B / sw), -lim, lim)
    return Wq, Bq, m, r, t


def quantise(p: np.ndarray, feats: np.ndarray, bins: np.ndarray, pow2: bool = True, rmax: int = 22,
             pair: str = "min") -> bytes:
    """int8 model blob from float parameters; activation scales from the
    float forward pass over the calibration samples (feats int8 [N, 27]).
    Hidden activations are unsigned bytes (0 .. A_MAX = 255).

    pow2: the hidden layers' requantisation multipliers are 1 (a shift by r
    alone, the fast path of the library's estimator); each hidden activation
    step then becomes sw 2^r, and the next layer's float weights are scaled
    by that actual step before they are quantised, so the powers of two cost
    activation resolution and nothing else.  pair: see _pow2_shift."""
    amax = model_format.A_MAX
    P = unflatten(p.astype(np.float64))
    x = feats.astype(np.float64) / 128.0
    h1 = x @ P["W1"].T + P["B1"][bins]
    s1 = np.maximum(np.percentile(np.maximum(h1, 0), 99.99, axis=0), 1e-9) / amax
    W1p, B1q, m1, r1, t1 = _hidden_layer(P["W1"] / 128.0, P["B1"], s1, pow2, rmax, pair)
    W1q = np.zeros((32, 32), np.int64)
    W1q[:, :27] = W1p
    a1q = np.clip(np.round(np.maximum(h1, 0) / t1), 0, amax) * t1  # activations as the model will see them
    a2 = np.maximum(a1q @ P["W2"].T + P["B2"], 0)
    s2 = np.maximum(np.percentile(a2, 99.99, axis=0), 1e-9) / amax
    W2q, B2q, m2, r2, t2 = _hidden_layer(P["W2"] * t1[None, :], P["B2"], s2, pow2, rmax, pair)
    W3e = P["W3"] * t2[None, :]
    sw3 = np.maximum(np.abs(W3e).max(axis=1), 1e-12) / 127.0
    W3q = np.zeros((16, 32), np.int64)
    W3q[:3] = np.clip(np.round(W3e / sw3[:, None]), -127, 127)
    B3q = np.zeros(16, np.int64)
    B3q[:3] = np.clip(np.round(P["B3"] / sw3), -(1 << 18), 1 << 18)
    m3 = np.ones(16, np.int64)
    r3 = np.ones(16, np.int64)
    m3[:3], r3[:3] = _mult_shift(sw3 * 65536.0, rmax=22)
    return model_format.pack({"W1": W1q, "B1": B1q, "m1": m1, "r1": r1, "W2": W2q, "B2": B2q, "m2": m2, "r2": r2,
                              "W3": W3q, "B3": B3q, "m3": m3, "r3": r3})


def make_samples(codec, specs, n_samples: int, seed: int):
    """Encode the training images with the plain encoder and draw n_samples
    pixels without replacement across them; returns the sample records."""
    codec.set_estimator(0)
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [sp.H * sp.W for sp in specs]
    total = sum(sizes)
    pick = np.sort(rng.choice(total, size=min(n_samples, total), replace=False))
    recs = []
    start = 0
    for sp, npx in zip(specs, sizes):
        x = torch.from_numpy(sp.make()).cuda()
        sdr, hdr, resid = codec.encode_enh(x, sp.q)
        k_img = int(rdl.header_from_bytes(hdr)["k_img"])
        sel = pick[(pick >= start) & (pick < start + npx)] - start
        idx = torch.from_numpy(sel.astype(np.int64)).cuda()
        recs.append(codec.train_samples(x, sdr, k_img, idx))
        start += npx
    torch.cuda.synchronize()
    return torch.cat(recs)


def train(codec, samples: torch.Tensor, epochs: int = 4, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
          log=print) -> np.ndarray:
    params = torch.from_numpy(init_params(seed)).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    n = samples.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    step = 0
    steps_per_epoch = (n + batch - 1) // batch
    for ep in range(epochs):
        order = torch.randperm(n, generator=g).cuda()
        data = samples[order].contiguous()
        tot = 0.0
        for k in range(steps_per_epoch):
            step += 1
            frac = step / (epochs * steps_per_epoch)
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * frac))  # cosine decay
            codec.train_step(params, m, v, data, k * batch, batch, lr_t, step, loss_out=loss)
            if k % 200 == 0 or k == steps_per_epoch - 1:
                tot = float(loss.item()) / (3 * min(batch, n - k * batch))
                log("epoch %d step %d/%d  mse(M/256) %.6f  (rms %.2f codes)" % (ep, k, steps_per_epoch, tot,
                                                                             256 * math.sqrt(tot)))
    torch.cuda.synchronize()
    return params.cpu().numpy()


def bits_per_pixel(codec, specs, learned: bool) -> float:
    codec.set_estimator(1 if learned else 0)
    tot_bits = 0.0
    tot_px = 0
    for sp in specs:
        x = torch.from_numpy(sp.make()).cuda()
        sdr, hdr, resid = codec.encode_enh(x, sp.q)
        h = codec.resid_hist(resid, sp.H, sp.W).cpu().numpy().astype(np.float64)
        for c in range(3):
            p = h[c][h[c] > 0] / h[c].sum()
            tot_bits += float(-(p * np.log2(p)).sum()) * sp.H * sp.W
        tot_px += sp.H * sp.W
    codec.set_estimator(0)
    return tot_bits / tot_px


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--samples", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval", type=int, default=16, help="number of 1920x1080 evaluation images")
    ap.add_argument("--params-out", default="", help="also save the float parameters (.npy)")
    ap.add_argument("--train-set", choices=("config2", "wide"), default="config2",
                    help="config2: the two 3840x2160 images of the single-image workload's generator; wide: those "
                         "plus eight images over the batch workloads' parameter ranges")
    ap.add_argument("--rmax", type=int, default=22,
                    help="largest hidden shift of a power-of-two model (22: the library's power-of-two paths)")
    ap.add_argument("--pair", choices=("max", "min", "none"), default="min",
                    help="shift shared by each hidden neuron pair (2k, 2k + 1): the larger or smaller of the two "
                         "(the library's fastest path), or none")
    ap.add_argument("--general", action="store_true",
                    help="general requantisation multipliers instead of powers of two")
    ap.add_argument("--params-in", default="",
                    help="quantise these float parameters (.npy) instead of training; the samples are drawn for "
                         "calibration only")
    args = ap.parse_args()
    t0 = time.time()
    codec = rdl.Codec(0)
    specs = synth.learned_train_set() + (synth.learned_train_set_wide() if args.train_set == "wide" else [])
    n_samples = 200_000 if args.params_in else args.samples
    samples = make_samples(codec, specs, n_samples, seed=4000)
    print("samples: %d records in %.1f s" % (samples.shape[0], time.time() - t0), flush=True)
    if args.params_in:
        params = np.load(args.params_in)
    else:
        params = train(codec, samples, args.epochs, args.batch, args.lr, log=lambda s: print(s, flush=True))
    if args.params_out:
        np.save(args.params_out, params)
    calib = samples[:200_000].cpu().numpy()
    blob = quantise(params, calib[:, :27].view(np.int8), calib[:, 27].astype(np.int64), pow2=not args.general,
                    rmax=args.rmax, pair="" if args.pair == "none" else args.pair)
    with open(args.out, "wb") as fh:
        fh.write(blob)
    print("model written: %s (%d bytes, hash %016x) after %.1f s" % (args.out, len(blob), model_format.blob_hash(blob),
                                                                   time.time() - t0), flush=True)
    codec.set_model(blob)
    ev = synth.learned_eval_set()[: args.eval]
    b_slr = bits_per_pixel(codec, ev, False)
    b_l = bits_per_pixel(codec, ev, True)
    print("eval (%d x 1920x1080): bits/px SLR %.4f  learned+fallback %.4f" % (len(ev), b_slr, b_l), flush=True)


if __name__ == "__main__":
    main()
