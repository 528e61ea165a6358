"""Pins for two oracle parts that the closed-form models elsewhere cannot
reach: the learned estimator's requantisation rounding and the residual
histogram.  CPU only.

The learned estimator is an extension beyond the paper (its regression needs
no learning, Sec. I).  Its integer arithmetic, as the model format defines it:
per pixel, 27 features S - 128 of the 3x3 neighbourhood (border replicated),
a bin b = clamp(E - 136 + k_img + 24, 0, 31) choosing the first layer's bias
row, two hidden layers a = clamp((h m + 2^(r-1)) >> r, 0, 255), and an output
q8 = (o m3 + 2^(r3-1)) >> r3, M_L = clamp((q8 + 128) >> 8, 0, 255).

The reference below writes that arithmetic out again in numpy int64 matrix
products, without calling the oracle's estimator, and compares every output
byte.  The models are random (multipliers over [1, 1023], shifts over
[1, 28], biases within 2^18) plus probe neurons built so that h m lands
exactly on 2^(r-1) mod 2^r at the largest shifts.  Each test also shows that
its inputs discriminate: the reference with a rounding term dropped, or with
the bin offset moved by one, disagrees with the oracle on some pixel.  Each
such change was also made once in the C oracle itself (dropping 2^(r-1) in
the hidden requantisation, dropping the +128 of the output, moving the bin
offset to +23, moving the histogram's offset to +254), and each made the
matching test below fail.
"""
import numpy as np
import pytest

from paper_2309_11072_amd import model_format


def _rnd(v, r, half):
    """(v + 2^(r-1)) >> r per column (arithmetic shift), or v >> r without
    the rounding term."""
    r = np.asarray(r, np.int64)
    add = np.left_shift(np.int64(1), r - 1) if half else 0
    return np.right_shift(v + add, r)


def mlp_ref(S, E, k_img, P, half=True, out_half=True, bin_off=24, a_max=255):
    """Learned estimates M_L [H][W][3] in plain int64 numpy."""
    H, W, _ = S.shape
    feat = np.zeros((H * W, 32), np.int64)
    ys, xs = np.arange(H), np.arange(W)
    for k in range(9):
        dy, dx = k // 3 - 1, k % 3 - 1
        yy = np.clip(ys + dy, 0, H - 1)[:, None]
        xx = np.clip(xs + dx, 0, W - 1)[None, :]
        for c in range(3):
            feat[:, 3 * k + c] = (S[yy, xx, c].astype(np.int64) - 128).reshape(-1)
    b = np.clip(E.astype(np.int64).reshape(-1) - 136 + k_img + bin_off, 0, 31)
    W1, B1 = P["W1"].astype(np.int64), P["B1"].astype(np.int64)
    h1 = feat @ W1.T + B1[b]
    a1 = np.clip(_rnd(h1 * P["m1"].astype(np.int64), P["r1"], half), 0, a_max)
    h2 = a1 @ P["W2"].astype(np.int64).T + P["B2"].astype(np.int64)
    a2 = np.clip(_rnd(h2 * P["m2"].astype(np.int64), P["r2"], half), 0, a_max)
    o = a2 @ P["W3"][:3].astype(np.int64).T + P["B3"][:3].astype(np.int64)
    q8 = _rnd(o * P["m3"][:3].astype(np.int64), P["r3"][:3], half)
    m = np.right_shift(q8 + (128 if out_half else 0), 8)
    out = np.clip(m, 0, 255).reshape(H, W, 3).astype(np.uint8)
    trace = {"h1m": h1 * P["m1"].astype(np.int64), "h2m": h2 * P["m2"].astype(np.int64), "o": o, "q8": q8}
    return out, trace


def random_model(seed):
    """A random model inside the library's limits (m in [1, 2^10), r in
    [1, 28], |B| <= 2^18), its multipliers scaled so that most neurons
    neither die nor saturate, plus two probe neurons.

    Probe neuron 0 of layer 1 reads only the centre pixel's G (weight 1) with
    bias 2^18 - 3, multiplier 512 and shift 28: h m = 2^27 + 512 (S_G - 131),
    exactly half of 2^28 where S_G = 131, so a1[0] = [S_G >= 131] with the
    rounding term and 0 everywhere without it.  Probe neuron 0 of layer 2
    reads a1[0] (weight 127) with bias 2^18 - 127, multiplier 512 and shift
    28: h m = 2^27 exactly when a1[0] = 1, so a2[0] = a1[0] with the rounding
    term and 0 without it."""
    rng = np.random.default_rng(seed)
    P = {}
    P["W1"] = rng.integers(-127, 128, (32, 32))
    P["B1"] = rng.integers(-(1 << 15), 1 << 15, (32, 32))
    P["W2"] = rng.integers(-127, 128, (32, 32))
    P["B2"] = rng.integers(-(1 << 15), 1 << 15, 32)
    P["W3"] = rng.integers(-127, 128, (16, 32))
    P["B3"] = rng.integers(-(1 << 18), 1 << 18, 16)
    for layer, scale in (("1", 64 / 30000.0), ("2", 64 / 25000.0)):
        r = rng.permutation(np.concatenate([np.arange(1, 29), rng.integers(1, 29, 4)]))  # every shift
        m = np.clip(np.round(scale * np.exp2(r) * rng.uniform(0.5, 2.0, 32)), 1, 1023).astype(np.int64)
        P["m" + layer], P["r" + layer] = m, r
    # probe neurons (layer 1 neuron 0, layer 2 neuron 0)
    P["W1"][0] = 0
    P["W1"][0, 13] = 1               # feature 13 = centre pixel, G
    P["B1"][:, 0] = (1 << 18) - 3    # h = 2^18 - 3 + (S_G - 128): 2^18 at S_G = 131
    P["m1"][0], P["r1"][0] = 512, 28
    P["W2"][0] = 0
    P["W2"][0, 0] = 127
    P["B2"][0] = (1 << 18) - 127
    P["m2"][0], P["r2"][0] = 512, 28
    # outputs: from the spread of o over a calibration image, m3 / 2^r3 and
    # B3 such that q8 spans the mantissa range in Q8 (centre 2^15, standard
    # deviation 20000, about 78 codes)
    P["W3"][3:] = 0
    P["B3"], P["m3"], P["r3"] = np.zeros(16, np.int64), np.ones(16, np.int64), np.ones(16, np.int64)
    S = rng.integers(0, 256, (64, 64, 3)).astype(np.uint8)
    o = mlp_ref(S, rng.integers(100, 160, (64, 64)), 0, P)[1]["o"]
    for c in range(3):
        sc = 20000.0 / max(float(o[:, c].std()), 1.0)
        rmax = int(np.clip(np.floor(np.log2(1023.0 / sc)), 1, 28))
        r3 = int(rng.integers(max(1, rmax - 3), rmax + 1))
        P["r3"][c] = r3
        P["m3"][c] = int(np.clip(round(sc * 2.0 ** r3), 1, 1023))
        P["B3"][c] = int(np.clip(round(32768.0 * 2.0 ** r3 / P["m3"][c] - np.median(o[:, c])), -(1 << 18), 1 << 18))
    return P


def _image(rng, H, W):
    S = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    x = rng.integers(0, 256, (H, W, 4)).astype(np.uint8)
    return S, x


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_mlp_requant_rounding_vs_int64_brute_force(O, seed):
    """The oracle's learned estimate equals the int64 numpy reference at
    every pixel of four sizes (1x1, 7x9, 33x47, 96x80: borders on every side),
    for three random models and three k_img.  The inputs contain exact
    half-way products h m = 2^(r-1) mod 2^r in both hidden layers (at shifts
    up to 28) and outputs q8 = 128 mod 256, and dropping either rounding term,
    moving the bin offset, clamping the hidden activations at 127 (the first
    format version) or not at all changes some estimate."""
    P = random_model(seed)
    blob = model_format.pack(P)
    rng = np.random.default_rng(seed + 100)
    half_hits = {"h1m": set(), "h2m": set()}
    q8_hits = 0
    differs = {"half": 0, "out_half": 0, "bin": 0, "a_max_127": 0, "no_upper_clamp": 0}
    for H, W in [(1, 1), (7, 9), (33, 47), (96, 80)]:
        S, x = _image(rng, H, W)
        for k_img in (-9, 0, 13):
            got = O.mlp_estimate(S, x, k_img, blob)
            ref, tr = mlp_ref(S, x[..., 3], k_img, P)
            assert np.array_equal(got, ref), (H, W, k_img)
            for key, rk in (("h1m", P["r1"]), ("h2m", P["r2"])):
                rk = np.asarray(rk, np.int64)
                hm = tr[key]
                on_half = (hm & ((np.int64(1) << rk) - 1)) == (np.int64(1) << (rk - 1))
                for n in np.nonzero(on_half.any(axis=0))[0]:
                    half_hits[key].add(int(rk[n]))
            q8_hits += int(((tr["q8"] & 255) == 128).sum())
            differs["half"] += int((mlp_ref(S, x[..., 3], k_img, P, half=False)[0] != got).any())
            differs["out_half"] += int((mlp_ref(S, x[..., 3], k_img, P, out_half=False)[0] != got).any())
            differs["bin"] += int((mlp_ref(S, x[..., 3], k_img, P, bin_off=23)[0] != got).any())
            differs["a_max_127"] += int((mlp_ref(S, x[..., 3], k_img, P, a_max=127)[0] != got).any())
            differs["no_upper_clamp"] += int((mlp_ref(S, x[..., 3], k_img, P, a_max=1 << 40)[0] != got).any())
    # exact half-way products occurred at small and at the largest shifts
    for key in half_hits:
        assert min(half_hits[key]) <= 4 and max(half_hits[key]) == 28, (key, sorted(half_hits[key]))
    assert q8_hits >= 10
    assert all(v > 0 for v in differs.values()), differs


def test_mlp_probe_neurons_need_the_rounding_term(O):
    """The probe neurons alone: every other weight zero and output R reading
    a2[0] only (W3[0][0] = 127, B3[0] = 1, m3 = 2, r3 = 1, so q8 = o =
    127 a2[0] + 1 and M_L[R] = (q8 + 128) >> 8 = a2[0]).  M_L[R] is 1 exactly
    where the centre pixel's S_G reaches 131: the half-way product at shift
    28 rounds up in both hidden layers, and q8 = 128 rounds up at the output.
    Without any one of the three rounding steps it stays 0."""
    P = random_model(5)
    for k in ("W1", "W2", "W3"):
        keep = P[k][0].copy()
        P[k][:] = 0
        if k != "W3":
            P[k][0] = keep
    P["W3"][0, 0] = 127
    P["B3"][:] = 0
    P["B3"][0] = 1
    P["m3"][:3], P["r3"][:3] = 2, 1
    blob = model_format.pack(P)
    S = np.zeros((16, 16, 3), np.uint8)
    S[..., 1] = (120 + np.arange(16 * 16) % 24).reshape(16, 16)
    x = np.zeros((16, 16, 4), np.uint8)
    got = O.mlp_estimate(S, x, 0, blob)
    exp = (S[..., 1] >= 131).astype(np.uint8)
    assert exp.min() == 0 and exp.max() == 1
    assert np.array_equal(got[..., 0], exp)
    assert not got[..., 1:].any()
    assert np.array_equal(got, mlp_ref(S, x[..., 3], 0, P)[0])
    assert not mlp_ref(S, x[..., 3], 0, P, half=False)[0].any()
    assert not mlp_ref(S, x[..., 3], 0, P, out_half=False)[0].any()


def test_resid_hist_vs_bincount(O):
    """hist[c][r + 255] of the oracle equals numpy's bincount of r + 255 per
    channel, on planes that include both ends of the range (+-255), a
    constant plane and random values."""
    rng = np.random.default_rng(41)
    for H, W in [(1, 1), (5, 7), (64, 97)]:
        n = H * W
        r = rng.integers(-255, 256, (3, n)).astype(np.int16)
        r[0, 0] = -255
        r[1, -1] = 255
        if n > 1:
            r[2, :] = 255 if n % 2 else -255
        buf = np.zeros(7 * n, np.uint8)
        buf[:6 * n] = r.reshape(-1).view(np.uint8)
        got = O.resid_hist(buf, n)
        for c in range(3):
            exp = np.bincount(r[c].astype(np.int64) + 255, minlength=511)
            assert np.array_equal(got[c], exp), (H, W, c)
        assert got.sum() == 3 * n
