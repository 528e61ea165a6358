"""Pins of the oracle's entropy code of the enhancement layer (static rANS,
Duda 2013, range variant; 64 interleaved states per group).

The pins rest on facts outside the oracle's own code: hand-worked coder
states for one- and two-pixel layers, the frequency rule's invariants and its
proven cost bound against the zeroth-order entropy, round trips over edge
cases, and coding efficiency against the information content of the model."""
import math

import numpy as np
import pytest

from paper_2309_11072_amd import synth

M = 1 << 15
HDR = 4136


def layer(r, E):
    """Enhancement-layer bytes from residual planes r[3][H][W] and E[H][W]."""
    r = np.ascontiguousarray(r, np.int16)
    return np.concatenate([r.reshape(-1).view(np.uint8), np.ascontiguousarray(E, np.uint8).reshape(-1)])


def u16(st, off):
    return int.from_bytes(st[off:off + 2], "little")


def u32(st, off):
    return int.from_bytes(st[off:off + 4], "little")


def u64(st, off):
    return int.from_bytes(st[off:off + 8], "little")


def payload_words(st, G):
    base = HDR + 32 * G
    return [u16(st, base + 2 * k) for k in range((len(st) - base) // 2)]


def test_one_pixel_stream_layout(O):
    """1 x 1 layer: every plane has one symbol, so f = M and coding leaves each
    state at L = 2^16; each plane's group holds 64 flushed states (1, 0)."""
    st = O.ent_encode(layer(np.array([[[3]], [[-7]], [[0]]]), np.array([[131]])), 1, 1, log2_k=8)
    assert len(st) == HDR + 32 + 2 * 4 * 128
    assert (u32(st, 0), u32(st, 4), u32(st, 8), u32(st, 12)) == (0x454C4452, 1, 1, 1)
    assert (u32(st, 16), u32(st, 20), u32(st, 24), u64(st, 32)) == (8, 15, 1, len(st))
    for p, sym in enumerate([3 + 255, -7 + 255, 255, 131]):
        f = [u16(st, 40 + 2 * (512 * p + s)) for s in range(512)]
        assert f[sym] == M and sum(f) == M
        assert u64(st, HDR + 8 * p) == 128 * p
    assert payload_words(st, 1) == [1, 0] * (64 * 4)


def test_two_pixel_states_by_hand(O):
    """1 x 2 layer with E = (a, b), a < b: counts (1, 1) give
    f = 1 + floor((2^15 - 2) / 2) = 16384 each, c = (0, 16384).  Lane 0 codes a:
    65536 -> (65536 div 16384) 2^15 + 0 + 0 = 131072 = (2, 0); lane 1 codes b:
    4 * 2^15 + 16384 = 147456 = (2, 16384).  Residual planes are constant."""
    st = O.ent_encode(layer(np.zeros((3, 1, 2)), np.array([[100, 200]])), 1, 2, log2_k=4, predict=False)
    assert u32(st, 28) == 0
    fe = [u16(st, 40 + 2 * (512 * 3 + s)) for s in range(256)]
    assert fe[100] == fe[200] == 16384 and sum(fe) == M
    w = payload_words(st, 1)
    assert len(w) == 4 * 128
    assert w[3 * 128:4 * 128] == [2, 0, 2, 16384] + [1, 0] * 62
    assert w[:128] == [1, 0] * 64  # constant residual planes cost nothing


def test_exponent_prediction_by_hand(O):
    """2 x 2 exponents [[100, 200], [50, 49]] coded as left differences: each
    row starts with its own value, so the symbols are 100, 100, 50, 255
    (49 - 50 mod 256).  Counts (2, 1, 1), P = 3, N = 4: f = 1 + floor(h 32765 / 4)
    = 16383, 8192, 8192, and the remainder 1 goes to symbol 100."""
    E = np.array([[100, 200], [50, 49]])
    st = O.ent_encode(layer(np.zeros((3, 2, 2)), E), 2, 2, log2_k=4)
    assert u32(st, 28) == 1
    fe = [u16(st, 40 + 2 * (512 * 3 + s)) for s in range(256)]
    assert (fe[100], fe[50], fe[255]) == (16384, 8192, 8192) and sum(fe) == M
    assert np.array_equal(O.ent_decode(st, 2, 2), layer(np.zeros((3, 2, 2)), E))
    # one row: 100, 100 is a single symbol, every state stays at L
    st = O.ent_encode(layer(np.zeros((3, 1, 2)), np.array([[100, 200]])), 1, 2, log2_k=4)
    assert u16(st, 40 + 2 * (512 * 3 + 100)) == M
    assert payload_words(st, 1)[3 * 128:] == [1, 0] * 64


@pytest.mark.parametrize("H,W", [(1, 1), (5, 1), (1, 300), (37, 41), (120, 160)])
def test_exponent_prediction_counts(O, H, W):
    """The exponent plane's frequencies are the rule applied to the counts of
    the left differences (numpy, row by row); the residual planes' tables and
    the decoded layer do not depend on the prediction."""
    x = synth.generate(H, W, 4.0, seed=H + 7 * W, spec_frac=0.05)
    E = x[..., 3].astype(np.int64)
    d = E.copy()
    d[:, 1:] = (E[:, 1:] - E[:, :-1]) % 256
    want = O.ent_freqs(np.bincount(d.reshape(-1), minlength=256))
    rng = np.random.default_rng(H * W)
    res = layer(np.clip(np.round(rng.laplace(0, 3, (3, H, W))), -255, 255), E)
    st1 = O.ent_encode(res, H, W, 4, predict=True)
    st0 = O.ent_encode(res, H, W, 4, predict=False)
    assert (u32(st1, 28), u32(st0, 28)) == (1, 0)
    f1 = np.array([u16(st1, 40 + 2 * (512 * 3 + s)) for s in range(256)])
    assert np.array_equal(f1, want)
    assert st1[40:40 + 3 * 1024] == st0[40:40 + 3 * 1024]
    assert np.array_equal(O.ent_decode(st1, H, W), res) and np.array_equal(O.ent_decode(st0, H, W), res)


def _info(h, f):
    m = h > 0
    return float((h[m] * np.log2(M / f[m].astype(np.float64))).sum())


def _h0(h):
    m = h > 0
    n = h.sum()
    return float((h[m] * np.log2(n / h[m].astype(np.float64))).sum())


@pytest.mark.parametrize("seed", range(6))
def test_frequency_invariants_and_cost_bound(O, seed):
    """Sum 2^15, support equal to the present symbols, monotone in the count,
    and N H0 <= sum h log2(M/f) < N H0 + N log2(M/(M-P)): every present f is at
    least h (M - P) / N, so no symbol pays more than that factor over h / N."""
    rng = np.random.default_rng(seed)
    nsym = 511 if seed % 2 == 0 else 256
    kind = seed % 3
    if kind == 0:
        h = rng.integers(0, 1000, nsym) * (rng.random(nsym) < 0.5)
    elif kind == 1:
        h = np.bincount(np.clip(np.round(rng.laplace(nsym // 2, 4, 100000)), 0, nsym - 1).astype(int),
                        minlength=nsym)
    else:
        h = np.ones(nsym, np.int64)
        h[7] = 2 ** 31 - nsym
    h = h.astype(np.int64)
    if h.sum() == 0:
        h[0] = 1
    f = O.ent_freqs(h).astype(np.int64)
    P = int((h > 0).sum())
    assert f.sum() == M
    assert np.array_equal(f > 0, h > 0)
    order = np.argsort(h, kind="stable")
    assert np.all(np.diff(f[order]) >= 0), "frequencies must not decrease with the count"
    n = h.sum()
    lo = _h0(h)
    cost = _info(h, f)
    assert lo - 1e-6 * n <= cost < lo + n * math.log2(M / (M - P)) + 1e-6 * n


def test_group_size_limits(O):
    x = _rand_layer(np.random.default_rng(2), 3, 4, "laplace")
    for k in (3, 13):
        assert O.ent_bound(3, 4, k) == -1
        with pytest.raises(ValueError, match="-1"):
            O.ent_encode(x, 3, 4, k)


def test_single_symbol_takes_the_whole_scale(O):
    for s in (0, 255, 510):
        h = np.zeros(511, np.int64)
        h[s] = 12345
        f = O.ent_freqs(h)
        assert f[s] == M and f.sum() == M


def _rand_layer(rng, H, W, kind):
    if kind == "laplace":
        r = np.clip(np.round(rng.laplace(0, 3, (3, H, W))), -255, 255)
        E = rng.integers(120, 140, (H, W))
    elif kind == "wide":
        r = rng.integers(-255, 256, (3, H, W))
        E = rng.integers(0, 256, (H, W))
    elif kind == "extreme":
        r = rng.choice([-255, 255], (3, H, W))
        E = rng.choice([0, 255], (H, W))
    else:  # constant
        r = np.full((3, H, W), -4)
        E = np.full((H, W), 255)
    return layer(r, E)


@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (1, 1025), (64, 65), (33, 257)])
@pytest.mark.parametrize("log2_k", [4, 5, 8, 12])
@pytest.mark.parametrize("kind", ["laplace", "wide", "extreme", "constant"])
@pytest.mark.parametrize("predict", [True, False])
def test_round_trip(O, H, W, log2_k, kind, predict):
    rng = np.random.default_rng(H * 1000 + W + log2_k)
    x = _rand_layer(rng, H, W, kind)
    st = O.ent_encode(x, H, W, log2_k, predict=predict)
    assert len(st) <= O.ent_bound(H, W, log2_k)
    G = -(-H * W // (64 << log2_k))
    starts = [u64(st, HDR + 8 * k) for k in range(4 * G)] + [(len(st) - HDR - 32 * G) // 2]
    assert starts[0] == 0 and all(b - a >= 128 for a, b in zip(starts, starts[1:]))
    assert np.array_equal(O.ent_decode(st, H, W), x)


def test_encoder_output_round_trip_and_rate(O):
    """A real enhancement layer (oracle encoder, 96 x 80, q = 75) round-trips and
    its residual planes code within 2 % plus the flushed states of H0."""
    x = synth.generate(96, 80, 4.0, seed=77, spec_frac=0.05)
    ref = O.encode_enh(x, 75)
    H, W = 96, 80
    res = np.ascontiguousarray(ref["resid"]).view(np.uint8).reshape(-1)
    st = O.ent_encode(res, H, W, 4)
    assert np.array_equal(O.ent_decode(st, H, W), res)
    G = -(-H * W // (64 << 4))
    h = O.resid_hist(ref["resid"], H * W)
    bits_planes = sum(_h0(hc) for hc in h)
    w = payload_words(st, G)
    starts = [u64(st, HDR + 8 * k) for k in range(4 * G)] + [len(w)]
    coded = 16 * (starts[3 * G] - starts[0]) - 3 * G * 64 * 32
    assert coded <= 1.02 * bits_planes + 3 * G * 64 * 16


def test_coding_efficiency(O):
    """300,000 Laplacian residuals per plane: the words emitted while coding
    (flushed states excluded) stay within 0.2 % of sum log2(M / f), the
    information content under the stream's own frequencies."""
    rng = np.random.default_rng(3)
    H, W = 300, 1000
    x = _rand_layer(rng, H, W, "laplace")
    log2_k = 10
    st = O.ent_encode(x, H, W, log2_k)
    G = -(-H * W // (64 << log2_k))
    w = payload_words(st, G)
    starts = [u64(st, HDR + 8 * k) for k in range(4 * G)] + [len(w)]
    r = x[:6 * H * W].view(np.int16).reshape(3, H * W)
    for p in range(3):
        h = np.bincount(r[p].astype(np.int64) + 255, minlength=511)
        f = np.array([u16(st, 40 + 2 * (512 * p + s)) for s in range(511)], np.int64)
        info = _info(h, f)
        emitted = 16 * (starts[(p + 1) * G] - starts[p * G] - 128 * G)
        assert abs(emitted - info) <= 0.002 * info + G * 64 * 32, (p, emitted, info)


def test_rejects_out_of_range_and_corrupt_streams(O):
    r = np.zeros((3, 4, 5), np.int16)
    r[1, 2, 3] = 256
    with pytest.raises(ValueError, match="-3"):
        O.ent_encode(layer(r, np.zeros((4, 5))), 4, 5, 4)
    x = _rand_layer(np.random.default_rng(1), 40, 30, "laplace")
    st = bytearray(O.ent_encode(x, 40, 30, 4))
    bad = bytearray(st)
    bad[0] ^= 1
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(bad), 40, 30)
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(st), 40, 31)
    bad = bytearray(st)
    bad[28] = 4  # unknown flag
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(bad), 40, 30)
    bad = bytearray(st)
    bad[28] = 3  # the context flag on a stream without context tables (too short for their header)
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(bad), 40, 30, sdr=np.zeros((40, 30, 3), np.uint8))
    bad = bytearray(st)
    bad[40 + 2 * 300] ^= 1  # frequencies no longer sum to 2^15
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(bad), 40, 30)
    bad = bytearray(st)
    bad[HDR + 8] += 1  # group 1 starts a word later: group 0 ends before its recorded end
    with pytest.raises(ValueError, match="-6"):
        O.ent_decode(bytes(bad), 40, 30)
