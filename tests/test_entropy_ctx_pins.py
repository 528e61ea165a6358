"""Pins of the oracle's residual contexts in the entropy code (stream flag
bit 1): each residual of channel p is coded with the table of its context
k = S[i][p] >> 5, S the decoded base layer; 8 tables per channel, the
exponent plane's table last.

They rest on facts outside the context code itself: with one context per
channel the stream must be the plain stream (already pinned by hand-worked
states) with the tables moved, a channel whose residual is a function of its
context costs nothing beyond the flushed states, round trips over edge cases,
and the rate against the conditional zeroth-order entropy."""
import numpy as np
import pytest

from paper_2309_11072_amd import synth

M = 1 << 15
HDR, HDR_CTX = 4136, 25640


def layer(r, E):
    r = np.ascontiguousarray(r, np.int16)
    return np.concatenate([r.reshape(-1).view(np.uint8), np.ascontiguousarray(E, np.uint8).reshape(-1)])


def u16(st, off):
    return int.from_bytes(st[off:off + 2], "little")


def u32(st, off):
    return int.from_bytes(st[off:off + 4], "little")


def u64(st, off):
    return int.from_bytes(st[off:off + 8], "little")


def table(st, t):
    return np.array([u16(st, 40 + 2 * (512 * t + s)) for s in range(512)])


def rand_layer(rng, H, W, kind="laplace"):
    if kind == "laplace":
        r = np.clip(np.round(rng.laplace(0, 3, (3, H, W))), -255, 255)
        E = rng.integers(120, 140, (H, W))
    elif kind == "wide":
        r = rng.integers(-255, 256, (3, H, W))
        E = rng.integers(0, 256, (H, W))
    else:  # extreme
        r = rng.choice([-255, 255], (3, H, W))
        E = rng.choice([0, 255], (H, W))
    return layer(r, E)


@pytest.mark.parametrize("ctx", [(0, 0, 0), (1, 7, 3), (5, 2, 6)])
def test_one_context_per_channel_is_the_plain_stream(O, ctx):
    """When every pixel of channel p falls in context k_p, table 8 p + k_p is
    the plain stream's table p, every other residual table is empty, and the
    group table and payload are the plain stream's word for word.  Distinct
    k_p per channel pin which SDRI channel selects the context."""
    rng = np.random.default_rng(sum(ctx))
    H, W = 37, 101
    x = rand_layer(rng, H, W)
    sdr = np.stack([rng.integers(32 * k, 32 * k + 32, (H, W)) for k in ctx], axis=-1).astype(np.uint8)
    for predict in (True, False):
        plain = O.ent_encode(x, H, W, 4, predict=predict)
        st = O.ent_encode(x, H, W, 4, predict=predict, sdr=sdr)
        assert u32(st, 28) == u32(plain, 28) | 2
        assert u64(st, 32) == len(st) == len(plain) + HDR_CTX - HDR
        for p in range(3):
            for k in range(8):
                want = table(plain, p) if k == ctx[p] else np.zeros(512)
                assert np.array_equal(table(st, 8 * p + k), want), (p, k)
        assert np.array_equal(table(st, 24), table(plain, 3))
        assert st[HDR_CTX:] == plain[HDR:]
        assert np.array_equal(O.ent_decode(st, H, W, sdr=sdr), x)


def test_residual_determined_by_its_context_costs_only_the_states(O):
    """Channel 0's residual is 0 where S_0 < 32 and 100 where S_0 >= 224, so
    tables 0 and 7 each hold one symbol with f = M; channels 1 and 2 and E are
    constant.  Coding a symbol of frequency M leaves a state unchanged, so
    every group is its 64 flushed states (1, 0) and nothing else."""
    H, W = 9, 130
    s0 = np.where((np.arange(H * W) % 3) == 0, 250, 7).reshape(H, W)
    sdr = np.stack([s0, np.full((H, W), 100), np.full((H, W), 31)], axis=-1).astype(np.uint8)
    r = np.zeros((3, H, W), np.int64)
    r[0] = np.where(s0 >= 224, 100, 0)
    r[1] = -3
    r[2] = 9
    x = layer(r, np.full((H, W), 140))
    st = O.ent_encode(x, H, W, 4, predict=False, sdr=sdr)
    G = -(-H * W // (64 << 4))
    assert len(st) == HDR_CTX + 32 * G + 2 * 4 * G * 128
    assert table(st, 0)[255] == M and table(st, 7)[355] == M
    assert table(st, 8 + 3)[252] == M and table(st, 16 + 0)[264] == M and table(st, 24)[140] == M
    used = {0, 7, 11, 16, 24}
    for t in range(25):
        assert table(st, t).sum() == (M if t in used else 0), t
    words = [u16(st, HDR_CTX + 32 * G + 2 * k) for k in range((len(st) - HDR_CTX - 32 * G) // 2)]
    assert words == [1, 0] * (64 * 4 * G)
    assert np.array_equal(O.ent_decode(st, H, W, sdr=sdr), x)


@pytest.mark.parametrize("H,W", [(1, 1), (7, 9), (1, 1025), (64, 65), (33, 257)])
@pytest.mark.parametrize("log2_k", [4, 8, 12])
@pytest.mark.parametrize("kind", ["laplace", "wide", "extreme"])
@pytest.mark.parametrize("sdr_kind", ["uniform", "two"])
def test_round_trip(O, H, W, log2_k, kind, sdr_kind):
    rng = np.random.default_rng(H * 7 + W + log2_k)
    x = rand_layer(rng, H, W, kind)
    if sdr_kind == "uniform":
        sdr = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    else:  # two contexts per channel, the others empty
        sdr = rng.choice(np.array([40, 200], np.uint8), (H, W, 3))
    for predict in (True, False):
        st = O.ent_encode(x, H, W, log2_k, predict=predict, sdr=sdr)
        assert len(st) <= O.ent_bound(H, W, log2_k, contexts=True)
        assert np.array_equal(O.ent_decode(st, H, W, sdr=sdr), x)


def test_rate_against_the_conditional_entropy(O):
    """A real layer (oracle encoder, 256 x 320, q 60): the residual planes
    code within 2 % (plus the flushed states) of sum over tables of N_t H0_t,
    and that payload is smaller than the plain stream's (conditioning on the
    context lowers the entropy here by far more than the rounding)."""
    H, W = 256, 320
    x = synth.generate(H, W, 3.5, seed=78, spec_frac=0.0)
    ref = O.encode_enh(x, 60)
    res = np.ascontiguousarray(ref["resid"]).view(np.uint8).reshape(-1)
    sdr = ref["sdr"]
    st = O.ent_encode(res, H, W, 4, sdr=sdr)
    plain = O.ent_encode(res, H, W, 4)
    assert np.array_equal(O.ent_decode(st, H, W, sdr=sdr), res)
    r, _ = O.split_resid(ref["resid"], H, W)
    cond = 0.0
    for p in range(3):
        ctx = sdr[..., p] >> 5
        for k in range(8):
            v = r[p][ctx == k].astype(np.int64) + 255
            if v.size:
                h = np.bincount(v, minlength=511)
                m = h > 0
                cond += float((h[m] * np.log2(v.size / h[m])).sum())
    G = -(-H * W // (64 << 4))
    start = lambda s, d, k: u64(s, d + 8 * k)  # noqa: E731
    coded = 16 * (start(st, HDR_CTX, 3 * G) - start(st, HDR_CTX, 0)) - 3 * G * 64 * 32
    assert coded <= 1.02 * cond + 3 * G * 64 * 16
    assert start(st, HDR_CTX, 3 * G) < start(plain, HDR, 3 * G)


def test_corrupt_and_mismatched_inputs(O):
    """A symbol whose context table is empty (decoded against another SDRI)
    and a context table that sums to neither 0 nor M are rejected; the stream
    cannot be decoded without the SDRI, nor encoded without it."""
    rng = np.random.default_rng(5)
    H, W = 20, 30
    x = rand_layer(rng, H, W)
    sdr = np.full((H, W, 3), 10, np.uint8)
    st = O.ent_encode(x, H, W, 4, sdr=sdr)
    with pytest.raises(ValueError, match="-6"):
        O.ent_decode(st, H, W, sdr=np.full((H, W, 3), 200, np.uint8))
    with pytest.raises(ValueError, match="-1"):
        O.ent_decode(st, H, W)
    bad = bytearray(st)
    bad[40 + 2 * 512 * 3] = 1  # table 3 (channel 0, context 3) was empty
    with pytest.raises(ValueError, match="-5"):
        O.ent_decode(bytes(bad), H, W, sdr=sdr)
    with pytest.raises(ValueError):
        O.ent_decode(st[:HDR_CTX - 1], H, W, sdr=sdr)
