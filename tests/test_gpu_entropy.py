"""GPU entropy code of the enhancement layer against the oracle: the code
stream must equal the oracle's byte for byte, and the GPU decoder must return
the layer exactly.  Layers come from the GPU encoder (the 3840 x 2160 image)
or are drawn directly (residual planes and exponents of chosen spreads), with
sizes that leave ragged last groups and lanes."""
import numpy as np
import pytest
import torch

from paper_2309_11072_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rdl_mod():
    from paper_2309_11072_amd import rdl
    return rdl


@pytest.fixture(scope="module")
def codec(rdl_mod):
    c = rdl_mod.Codec(0)
    yield c
    c.close()


def make_layer(H, W, seed, spread=3.0, e_lo=110, e_hi=150, outlier=0.0):
    rng = np.random.default_rng(seed)
    r = np.clip(np.round(rng.laplace(0, spread, (3, H, W))), -255, 255)
    if outlier:
        m = rng.random((3, H, W)) < outlier
        r[m] = rng.integers(-255, 256, int(m.sum()))
    E = rng.integers(e_lo, e_hi, (H, W))
    return np.concatenate([r.astype(np.int16).reshape(-1).view(np.uint8), E.astype(np.uint8).reshape(-1)])


def gpu_roundtrip(codec, O, x, H, W, log2_k, offset=0, predict=True):
    """offset: place the layer that many bytes into a device buffer (a layer
    that is not 16-byte aligned takes the library's narrow-load histogram);
    predict: the exponents as left differences (the library's default)."""
    if offset:
        buf = torch.zeros(x.size + offset, dtype=torch.uint8, device="cuda")
        buf[offset:] = torch.from_numpy(x).cuda()
        d = buf[offset:]
    else:
        d = torch.from_numpy(x).cuda()
    codec.set_ent_predict(predict)
    try:
        code = codec.ent_encode(d, H, W, log2_k)
    finally:
        codec.set_ent_predict(True)
    got = code.cpu().numpy().tobytes()
    ref = O.ent_encode(x, H, W, log2_k, predict=predict)
    assert len(got) == len(ref), (len(got), len(ref))
    assert got == ref
    status = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    back = codec.ent_decode(code, H, W, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(back, d)
    return code


CASES = [
    (1, 1, 4, 3.0), (7, 9, 4, 3.0), (1, 1025, 4, 3.0), (33, 257, 5, 0.5), (64, 65, 8, 20.0),
    (97, 131, 4, 3.0), (300, 401, 8, 3.0), (512, 384, 12, 6.0), (1081, 1919, 8, 3.0),
]


@pytest.mark.parametrize("H,W,log2_k,spread", CASES)
def test_stream_equals_oracle_and_decodes(codec, O, H, W, log2_k, spread):
    _say("entropy case", H, W, log2_k, spread)
    gpu_roundtrip(codec, O, make_layer(H, W, H * 7 + W, spread), H, W, log2_k)


def test_wide_and_degenerate_planes(codec, O):
    _say("entropy: wide / outliers / constant planes")
    gpu_roundtrip(codec, O, make_layer(200, 300, 1, spread=200.0, e_lo=0, e_hi=256), 200, 300, 6)
    gpu_roundtrip(codec, O, make_layer(200, 300, 2, outlier=0.01), 200, 300, 8)
    H, W = 150, 170
    r = np.full((3, H, W), -255, np.int16)
    r[1] = 255
    r[2, ::7, ::3] = 0
    x = np.concatenate([r.reshape(-1).view(np.uint8), np.full(H * W, 255, np.uint8)])
    gpu_roundtrip(codec, O, x, H, W, 4)


@pytest.mark.parametrize("H,W,offset", [(3, 5, 0), (97, 131, 2), (300, 401, 6), (17, 1, 0), (4, 4, 0)])
def test_histogram_paths(codec, O, H, W, offset):
    """Both histogram kernels: 16-byte loads (aligned layer, at least 16 pixels)
    and 2-byte loads (any other), with residual and exponent tails."""
    _say("entropy histogram path", H, W, offset)
    gpu_roundtrip(codec, O, make_layer(H, W, 31 * H + W, spread=5.0, e_lo=0, e_hi=256), H, W, 4, offset=offset)


def smooth_layer(H, W, seed):
    """Residuals as make_layer's, exponents of the synthetic image generator
    (smooth, with the runs and steps the differences code)."""
    x = make_layer(H, W, seed)
    x[6 * H * W:] = synth.generate(H, W, 4.0, seed=seed, spec_frac=0.05)[..., 3].reshape(-1)
    return x


@pytest.mark.parametrize("H,W", [(1, 1), (1, 17), (17, 1), (3, 5), (5, 4097), (97, 131), (2, 70000), (700, 1510)])
@pytest.mark.parametrize("predict", [True, False])
def test_exponent_prediction(codec, O, H, W, predict):
    """Exponents as left differences and as they are: the stream equals the
    oracle's and decodes exactly; rows inside one lane (W = 1, 5), rows across
    tiles (70,000 wide) and more tiles than one carry chunk (700 x 1510)."""
    _say("entropy prediction", H, W, predict)
    gpu_roundtrip(codec, O, smooth_layer(H, W, H + 3 * W), H, W, 4, predict=predict)
    if H * W >= 16:
        gpu_roundtrip(codec, O, smooth_layer(H, W, H + 5 * W), H, W, 8, offset=2, predict=predict)


def test_prediction_switch(codec, rdl_mod):
    assert codec._L.rdl_set_ent_predict(codec._h, 2) == rdl_mod.RDL_EINVAL
    assert codec._L.rdl_set_ent_predict(None, 1) == rdl_mod.RDL_EINVAL


def test_workspace_reuse_across_sizes(codec, O):
    """Calls of growing and shrinking sizes on one context: each stream equals
    the oracle's (the histograms are cleared between calls)."""
    for H, W, k in [(50, 60, 4), (700, 900, 8), (50, 60, 4), (31, 33, 12)]:
        _say("entropy reuse", H, W, k)
        gpu_roundtrip(codec, O, make_layer(H, W, H + W + k), H, W, k)


def test_encoder_layer_3840x2160(codec, O):
    """The GPU encoder's layer of the 3840 x 2160 image (sigma_L = 4, 5 %
    speculars, q = 75), coded at the default group size and at the largest."""
    sp = synth.image_3840x2160()
    x = sp.make()
    H, W = sp.H, sp.W
    d = torch.from_numpy(x).cuda()
    sdr, hdr, resid = codec.encode_enh(d, sp.q)
    torch.cuda.synchronize()
    layer = resid.cpu().numpy()
    for k in (8, 12):
        _say("entropy 3840x2160 log2_k", k)
        code = gpu_roundtrip(codec, O, layer, H, W, k)
        hist = codec.resid_hist(resid, H, W).cpu().numpy()
        h0 = sum(float(-(h[h > 0] / h.sum() * np.log2(h[h > 0] / h.sum())).sum()) for h in hist)
        G = -(-H * W // (64 << k))
        coded_planes = 8 * (code.numel() - 4136 - 32 * G)  # all four planes
        assert coded_planes < (h0 + 8.0) * H * W  # residual H0 + at most 8 bits for E and overheads


def test_out_of_range_residual_gives_no_stream(codec, rdl_mod):
    H, W = 40, 50
    x = make_layer(H, W, 5)
    r = x[:6 * H * W].view(np.int16)
    r[1234] = 300
    d = torch.from_numpy(x).cuda()
    out = torch.empty(codec.ent_bound(H, W, 8), dtype=torch.uint8, device="cuda")
    n = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    codec.ent_encode_into(d, H, W, out, n, 8)
    torch.cuda.synchronize()
    assert int(n.item()) == 0
    assert int.from_bytes(out[:4].cpu().numpy().tobytes(), "little") == 0
    with pytest.raises(rdl_mod.RdlError):
        codec.ent_encode(d, H, W, 8)
    # a valid layer afterwards still codes (the flags are per call)
    r[1234] = 0
    d = torch.from_numpy(x).cuda()
    codec.ent_encode(d, H, W, 8)


def test_corrupt_streams_are_reported(codec, O, rdl_mod):
    H, W = 90, 110
    x = make_layer(H, W, 9)
    code = gpu_roundtrip(codec, O, x, H, W, 4)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    # host header check: wrong size, broken frequency sum
    with pytest.raises(rdl_mod.RdlError):
        codec.ent_decode(code, H, W + 1)
    bad = code.clone()
    bad[40 + 2 * 600] ^= 1
    with pytest.raises(rdl_mod.RdlError):
        codec.ent_decode(bad, H, W)
    bad = code.clone()
    bad[28] = 2  # unknown flag
    with pytest.raises(rdl_mod.RdlError):
        codec.ent_decode(bad, H, W)
    # device checks: a group offset one word late, a truncated group
    G = -(-H * W // (64 << 4))
    bad = code.clone()
    bad[4136 + 8] += 1
    codec.ent_decode(bad, H, W, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == rdl_mod.RDL_ECORRUPT
    bad = code.clone()
    bad[4136 + 8 * (4 * G - 1):4136 + 8 * 4 * G] = torch.tensor(
        np.frombuffer(np.uint64(1 << 40).tobytes(), np.uint8).copy(), device="cuda")
    status.zero_()
    codec.ent_decode(bad, H, W, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == rdl_mod.RDL_ECORRUPT
    # the intact stream still decodes with status OK
    codec.ent_decode(code, H, W, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0


def test_max_size_layer(codec, O):
    """4321 x 7679 (33 MP, ragged): the stream equals the oracle's at the
    smallest and the largest group size."""
    H, W = 4321, 7679
    x = make_layer(H, W, 4321, spread=4.0, e_lo=100, e_hi=160, outlier=0.001)
    for k in (4, 12):
        _say("entropy max size log2_k", k)
        gpu_roundtrip(codec, O, x, H, W, k)
