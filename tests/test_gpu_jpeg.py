"""GPU JPEG file of the base layer against the oracle's writer, byte for
byte, and read back by an independent decoder (libjpeg through Pillow)."""
import io

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


def coefficients(codec, H, W, q, seed):
    x = synth.generate(H, W, 3.5, seed=seed, spec_frac=0.05)
    d = torch.from_numpy(x).cuda()
    ks = codec.stage_keystat(d)
    sdr, _, dct = codec.stage_tmo_base(d, q, ks, want_dct=True)
    return sdr, dct


def check(codec, O, H, W, q, seed, offset=0):
    sdr, dct = coefficients(codec, H, W, q, seed)
    if offset:
        buf = torch.zeros(dct.numel() + offset // 2, dtype=torch.int16, device="cuda")
        buf[offset // 2:] = dct.reshape(-1)
        dct = buf[offset // 2:].reshape(dct.shape)
    jp = codec.jpeg_encode(dct, H, W, q).cpu().numpy().tobytes()
    ref = O.jpeg_write(dct.cpu().numpy(), H, W, q)
    assert len(jp) == len(ref), (len(jp), len(ref))
    assert jp == ref
    PIL = pytest.importorskip("PIL.Image")
    im = PIL.open(io.BytesIO(jp))
    im.load()
    assert im.size == (W, H)
    d = np.abs(np.asarray(im.convert("RGB")).astype(int) - sdr.cpu().numpy().astype(int))
    assert d.max() <= 3 and d.mean() <= 0.5
    return len(jp)


@pytest.mark.parametrize("H,W,q", [(1, 1, 75), (7, 9, 50), (8, 8, 100), (61, 83, 90), (217, 301, 1),
                                   (256, 384, 100), (1081, 1921, 75)])
def test_file_equals_oracle(codec, O, H, W, q):
    _say("jpeg", H, W, q)
    check(codec, O, H, W, q, H + 3 * W)


def test_unaligned_coefficients_and_reuse(codec, O):
    for H, W, q, off in [(97, 131, 60, 2), (480, 640, 95, 0), (33, 65, 20, 6), (2, 2, 100, 0)]:
        _say("jpeg reuse / alignment", H, W, q, off)
        check(codec, O, H, W, q, H * W + q, offset=off)


def test_full_size_3840x2160(codec, O):
    sp = synth.image_3840x2160()
    _say("jpeg 3840x2160")
    n = check(codec, O, sp.H, sp.W, sp.q, sp.seed)
    _say("bytes", n, "bits/px %.3f" % (8 * n / (sp.H * sp.W)))


def test_batched_encoder_writes_the_coefficients(codec, O):
    """rdl_image.dct: the batched encoder also writes the quantised
    coefficients, equal to the stage kernel's, and leaves S and the layer
    unchanged; encode_files returns the JPEG file and the coded layer."""
    specs = [(61, 83, 75), (217, 301, 40), (8, 8, 95), (480, 641, 60)]
    items, ref = [], []
    for k, (H, W, q) in enumerate(specs):
        x = synth.generate(H, W, 3.5, seed=600 + k, spec_frac=0.05)
        d = torch.from_numpy(x).cuda()
        sdr, hdr, resid = codec.alloc_outputs(H, W)
        dct = torch.full((3, (H + 7) // 8 * 8, (W + 7) // 8 * 8), 12345, dtype=torch.int16, device="cuda")
        items.append((d, q, sdr, hdr, resid, dct))
        s2, h2, r2 = codec.encode_enh(d, q)
        ks = codec.stage_keystat(d)
        _, _, dct_ref = codec.stage_tmo_base(d, q, ks, want_dct=True)
        ref.append((s2.clone(), r2.clone(), dct_ref))
    codec.encode_batch(items)
    torch.cuda.synchronize()
    for (d, q, sdr, hdr, resid, dct), (s2, r2, dref) in zip(items, ref):
        assert torch.equal(dct, dref) and torch.equal(sdr, s2) and torch.equal(resid, r2)
    d, q = items[1][0], items[1][1]
    H, W = d.shape[:2]
    jpg, hdr, code = codec.encode_files(d, q)
    assert jpg.cpu().numpy().tobytes() == O.jpeg_write(items[1][5].cpu().numpy(), H, W, q)
    assert torch.equal(codec.ent_decode(code, H, W), items[1][4])


def test_large_counts_take_64_bit_keys(codec, O):
    """At q = 100 the chroma AC table of a 3840 x 2160 image counts more than
    2^22 symbols (one per nonzero AC coefficient at least), so the table
    builder keys its merges with 64-bit values instead of 32-bit ones; the
    file must still equal the oracle's."""
    H, W, q = 2160, 3840, 100
    _say("jpeg 64-bit keys", H, W, q)
    sdr, dct = coefficients(codec, H, W, q, 4242)
    d = dct.cpu().numpy()
    ac = d[1:].reshape(2, H // 8, 8, W // 8, 8).transpose(0, 1, 3, 2, 4).reshape(2, -1, 64)[:, :, 1:]
    assert int((ac != 0).sum()) >= 1 << 22
    jp = codec.jpeg_encode(dct, H, W, q).cpu().numpy().tobytes()
    assert jp == O.jpeg_write(d, H, W, q)


def test_coefficients_in_graph_mode(codec):
    """The coefficient output through a captured graph: two replays with the
    coefficients cleared in between (eager work between them) equal the
    direct launch's; a plan without coefficients stays a plan of its own."""
    H, W, q = 217, 301, 70
    d = torch.from_numpy(synth.generate(H, W, 3.5, seed=77, spec_frac=0.05)).cuda()
    shape = (3, (H + 7) // 8 * 8, (W + 7) // 8 * 8)
    sdr, hdr, resid = codec.alloc_outputs(H, W)
    want = torch.zeros(shape, dtype=torch.int16, device="cuda")
    codec.encode_batch([(d, q, sdr, hdr, resid, want)])
    torch.cuda.synchronize()
    codec.set_launch_mode(graph=True)
    try:
        dct = torch.zeros(shape, dtype=torch.int16, device="cuda")
        s2, h2, r2 = codec.alloc_outputs(H, W)
        for rep in range(2):
            dct.fill_(7)
            torch.cuda.synchronize()
            codec.encode_batch([(d, q, s2, h2, r2, dct)])
            torch.cuda.synchronize()
            assert torch.equal(dct, want), rep
            assert torch.equal(s2, sdr) and torch.equal(r2, resid)
        dct.fill_(7)
        codec.encode_batch([(d, q, s2, h2, r2)])  # no coefficients: its own plan
        torch.cuda.synchronize()
        assert bool((dct == 7).all()) and torch.equal(r2, resid)
    finally:
        codec.set_launch_mode(graph=False)
