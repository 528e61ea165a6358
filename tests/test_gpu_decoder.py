"""GPU decoders against the oracle: the base layer rebuilt from its quantised
coefficients must equal the encoder's S byte for byte, and the batched
decoder (coefficients -> S -> RGBE, or S -> RGBE) must return every image
exactly, plain and learned, with per-image status."""
import os

import numpy as np
import pytest
import torch

from paper_2309_11072_amd import synth

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2309_11072_amd",
                     "mlp_model.bin")


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


def coefficients(codec, d, q):
    """S and the quantised coefficients of image d (stage kernels of the encoder)."""
    ks = codec.stage_keystat(d)
    sdr, _, dct = codec.stage_tmo_base(d, q, ks, want_dct=True)
    return sdr, dct


@pytest.mark.parametrize("H,W,q", [(1, 1, 75), (7, 9, 30), (61, 83, 75), (256, 384, 95), (1081, 1921, 50), (33, 2050, 1)])
def test_base_decode_equals_encoder_and_oracle(codec, O, H, W, q):
    _say("base decode", H, W, q)
    x = synth.generate(H, W, 3.5, seed=H * 31 + W, spec_frac=0.05)
    d = torch.from_numpy(x).cuda()
    sdr, hdr, resid = codec.encode_enh(d, q)
    s_ref, dct = coefficients(codec, d, q)
    status = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    out = torch.full((H, W, 3), 0xAA, dtype=torch.uint8, device="cuda")
    codec.base_decode(dct, hdr, H, W, out=out, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(s_ref, sdr)
    assert torch.equal(out, sdr), "base decode differs from the encoder's S"
    assert np.array_equal(out.cpu().numpy(), O.base_decode(dct.cpu().numpy(), H, W, q))


def _items(codec, specs, with_dct):
    imgs, items, keep = [], [], []
    for k, s in enumerate(specs):
        d = s.make_torch()
        sdr, hdr, resid = codec.alloc_outputs(s.H, s.W)
        imgs.append(d)
        items.append((d, s.q, sdr, hdr, resid))
    codec.encode_batch(items)
    torch.cuda.synchronize()
    dec = []
    for k, (d, q, sdr, hdr, resid) in enumerate(items):
        H, W = d.shape[:2]
        out = torch.full((H, W, 4), 0x55, dtype=torch.uint8, device="cuda")
        st = torch.full((1,), 77, dtype=torch.int32, device="cuda")
        if with_dct(k):
            s_ref, dct = coefficients(codec, d, q)
            assert torch.equal(s_ref, sdr)
            s_in = torch.full_like(sdr, 0xAA)  # written by the batch decoder
            dec.append((dct, s_in, hdr, resid, out, st))
        else:
            dec.append((None, sdr, hdr, resid, out, st))
        keep.append(sdr)
    return imgs, dec, keep


def _specs(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(1, 1), (7, 9), (61, 83), (480, 640), (1080, 1920), (33, 1025), (517, 389), (8, 8)]
    out = []
    for k in range(n):
        H, W = sizes[k % len(sizes)]
        out.append(synth.ImageSpec(H, W, float(rng.uniform(1.5, 4.5)), int(rng.integers(30, 99)), 9000 + seed + k, 0.05))
    return out


def test_decode_batch_plain(codec):
    specs = _specs(12, 1)
    imgs, dec, keep = _items(codec, specs, lambda k: k % 2 == 0)
    _say("decode batch, plain:", len(dec))
    codec.decode_batch(dec)
    torch.cuda.synchronize()
    for im, (dct, s, hdr, resid, out, st), sdr in zip(imgs, dec, keep):
        assert int(st.item()) == 0
        assert torch.equal(s, sdr), "S rebuilt from the coefficients"
        assert torch.equal(out, im), "lossless"


def test_decode_batch_learned(codec, rdl_mod):
    blob = open(MODEL, "rb").read()
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        specs = _specs(8, 2)
        imgs, dec, keep = _items(codec, specs, lambda k: k % 3 != 1)
        flagged = sum(int(rdl_mod.header_from_bytes(it[2])["flag"].sum()) for it in dec)
        _say("decode batch, learned: regions flagged", flagged)
        assert flagged > 0
        codec.decode_batch(dec)
        torch.cuda.synchronize()
        for im, (dct, s, hdr, resid, out, st) in zip(imgs, dec):
            assert int(st.item()) == 0
            assert torch.equal(out, im)
    finally:
        codec.set_estimator(0)


def test_decode_batch_reports_corrupt_headers_per_image(codec, rdl_mod):
    specs = _specs(4, 3)
    imgs, dec, keep = _items(codec, specs, lambda k: True)
    hdr1 = dec[1][2]
    bad = hdr1.clone()
    q_off = rdl_mod.HEADER_DTYPE.fields["q"][1]
    bad[q_off:q_off + 4] = 0  # quality 0
    dec[1] = (dec[1][0], dec[1][1], bad, dec[1][3], dec[1][4], dec[1][5])
    codec.decode_batch(dec)
    torch.cuda.synchronize()
    sts = [int(it[5].item()) for it in dec]
    assert sts[1] == rdl_mod.RDL_ECORRUPT
    for k in (0, 2, 3):
        assert sts[k] == 0 and torch.equal(dec[k][4], imgs[k])


def test_decode_enh_sets_status_ok(codec):
    x = synth.generate(40, 50, 3.0, seed=4, spec_frac=0.05)
    d = torch.from_numpy(x).cuda()
    sdr, hdr, resid = codec.encode_enh(d, 75)
    st = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    back = codec.decode_enh(sdr, hdr, resid, 40, 50, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and torch.equal(back, d)
