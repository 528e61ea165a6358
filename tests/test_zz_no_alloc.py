"""GPU check of the allocation-free batched encoder (rdl_encode_batch_noalloc,
for callers that cannot allocate device memory): through the C ABI, its
outputs equal rdl_encode_batch's byte for byte on two calls in a row, the
second with fewer and smaller images, so that the static scratch it shares
between calls must have been cleared.  Outputs are poisoned before every
call.  The three SLR-family estimator settings are covered (SLR per region,
SLR without the Gaussian filter, one line per channel).  Its limits (image
count, learned estimator) are rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

from paper_2309_11072_amd import synth

pytestmark = pytest.mark.gpu

# (H, W, sigma_L, q, seed): the first call has a 4.3 Mpx image (the fit's
# large workgroups) and ragged smaller ones; the second call is smaller.
FIRST = [(1800, 2400, 4.0, 75, 9101), (480, 640, 1.5, 50, 9102), (131, 203, 3.0, 95, 9103)]
SECOND = [(61, 83, 2.5, 30, 9104), (17, 1029, 5.0, 98, 9105)]


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


def _items(codec, specs, poison):
    items = []
    for H, W, s, q, sd in specs:
        x = torch.from_numpy(synth.generate(H, W, s, seed=sd, spec_frac=0.05)).cuda()
        sdr, hdr, resid = codec.alloc_outputs(H, W)
        for t in (sdr, hdr, resid):
            t.fill_(poison)
        items.append((x, q, sdr, hdr, resid))
    return items


def _same(a, b):
    for (xa, qa, *oa), (xb, qb, *ob) in zip(a, b):
        for ta, tb, name in zip(oa, ob, ("S", "header", "residual and exponent planes")):
            assert torch.equal(ta, tb), name


@pytest.mark.parametrize("mode", ["slr", "slr_no_gf", "global_line"])
def test_noalloc_equals_batch_encoder_on_two_calls(rdl_mod, codec, mode):
    est, gf = {"slr": (0, True), "slr_no_gf": (0, False), "global_line": (2, True)}[mode]
    codec.set_estimator(est)
    codec.set_gf(gf)
    try:
        for call, specs in enumerate((FIRST, SECOND)):
            _say("noalloc %s call %d: %s" % (mode, call, [(H, W, q) for H, W, _, q, _ in specs]))
            ref = _items(codec, specs, 0x55)
            got = [(x, q, *(torch.full_like(t, 0xAA) for t in o)) for x, q, *o in ref]
            codec.encode_batch(ref)
            codec.encode_batch_noalloc(got)
            torch.cuda.synchronize()
            _same(got, ref)
            for x, q, sdr, hdr, resid in got:
                H, W = int(x.shape[0]), int(x.shape[1])
                assert torch.equal(codec.decode_enh(sdr, hdr, resid, H, W), x), "lossless"
    finally:
        codec.set_estimator(0)
        codec.set_gf(True)


def test_noalloc_single_image_repeated(rdl_mod, codec):
    """The same image twice in a row: the second call starts from the first
    call's scratch contents and must still give the same bytes."""
    items = _items(codec, [(255, 257, 3.0, 75, 9106)], 0x55)
    ref = [(x, q, *(torch.full_like(t, 0x11) for t in o)) for x, q, *o in items]
    codec.encode_batch(ref)
    for rep in range(2):
        got = [(x, q, *(torch.full_like(t, 0xAA) for t in o)) for x, q, *o in items]
        codec.encode_batch_noalloc(got)
        torch.cuda.synchronize()
        _same(got, ref)


def test_noalloc_rejects_its_limits(rdl_mod, codec):
    n = rdl_mod.NOALLOC_MAX_IMAGES + 1
    items = _items(codec, [(8, 8, 2.0, 75, 9200 + k) for k in range(n)], 0)
    with pytest.raises(rdl_mod.RdlError) as e:
        codec.encode_batch_noalloc(items)
    assert e.value.code == rdl_mod.RDL_ENOMEM and str(rdl_mod.NOALLOC_MAX_IMAGES) in str(e.value)
    codec.encode_batch_noalloc(items[:-1])  # exactly the limit is accepted
    torch.cuda.synchronize()
    for x, q, sdr, hdr, resid in items[:-1]:
        assert torch.equal(codec.decode_enh(sdr, hdr, resid, 8, 8), x)
    blob = open(__import__("os").path.join(__import__("os").path.dirname(rdl_mod.__file__), "mlp_model.bin"),
                "rb").read()
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        with pytest.raises(rdl_mod.RdlError) as e:
            codec.encode_batch_noalloc(items[:1])
        assert e.value.code == rdl_mod.RDL_EUNSUPPORTED
    finally:
        codec.set_estimator(0)
