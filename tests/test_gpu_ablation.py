"""GPU ablation encoders (one line per channel, no estimator, the Gaussian
filter off) against the oracle, byte for byte, and their decoding."""
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


@pytest.fixture
def mode(codec):
    def set_mode(est, gf):
        codec.set_estimator(est)
        codec.set_gf(gf)
    yield set_mode
    codec.set_estimator(0)
    codec.set_gf(True)


@pytest.mark.parametrize("est", [0, 2, 3])
@pytest.mark.parametrize("gf", [True, False])
@pytest.mark.parametrize("H,W,q", [(61, 83, 75), (217, 301, 40), (1080, 1921, 90)])
def test_mode_equals_oracle(codec, O, rdl_mod, mode, est, gf, H, W, q):
    _say("ablation", est, gf, H, W, q)
    x = synth.generate(H, W, 3.5, seed=H + W + est, spec_frac=0.05)
    mode(est, gf)
    d = torch.from_numpy(x).cuda()
    sdr, hdr, resid = codec.encode_enh(d, q)
    torch.cuda.synchronize()
    ref = O.encode_mode(x, q, est, gf)
    h = rdl_mod.header_from_bytes(hdr)
    assert int(h["estimator"]) == est | (0 if gf else rdl_mod.EST_GF_OFF)
    assert np.array_equal(sdr.cpu().numpy(), ref["sdr"])
    assert np.array_equal(h["a_q"], ref["a_q"]) and np.array_equal(h["b_q"], ref["b_q"])
    assert np.array_equal(h["present"], ref["present"])
    assert np.array_equal(resid.cpu().numpy(), ref["resid"])
    st = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    back = codec.decode_enh(sdr, hdr, resid, H, W, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and torch.equal(back, d)


def test_mixed_modes_decode_in_one_batch(codec, mode):
    """Headers of every mode decode together (the filter switch is per image)."""
    items, imgs = [], []
    for k, (est, gf) in enumerate([(0, True), (2, False), (3, False), (0, False), (2, True), (3, True)]):
        mode(est, gf)
        x = synth.generate(47 + 9 * k, 53 + 4 * k, 3.0, seed=70 + k, spec_frac=0.05)
        d = torch.from_numpy(x).cuda()
        sdr, hdr, resid = codec.encode_enh(d, 60)
        out = torch.empty_like(d)
        st = torch.full((1,), 77, dtype=torch.int32, device="cuda")
        items.append((None, sdr.clone(), hdr.clone(), resid.clone(), out, st))
        imgs.append(d)
    mode(0, True)
    codec.decode_batch(items)
    torch.cuda.synchronize()
    for d, it in zip(imgs, items):
        assert int(it[5].item()) == 0 and torch.equal(it[4], d)


def test_mode_arguments(codec, rdl_mod, mode):
    with pytest.raises(rdl_mod.RdlError):
        codec.set_estimator(4)
    assert codec._L.rdl_set_gf(codec._h, 2) == rdl_mod.RDL_EINVAL
    # the learned estimator needs the filter
    import os
    blob = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2309_11072_amd",
                             "mlp_model.bin"), "rb").read()
    codec.set_model(blob)
    try:
        mode(1, False)
        d = torch.from_numpy(synth.generate(16, 16, 3.0, seed=1)).cuda()
        with pytest.raises(rdl_mod.RdlError) as ei:
            codec.encode_enh(d, 75)
        assert ei.value.code == rdl_mod.RDL_EUNSUPPORTED
    finally:
        codec.set_estimator(0)
        codec.set_model(None)
