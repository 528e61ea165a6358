"""Seeded randomized parity sweep: image sizes from 1 to 300 pixels on either
side (ragged against every tile and strip), qualities 1 to 100, exponent
spreads, specular fractions and random learned models; every output of the
GPU encoder equals the oracle's and every stream decodes losslessly."""
import numpy as np
import pytest
import torch

from paper_2309_11072_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rdl_mod():
    from paper_2309_11072_amd import rdl
    return rdl


@pytest.fixture(scope="module")
def codec(rdl_mod):
    c = rdl_mod.Codec(0)
    yield c
    c.close()


def _cases(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        H, W = (int(v) for v in rng.integers(1, 301, 2))
        out.append((H, W, float(rng.uniform(0.5, 6.0)), int(rng.integers(1, 101)),
                    float(rng.choice([0.0, 0.01, 0.1])), 9000 + k))
    return out


@pytest.mark.parametrize("learned", [False, True], ids=["slr", "learned"])
def test_random_sweep_matches_oracle(codec, rdl_mod, O, learned):
    for k, (H, W, sig, q, spec, seed) in enumerate(_cases(16, 77 + learned)):
        print("sweep", "learned" if learned else "slr", k, H, W, sig, q, spec, flush=True)
        x = synth.generate(H, W, sig, seed=seed, spec_frac=spec)
        d = torch.from_numpy(x).cuda()
        out = codec.alloc_outputs(H, W)
        for t in out:
            t.fill_(0xAA)
        if learned:
            blob = synth.random_model(seed, rq=("general", "pow2", "pair")[seed % 3])
            codec.set_model(blob)
            codec.set_estimator(1)
        try:
            sdr, hdr, resid = codec.encode_enh(d, q, out=out)
            torch.cuda.synchronize()
            ref = O.encode_learned(x, q, blob) if learned else O.encode_enh(x, q)
            h = rdl_mod.header_from_bytes(hdr)
            assert np.array_equal(sdr.cpu().numpy(), ref["sdr"]), k
            assert np.array_equal(resid.cpu().numpy(), ref["resid"]), k
            assert np.array_equal(h["a_q"], ref["a_q"]) and np.array_equal(h["b_q"], ref["b_q"]), k
            if learned:
                assert np.array_equal(h["flag"], ref["flag"]), k
            back = codec.decode_enh(sdr, hdr, resid, H, W)
            assert torch.equal(back, d), k
        finally:
            codec.set_estimator(0)
