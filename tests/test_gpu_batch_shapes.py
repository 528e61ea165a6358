"""GPU parity of a mixed batch at the batch workloads' real shapes: one image
above 4 Mpx (so the launch's fit takes the 16-wave x 8-row workgroups of the
large size classes) and smaller ones of ragged sizes, encoded in one call,
in direct and in graph launch mode, with the plain SLR estimator and with the
learned estimator plus per-region SLR fallback (the library's trained model).
Launch shapes are first tuned on the largest image, as the benchmark does.
Every output of every image (S, the residual and exponent planes, the
header's coefficients, presence flags, key fields and region flags) is
compared with the oracle, and the batch is decoded losslessly."""
import os

import numpy as np
import pytest
import torch

from paper_2309_11072_amd import synth

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2309_11072_amd",
                     "mlp_model.bin")
# (H, W, sigma_L, q, seed): 2400 x 1800 = 4.32 Mpx, then 0.3-0.8 Mpx and
# two small ragged images
SPECS = [(1800, 2400, 4.0, 75, 8101), (480, 640, 1.5, 50, 8102), (751, 1001, 3.0, 95, 8103),
         (129, 200, 2.5, 30, 8104), (37, 1031, 5.0, 98, 8105)]


@pytest.fixture(scope="module")
def rdl_mod():
    from paper_2309_11072_amd import rdl
    return rdl


@pytest.fixture(scope="module")
def codec(rdl_mod):
    c = rdl_mod.Codec(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def images():
    return [synth.generate(H, W, s, seed=sd, spec_frac=0.05) for H, W, s, q, sd in SPECS]


def _say(*a):
    print(*a, flush=True)


def _check(rdl_mod, x, q, out, ref, learned):
    sdr, hdr, resid = out
    h = rdl_mod.header_from_bytes(hdr)
    assert np.array_equal(sdr.cpu().numpy(), ref["sdr"]), "S"
    assert np.array_equal(resid.cpu().numpy(), ref["resid"]), "residual and exponent planes"
    assert np.array_equal(h["a_q"], ref["a_q"]) and np.array_equal(h["b_q"], ref["b_q"]), "coefficients"
    assert np.array_equal(h["present"], ref["present"]), "present"
    assert int(h["k_img"]) == ref["k_img"] and int(h["q"]) == q
    if learned:
        assert np.array_equal(h["flag"], ref["flag"]), "region flags"
        assert int(h["estimator"]) == 1
    else:
        assert not h["flag"].any() and int(h["estimator"]) == 0
        assert int(h["lambda_sum"]) == ref["lambda_sum"] and int(h["n_lit"]) == ref["n_lit"]


@pytest.mark.parametrize("learned", [False, True], ids=["slr", "learned"])
def test_mixed_batch_direct_and_graph_match_oracle(codec, rdl_mod, O, images, learned):
    blob = open(MODEL, "rb").read()
    devs = [torch.from_numpy(x).cuda() for x in images]
    H0, W0, _, q0, _ = SPECS[0]
    _say("autotune on", H0, W0)
    codec.set_estimator(0)
    codec.autotune(devs[0], q0, codec.alloc_outputs(H0, W0), reps=2)
    refs = []
    for x, (H, W, s, q, sd) in zip(images, SPECS):
        _say("oracle", "learned" if learned else "slr", H, W)
        refs.append(O.encode_learned(x, q, blob) if learned else O.encode_enh(x, q))
    if learned:
        codec.set_model(blob)
        codec.set_estimator(1)
    try:
        outs = [codec.alloc_outputs(H, W) for H, W, s, q, sd in SPECS]
        items = [(d, sp[3]) + tuple(o) for d, sp, o in zip(devs, SPECS, outs)]
        for graph in (False, True):
            codec.set_launch_mode(graph)
            # graph mode: the first call captures the plan's graph, the
            # later ones replay it
            for rep in range(3):
                _say("batch", "graph" if graph else "direct", "call", rep)
                for o in outs:
                    for t in o:
                        t.fill_(0xAA)
                codec.encode_batch(items)
                torch.cuda.synchronize()
                for x, sp, o, ref in zip(images, SPECS, outs, refs):
                    _check(rdl_mod, x, sp[3], o, ref, learned)
        # the batch decodes losslessly
        backs = [torch.empty_like(d) for d in devs]
        codec.decode_batch([(None, o[0], o[1], o[2], b, None) for o, b in zip(outs, backs)])
        torch.cuda.synchronize()
        for d, b in zip(devs, backs):
            assert torch.equal(d, b)
    finally:
        codec.set_launch_mode(False)
        codec.set_estimator(0)


def test_learned_launch_of_2p25_pixels_matches_oracle(codec, rdl_mod, O, images):
    """A learned launch of at least 2^25 pixels, where the estimator's and the
    learned decoder's workgroups take 12 tiles of 16 rows instead of 8: one
    5800 x 5800 image (33.6 Mpx, drawn on the GPU) plus the four smaller
    images above, in one call.  The four small images' outputs are compared
    with the oracle (the large one would take the oracle about a minute), and
    the whole batch, the large image included, decodes losslessly in one
    call (the decoder's launch is as large)."""
    blob = open(MODEL, "rb").read()
    big = synth.generate_torch(5800, 5800, 3.0, seed=8110, spec_frac=0.05)
    small = [(torch.from_numpy(x).cuda(), sp) for x, sp in zip(images[1:], SPECS[1:])]
    assert 5800 * 5800 + sum(sp[0] * sp[1] for _, sp in small) >= 1 << 25
    refs = []
    for x, sp in zip(images[1:], SPECS[1:]):
        _say("oracle learned", sp[0], sp[1])
        refs.append(O.encode_learned(x, sp[3], blob))
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        outs = [codec.alloc_outputs(5800, 5800)] + [codec.alloc_outputs(sp[0], sp[1]) for _, sp in small]
        items = [(big, 75) + tuple(outs[0])] + [(d, sp[3]) + tuple(o) for (d, sp), o in zip(small, outs[1:])]
        for rep in range(2):
            _say("large learned launch, call", rep)
            for o in outs:
                for t in o:
                    t.fill_(0xAA)
            codec.encode_batch(items)
            torch.cuda.synchronize()
            for (d, sp), o, x, ref in zip(small, outs[1:], images[1:], refs):
                _check(rdl_mod, x, sp[3], o, ref, True)
        assert rdl_mod.header_from_bytes(outs[0][1])["flag"].any(), "the large image has learned regions"
        devs = [big] + [d for d, _ in small]
        backs = [torch.empty_like(d) for d in devs]
        codec.decode_batch([(None, o[0], o[1], o[2], b, None) for o, b in zip(outs, backs)])
        torch.cuda.synchronize()
        for d, b in zip(devs, backs):
            assert torch.equal(d, b)
    finally:
        codec.set_estimator(0)
