"""GPU parity of the learned estimator path: int8 MLP inference on MFMA, the
per-region entropy-cost selection and the learned encoder/decoder equal the
CPU oracle bit for bit, on seeded random models (test inputs), over sizes with
ragged edges and the degenerate cases."""
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _say(*a):
    print(*a, flush=True)


CASES = [("1x1", (1, 1), 2.0, 75, 11), ("7x9", (7, 9), 3.0, 50, 12), ("64x64", (64, 64), 2.5, 90, 13),
         ("65x130", (65, 130), 4.0, 75, 14), ("100x77", (100, 77), 1.5, 30, 15), ("200x301", (200, 301), 3.5, 85, 16)]


@pytest.mark.parametrize("name,shape,sig,q,ms", CASES, ids=[c[0] for c in CASES])
def test_learned_encode_decode_match_oracle(codec, rdl_mod, O, name, shape, sig, q, ms):
    H, W = shape
    # the models take every requantisation path: general multipliers, powers
    # of two with per-neuron shifts, and powers of two with paired shifts
    rq = ("general", "pow2", "pair")[ms % 3]
    _say("learned", name, q, "model", ms, rq)
    x = synth.generate(H, W, sig, seed=700 + ms, spec_frac=0.05)
    blob = synth.random_model(ms, rq=rq)
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        d = _dev(x)
        out = codec.alloc_outputs(H, W)
        for t in out:
            t.fill_(0xAA)
        for _ in range(3):  # the first call builds the plan, the later ones reuse it
            sdr, hdr, resid = codec.encode_enh(d, q, out=out)
        torch.cuda.synchronize()
        ref = O.encode_learned(x, q, blob)
        h = rdl_mod.header_from_bytes(hdr)
        assert np.array_equal(sdr.cpu().numpy(), ref["sdr"])
        assert np.array_equal(h["flag"], ref["flag"]), "region selection"
        assert np.array_equal(resid.cpu().numpy(), ref["resid"]), "residuals"
        assert h["estimator"] == 1 and h["model_hash"] == int(np.frombuffer(blob[8:16], "<u8")[0])
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        back = codec.decode_enh(sdr, hdr, resid, H, W, status=status)
        assert np.array_equal(back.cpu().numpy(), x), "GPU round trip"
        assert int(status.item()) == 0
        # the GPU decoder on the oracle's stream (same header bytes)
        back2 = codec.decode_enh(_dev(ref["sdr"]), hdr, _dev(ref["resid"]), H, W)
        assert np.array_equal(back2.cpu().numpy(), x)
    finally:
        codec.set_estimator(0)


def test_learned_random_words(codec, rdl_mod, O):
    rng = np.random.default_rng(41)
    x = rng.integers(0, 256, (29, 70, 4)).astype(np.uint8)
    blob = synth.random_model(41)
    _say("learned random words")
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        sdr, hdr, resid = codec.encode_enh(_dev(x), 60)
        ref = O.encode_learned(x, 60, blob)
        assert np.array_equal(resid.cpu().numpy(), ref["resid"])
        assert np.array_equal(rdl_mod.header_from_bytes(hdr)["flag"], ref["flag"])
        assert np.array_equal(codec.decode_enh(sdr, hdr, resid, 29, 70).cpu().numpy(), x)
    finally:
        codec.set_estimator(0)


@pytest.mark.parametrize("kind", ["general", "pow2", "pair"])
def test_learned_batch_matches_oracle(codec, O, kind):
    specs = [(40, 90, 2.0, 55), (70, 33, 4.0, 90), (129, 66, 1.5, 30)]
    blob = synth.random_model(51, rq=kind)
    _say("learned batch", kind)
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        xs = [synth.generate(H, W, s, seed=950 + k, spec_frac=0.05) for k, (H, W, s, q) in enumerate(specs)]
        items = []
        for x, (H, W, s, q) in zip(xs, specs):
            items.append((_dev(x), q) + tuple(codec.alloc_outputs(H, W)))
        for rep in range(3):
            codec.encode_batch(items)
            torch.cuda.synchronize()
            for x, it, (H, W, s, q) in zip(xs, items, specs):
                ref = O.encode_learned(x, q, blob)
                assert np.array_equal(it[4].cpu().numpy(), ref["resid"]), (rep, H, W)
    finally:
        codec.set_estimator(0)


def test_model_validation_and_decoder_checks(codec, rdl_mod):
    from paper_2309_11072_amd import model_format
    _say("model validation")
    blob = bytearray(synth.random_model(61))
    bad = bytearray(blob)
    bad[100] ^= 1  # body changed, hash not
    with pytest.raises(rdl_mod.RdlError):
        codec.set_model(bytes(bad))
    p = model_format.unpack(bytes(blob))
    p["m1"][3] = 1 << 10  # beyond the multiplier limit
    with pytest.raises(rdl_mod.RdlError):
        codec.set_model(model_format.pack(p))
    p["m1"][3] = (1 << 10) - 1  # at it
    codec.set_model(model_format.pack(p))
    old = bytearray(blob)
    old[4] = 1  # the first format version (activations clamped at 127) is refused
    with pytest.raises(rdl_mod.RdlError):
        codec.set_model(bytes(old))
    codec.set_model(None)
    with pytest.raises(rdl_mod.RdlError):
        codec.set_estimator(1)
    # a learned stream decoded with another model is rejected
    x = synth.generate(30, 40, 3.0, seed=62)
    codec.set_model(bytes(blob))
    codec.set_estimator(1)
    sdr, hdr, resid = codec.encode_enh(_dev(x), 75)
    codec.set_estimator(0)
    codec.set_model(synth.random_model(63))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    codec.decode_enh(sdr, hdr, resid, 30, 40, status=status)
    assert int(status.item()) == rdl_mod.RDL_ECORRUPT
    codec.set_model(None)
    status.zero_()
    codec.decode_enh(sdr, hdr, resid, 30, 40, status=status)
    assert int(status.item()) == rdl_mod.RDL_ECORRUPT


def test_training_step_deterministic_and_learns(codec):
    """Two identical short trainings give identical parameters (the gradient
    reduction order is fixed); the loss falls; the quantised model encodes
    losslessly."""
    from paper_2309_11072_amd import train
    _say("training")
    specs = [synth.ImageSpec(256, 384, 4.0, 75, 4200, 0.05)]
    samples = train.make_samples(codec, specs, 60000, seed=1)
    log = []
    p1 = train.train(codec, samples, epochs=2, batch=4096, lr=3e-3, seed=3, log=log.append)
    p2 = train.train(codec, samples, epochs=2, batch=4096, lr=3e-3, seed=3, log=lambda s: None)
    assert np.array_equal(p1, p2)
    first = float(log[0].split("mse(M/256) ")[1].split()[0])
    last = float(log[-1].split("mse(M/256) ")[1].split()[0])
    assert last < 0.5 * first
    calib = samples[:20000].cpu().numpy()
    blob = train.quantise(p1, calib[:, :27].view(np.int8), calib[:, 27].astype(np.int64))
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        x = synth.generate(90, 120, 4.0, seed=4201, spec_frac=0.05)
        d = _dev(x)
        sdr, hdr, resid = codec.encode_enh(d, 75)
        assert torch.equal(codec.decode_enh(sdr, hdr, resid, 90, 120), d)
    finally:
        codec.set_estimator(0)


def test_learned_graph_mode_replays_match_oracle(codec, rdl_mod, O):
    """The learned encoder captured as a graph: every replay equals the oracle
    (its record cursors, histograms and flags are rebuilt or cleared each time)."""
    H, W, q, ms = 150, 222, 60, 21
    _say("learned graph mode", H, W)
    x = synth.generate(H, W, 3.0, seed=7021, spec_frac=0.05)
    blob = synth.random_model(ms)
    codec.set_model(blob)
    codec.set_estimator(1)
    codec.set_launch_mode(True)
    try:
        ref = O.encode_learned(x, q, blob)
        d = _dev(x)
        out = codec.alloc_outputs(H, W)
        for rep in range(3):
            for t in out:
                t.fill_(0xAA)
            sdr, hdr, resid = codec.encode_enh(d, q, out=out)
            torch.cuda.synchronize()
            h = rdl_mod.header_from_bytes(hdr)
            assert np.array_equal(h["flag"], ref["flag"]), rep
            assert np.array_equal(resid.cpu().numpy(), ref["resid"]), rep
            assert np.array_equal(sdr.cpu().numpy(), ref["sdr"]), rep
    finally:
        codec.set_launch_mode(False)
        codec.set_estimator(0)


def test_learned_plan_eviction_reuses_buffers(codec, rdl_mod, O):
    """Twelve image sets, more than the context keeps plans for, in an order
    whose sizes grow and shrink: every new plan past the eighth takes over the
    evicted plan's buffers when they are large enough (else allocates), and
    each encode still equals the oracle, on the first pass and on the second
    (the evicted plans rebuilt), directly and through graphs."""
    sizes = [(20, 30), (60, 90), (15, 17), (90, 120), (33, 33), (120, 150), (9, 70), (70, 9),
             (100, 140), (8, 8), (130, 160), (40, 41)]
    blob = synth.random_model(71, rq="pair")
    _say("learned plan eviction: 12 sets, twice")
    codec.set_model(blob)
    codec.set_estimator(1)
    try:
        xs = [synth.generate(H, W, 3.0, seed=1200 + k, spec_frac=0.05) for k, (H, W) in enumerate(sizes)]
        qs = [40 + 5 * k for k in range(len(sizes))]
        refs = [O.encode_learned(x, q, blob) for x, q in zip(xs, qs)]
        devs = [_dev(x) for x in xs]
        outs = [codec.alloc_outputs(H, W) for H, W in sizes]
        for graph in (False, True):
            codec.set_launch_mode(graph)
            for k in list(range(len(sizes))) * 2:
                for t in outs[k]:
                    t.fill_(0xAA)
                sdr, hdr, resid = codec.encode_enh(devs[k], qs[k], out=outs[k])
                torch.cuda.synchronize()
                assert np.array_equal(resid.cpu().numpy(), refs[k]["resid"]), (graph, k)
                assert np.array_equal(rdl_mod.header_from_bytes(hdr)["flag"], refs[k]["flag"]), (graph, k)
    finally:
        codec.set_launch_mode(False)
        codec.set_estimator(0)
