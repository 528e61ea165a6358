#!/usr/bin/env python3
"""Throughput of the MI355X encoder for dual-layer lossless Radiance coding.

One step = one full encode (key statistic, tone map + JPEG-style base layer,
GF + regression sums, coefficient solve, residuals) of one 3840x2160 synthetic
RGBE image (sigma_L 4, 5% speculars at +10 stops, q 75) already resident in
HBM, one launch per stage kernel on the stream (the faster of the two launch
modes; the graph replay is timed beside it); outputs stay in HBM.  Prints one
JSON line.

Also measured, outside the timed region:
  * per-kernel durations (each stage launched back to back between HIP events
    on the encoder's stream) -> roofline of the dominant kernel;
  * the lossless round trip through the GPU decoder, residual bits/pixel;
  * the entropy code of the image's enhancement layer (static rANS): encode
    and decode times, coded bits/pixel against the planes' H0, round trip;
  * the batched decoder, quantised coefficients -> S -> RGBE, on the image
    and on the 64-image batch;
  * the base layer written as a JPEG file, and the size of the whole
    dual-layer stream (JPEG + entropy-coded enhancement layer);
  * the ablations (SLR without the Gaussian filter, one line per channel, no
    estimator) and a quality sweep: residual bits/pixel on the image;
  * the batched encoder on 64 uneven images (~275 Mpx, one launch per stage);
  * the learned estimator with per-region SLR fallback: bits/pixel against
    plain SLR on 16 held-out 1920x1080 images, and its throughput;
  * 256 uneven images of 1 to 33 MP (~4.4 Gpx) batched, plain and learned:
    Mpixel/s, GB/s, bits/pixel, lossless round trip of every image;
  * the CPU oracle on the host's cores, on the same image (cpu_baseline).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
# Vector ALU peak counting a multiply-add as two operations and no packed
# (two-wide) FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic HBM bytes per pixel of each stage (inputs read once, outputs
# written once): RGBE 4 B, S 3 B, residual planes 6 B, E plane 1 B.
ALGO_BYTES_PER_PX = {"keystat": 4, "tmo_base": 4 + 3, "fit_sums": 3 + 4, "resid": 3 + 4 + 6 + 1}
PIPELINE_BYTES_PER_PX = 4 + 3 + 6 + 1
# Algorithmic operations per pixel of the tone map + base layer (a
# multiply-add counts two): TMO 57, forward colour 21, FDCT 66, quantise and
# dequantise 27, IDCT with level shift and clamp 72, inverse colour 20.
TMO_BASE_OPS_PER_PX = 57 + 21 + 66 + 27 + 72 + 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_encode_3840x2160.md")


def entropy_bits(hist_row):
    n = float(sum(hist_row))
    if n <= 0:
        return 0.0
    return -sum((h / n) * math.log2(h / n) for h in hist_row if h)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rdl_kernels.hip", "rdl_internal.h"):
        with open(os.path.join(ROOT, "paper_2309_11072_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic():
    """HBM bytes per launch of each stage kernel from the committed counter
    summary, or None when the kernels changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    data = json.loads(m.group(1))
    if data.get("source_sha256") != kernel_source_hash():
        return None
    return data


def _oracle_worker(path, q, go, out):
    import numpy as np
    from oracle import oracle as O
    x = np.load(path)
    O.encode_enh(x[:8, :8], q)  # library loaded and warm
    out.put(("ready", 0.0, 0.0))
    go.wait()
    t0 = time.time()
    O.encode_enh(x, q)
    out.put(("done", t0, time.time()))


def cpu_baseline(x, q, budget_s):
    """The oracle as it stands (single-threaded C): first one process on the
    whole benchmark image, then as many concurrent processes as the host
    offers (at most 16, and as many as fit the budget), each encoding its own
    copy, released together once all are loaded.  The worker processes are
    started before this process touches the GPU."""
    import multiprocessing as mp
    import numpy as np
    from oracle import oracle as O
    O.build()
    H, W = x.shape[:2]
    fd, path = tempfile.mkstemp(suffix=".npy")
    os.close(fd)
    ctx = mp.get_context("spawn")

    def run(n):
        go, out = ctx.Event(), ctx.Queue()
        procs = [ctx.Process(target=_oracle_worker, args=(path, q, go, out)) for _ in range(n)]
        for p in procs:
            p.start()
        for _ in procs:
            out.get(timeout=600)
        go.set()
        spans = [out.get(timeout=600)[1:] for _ in procs]
        for p in procs:
            p.join()
        return max(e for _, e in spans) - min(s for s, _ in spans)

    try:
        np.save(path, x)
        t1 = run(1)
        # as many encodes as fit the budget, one per core, at most 16 cores
        n = max(1, min(16, os.cpu_count() or 1, int(budget_s / max(t1, 1e-3))))
        wall = run(n)
    finally:
        os.unlink(path)
    return {"value": round(n * H * W / wall / 1e6, 4), "unit": "Mpixel/s", "cores": n, "kind": "oracle",
            "sample": "%d concurrent full encodes of the %dx%d benchmark image by the C oracle (one thread each, "
                      "timed from a common start), %.2f s; one alone: %.2f s" % (n, W, H, wall, t1),
            "single_thread_Mpixel_s": round(H * W / t1 / 1e6, 4)}


def say(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def time_calls(fn, steps, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def tune_classes(codec, imgs, specs, items):
    """One autotuning per size class floor(log2(H W)), on its largest image."""
    best = {}
    for im, s, it in zip(imgs, specs, items):
        c = (s.H * s.W).bit_length() - 1
        if c not in best or s.H * s.W > best[c][0]:
            best[c] = (s.H * s.W, im, s.q, it[2:])
    for _, im, qq, o in best.values():
        codec.autotune(im, qq, o, reps=5)
    return len(best)


def cond_bits(resid, H, W):
    """Bits/pixel of the three residual planes coded given the exponent:
    sum over (channel, E) of sum_v h log2(n_E / h), over H W (computed on the
    GPU from the residual buffer).  This is the code length the per-region
    estimator selection minimises."""
    import torch
    npx = H * W
    r = resid[:6 * npx].view(torch.int16).reshape(3, npx).long()
    E = resid[6 * npx:7 * npx].long()
    tot = 0.0
    for c in range(3):
        h = torch.bincount(E * 511 + r[c] + 255, minlength=256 * 511).reshape(256, 511).double()
        n = h.sum(dim=1, keepdim=True)
        nz = h > 0
        tot += float((h[nz] * torch.log2((n.expand_as(h))[nz] / h[nz])).sum())
    return tot / npx


def resid_bits(codec, resid, H, W):
    h = codec.resid_hist(resid, H, W).cpu().numpy()
    return sum(entropy_bits(h[c].tolist()) for c in range(3))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=40.0,
                    help="oracle budget in CPU-seconds (0 = skip; skip it under a profiler, which starts the GPU "
                         "before the oracle's worker processes would start)")
    ap.add_argument("--profile-reps", type=int, default=50)
    ap.add_argument("--batch-steps", type=int, default=10, help="timed launches of the 64-image batch (0 = skip)")
    ap.add_argument("--learned-steps", type=int, default=20, help="timed learned encodes (0 = skip)")
    ap.add_argument("--large-steps", type=int, default=3,
                    help="timed launches of the 256-image batch, plain and learned (0 = skip)")
    ap.add_argument("--entropy-steps", type=int, default=50,
                    help="timed entropy encodes/decodes of the image's enhancement layer (0 = skip)")
    ap.add_argument("--decode-steps", type=int, default=20,
                    help="timed batched decodes (coefficients -> S -> RGBE) of the image and the 64-image batch (0 = skip)")
    ap.add_argument("--ablation", type=int, default=1, help="bits/pixel of the ablations and the quality sweep (0 = skip)")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch shapes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: images shard across GPUs without any exchange, and this build "
              "has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2309_11072_amd import rdl, synth

    sp = synth.image_3840x2160()
    H, W, q = sp.H, sp.W, sp.q
    x = sp.make()
    print("bench: workload %dx%d q=%d generated" % (W, H, q), file=sys.stderr, flush=True)
    cpu = cpu_baseline(x, q, args.cpu_seconds) if args.cpu_seconds > 0 else None
    if cpu:
        print("bench: cpu oracle %.3f Mpixel/s on %d cores" % (cpu["value"], cpu["cores"]), file=sys.stderr,
              flush=True)

    import torch
    codec = rdl.Codec(0)
    d = torch.from_numpy(x).cuda()
    out = codec.alloc_outputs(H, W)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_tune:
        tuned = codec.autotune(d, q, out, reps=20)
        print("bench: tuned %s" % tuned, file=sys.stderr, flush=True)

    for _ in range(max(args.warmup, 3)):
        codec.encode_enh(d, q, out=out)
    w0 = time.perf_counter()
    ms_step = time_calls(lambda: codec.encode_enh(d, q, out=out), args.steps, stream)
    wall = time.perf_counter() - w0
    mpx_s = H * W / (ms_step * 1e-3) / 1e6
    print("bench: %.4f ms/step (%.1f Mpixel/s), wall %.3f s" % (ms_step, mpx_s, wall), file=sys.stderr, flush=True)
    # the other launch mode, outside the timed region: the same plan replayed
    # as a captured graph
    codec.set_launch_mode(True)
    for _ in range(3):
        codec.encode_enh(d, q, out=out)
    ms_graph = time_calls(lambda: codec.encode_enh(d, q, out=out), args.steps, stream)
    codec.set_launch_mode(False)

    # ---- outside the timed region -----------------------------------------
    sdr, hdr, resid = out
    lossless = bool(torch.equal(codec.decode_enh(sdr, hdr, resid, H, W), d))
    bpp = resid_bits(codec, resid, H, W)
    e_bits = entropy_bits(np.bincount(x[..., 3].reshape(-1), minlength=256).tolist())
    h = rdl.header_from_bytes(hdr)

    say("decode and bits/pixel done")
    stage_ms = codec.profile_encode(d, q, out, reps=args.profile_reps)
    say("stage times %s" % {k: round(v * 1000, 1) for k, v in stage_ms.items()})
    dom = max((k for k in stage_ms if k in ALGO_BYTES_PER_PX), key=lambda k: stage_ms[k])
    t_dom = stage_ms[dom] * 1e-3
    traffic = committed_traffic()
    tr = traffic["kernels"].get("k_" + dom, {}).get("bytes") if traffic else None
    hbm_gbps = ALGO_BYTES_PER_PX[dom] * H * W / t_dom / 1e9
    if dom == "tmo_base":
        achieved = TMO_BASE_OPS_PER_PX * H * W / t_dom / 1e12
        roofline = {"kernel": "k_tmo_base", "bound": "alu", "achieved": round(achieved, 2), "peak": ALU_PEAK_TOPS,
                    "unit": "TOP/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": tr,
                    "ops_per_px": TMO_BASE_OPS_PER_PX, "avg_ms": round(stage_ms[dom], 5),
                    "hbm_GBps": round(hbm_gbps, 1), "hbm_frac": round(hbm_gbps / HBM_PEAK_GBPS, 4)}
    else:
        roofline = {"kernel": "k_" + dom, "bound": "hbm", "achieved": round(hbm_gbps, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(hbm_gbps / HBM_PEAK_GBPS, 4), "traffic": tr,
                    "bytes_per_px": ALGO_BYTES_PER_PX[dom], "avg_ms": round(stage_ms[dom], 5)}
    pipe_gbps = PIPELINE_BYTES_PER_PX * H * W / (ms_step * 1e-3) / 1e9

    # ---- entropy code of the enhancement layer (static rANS) -----------------
    entropy = None
    if args.entropy_steps > 0:
        k = rdl.ENT_LOG2K_DEFAULT
        code = torch.empty(codec.ent_bound(H, W, k), dtype=torch.uint8, device="cuda")
        clen = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(3):
            codec.ent_encode_into(resid, H, W, code, clen, k)
        ms_e = time_calls(lambda: codec.ent_encode_into(resid, H, W, code, clen, k), args.entropy_steps, stream)
        nbytes = int(clen.item())
        cview = code[:nbytes]
        chdr = cview[:rdl.ENT_HEADER_BYTES].cpu().numpy()
        back = torch.empty_like(resid)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        for _ in range(3):
            codec.ent_decode(cview, H, W, out=back, status=st, header=chdr)
        ms_d = time_calls(lambda: codec.ent_decode(cview, H, W, out=back, status=st, header=chdr),
                          args.entropy_steps, stream)
        ok = bool(torch.equal(back, resid)) and int(st.item()) == 0
        npx = H * W
        # the same layer with the exponents coded as they are, and the H0 of
        # their left differences (statistics of the stream, not timed)
        codec.set_ent_predict(False)
        codec.ent_encode_into(resid, H, W, code, clen, k)
        codec.set_ent_predict(True)
        nbytes_plain = int(clen.item())
        e_pl = resid[6 * npx:].view(H, W).to(torch.int32)
        e_d = e_pl.clone()
        e_d[:, 1:] = (e_pl[:, 1:] - e_pl[:, :-1]) & 255
        p_d = torch.bincount(e_d.reshape(-1), minlength=256).double() / npx
        e_d_bits = float(-(p_d[p_d > 0] * torch.log2(p_d[p_d > 0])).sum())
        entropy = {"workload": "the 3840x2160 image's enhancement layer (3 int16 residual planes + the exponent "
                               "plane as left differences), static rANS, 64 interleaved states per group of %d "
                               "symbols" % (64 << k),
                   "log2_k": k, "ms_encode": round(ms_e, 5), "Mpixel_s_encode": round(npx / (ms_e * 1e-3) / 1e6, 1),
                   "ms_decode": round(ms_d, 5), "Mpixel_s_decode": round(npx / (ms_d * 1e-3) / 1e6, 1),
                   "bytes": nbytes, "bits_per_pixel_coded": round(8 * nbytes / npx, 4),
                   "bits_per_pixel_h0": round(bpp + e_d_bits, 4),
                   "bits_per_pixel_h0_plain_exponents": round(bpp + e_bits, 4),
                   "bits_per_pixel_coded_plain_exponents": round(8 * nbytes_plain / npx, 4), "lossless": ok,
                   "encode_plus_entropy_ms": round(ms_step + ms_e, 5),
                   "encode_plus_entropy_Mpixel_s": round(npx / ((ms_step + ms_e) * 1e-3) / 1e6, 1)}
        say("entropy code: %.1f us encode, %.1f us decode, %.4f bits/px (H0 %.4f; plain exponents %.4f)" % (
            ms_e * 1e3, ms_d * 1e3, entropy["bits_per_pixel_coded"], entropy["bits_per_pixel_h0"],
            entropy["bits_per_pixel_coded_plain_exponents"]))
        del code, back

    # ---- ablations (the comparisons of Table I) and a quality sweep (Fig. 4) --
    ablation = None
    if args.ablation:
        outa = codec.alloc_outputs(H, W)
        rows = {}
        for name, est, gf in (("slr_gf (proposed)", 0, True), ("slr_no_gf", 0, False), ("global_line_gf", 2, True),
                              ("no_slrme (M* = S, no GF)", 3, False)):
            codec.set_estimator(est)
            codec.set_gf(gf)
            codec.encode_enh(d, q, out=outa)
            ms_m = time_calls(lambda: codec.encode_enh(d, q, out=outa), 5, stream)
            ok_m = bool(torch.equal(codec.decode_enh(*outa, H, W), d))
            rows[name] = {"bits_per_pixel": round(resid_bits(codec, outa[2], H, W), 4),
                          "bits_per_pixel_given_E": round(cond_bits(outa[2], H, W), 4), "ms": round(ms_m, 4),
                          "lossless": ok_m}
        sweep = {}
        for qq in (10, 30, 50, 70, 90, 100):
            row = {}
            for name, est, gf in (("slr_gf", 0, True), ("no_slrme", 3, False)):
                codec.set_estimator(est)
                codec.set_gf(gf)
                codec.encode_enh(d, qq, out=outa)
                row[name] = round(resid_bits(codec, outa[2], H, W), 4)
            sweep[str(qq)] = row
        codec.set_estimator(0)
        codec.set_gf(True)
        ablation = {"workload": "the 3840x2160 image, residual bits/pixel (sum of the three planes' H0; exponent plane "
                                "%.4f bits/pixel in every mode)" % e_bits, "q": q, "modes": rows,
                    "quality_sweep_bits_per_pixel": sweep}
        say("ablation: %s" % {k: v["bits_per_pixel"] for k, v in rows.items()})
        del outa

    # ---- decoder: quantised coefficients -> S -> RGBE ------------------------
    decoder = None
    jpeg = None
    if args.decode_steps > 0:
        ks = codec.stage_keystat(d)
        s_ref, _, dct = codec.stage_tmo_base(d, q, ks, want_dct=True)
        # the base layer as a JPEG file (baseline, optimised Huffman tables)
        jbuf = torch.empty(codec.jpeg_bound(H, W), dtype=torch.uint8, device="cuda")
        jlen = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(3):
            codec.jpeg_encode_into(dct, H, W, q, jbuf, jlen)
        ms_j = time_calls(lambda: codec.jpeg_encode_into(dct, H, W, q, jbuf, jlen), args.decode_steps, stream)
        jbytes = int(jlen.item())
        jpeg = {"workload": "the 3840x2160 image's base layer: quantised coefficients -> baseline JFIF file "
                            "(Huffman tables optimised per image, one scan per component)",
                "ms": round(ms_j, 5), "Mpixel_s": round(H * W / (ms_j * 1e-3) / 1e6, 1), "bytes": jbytes,
                "bits_per_pixel": round(8 * jbytes / (H * W), 4)}
        if entropy is not None:
            jpeg["dual_layer_bits_per_pixel"] = round(jpeg["bits_per_pixel"] + entropy["bits_per_pixel_coded"], 4)
            jpeg["dual_layer_encode_ms"] = round(ms_step + ms_j + entropy["ms_encode"], 5)
            jpeg["dual_layer_Mpixel_s"] = round(H * W / (jpeg["dual_layer_encode_ms"] * 1e-3) / 1e6, 1)
        say("jpeg: %.1f us, %.4f bits/px" % (ms_j * 1e3, jpeg["bits_per_pixel"]))
        del jbuf
        s_dec = torch.empty_like(sdr)
        rgbe_dec = torch.empty_like(d)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        item = [(dct, s_dec, hdr, resid, rgbe_dec, st)]
        for _ in range(3):
            codec.decode_batch(item)
        ms_full = time_calls(lambda: codec.decode_batch(item), args.decode_steps, stream)
        ms_base = time_calls(lambda: codec.base_decode(dct, hdr, H, W, out=s_dec), args.decode_steps, stream)
        ms_enh = time_calls(lambda: codec.decode_enh(sdr, hdr, resid, H, W, out=rgbe_dec), args.decode_steps, stream)
        codec.decode_batch(item)
        ok = bool(torch.equal(rgbe_dec, d)) and bool(torch.equal(s_dec, sdr)) and int(st.item()) == 0
        decoder = {"workload": "the 3840x2160 image: base layer from its quantised coefficients, then the enhancement layer",
                   "ms_per_image": round(ms_full, 5), "Mpixel_s": round(H * W / (ms_full * 1e-3) / 1e6, 1),
                   "ms_base_layer": round(ms_base, 5), "ms_enhancement_layer": round(ms_enh, 5), "lossless": ok}
        say("decoder: %.1f us per image (base %.1f us, enhancement %.1f us)" % (ms_full * 1e3, ms_base * 1e3,
                                                                            ms_enh * 1e3))
        del dct, s_dec, rgbe_dec

    # plain device copy of 1 GiB for scale (reads + writes 2 GiB)
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    copy_gbps = 2 * (1 << 30) / (time_calls(lambda: b.copy_(a), 5, stream) * 1e-3) / 1e9
    del a, b

    # ---- batch: 64 uneven images, one launch per stage ----------------------
    batch = None
    if args.batch_steps > 0:
        specs = synth.batch_64_uneven()
        imgs = []
        for k, s in enumerate(specs):
            imgs.append(s.make_torch())
            if k % 16 == 15:
                say("batch images generated: %d" % (k + 1))
        items = [(im, s.q) + tuple(codec.alloc_outputs(s.H, s.W)) for im, s in zip(imgs, specs)]
        npx = sum(s.H * s.W for s in specs)
        if not args.no_tune:
            say("batch tuned for %d size classes" % tune_classes(codec, imgs, specs, items))
        for _ in range(3):
            codec.encode_batch(items)
        ms_b = time_calls(lambda: codec.encode_batch(items), args.batch_steps, stream)
        ok = all(torch.equal(codec.decode_enh(it[2], it[3], it[4], s.H, s.W), im)
                 for it, s, im in zip(items, specs, imgs))
        gbps_b = PIPELINE_BYTES_PER_PX * npx / (ms_b * 1e-3) / 1e9
        batch = {"workload": "64 uneven RGBE images of 0.3 to 8.3 MP (sigma_L 1.5-4, q 50-95, drawn on the GPU), one launch "
                             "per stage, plain SLR", "images": len(specs), "Mpixel": round(npx / 1e6, 2),
                 "ms_per_step": round(ms_b, 4), "Mpixel_s": round(npx / (ms_b * 1e-3) / 1e6, 1),
                 "pipeline_algorithmic_GBps": round(gbps_b, 1), "pipeline_frac_of_hbm": round(gbps_b / HBM_PEAK_GBPS, 4),
                 "lossless": ok}
        print("bench: batch %.3f ms (%.1f Mpixel/s)" % (ms_b, batch["Mpixel_s"]), file=sys.stderr, flush=True)
        if args.decode_steps > 0:
            dec = []
            for (im, qq, sdr_b, hdr_b, resid_b), s in zip(items, specs):
                ks = codec.stage_keystat(im)
                _, _, dct_b = codec.stage_tmo_base(im, qq, ks, want_dct=True)
                dec.append((dct_b, torch.empty_like(sdr_b), hdr_b, resid_b, torch.empty_like(im),
                            torch.zeros(1, dtype=torch.int32, device="cuda")))
            for _ in range(2):
                codec.decode_batch(dec)
            ms_db = time_calls(lambda: codec.decode_batch(dec), max(3, args.decode_steps // 4), stream)
            okd = all(torch.equal(dv[4], im) and torch.equal(dv[1], it[2]) and int(dv[5].item()) == 0
                      for dv, it, im in zip(dec, items, imgs))
            batch["decode"] = {"what": "quantised coefficients -> S -> RGBE, one launch per stage for the 64 images",
                               "ms": round(ms_db, 4), "Mpixel_s": round(npx / (ms_db * 1e-3) / 1e6, 1), "lossless": okd}
            say("batch decode %.3f ms (%.1f Mpixel/s)" % (ms_db, batch["decode"]["Mpixel_s"]))
            del dec
        del imgs, items

    # ---- learned estimator with per-region SLR fallback ----------------------
    learned = None
    model_path = os.path.join(ROOT, "paper_2309_11072_amd", "mlp_model.bin")
    if os.path.exists(model_path) and args.learned_steps > 0:
        with open(model_path, "rb") as fh:
            codec.set_model(fh.read())
        say("learned estimator: evaluating")
        bits = {0: 0.0, 1: 0.0}
        cbits = {0: 0.0, 1: 0.0}
        npx_eval = 0
        ok = True
        regions = [0, 0]
        for s in synth.learned_eval_set():
            xe = torch.from_numpy(s.make()).cuda()
            oe = codec.alloc_outputs(s.H, s.W)
            for mode in (0, 1):
                codec.set_estimator(mode)
                codec.encode_enh(xe, s.q, out=oe)
                bits[mode] += resid_bits(codec, oe[2], s.H, s.W) * s.H * s.W
                cbits[mode] += cond_bits(oe[2], s.H, s.W) * s.H * s.W
                if mode == 1:
                    ok &= bool(torch.equal(codec.decode_enh(oe[0], oe[1], oe[2], s.H, s.W), xe))
                    he = rdl.header_from_bytes(oe[1])
                    regions[0] += int(he["flag"].sum())
                    regions[1] += int(3 * he["n_regions"])
            npx_eval += s.H * s.W
        codec.set_estimator(1)
        outl = codec.alloc_outputs(H, W)
        for _ in range(3):
            codec.encode_enh(d, q, out=outl)
        ms_l = time_calls(lambda: codec.encode_enh(d, q, out=outl), args.learned_steps, stream)
        ok &= bool(torch.equal(codec.decode_enh(outl[0], outl[1], outl[2], H, W), d))
        codec.set_estimator(0)
        learned = {"eval": "16 held-out 1920x1080 images (sigma_L 4, 5% speculars, q 75)",
                   "bits_per_pixel_slr": round(bits[0] / npx_eval, 4),
                   "bits_per_pixel_learned": round(bits[1] / npx_eval, 4),
                   "bits_per_pixel_given_E_slr": round(cbits[0] / npx_eval, 4),
                   "bits_per_pixel_given_E_learned": round(cbits[1] / npx_eval, 4),
                   "regions_learned": regions[0], "regions": regions[1], "lossless": ok,
                   "Mpixel_s": round(H * W / (ms_l * 1e-3) / 1e6, 1), "ms_per_step": round(ms_l, 5),
                   "throughput_workload": "the 3840x2160 benchmark image",
                   "model_hash": "%016x" % int(rdl.header_from_bytes(outl[1])["model_hash"])}
        del outl

    # ---- 256 uneven images up to 33 MP: learned + fallback vs plain SLR ------
    large = None
    if learned is not None and args.large_steps > 0:
        torch.cuda.empty_cache()
        specs = synth.batch_256_large()
        imgs = []
        for k, s in enumerate(specs):
            imgs.append(s.make_torch())
            if k % 64 == 63:
                say("large batch images generated: %d" % (k + 1))
        items = [(im, s.q) + tuple(codec.alloc_outputs(s.H, s.W)) for im, s in zip(imgs, specs)]
        npx = sum(s.H * s.W for s in specs)
        if not args.no_tune:
            say("large batch tuned for %d size classes" % tune_classes(codec, imgs, specs, items))
        res = {}
        for mode in (0, 1):
            codec.set_estimator(mode)
            for _ in range(2):
                codec.encode_batch(items)
            ms = time_calls(lambda: codec.encode_batch(items), args.large_steps, stream)
            bits = sum(resid_bits(codec, it[4], s.H, s.W) * s.H * s.W for it, s in zip(items, specs)) / npx
            cb = sum(cond_bits(it[4], s.H, s.W) * s.H * s.W for it, s in zip(items, specs)) / npx
            ok = all(torch.equal(codec.decode_enh(it[2], it[3], it[4], s.H, s.W), im)
                     for it, s, im in zip(items, specs, imgs))
            flagged = sum(int(rdl.header_from_bytes(it[3])["flag"].sum()) for it in items) if mode else 0
            res[mode] = (ms, bits, ok, flagged, cb)
            say("large batch, %s: %.2f ms (%.1f Mpixel/s)" % ("learned" if mode else "plain", ms,
                                                             npx / (ms * 1e-3) / 1e6))
        codec.set_estimator(0)
        large = {"workload": "256 uneven RGBE images of 1 to 33 MP (sigma_L 1-5, q 30-98, drawn on the "
                             "GPU), one launch per stage", "images": len(specs), "Mpixel": round(npx / 1e6, 1)}
        for mode, name in ((0, "slr"), (1, "learned")):
            ms, bits, ok, flagged, cb = res[mode]
            gbps = PIPELINE_BYTES_PER_PX * npx / (ms * 1e-3) / 1e9
            large[name] = {"ms_per_step": round(ms, 3), "Mpixel_s": round(npx / (ms * 1e-3) / 1e6, 1),
                           "pipeline_algorithmic_GBps": round(gbps, 1), "bits_per_pixel": round(bits, 4),
                           "bits_per_pixel_given_E": round(cb, 4),
                           "lossless": ok}
        large["learned"]["regions_learned"] = res[1][3]
        del imgs, items
        torch.cuda.empty_cache()

    line = {
        "metric": "encoded Mpixel/s on 1 MI355X + residual bits/pixel, learned vs SLR, lossless",
        "value": round(mpx_s, 2), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32+fp32", "data": "synthetic",
        "config": {"workload": "single 3840x2160 RGBE image, sigma_L 4, 5% speculars at +10 stops, JPEG q 75, "
                               "plain SLR estimator (direct stage launches)", "H": H, "W": W, "q": q, "seed": sp.seed,
                   "tuning": tuned},
        "lossless": lossless,
        "graph_replay_ms_per_step": round(ms_graph, 5),
        "bits_per_pixel": {"slr": round(bpp, 4), "e_plane": round(e_bits, 4)},
        "n_regions": int(h["n_regions"]),
        "pipeline_algorithmic_GBps": round(pipe_gbps, 1),
        "pipeline_frac_of_hbm": round(pipe_gbps / HBM_PEAK_GBPS, 4),
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "device_copy_GBps": round(copy_gbps, 1),
        "entropy": entropy,
        "decoder": decoder,
        "jpeg": jpeg,
        "ablation": ablation,
        "batch": batch,
        "learned": learned,
        "large_batch": large,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
