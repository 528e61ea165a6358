"""CPU model of the memory accesses of the strip walk shared by the fit and
residual kernels (the same index arithmetic as the HIP code, lane by lane):
every read and write must fall inside its buffer, for every lane, row and
launch shape, on widths of every residue mod 4 and on S buffers whose rows do
not start on dword boundaries.  No GPU is needed; this runs before a changed
walk ever reaches one."""
import numpy as np
import pytest

STRIP_W, STRIP_WAVES, WALK_CH = 256, 4, 4


def walk_accesses(H, W, srh, sdr_base, rgbe_base, resid_base, waves=STRIP_WAVES):
    """Yields (buffer, first byte, last byte + 1) for every access."""
    nsx = (W + STRIP_W - 1) // STRIP_W
    nwg = ((H + srh * waves - 1) // (srh * waves)) * nsx
    end = sdr_base + 3 * H * W
    npx = H * W
    for wgl in range(nwg):
        sy, sx = divmod(wgl, nsx)
        x0 = sx * STRIP_W
        for wave in range(waves):
            ya = (sy * waves + wave) * srh
            if ya >= H:
                continue
            yb = min(ya + srh, H)
            lanes = np.arange(64)
            x = x0 + 4 * lanes
            hx = np.where(lanes == 0, max(x0 - 1, 0), min(x0 + STRIP_W, W - 1))
            xo3, ho3, xo4 = 3 * x, 3 * hx, 4 * x
            fx = x + 4 <= W
            last = sdr_base + (H - 1) * 3 * W
            shl = (last + xo3) & 3
            fast_last = fx & (xo3 - shl + 16 <= 3 * W)

            def s_row(yy):
                row = sdr_base + yy * 3 * W
                fast = fx if yy < H - 1 else fast_last
                sh = (row + xo3) & 3
                for l in range(64):
                    if fast[l]:
                        a = row + xo3[l] - sh[l]
                        yield ("sdr", a, a + 16)
                    else:
                        for j in range(4):
                            a = row + 3 * min(x[l] + j, W - 1)
                            yield ("sdr", a, a + 3)
                    yield ("sdr", row + ho3[l], row + ho3[l] + 3)

            def rgbe_row(yy):
                row = rgbe_base + yy * 4 * W
                for l in range(64):
                    p = row + xo4[l]
                    if fx[l] and (p & 15) == 0:
                        yield ("rgbe", p, p + 16)
                    else:
                        for j in range(4):
                            a = row + 4 * min(x[l] + j, W - 1)
                            yield ("rgbe", a, a + 4)

            yield from s_row(max(ya - 1, 0))
            yield from s_row(ya)
            for y0 in range(ya, yb, WALK_CH):
                for k in range(WALK_CH):
                    yield from s_row(min(min(y0 + k + 1, yb), H - 1))
                    yield from rgbe_row(min(y0 + k, yb - 1))
                for k in range(WALK_CH):
                    y = y0 + k
                    if y >= yb:
                        continue
                    al = (W & 3) == 0 and (resid_base & 7) == 0
                    for l in range(64):
                        if x[l] >= W:
                            continue
                        if al and x[l] + 4 <= W:
                            for c in range(3):
                                a = resid_base + 2 * (c * npx + y * W + x[l])
                                yield ("resid", a, a + 8)
                            a = resid_base + 6 * npx + y * W + x[l]
                            yield ("resid", a, a + 4)
                        else:
                            for j in range(min(4, W - x[l])):
                                for c in range(3):
                                    a = resid_base + 2 * (c * npx + y * W + x[l] + j)
                                    yield ("resid", a, a + 2)
                                a = resid_base + 6 * npx + y * W + x[l] + j
                                yield ("resid", a, a + 1)


SHAPES = [(1, 1), (1, 4), (1, 5), (2, 7), (7, 9), (9, 17), (5, 256), (3, 257), (6, 258), (4, 259), (33, 40),
          (17, 513), (2, 1023)]


@pytest.mark.parametrize("H,W", SHAPES, ids=["%dx%d" % s for s in SHAPES])
@pytest.mark.parametrize("srh,waves", [(2, 4), (8, 4), (32, 4), (8, 16), (16, 8)])
def test_strip_walk_stays_inside_buffers(H, W, srh, waves):
    bases = {"sdr": 4096, "rgbe": 1 << 20, "resid": 1 << 24}
    sizes = {"sdr": 3 * H * W, "rgbe": 4 * H * W, "resid": 7 * H * W}
    for sdr_off in (0, 4, 8):   # S buffers start on dword boundaries (the API requires it)
        for res_off in (0, 2):
            b = dict(bases, sdr=bases["sdr"] + sdr_off, resid=bases["resid"] + res_off)
            for buf, lo, hi in walk_accesses(H, W, srh, b["sdr"], b["rgbe"], b["resid"], waves):
                assert b[buf] <= lo and hi <= b[buf] + sizes[buf], (buf, lo - b[buf], hi - b[buf], sizes[buf])


# ---------------------------------------------------------------------------
# Learned path: exponent buckets of residual records.  k_solve turns the
# region sizes n_e into bucket starts and the first histogram workgroup of
# each exponent (prefixes over ceil(n_e / LCH)); k_learn reserves records per
# tile with atomics on the bucket cursors; k_lhist maps its workgroup to an
# exponent by binary search and histograms LCH records of that bucket.
LCH = 32768


def bucket_table(ne):
    """The uint32 table k_solve writes: cursors, first workgroups (+ total),
    bucket starts."""
    ne = [int(v) for v in ne]
    start = np.concatenate([[0], np.cumsum(ne)[:-1]]).astype(np.int64)
    nc = [(v + LCH - 1) // LCH for v in ne]
    fw = np.concatenate([[0], np.cumsum(nc)]).astype(np.int64)
    return start.copy(), fw, start


def lhist_ranges(ne, nwg):
    """(e, first record, count) of each histogram workgroup that runs."""
    _, fw, start = bucket_table(ne)
    out = []
    for g in range(nwg):
        if g >= fw[256]:
            continue
        lo, hi = 0, 256
        while hi - lo > 1:
            mid = (lo + hi) >> 1
            if fw[mid] <= g:
                lo = mid
            else:
                hi = mid
        e = lo
        k = g - fw[e]
        first = int(start[e]) + k * LCH
        cnt = min(LCH, ne[e] - k * LCH)
        out.append((e, first, cnt))
    return out


@pytest.mark.parametrize("case", ["one", "spread", "multiples", "sparse", "4k"])
def test_learned_buckets_cover_each_record_once(case):
    rng = np.random.default_rng(11)
    if case == "one":
        ne = np.zeros(256, np.int64); ne[0] = 1
    elif case == "spread":
        ne = rng.integers(0, 5000, 256)
    elif case == "multiples":
        ne = np.zeros(256, np.int64); ne[[3, 100, 255]] = [LCH, 2 * LCH, 3 * LCH]
    elif case == "sparse":
        ne = np.zeros(256, np.int64); ne[rng.choice(256, 40, replace=False)] = rng.integers(1, 200000, 40)
    else:
        ne = np.zeros(256, np.int64); ne[110:160] = rng.multinomial(3840 * 2160, np.ones(50) / 50)
    npx = int(ne.sum())
    nwg = (npx + LCH - 1) // LCH + 256  # the grid of wgs_lhist
    runs = lhist_ranges(ne, nwg)
    seen = np.zeros(npx, np.int32)
    for e, first, cnt in runs:
        assert 0 < cnt <= LCH and first >= 0 and first + cnt <= npx
        seen[first:first + cnt] += 1
    assert np.all(seen == 1), "every record in exactly one histogram workgroup"
    assert len(runs) <= nwg
    # the workgroup's records all belong to its exponent's bucket
    _, _, start = bucket_table(ne)
    for e, first, cnt in runs:
        assert start[e] <= first and first + cnt <= start[e] + ne[e]


def test_learned_reservation_stays_in_bucket():
    """k_learn's tiles (16 x 64 px) rank their pixels of each exponent, then
    reserve that many records of it with one atomic on its cursor, the tiles
    in any order; with reservations summing to n_e every index lands inside
    bucket e, exactly once."""
    rng = np.random.default_rng(5)
    H, W = 200, 333
    E = rng.integers(120, 140, (H, W))
    E[rng.random((H, W)) < 0.05] += 10
    ne = np.bincount(E.reshape(-1), minlength=256)
    cur, _, start = bucket_table(ne)
    tiles = [(ty, tx) for ty in range(0, H, 16) for tx in range(0, W, 64)]
    rng.shuffle(tiles)
    hit = np.zeros(H * W, np.int32)
    for ty, tx in tiles:
        t = E[ty:ty + 16, tx:tx + 64].reshape(-1)
        rank = {}
        idx = []
        for e in t:
            r = rank.get(e, 0)
            rank[e] = r + 1
            idx.append((e, r))
        base = {}
        for e, c in rank.items():
            base[e] = cur[e]
            cur[e] += c
        for e, r in idx:
            k = base[e] + r
            assert start[e] <= k < start[e] + ne[e] and k < H * W
            hit[k] += 1
    assert np.all(hit == 1)


# ---------------------------------------------------------------- JPEG writer: word ownership
def jpeg_emit_words(lengths):
    """Model of k_jpg_emit's stores: block b covers bits [pos_b, pos_b + len_b);
    it ORs its first word and its last partial word and plain-stores the words
    it fills completely past its first.  Returns (plain, ored) lists of
    (block, word)."""
    plain, ored = [], []
    pos = 0
    for b, n in enumerate(lengths):
        first = pos >> 5
        nacc = pos & 31
        w = first
        for _ in range(n):  # bit by bit: a word goes out when 32 bits are pending
            nacc += 1
            if nacc == 32:
                (ored if w == first else plain).append((b, w))
                w += 1
                nacc = 0
        if nacc:
            ored.append((b, w))
        pos += n
    return plain, ored, pos


@pytest.mark.parametrize("seed", range(20))
def test_jpeg_emit_plain_stores_are_exclusive(seed):
    """Every plain-stored word lies wholly inside one block's bit range (no
    other block touches it), and every word of the scan is written; shared
    words are only ever ORed."""
    rng = np.random.default_rng(seed)
    lengths = list(rng.integers(0, 120, int(rng.integers(1, 60))))
    lengths[int(rng.integers(len(lengths)))] = 0  # a block of no bits (the encoder makes none) is harmless too
    plain, ored, total = jpeg_emit_words(lengths)
    owners = {}
    for b, w in plain + ored:
        owners.setdefault(w, []).append(b)
    starts = np.concatenate([[0], np.cumsum(lengths)])
    for b, w in plain:
        assert starts[b] <= 32 * w and 32 * (w + 1) <= starts[b + 1], "plain store outside its block"
        assert owners[w] == [b], "a plain-stored word is touched by another block"
    assert set(owners) == set(range((total + 31) // 32)), "every word of the scan is written"


# ---------------------------------------------------------------- entropy decoder: ring of words
def test_entropy_decoder_ring_reads_stay_inside():
    """Model of k_ent_dec's ring: words [b, b + 512) in LDS, the next 256 in
    registers; before a step, pos >= b + 256 moves b by 256.  For any sequence
    of per-step consumptions (0..64 words), every word a step reads was put in
    the ring and not overwritten."""
    rng = np.random.default_rng(7)
    for trial in range(200):
        w0 = int(rng.integers(0, 1000))
        b = pos = w0 + 128
        ring_lo, ring_hi = b, b + 512          # words currently held
        for step in range(400):
            if pos >= b + 256:
                b += 256
                ring_lo, ring_hi = b, b + 512
            k = int(rng.integers(0, 65)) if trial % 2 else int(rng.choice([0, 64]))
            assert ring_lo <= pos and pos + k <= ring_hi, (trial, step, pos, k, b)
            pos += k


# ---------------------------------------------------------------- enhancement decoder: wide accesses
@pytest.mark.parametrize("W", [4, 8, 12, 256, 260, 1024, 3840])
@pytest.mark.parametrize("H", [1, 3, 17])
def test_decode_wide_accesses_stay_inside(H, W):
    """k_decode reads 4 exponent bytes and 3 x 8 residual bytes per lane and
    row, and stores 16 bytes of RGBE, only when W % 4 == 0 and the lane's four
    pixels are inside: every such access lies inside its plane and row and
    on its alignment."""
    npx = H * W
    assert W % 4 == 0
    for y in range(H):
        for x in range(0, W, 4):
            off = y * W + x
            e_byte = 6 * npx + off
            assert e_byte % 4 == 0 and e_byte + 4 <= 7 * npx
            for c in range(3):
                r_byte = 2 * (c * npx + off)
                assert r_byte % 8 == 0 and r_byte + 8 <= 2 * (c + 1) * npx
            o_byte = 4 * off
            assert o_byte % 16 == 0 and o_byte + 16 <= 4 * npx


# ---- left differences of the exponent plane ---------------------------------
def _seg_join(a, b):
    return b if b & 256 else ((a + b) & 255) | (a & 256)


def _block_excl_scan(vals, nw=4):
    """The workgroup scan as the kernel runs it: per wave the shuffle-up
    ladder (offsets 1 .. 32), then the waves' totals joined in order."""
    n = 64 * nw
    vals = list(vals) + [0] * (n - len(vals))
    inc = list(vals)
    for w in range(nw):
        lanes = inc[64 * w:64 * w + 64]
        off = 1
        while off < 64:
            lanes = [_seg_join(lanes[l - off], lanes[l]) if l >= off else lanes[l] for l in range(64)]
            off <<= 1
        inc[64 * w:64 * w + 64] = lanes
    sh = [inc[64 * w + 63] for w in range(nw)]
    out, total = [], 0
    for k in range(nw):
        total = _seg_join(total, sh[k])
    for t in range(n):
        w, l = divmod(t, 64)
        before = 0
        for k in range(w):
            before = _seg_join(before, sh[k])
        ex = inc[t - 1] if l else 0
        out.append(_seg_join(before, ex))
    return out, total


def _chunk(N, W, lead, t, touched):
    """echunk_load: (i0, col0, full, indices read); records the bytes read."""
    i0 = 16 * t - lead
    full = i0 >= 0 and i0 + 16 <= N
    m = abs(i0) % W
    col0 = W - m if i0 < 0 and m else m
    idx = [i0 + k for k in range(16) if 0 <= i0 + k < N]
    if full:
        assert (lead + i0) % 16 == 0  # the 16-byte access is aligned
    touched.update(idx)
    return i0, col0, full


def _undo_model(d, W, lead):
    """k_ent_eseg, k_ent_ecarry and k_ent_eundo on a flat plane d (uint8) at
    an address with the given lead; checks every access stays in the plane."""
    N = d.size
    ntiles = (N + lead + 4095) // 4096
    assert ntiles <= (N + 15 + 4095) // 4096  # the workspace holds 2 values per tile for any lead
    touched = set()
    lanes = []
    for t in range(ntiles * 256):
        i0, col0, full = _chunk(N, W, lead, t, touched)
        v = [int(d[i0 + k]) if 0 <= i0 + k < N else 0 for k in range(16)]
        seg, col = 0, col0
        for k in range(16):
            if 0 <= i0 + k < N:
                seg = (v[k] | 256) if col == 0 else _seg_join(seg, v[k])
            col = 0 if col + 1 == W else col + 1
        lanes.append((i0, col0, v, seg))
    assert touched == set(range(N))
    tile_seg, tile_ex = [], []
    for b in range(ntiles):
        ex, tot = _block_excl_scan([ln[3] for ln in lanes[256 * b:256 * b + 256]])
        tile_seg.append(tot)
        tile_ex.append(ex)
    carry, run = [], 0
    for b0 in range(0, ntiles, 1024):
        ex, tot = _block_excl_scan(tile_seg[b0:b0 + 1024], nw=16)
        carry += [_seg_join(run, e) for e in ex[:min(1024, ntiles - b0)]]
        run = _seg_join(run, tot)
    if W <= 4096:  # the kernel's direct carry: the previous tile's value
        assert carry == [0] + tile_seg[:-1]
    out = np.full(N, -1, np.int64)
    for t, (i0, col, v, _) in enumerate(lanes):
        b = t // 256
        acc = _seg_join(carry[b], tile_ex[b][t % 256]) & 255
        for k in range(16):
            acc = (v[k] if col == 0 else acc + v[k]) & 255
            if 0 <= i0 + k < N:
                assert out[i0 + k] < 0  # written once
                out[i0 + k] = acc
            col = 0 if col + 1 == W else col + 1
    return out


def _diff_model(E, W, lead):
    """k_ent_ediff: d of every chunk, with the previous byte read from before
    the chunk only past a row's first pixel."""
    N = E.size
    out = np.full(N, -1, np.int64)
    touched = set()
    for t in range((N + lead + 4095) // 4096 * 256):
        i0, col, full = _chunk(N, W, lead, t, touched)
        if i0 >= N:
            continue
        prev = int(E[i0 - 1]) if i0 >= 1 else 0
        for k in range(16):
            i = i0 + k
            v = int(E[i]) if 0 <= i < N else 0
            dv = (v if col == 0 else v - prev) & 255
            prev = v
            if 0 <= i < N:
                out[i] = dv
            col = 0 if col + 1 == W else col + 1
    assert touched == set(range(N))
    return out


_SMALL = [(1, 1), (1, 2), (3, 1), (1, 17), (5, 4097), (300, 37), (2, 70000), (41, 1000)]


@pytest.mark.parametrize("H,W,lead", [(H, W, lead) for H, W in _SMALL for lead in (0, 6, 15)]
                         + [(700, 1510, 15), (1100, 3900, 6)])
def test_exponent_difference_kernels_model(H, W, lead):
    """The encoder's differences and the decoder's segmented scan (lanes,
    waves, tiles, carry chunks of 1024 tiles) give d and back E exactly, for a
    plane at any address mod 16: rows inside one lane (W = 1, 2, 37), rows
    across tiles (70,000 wide), 1100 x 3900 needs two carry chunks; with rows
    of at most 4096 pixels the carry is the previous tile's value."""
    rng = np.random.default_rng(H * W + lead)
    E = rng.integers(0, 256, (H, W))
    E[:, W // 3:] = E[:, W // 3:] // 64 + 120  # runs of close values too
    d = E.copy()
    d[:, 1:] = (E[:, 1:] - E[:, :-1]) % 256
    flat = E.reshape(-1).astype(np.uint8)
    assert np.array_equal(_diff_model(flat, W, lead), d.reshape(-1))
    assert np.array_equal(_undo_model(d.reshape(-1).astype(np.uint8), W, lead), E.reshape(-1))


# ---- learned path: the residual patch ----------------------------------------
KS_PX_PER_WG, PATCH_THREADS, PATCH_PAIRS = 32768, 1024, 8


@pytest.mark.parametrize("npx", [1, 2, 3, 63, 4095, 4097, 32767, 32768, 32769, 65535, 7 * 9, 3840 * 2160,
                                 4492 * 5989])
def test_resid_patch_covers_each_pixel_once(npx):
    """k_resid_patch: workgroup g of an image (ceil(npx / KS_PX_PER_WG) of
    them) takes the pixel pairs starting at g KS_PX_PER_WG + it 16384 +
    2 (j 1024 + lane) while they lie wholly below pe = npx rounded down to
    even; its 16-bit exponent loads start at an even offset clamped to pe - 2,
    so they stay 2-byte aligned and inside the plane; an odd image's last
    pixel goes to thread 0 of the workgroup that holds it.  Every pixel is
    taken exactly once, so the residual stores c npx + p stay inside the
    planes."""
    nwg = (npx + KS_PX_PER_WG - 1) // KS_PX_PER_WG
    pe = npx & ~1
    lanes = np.arange(PATCH_THREADS, dtype=np.int64)
    seen = np.zeros(npx, np.int32)
    step = 2 * PATCH_THREADS * PATCH_PAIRS
    for g in range(nwg):
        base = g * KS_PX_PER_WG + 2 * lanes
        for it in range(KS_PX_PER_WG // step):
            p0 = base + it * step
            live = p0 < pe
            if pe >= 2:
                for j in range(PATCH_PAIRS):
                    q = np.minimum(p0 + 2 * j * PATCH_THREADS, pe - 2)
                    assert (q % 2 == 0).all() and q.min() >= 0 and (q + 2).max() <= npx
            if not live.any():
                break
            for j in range(PATCH_PAIRS):
                p = p0[live] + 2 * j * PATCH_THREADS
                ok = p[p < pe]
                np.add.at(seen, ok, 1)
                np.add.at(seen, ok + 1, 1)
        if npx % 2 and (npx - 1) // KS_PX_PER_WG == g:
            seen[npx - 1] += 1
    assert (seen == 1).all()


@pytest.mark.parametrize("H,W", [(1, 1), (1, 2), (2, 3), (3, 5), (17, 129), (64, 66), (5, 1001)])
def test_learn_s_word_loads(H, W):
    """k_learn's S tile fetch: for every pixel, two dwords from the dword
    boundary at or below its first byte, byte-aligned by its offset, give
    its three bytes whenever those 8 bytes end inside S (S starts on a dword
    boundary); otherwise the three bytes are read one by one.  The two dword
    loads never touch a byte outside S."""
    rng = np.random.default_rng(H * 1000 + W)
    n = 3 * H * W
    S = rng.integers(0, 256, n, dtype=np.uint64)
    fast = 0
    for px in range(H * W):
        p = 3 * px
        sh = p & 3
        q = p - sh
        want = int(S[p]) | int(S[p + 1]) << 8 | int(S[p + 2]) << 16
        if q + 8 <= n:
            lo = sum(int(S[q + k]) << (8 * k) for k in range(4))
            hi = sum(int(S[q + 4 + k]) << (8 * k) for k in range(4))
            got = (((hi << 32) | lo) >> (8 * sh)) & 0xFFFFFF
            assert q >= 0 and got == want, (px, sh)
            fast += 1
    assert fast >= H * W - 3
