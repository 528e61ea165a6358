"""Pins of the oracle's base-layer JPEG writer (baseline sequential, ITU-T
T.81, JFIF): an independent decoder (libjpeg through Pillow) reads every file
back to within a few codes of the normative base layer S, the quantisation
tables it reads equal the writer's, and the Huffman tables of Annex K.2 cost
what an optimal prefix code with the reserved code point costs, never exceed
16 bits and leave the all-ones code unused."""
import heapq
import io
import itertools

import numpy as np
import pytest

from paper_2309_11072_amd import synth

PIL = pytest.importorskip("PIL.Image")


def base_layer(O, H, W, q, seed):
    x = synth.generate(H, W, 3.5, seed=seed, spec_frac=0.05)
    lam, n = O.keystat(x)
    kp = O.key_params(lam, n)
    s0 = O.tmo(x, kp[0], kp[2], n)
    return O.base_layer(s0, q, want_dct=True)


@pytest.mark.parametrize("H,W,q", [(1, 1, 75), (7, 9, 50), (8, 8, 100), (61, 83, 90), (217, 301, 1), (129, 257, 30)])
def test_libjpeg_decodes_the_file(O, H, W, q):
    """libjpeg's decoder (its own IDCT and colour conversion, rounding
    differently from the normative integer path) returns the base layer within
    3 codes, 0.5 on average; one wrong bit would desynchronise the scan."""
    S, dct = base_layer(O, H, W, q, H * 7 + W)
    jp = O.jpeg_write(dct, H, W, q)
    im = PIL.open(io.BytesIO(jp))
    im.load()
    assert im.format == "JPEG" and im.size == (W, H) and im.mode == "RGB"
    d = np.abs(np.asarray(im.convert("RGB")).astype(int) - S.astype(int))
    assert d.max() <= 3 and d.mean() <= 0.5


def test_quantisation_tables_read_back(O):
    H, W, q = 40, 48, 65
    S, dct = base_layer(O, H, W, q, 5)
    im = PIL.open(io.BytesIO(O.jpeg_write(dct, H, W, q)))
    qt = im.quantization
    for t in (0, 1):
        want = O.quant_table(q, bool(t)).reshape(-1)
        got = np.array(qt[t]).reshape(-1)
        # Pillow lists a table in natural order (it undoes the file's zig-zag)
        assert np.array_equal(np.sort(got), np.sort(want)) and np.array_equal(got, want)


def test_file_structure(O):
    """Markers in order: SOI, APP0 (JFIF), DQT, SOF0, DHT, SOS x 3 with their
    component and table selectors, EOI."""
    H, W, q = 30, 50, 80
    _, dct = base_layer(O, H, W, q, 9)
    jp = O.jpeg_write(dct, H, W, q)
    assert jp[:2] == b"\xff\xd8" and jp[-2:] == b"\xff\xd9" and jp[6:11] == b"JFIF\x00"
    pos, seen, sos = 2, [], []
    while True:
        m = jp[pos:pos + 2]
        assert m[0] == 0xFF
        if m[1] == 0xD9:
            break
        ln = int.from_bytes(jp[pos + 2:pos + 4], "big")
        seen.append(m[1])
        if m[1] == 0xC0:
            assert jp[pos + 4] == 8 and int.from_bytes(jp[pos + 5:pos + 7], "big") == H
            assert int.from_bytes(jp[pos + 7:pos + 9], "big") == W and jp[pos + 9] == 3
        if m[1] == 0xDA:
            sos.append((jp[pos + 5], jp[pos + 6]))
            pos += 2 + ln
            while not (jp[pos] == 0xFF and jp[pos + 1] not in (0x00,)):  # entropy-coded data
                pos += 2 if jp[pos] == 0xFF else 1
            continue
        pos += 2 + ln
    assert seen == [0xE0, 0xDB, 0xC0, 0xC4, 0xDA, 0xDA, 0xDA]
    assert sos == [(1, 0x00), (2, 0x11), (3, 0x11)]


def _code_lengths(bits, huffval):
    lens = {}
    k = 0
    for L, cnt in enumerate(bits, start=1):
        for _ in range(int(cnt)):
            lens[int(huffval[k])] = L
            k += 1
    return lens


def _optimal_cost(freqs):
    """Cost of an optimal binary prefix code (heap Huffman), no length limit."""
    if len(freqs) == 1:
        return freqs[0]
    h = list(freqs)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(8))
def test_huffman_table_is_optimal_with_the_reserved_point(O, seed):
    """Annex K.2 adds a symbol of count 1 (the all-ones code point) and builds
    a Huffman code: with no length above 16 its cost over the real symbols is
    an optimal code's cost for counts + {1} minus the reserved symbol's part."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 40))
    freq = np.zeros(256, np.int64)
    syms = rng.choice(256, k, replace=False)
    freq[syms] = rng.integers(1, 5000, k)
    bits, hv = O.jpeg_huff_table(freq)
    lens = _code_lengths(bits, hv)
    assert sorted(lens) == sorted(int(s) for s in syms)
    assert max(lens.values()) <= 16
    kraft = sum(2.0 ** -L for L in lens.values())
    assert kraft < 1.0  # the all-ones code of the longest length stays free
    cost = sum(int(freq[s]) * L for s, L in lens.items())
    # The reserved symbol takes one of the longest codes; with it the code is complete.
    Lmax = max(lens.values())
    assert cost + Lmax == _optimal_cost([int(f) for f in freq[syms]] + [1])


def test_huffman_lengths_are_limited_to_16(O):
    """Counts 1, 2, 4, ..., 2^23 make an unlimited Huffman code a chain 24 bits
    deep; Figure K.3 limits it to 16 and the code stays prefix-free with every
    symbol coded."""
    freq = np.zeros(256, np.int64)
    freq[:24] = 2 ** np.arange(24)
    bits, hv = O.jpeg_huff_table(freq)
    lens = _code_lengths(bits, hv)
    assert len(lens) == 24 and max(lens.values()) == 16
    assert sum(2.0 ** -L for L in lens.values()) < 1.0


def test_code_sizes_above_32_are_listed(O):
    """Counts 1, 2, 4, ..., 2^39 (40 symbols; with the reserved point each
    merge joins the chain to the next symbol) make Figure K.1's code sizes
    run to 40, past 32, where Figure K.2's arrays end; with the histogram and
    Figure K.3 extended to the longest size every symbol is listed once, with
    a code of at most 16 bits, and the code stays prefix-free."""
    freq = np.zeros(256, np.int64)
    freq[:40] = 2 ** np.arange(40, dtype=np.int64)
    bits, hv = O.jpeg_huff_table(freq)
    lens = _code_lengths(bits, hv)
    assert sorted(lens) == list(range(40)) and max(lens.values()) <= 16
    assert sum(2.0 ** -L for L in lens.values()) < 1.0


def test_codes_are_canonical_and_prefix_free(O):
    rng = np.random.default_rng(3)
    freq = np.zeros(256, np.int64)
    freq[rng.choice(256, 60, replace=False)] = rng.integers(1, 100, 60)
    bits, hv = O.jpeg_huff_table(freq)
    lens = _code_lengths(bits, hv)
    codes, c, k = {}, 0, 0
    for L, cnt in enumerate(bits, start=1):
        for _ in range(int(cnt)):
            codes[int(hv[k])] = format(c, "0%db" % L)
            c += 1
            k += 1
        c <<= 1
    for a, b in itertools.permutations(codes.values(), 2):
        assert not b.startswith(a)
    assert all(set(cw) != {"1"} or len(cw) < 16 for cw in codes.values())
    assert len(codes) == len(lens)
