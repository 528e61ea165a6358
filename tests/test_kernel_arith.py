"""CPU checks of integer identities the HIP kernels rely on, written out here
with numpy (no GPU, no oracle): each kernel form must equal the plain
definition on every input it can receive."""
import numpy as np
import pytest

AQ_MAX = 255 << 22
BQ_MIN, BQ_MAX = -65025 << 14, 65280 << 14


def mstar_def(aq, bq, s):
    """Eq. 8 with the fixed-point coefficients: clamp(floor((a_q s + 2^8 b_q + 2^21) / 2^22), 0, 255)."""
    v = (aq.astype(np.int64) * s + bq.astype(np.int64) * 256 + (1 << 21)) >> 22
    return np.clip(v, 0, 255)


def mstar_kernel(aq, bq, s):
    """The residual kernel's 32-bit form: x = ah (low 24 bits, signed) | al << 24,
    y = b_q + 2^13; v = mul_i24(x, s) + y; u = (al s) >> 8; clamp((v + u) >> 14)."""
    aq = aq.astype(np.int64)
    ah = aq >> 8
    al = aq & 255
    x = (ah & 0xFFFFFF) | (al << 24)
    x24 = ((x & 0xFFFFFF) ^ 0x800000) - 0x800000          # sign-extend bits 0..23
    v = x24 * s + (bq.astype(np.int64) + 8192)
    assert np.all(np.abs(v) < 2 ** 31), "32-bit overflow"
    u = (((x >> 24) & 255) * s) >> 8
    t = v + u
    assert np.all(np.abs(t) < 2 ** 31)
    return np.clip(t >> 14, 0, 255)


def test_mstar_32bit_form_equals_definition():
    rng = np.random.default_rng(7)
    edges_a = np.array([-AQ_MAX, -AQ_MAX + 1, -(1 << 22), -255, -1, 0, 1, 255, 256, 1 << 22, AQ_MAX - 1, AQ_MAX])
    edges_b = np.array([BQ_MIN, BQ_MIN + 1, -(1 << 14), -1, 0, 1, 8191, 8192, 1 << 14, BQ_MAX - 1, BQ_MAX])
    s = np.arange(256, dtype=np.int64)[None, :]
    A, B = np.meshgrid(edges_a, edges_b, indexing="ij")
    A, B = A.reshape(-1, 1), B.reshape(-1, 1)
    assert np.array_equal(mstar_kernel(A, B, s), mstar_def(A, B, s))
    A = rng.integers(-AQ_MAX, AQ_MAX + 1, (4000, 1))
    B = rng.integers(BQ_MIN, BQ_MAX + 1, (4000, 1))
    assert np.array_equal(mstar_kernel(A, B, s), mstar_def(A, B, s))
    # near the rounding boundaries: a_q s + 2^8 b_q + 2^21 = k 2^22 + {-1, 0, 1}
    A = rng.integers(-AQ_MAX, AQ_MAX + 1, (4000, 1))
    S = rng.integers(0, 256, (4000, 1))
    K = rng.integers(-200, 400, (4000, 1))
    for off in (-1, 0, 1):
        Bn = (K * (1 << 22) + off - (1 << 21) - A * S) // 256
        keep = (Bn >= BQ_MIN) & (Bn <= BQ_MAX)
        a, b = A[keep][:, None], Bn[keep][:, None]
        assert np.array_equal(mstar_kernel(a, b, s), mstar_def(a, b, s))


def test_mstar_regression_lines_through_pixels():
    """Coefficients as the solve makes them (least-squares lines through
    8-bit data) stay within the kernel's bounds."""
    rng = np.random.default_rng(11)
    for _ in range(2000):
        n = int(rng.integers(2, 40))
        sv = rng.integers(0, 256, n)
        mv = rng.integers(0, 256, n)
        num = n * int((sv * mv).sum()) - int(sv.sum()) * int(mv.sum())
        den = n * int((sv * sv).sum()) - int(sv.sum()) ** 2
        if den == 0:
            continue
        aq = (2 * (num << 22) + den) // (2 * den)
        bq = (2 * ((int(mv.sum()) << 22) - aq * int(sv.sum())) + 256 * n) // (2 * 256 * n)
        assert -AQ_MAX <= aq <= AQ_MAX and BQ_MIN <= bq <= BQ_MAX


def test_gf_packed_fields_never_carry():
    """The GF adds (1,6,1) x (1,6,1) weighted 8-bit values in 16-bit lanes:
    the largest sum, 64 * 255 + 32, stays below 2^16, and >> 6 of it is 255."""
    top = 64 * 255 + 32
    assert top < 1 << 16 and top >> 6 == 255


# ---------------------------------------------------------------------------
# Base layer: bound of the quantiser's input and its signed magic-multiplier form.
def dct_basis():
    """K[u][x] = round(2^13 c_u cos((2x + 1) u pi / 16)), c_0 = 1/sqrt(8), else 1/2."""
    import math
    return np.array([[round(8192 * (math.sqrt(1 / 8) if u == 0 else 0.5) * math.cos((2 * x + 1) * u * math.pi / 16))
                      for x in range(8)] for u in range(8)], dtype=np.int64)


def test_quantiser_input_bound():
    """f = F >> 15 of the integer FDCT (row pass (T + 2^10) >> 11, column pass
    + 2^14) stays within +-1024 for every 8x8 block of level-shifted samples in
    [-128, 128] (Y - 128 reaches 127, Cb - 128 and Cr - 128 reach 128).  Rows
    are independent inputs and both passes are monotone in them, so each
    column's extremes come from sign patterns: the maximum below is exact."""
    K = dct_basis()
    lo, hi = -128, 128
    best = 0
    for u in range(8):
        tmax = (int((K[u] * np.where(K[u] > 0, hi, lo)).sum()) + 1024) >> 11
        tmin = (int((K[u] * np.where(K[u] > 0, lo, hi)).sum()) + 1024) >> 11
        for v in range(8):
            fmax = (sum(int(K[v][y]) * (tmax if K[v][y] > 0 else tmin) for y in range(8)) + 16384) >> 15
            fmin = (sum(int(K[v][y]) * (tmin if K[v][y] > 0 else tmax) for y in range(8)) + 16384) >> 15
            best = max(best, abs(fmax), abs(fmin))
    assert best == 1024
    # brute force on random blocks never exceeds it
    rng = np.random.default_rng(3)
    X = rng.integers(lo, hi + 1, (2000, 8, 8))
    T = (np.einsum("ux,byx->byu", K, X) + 1024) >> 11
    F = (np.einsum("vy,byu->bvu", K, T) + 16384) >> 15
    assert np.abs(F).max() <= 1024


def test_quantiser_signed_magic_form_equals_definition():
    """sign(f) floor((|f| + h) / Q) == (a M + 2^11) >> 20 with a = f + h - e,
    e = [f < 0 and Q even], M = ceil(2^20 / Q), h = floor(Q / 2): every Q in
    [1, 255], every f in [-1024, 1024]; a and M fit the 24-bit multiplier and
    the sum 32 bits."""
    f = np.arange(-1024, 1025, dtype=np.int64)
    for Q in range(1, 256):
        h, M = Q // 2, ((1 << 20) + Q - 1) // Q
        ref = np.sign(f) * ((np.abs(f) + h) // Q)
        a = f + h - ((f < 0) & (Q % 2 == 0))
        assert np.abs(a).max() < 1 << 23 and M < 1 << 23
        t = a * M + 2048
        assert np.abs(t).max() < 1 << 31
        assert np.array_equal(t >> 20, ref), Q


def test_entropy_quotient_from_float_reciprocal():
    """The entropy encoder divides a state x in [2 f, 2^17 f) by a frequency f in
    [1, 2^15] as q = trunc(fl(fl(x) * r)), r = fl(1/f) lowered by 4 ulps, and
    one upward correction (IEEE single rounding, which numpy's float32
    follows).  The estimate never exceeds x / f and falls short by less than
    1, for every f with quotients spread over [2, 2^17) and remainders 0, 1,
    f/2, f - 1 and random ones; q and x - q f are then x div f and x mod f."""
    rng = np.random.default_rng(11)
    f = np.arange(1, (1 << 15) + 1, dtype=np.int64)
    ks = np.concatenate([[2, 3, 255, 256, 65535, 65536, (1 << 17) - 2, (1 << 17) - 1],
                         rng.integers(2, 1 << 17, 40)])
    rcp = (np.float32(1.0) / f.astype(np.float32)).astype(np.float32)
    rcp = (rcp.view(np.uint32) - 4).view(np.float32)
    for k in ks:
        for rem in (np.zeros_like(f), np.ones_like(f) % f, f // 2, f - 1, rng.integers(0, 1 << 15, f.size) % f):
            x = k * f + rem
            assert np.all((x >= 2 * f) & (x < (f << 17)) & (x < 2 ** 32))
            est = x.astype(np.float32) * rcp
            short = x / f - est.astype(np.float64)
            assert np.all(short >= 0) and np.all(short < 0.11)
            q = np.trunc(est).astype(np.int64)
            r = x - q * f
            assert np.all(r >= 0) and np.all(r < 2 * f) and np.all(r < 1 << 24)
            up = r >= f
            q = np.where(up, q + 1, q)
            r = np.where(up, r - f, r)
            assert np.array_equal(q, x // f) and np.array_equal(r, x % f)


def test_learned_output_rounding_fold():
    """The estimator's output step in one shift: for every accepted r3 (1..22)
    and multiplier, floor((floor((o m3 + 2^(r3-1)) / 2^r3) + 128) / 2^8) equals
    floor((o m3 + 2^(r3-1) + 2^(r3+7)) / 2^(r3+8)), and the folded numerator
    stays inside int32 for every o the model format allows
    (|o| <= 32 * 127 * 255 + 2^18, multipliers below 2^10)."""
    rng = np.random.default_rng(5)
    omax = 32 * 127 * 255 + (1 << 18)
    for r3 in range(1, 23):
        for m3 in (1, 2, 777, 1023):
            o = np.concatenate([rng.integers(-omax, omax + 1, 20000), [-omax, omax, 0, -1, 1]]).astype(np.int64)
            num = o * m3 + (1 << (r3 - 1))
            two_step = ((num >> r3) + 128) >> 8
            folded_num = num + (1 << (r3 + 7))
            assert np.array_equal(two_step, folded_num >> (r3 + 8)), (r3, m3)
            assert folded_num.max() < 2 ** 31 and folded_num.min() >= -2 ** 31, (r3, m3)
    # r3 = 23 would overflow at the bound: the library rejects it
    assert omax * 1023 + (1 << 22) + (1 << 30) >= 2 ** 31


def test_learned_general_requant_in_int32():
    """General multipliers: h m + 2^(r-1) stays inside int32 for every
    pre-activation the model format allows (|h| <= 32 * 127 * 255 + 2^18 in
    layer 2, less in layer 1), multiplier below 2^10 and shift up to 28; at
    multipliers up to 2^11 (the first format version's limit) it would not."""
    hmax = 32 * 127 * 255 + (1 << 18)
    assert hmax * 1023 + (1 << 27) < 2 ** 31
    assert hmax * 2047 >= 2 ** 31


def test_learned_offset_inputs():
    """Activations a in [0, 255] enter the next layer's signed-byte MFMA as
    a - 128 = a XOR 0x80, and the bias carried as b + 128 sum_k W[k] makes the
    product exact: sum_k W[k] (a_k - 128) + b + 128 sum_k W[k] = sum_k W[k] a_k
    + b, for random rows and activations including 0 and 255."""
    rng = np.random.default_rng(8)
    W = rng.integers(-127, 128, (200, 32)).astype(np.int64)
    a = rng.integers(0, 256, (200, 32)).astype(np.int64)
    a[0], a[1] = 0, 255
    b = rng.integers(-(1 << 18), (1 << 18) + 1, 200)
    signed = ((a ^ 0x80).astype(np.uint8)).view(np.int8).astype(np.int64)
    assert np.array_equal(signed, a - 128)
    lhs = (W * signed).sum(axis=1) + b + 128 * W.sum(axis=1)
    assert np.array_equal(lhs, (W * a).sum(axis=1) + b)


def test_learned_pow2_bias_fold():
    """With a hidden multiplier of 1 the rounding constant and the input offset
    of the next layer move into the bias: for every shift the power-of-two
    paths accept (r <= 22), clamp((h + 2^(r-1)) >> r, 0, 255) - 128 equals
    clamp((h + 2^(r-1) - 2^(r+7)) >> r, -128, 127), and the folded value stays
    inside int32 for every accepted bias; the pair path's one instruction
    (shift two values, saturate to int8, pack) gives the same bytes."""
    rng = np.random.default_rng(6)
    hmax = 32 * 127 * 128 + 128 * 32 * 127 + (1 << 18)
    for r in range(1, 23):
        h = np.concatenate([rng.integers(-hmax, hmax + 1, 5000),
                            (np.arange(-300, 300) << r) + rng.integers(-2, 3, 600)]).astype(np.int64)
        a = np.clip((h + (1 << (r - 1))) >> r, 0, 255)
        folded = h + (1 << (r - 1)) - (1 << (r + 7))
        assert np.array_equal(a - 128, np.clip(folded >> r, -128, 127)), r
        assert np.abs(folded).max() < 2 ** 31 and hmax + (1 << (r + 7)) < 2 ** 31, r
        # the packed pair: low byte from the first value, high from the second
        x, y = folded[0::2][:2500], folded[1::2][:2500]
        pk = (np.clip(x >> r, -128, 127) & 255) | ((np.clip(y >> r, -128, 127) & 255) << 8)
        assert np.array_equal(pk & 255, (a[0::2][:2500] - 128) & 255)
        assert np.array_equal(pk >> 8, (a[1::2][:2500] - 128) & 255)


# ---------------------------------------------------------------------------
# The context decoder's symbol lookup (k_ent_dec_ctx): per table the present
# symbols' first slots c (with M after the last), a bucket index per 16 slots
# marked by the last symbol whose c rounds up to the bucket, then a prefix
# maximum; a binary search between a bucket's entry and the next one.
def _ctx_tables(f):
    M = 1 << 15
    P = len(f)
    c = np.concatenate([[0], np.cumsum(f)[:-1]])
    pc = np.concatenate([c, [M]])
    bk = np.zeros(2048, np.int64)
    for j in range(P):
        b = (int(c[j]) + 15) >> 4
        if b < 2048 and ((int(c[j] + f[j]) + 15) >> 4) != b:
            bk[b] = j
    return pc, np.maximum.accumulate(bk)


@pytest.mark.parametrize("kind", ["flat", "peaked", "ones", "single"])
def test_context_decoder_lookup_finds_the_holder(kind):
    """For every slot the search stays inside the table (at most 17
    candidates, so 5 halvings) and ends at the symbol whose range holds it."""
    M = 1 << 15
    rng = np.random.default_rng(len(kind))
    if kind == "flat":
        h = rng.integers(1, 120, 400)
    elif kind == "peaked":
        h = np.maximum(1, (rng.laplace(0, 1, 300) ** 2 * 200).astype(np.int64))
    elif kind == "ones":
        h = np.ones(511, np.int64)
    else:
        h = np.array([12345])
    # present symbols' frequencies by the stream's rule: 1 + floor(h (M - P) / N),
    # the remainder to the largest count
    h = h.astype(np.int64)
    f = 1 + h * (M - len(h)) // h.sum()
    f[int(np.argmax(h))] += M - f.sum()
    assert f.min() >= 1 and f.sum() == M
    pc, bk = _ctx_tables(f)
    P = len(f)
    holder = np.searchsorted(pc[:-1], np.arange(M), side="right") - 1
    for slot in range(M):
        bb = slot >> 4
        lo, hi = int(bk[bb]), int(bk[bb + 1]) if bb < 2047 else P - 1
        assert 0 <= lo <= hi <= P - 1 and hi - lo <= 16
        while lo < hi:
            mid = (lo + hi + 1) >> 1
            if pc[mid] <= slot:
                lo = mid
            else:
                hi = mid - 1
        assert lo == holder[slot] and pc[lo] <= slot < pc[lo + 1]
