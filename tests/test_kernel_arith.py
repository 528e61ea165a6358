"""CPU checks of integer identities the HIP kernels rely on, written out here
with numpy (no GPU, no oracle): each kernel form must equal the plain
definition on every input it can receive."""
import numpy as np

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
    (|o| <= 32 * 127 * 127 + 2^18)."""
    rng = np.random.default_rng(5)
    omax = 32 * 127 * 127 + (1 << 18)
    for r3 in range(1, 23):
        for m3 in (1, 2, 777, 2047):
            o = np.concatenate([rng.integers(-omax, omax + 1, 20000), [-omax, omax, 0, -1, 1]]).astype(np.int64)
            num = o * m3 + (1 << (r3 - 1))
            two_step = ((num >> r3) + 128) >> 8
            folded_num = num + (1 << (r3 + 7))
            assert np.array_equal(two_step, folded_num >> (r3 + 8)), (r3, m3)
            assert folded_num.max() < 2 ** 31 and folded_num.min() >= -2 ** 31, (r3, m3)
    # r3 = 23 would overflow at the bound: the library rejects it
    assert omax * 2047 + (1 << 22) + (1 << 30) >= 2 ** 31


def test_learned_pow2_bias_fold():
    """With a hidden multiplier of 1 the rounding constant moves into the bias:
    (h m + 2^(r-1)) >> r = (h' ) >> r with h' = h + 2^(r-1), and h' stays inside
    int32 for every accepted bias and shift."""
    rng = np.random.default_rng(6)
    hmax = 27 * 128 * 127 + (1 << 18)
    for r in range(1, 29):
        h = rng.integers(-hmax, hmax + 1, 5000).astype(np.int64)
        assert np.array_equal((h * 1 + (1 << (r - 1))) >> r, (h + (1 << (r - 1))) >> r)
        assert hmax + (1 << (r - 1)) < 2 ** 31


def test_learned_packed_requantisation():
    """The 16-bit packed requantisation: for every shift r <= 8, saturating the
    pre-activation to int16 before the shift leaves clamp(h >> r, 0, 127)
    unchanged, over the whole range the model format allows (|h| < 2^31 after
    the rounding constant), and every pair of shifts fits the packed operand;
    at r = 9 the saturation would change it."""
    hs = np.concatenate([np.arange(-70000, 70000), np.array([-2 ** 31, 2 ** 31 - 1, -2 ** 20, 2 ** 20])]).astype(np.int64)
    sat = np.clip(hs, -32768, 32767)
    for r in range(1, 9):
        assert np.array_equal(np.clip(hs >> r, 0, 127), np.clip(sat >> r, 0, 127)), r
    assert not np.array_equal(np.clip(hs >> 9, 0, 127), np.clip(sat >> 9, 0, 127))
