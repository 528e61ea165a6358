/*
 * rdl_ent_oracle.c -- CPU oracle for the entropy code of the enhancement layer.
 *
 * TEST INFRASTRUCTURE ONLY, under the same rules as rdl_oracle.c: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it, and it shares no code, header or constant with the HIP library.
 *
 * The paper hands the residual planes and the exponent plane to an
 * off-the-shelf lossless image coder (JPEG 2000; Sec. IV, the second and
 * third encoders).  This extension codes them instead with a static rANS
 * coder, the range variant of asymmetric numeral systems (J. Duda,
 * "Asymmetric numeral systems", arXiv:1311.2540, 2013, Sec. 3 and 4), with 64
 * interleaved coder states per group of symbols so that groups and lanes
 * code in parallel.  The format below is defined by this encoder/decoder pair
 * and by the public header's description of it.
 *
 * Coder (Duda's range variant with 16-bit renormalisation):
 *   M = 2^15 (probability scale), L = 2^16; a state x lies in [L, 2^32).
 *   Frequencies f[s] > 0 sum to M; c[s] = sum of f[t], t < s.
 *   Encode s:  while x >= 2^17 f[s]: emit x mod 2^16, x = x div 2^16
 *              (at most once), then x = (x div f[s]) M + (x mod f[s]) + c[s].
 *   Decode:    slot = x mod M, s = the symbol with c[s] <= slot < c[s]+f[s],
 *              x = f[s] (x div M) + slot - c[s], and while x < L:
 *              x = x 2^16 + next word.
 *
 * Planes: p = 0, 1, 2 hold the residuals r of channel R, G, B as symbols
 * r + 255 (511 symbols); p = 3 holds the exponent E (256 symbols).  Each
 * plane is N = H W symbols in raster order.
 *
 * Exponent prediction (flags bit 0): the shared exponent changes little from
 * one pixel to the next, so plane 3 may instead hold the difference from the
 * left neighbour, (E[y][x] - E[y][x-1]) mod 256, with E[y][x] itself at
 * x = 0.  The residual planes are always coded as they are: they are close to
 * white (the JPEG quantisation error of the base layer plus the estimator's),
 * and differencing them raises their entropy.
 *
 * Residual contexts (flags bit 1): the residual of channel p at pixel i is
 * coded with the table of its context k = S[i][p] >> 5 (k = 0..7), S being
 * the decoded base layer (8-bit SDRI, H W x 3, channel-interleaved), which the
 * decoder holds before it reads this layer.  The residuals' spread depends on
 * where the tone curve put the pixel (how many mantissa steps one SDRI step
 * spans there), so 8 tables per channel fit the data better than one.
 * Symbols of all contexts stay interleaved in the same groups and lanes; only
 * the table used for a symbol changes.  The exponent plane keeps one table.
 *
 * Frequencies of a table, from its counts h[s] (P symbols present, N = sum of
 * h, the symbols coded with that table):
 *   f[s] = 0 where h[s] = 0, else 1 + floor(h[s] (M - P) / N);
 *   then the smallest s with the largest count takes the remainder M - sum f.
 *   A context table with N = 0 (no pixel in that context) is all zero.
 *
 * Groups: K = 2^log2_k steps (4 <= log2_k <= 12); a plane is cut into
 * G = ceil(N / 64K) groups of 64K consecutive symbols (the last one shorter).  Symbol i of a group
 * belongs to lane i mod 64 at step i div 64.  The encoder starts every lane
 * at x = L, runs the steps from last to first, and within a step the lanes
 * from 63 down to 0 (a lane without a symbol at that step skips it); at the
 * end it emits every lane's state, lanes 63 down to 0, low half first.  A
 * group's stored words are this emission sequence reversed, so that a decoder
 * reads them in order: lane 0..63 states (high, low), then for each step
 * from the first, the words of the lanes that renormalise, in lane order.
 *
 * Stream (little-endian):
 *   0 u32 magic 0x454C4452   4 u32 version 1    8 i32 H       12 i32 W
 *  16 i32 log2_k            20 i32 prob_bits 15 24 u32 G      28 u32 flags (0..3)
 *  32 u64 total bytes       40 u16 freq[T][512]  (unused entries 0)
 *  D = 40 + 1024 T: u64 start[4][G]: first word of each group, counted from the payload
 *  D + 32 G: payload, u16 words, groups in plane-major order.
 * T = 4 tables (plane p's at p) without contexts, D = 4136; with contexts
 * T = 25 (channel p, context k at 8 p + k; the exponents' at 24), D = 25640.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ENT_PB 15
#define ENT_M (1u << ENT_PB)
#define ENT_L (1u << 16)
#define ENT_HDR 4136
#define ENT_HDR_CTX 25640
#define ENT_MAGIC 0x454C4452u
#define ENT_NCTX 8

static int64_t hdr_bytes(int flags) { return (flags & 2) ? ENT_HDR_CTX : ENT_HDR; }
static int n_tables(int flags) { return (flags & 2) ? 3 * ENT_NCTX + 1 : 4; }
static int table_nsym(int flags, int t) { return t == n_tables(flags) - 1 ? 256 : 511; }

/* Table of symbol i of plane p. */
static int table_of(const uint8_t *sdr, int flags, int p, int64_t i)
{
    if (!(flags & 2)) return p;
    if (p == 3) return 3 * ENT_NCTX;
    return ENT_NCTX * p + (sdr[3 * i + p] >> 5);
}

static void put32(uint8_t *p, uint32_t v) { for (int k = 0; k < 4; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put64(uint8_t *p, uint64_t v) { for (int k = 0; k < 8; k++) p[k] = (uint8_t)(v >> (8 * k)); }
static void put16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static uint32_t get32(const uint8_t *p) { uint32_t v = 0; for (int k = 3; k >= 0; k--) v = v << 8 | p[k]; return v; }
static uint64_t get64(const uint8_t *p) { uint64_t v = 0; for (int k = 7; k >= 0; k--) v = v << 8 | p[k]; return v; }
static uint32_t get16(const uint8_t *p) { return (uint32_t)p[0] | (uint32_t)p[1] << 8; }

/* Symbol i of plane p, or -1 when a residual lies outside [-255, 255]. */
static int plane_sym(const uint8_t *resid, int64_t N, int W, int flags, int p, int64_t i)
{
    if (p == 3) {
        const uint8_t *E = resid + 6 * N;
        if (!(flags & 1) || i % W == 0) return E[i];
        return (E[i] - E[i - 1]) & 255;
    }
    int16_t r;
    memcpy(&r, resid + 2 * (p * N + i), 2);
    return (r < -255 || r > 255) ? -1 : r + 255;
}

/* Quantised frequencies of one table (rule in the file header). */
int oracle_ent_freqs(const int64_t *h, int nsym, uint16_t *f)
{
    int64_t N = 0, P = 0;
    for (int s = 0; s < nsym; s++) {
        if (h[s] < 0) return -1;
        N += h[s];
        P += h[s] > 0;
    }
    if (N == 0) return -1;  /* callers handle an unused context table themselves */
    int64_t sum = 0;
    int best = 0;
    for (int s = 0; s < nsym; s++) {
        int64_t v = h[s] ? 1 + h[s] * ((int64_t)ENT_M - P) / N : 0;
        f[s] = (uint16_t)v;
        sum += v;
        if (h[s] > h[best]) best = s;
    }
    f[best] = (uint16_t)(f[best] + ((int64_t)ENT_M - sum));
    return 0;
}

int64_t oracle_ent_groups(int H, int W, int log2_k)
{
    int64_t z = (int64_t)64 << log2_k, N = (int64_t)H * W;
    return (N + z - 1) / z;
}

/* Largest stream of an H x W layer: every symbol renormalises once (flags
 * bit 1: the larger header of the context tables). */
int64_t oracle_ent_bound(int H, int W, int log2_k, int flags)
{
    if (H < 1 || W < 1 || log2_k < 4 || log2_k > 12) return -1;
    int64_t G = oracle_ent_groups(H, W, log2_k), N = (int64_t)H * W;
    return hdr_bytes(flags) + 32 * G + 2 * (4 * N + 4 * G * 128);
}

/* Encode the enhancement layer resid (int16 r[3][H][W], then uint8 E[H][W]);
 * flags bit 0 codes the exponents as left differences, bit 1 codes each
 * residual with the table of its context from sdr (the decoded base layer,
 * H W x 3 bytes; unused otherwise).  Returns the stream length, -1 for bad
 * arguments, -2 when cap is too small, -3 when a residual lies outside
 * [-255, 255]. */
int64_t oracle_ent_encode(const void *resid_v, const uint8_t *sdr, int H, int W, int log2_k, int flags, uint8_t *out,
                          int64_t cap)
{
    const uint8_t *resid = (const uint8_t *)resid_v;
    if (!resid || !out || H < 1 || W < 1 || log2_k < 4 || log2_k > 12 || (flags & ~3) || ((flags & 2) && !sdr))
        return -1;
    const int64_t N = (int64_t)H * W, Z = (int64_t)64 << log2_k, G = oracle_ent_groups(H, W, log2_k);
    const int64_t D = hdr_bytes(flags);
    const int NT = n_tables(flags);
    if (cap < oracle_ent_bound(H, W, log2_k, flags)) return -2;
    memset(out, 0, D + 32 * G);
    int64_t h[3 * ENT_NCTX + 1][512];
    uint16_t f[3 * ENT_NCTX + 1][512];
    uint32_t c[3 * ENT_NCTX + 1][512];
    memset(h, 0, sizeof h);
    memset(f, 0, sizeof f);
    for (int p = 0; p < 4; p++)
        for (int64_t i = 0; i < N; i++) {
            int s = plane_sym(resid, N, W, flags, p, i);
            if (s < 0) return -3;
            h[table_of(sdr, flags, p, i)][s]++;
        }
    for (int t = 0; t < NT; t++) {
        int64_t n = 0;
        for (int s = 0; s < 512; s++) n += h[t][s];
        if (n && oracle_ent_freqs(h[t], table_nsym(flags, t), f[t])) return -1;
        uint32_t run = 0;
        for (int s = 0; s < 512; s++) {
            c[t][s] = run;
            run += f[t][s];
            put16(out + 40 + 2 * (512 * t + s), f[t][s]);
        }
    }
    uint16_t *emit = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(Z + 128));
    if (!emit) return -4;
    uint8_t *payload = out + D + 32 * G;
    int64_t words = 0;
    for (int p = 0; p < 4; p++) {
        for (int64_t g = 0; g < G; g++) {
            const int64_t base = g * Z, n = (N - base < Z) ? N - base : Z, T = (n + 63) / 64;
            uint32_t x[64];
            for (int j = 0; j < 64; j++) x[j] = ENT_L;
            int64_t ne = 0;
            for (int64_t t = T - 1; t >= 0; t--) {
                for (int j = 63; j >= 0; j--) {
                    const int64_t i = t * 64 + j;
                    if (i >= n) continue;
                    const int s = plane_sym(resid, N, W, flags, p, base + i);
                    const int tb = table_of(sdr, flags, p, base + i);
                    const uint32_t fs = f[tb][s];
                    if ((uint64_t)x[j] >= ((uint64_t)fs << 17)) {
                        emit[ne++] = (uint16_t)(x[j] & 0xFFFF);
                        x[j] >>= 16;
                    }
                    x[j] = (x[j] / fs) * ENT_M + (x[j] % fs) + c[tb][s];
                }
            }
            for (int j = 63; j >= 0; j--) {
                emit[ne++] = (uint16_t)(x[j] & 0xFFFF);
                emit[ne++] = (uint16_t)(x[j] >> 16);
            }
            put64(out + D + 8 * (p * G + g), (uint64_t)words);
            for (int64_t k = 0; k < ne; k++) put16(payload + 2 * (words + k), emit[ne - 1 - k]);
            words += ne;
        }
    }
    free(emit);
    const int64_t total = D + 32 * G + 2 * words;
    put32(out + 0, ENT_MAGIC);
    put32(out + 4, 1);
    put32(out + 8, (uint32_t)H);
    put32(out + 12, (uint32_t)W);
    put32(out + 16, (uint32_t)log2_k);
    put32(out + 20, ENT_PB);
    put32(out + 24, (uint32_t)G);
    put32(out + 28, (uint32_t)flags);
    put64(out + 32, (uint64_t)total);
    return total;
}

/* Decode a stream into resid (7 H W bytes); sdr (the decoded base layer)
 * is needed when the stream has flags bit 1.  Returns 0, or a negative code:
 * -1 bad arguments, -5 header mismatch, -6 corrupt group data (including a
 * symbol whose context table is empty). */
int oracle_ent_decode(const uint8_t *st, int64_t len, const uint8_t *sdr, int H, int W, void *resid_v)
{
    uint8_t *resid = (uint8_t *)resid_v;
    if (!st || !resid || H < 1 || W < 1 || len < 40) return -1;
    const int log2_k = (int)get32(st + 16);
    if (get32(st) != ENT_MAGIC || get32(st + 4) != 1 || (int)get32(st + 8) != H || (int)get32(st + 12) != W ||
        log2_k < 4 || log2_k > 12 || get32(st + 20) != ENT_PB)
        return -5;
    const uint32_t flags = get32(st + 28);
    if (flags > 3) return -5;
    if ((flags & 2) && !sdr) return -1;
    const int64_t D = hdr_bytes((int)flags);
    const int NT = n_tables((int)flags);
    if (len < D) return -5;
    const int64_t N = (int64_t)H * W, Z = (int64_t)64 << log2_k, G = oracle_ent_groups(H, W, log2_k);
    const int64_t total = (int64_t)get64(st + 32);
    if (get32(st + 24) != (uint32_t)G || total > len || total < D + 32 * G || (total - D - 32 * G) % 2)
        return -5;
    const int64_t nwords = (total - D - 32 * G) / 2;
    uint32_t f[3 * ENT_NCTX + 1][512], c[3 * ENT_NCTX + 1][513];
    for (int t = 0; t < NT; t++) {
        uint32_t run = 0;
        for (int s = 0; s < 512; s++) {
            f[t][s] = get16(st + 40 + 2 * (512 * t + s));
            if (s >= table_nsym((int)flags, t) && f[t][s]) return -5;
            c[t][s] = run;
            run += f[t][s];
        }
        c[t][512] = run;
        /* the exponents' table is always used; a context table may be empty */
        if (run != ENT_M && !(run == 0 && t < NT - 1 && (flags & 2))) return -5;
    }
    const uint8_t *payload = st + D + 32 * G;
    for (int p = 0; p < 4; p++) {
        for (int64_t g = 0; g < G; g++) {
            const int64_t k = p * G + g;
            const int64_t w0 = (int64_t)get64(st + D + 8 * k);
            const int64_t w1 = k + 1 < 4 * G ? (int64_t)get64(st + D + 8 * (k + 1)) : nwords;
            if (w0 < 0 || w1 > nwords || w1 - w0 < 128) return -6;
            const int64_t base = g * Z, n = (N - base < Z) ? N - base : Z, T = (n + 63) / 64;
            int64_t pos = w0;
            uint32_t x[64];
            for (int j = 0; j < 64; j++) {
                x[j] = get16(payload + 2 * pos) << 16 | get16(payload + 2 * (pos + 1));
                pos += 2;
            }
            for (int64_t t = 0; t < T; t++) {
                for (int j = 0; j < 64; j++) {
                    const int64_t i = t * 64 + j;
                    if (i >= n) continue;
                    const int tb = table_of(sdr, (int)flags, p, base + i);
                    if (c[tb][512] != ENT_M) return -6;
                    const uint32_t slot = x[j] % ENT_M;
                    int s = 0;
                    while (c[tb][s + 1] <= slot) s++;
                    x[j] = f[tb][s] * (x[j] / ENT_M) + slot - c[tb][s];
                    if (x[j] < ENT_L) {
                        if (pos >= w1) return -6;
                        x[j] = x[j] << 16 | get16(payload + 2 * pos);
                        pos++;
                    }
                    const int64_t at = base + i;
                    if (p == 3) {
                        resid[6 * N + at] = (uint8_t)s;
                    } else {
                        const int16_t r = (int16_t)(s - 255);
                        memcpy(resid + 2 * (p * N + at), &r, 2);
                    }
                }
            }
            if (pos != w1) return -6;
            for (int j = 0; j < 64; j++)
                if (x[j] != ENT_L) return -6;
        }
    }
    if (flags & 1) {  /* undo the left differences, row by row */
        uint8_t *E = resid + 6 * N;
        for (int64_t i = 0; i < N; i++)
            if (i % W) E[i] = (uint8_t)(E[i - 1] + E[i]);
    }
    return 0;
}
