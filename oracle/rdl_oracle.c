/*
 * rdl_oracle.c -- CPU oracle for the encoder of Suzuki et al., "Lightning-Fast
 * Dual-Layer Lossless Coding for Radiance Format HDR Images" (arXiv 2309.11072).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, scalar reference
 * that the GPU path is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the HIP library: every table below
 * is computed here, from its defining formula, at first use.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (float stays float on x86-64 SSE, FLT_EVAL_METHOD == 0; no FMA contraction).
 * `>>` on a negative signed integer is an arithmetic (floor) shift in gcc.
 *
 * Stages (each function names the passage it follows):
 *   C1  RGBE pixel unpack                     Sec. II.A, Fig. 1 caption
 *   C2  key statistic (log-average luminance) Sec. IV (Reinhard TMO), reading
 *   C3  TMO per pixel, Eq. 3 mantissa centre  Sec. II.A Eq. 3, Sec. IV
 *   C4  gamma + 8-bit quantisation            Sec. IV (silent) -> threshold count
 *   C5-C9 JPEG-style base layer round trip     Sec. II.B, Sec. IV (JPEG, Q)
 *   C10 Gaussian-filter restoration           Sec. III.B (GF pre-processing)
 *   C11 per-(channel, exponent) sums           Sec. III.B, Eq. 9-10
 *   C12 fixed-point coefficient solve          Sec. II.C Eq. 6-7, Sec. III.B-C
 *   C13 estimate + residual                    Sec. III.B Eq. 8
 *   C14 decode                                 Sec. I, Sec. III.C
 *   C15 residual zeroth-order entropy          (metric; not in the paper)
 *   C16 learned int8 estimator                 (extension; not in the paper)
 * Where the paper is silent the reading taken is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* Frozen tables, each computed from its formula in float64.                 */
/* ------------------------------------------------------------------------ */
static int32_t LOG2F[4096];  /* round(2^16 * log2(1 + (i + 0.5)/4096))       */
static float EXP2H[256];     /* fl32(2^(j/256))                              */
static float EXP2L[256];     /* fl32(2^(j/65536))                            */
static float TGAM[256];      /* TGAM[k] = fl32(((k - 0.5)/255)^2.2), k>=1    */
static int32_t KDCT[8][8];   /* round(2^13 * c_u * cos((2x+1) u pi / 16))    */
static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < 4096; i++)
        LOG2F[i] = (int32_t)llround(65536.0 * log2(1.0 + (i + 0.5) / 4096.0));
    for (int j = 0; j < 256; j++) {
        EXP2H[j] = (float)exp2(j / 256.0);
        EXP2L[j] = (float)exp2(j / 65536.0);
    }
    TGAM[0] = 0.0f; /* unused: the count starts at k = 1 */
    for (int k = 1; k < 256; k++) TGAM[k] = (float)pow((k - 0.5) / 255.0, 2.2);
    const double pi = 3.14159265358979323846;
    for (int u = 0; u < 8; u++)
        for (int x = 0; x < 8; x++) {
            double cu = (u == 0) ? sqrt(1.0 / 8.0) : 0.5;
            KDCT[u][x] = (int32_t)lround(8192.0 * cu * cos((2 * x + 1) * u * pi / 16.0));
        }
    tables_ready = 1;
}

/* Expose the tables so tests can regenerate them independently. */
void oracle_tables(int32_t *log2f, float *exp2h, float *exp2l, float *tgam, int32_t *kdct)
{
    init_tables();
    if (log2f) memcpy(log2f, LOG2F, sizeof LOG2F);
    if (exp2h) memcpy(exp2h, EXP2H, sizeof EXP2H);
    if (exp2l) memcpy(exp2l, EXP2L, sizeof EXP2L);
    if (tgam) memcpy(tgam, TGAM, sizeof TGAM);
    if (kdct) memcpy(kdct, KDCT, sizeof KDCT);
}

/* ------------------------------------------------------------------------ */
/* Small exact helpers                                                       */
/* ------------------------------------------------------------------------ */
static int64_t floor_div64(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static i128 floor_div128(i128 a, i128 b) /* b > 0 */
{
    i128 q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

/* rhu(x / y) = floor((2x + y) / (2y)): round half up, y > 0. */
static i128 rhu128(i128 x, i128 y) { return floor_div128(2 * x + y, 2 * y); }

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* C2: key statistic.  Reinhard's global operator scales luminance by        */
/* key / (log-average luminance).  The log is taken in Q16 fixed point so   */
/* the image-wide sum is exact and order-independent.  For a pixel with     */
/* E != 0 the luminance of the mantissa centres (M + 0.5) (Eq. 3) in units  */
/* of 2^-16 is Y = 13933 MR + 46871 MG + 4732 MB + 32768 (Rec. 709 weights, */
/* round(2^16 w), summing to 65536), and its absolute luminance is          */
/* Y * 2^(E - 136 - 16).  Pixels with E == 0 are black and left out.        */
/* ------------------------------------------------------------------------ */
static uint32_t lum_y(const uint8_t *px)
{
    return 13933u * px[0] + 46871u * px[1] + 4732u * px[2] + 32768u;
}

/* lambda(Y) ~= 2^16 * (log2(Y) - 16), Y in [2^15, 2^24). */
static int64_t lambda_q16(uint32_t Y)
{
    int p = 31;
    while (!((Y >> p) & 1u)) p--; /* floor(log2 Y) */
    uint32_t idx = (Y >> (p - 12)) & 4095u;
    return (int64_t)65536 * (p - 16) + LOG2F[idx];
}

void oracle_keystat(const uint8_t *rgbe, int64_t npx, int64_t *lambda_sum, int64_t *n_lit)
{
    init_tables();
    int64_t L = 0, N = 0;
    for (int64_t i = 0; i < npx; i++) {
        const uint8_t *px = rgbe + 4 * i;
        if (px[3] == 0) continue;
        L += (int64_t)65536 * ((int)px[3] - 136) + lambda_q16(lum_y(px));
        N += 1;
    }
    *lambda_sum = L;
    *n_lit = N;
}

/* Q = floor(-Lambda / N') = 2^16 k_img + f with f in [0, 2^16).
 * sigma = 0.18 * 2^(f / 2^16) from the two frozen exp2 tables.
 * The per-pixel scale is P = sigma * 2^(k_img + E - 136). */
void oracle_key_params(int64_t lambda_sum, int64_t n_lit, int32_t *k_img, int32_t *f_key, float *sigma)
{
    init_tables();
    if (n_lit <= 0) {
        *k_img = 0;
        *f_key = 0;
        *sigma = 0.0f;
        return;
    }
    int64_t Q = floor_div64(-lambda_sum, n_lit);
    int64_t k = Q >> 16;
    int64_t f = Q - k * 65536;
    float s = 0.18f * EXP2H[f >> 8];
    s = s * EXP2L[f & 255];
    *k_img = (int32_t)k;
    *f_key = (int32_t)f;
    *sigma = s;
}

/* C4: code = #{k in 1..255 : C >= TGAM[k]}, i.e. round(255 C^(1/2.2))
 * clamped to [0, 255], written as exact threshold comparisons. */
static int gamma_code(float C)
{
    int code = 0;
    for (int k = 1; k < 256; k++)
        if (C >= TGAM[k]) code++;
    return code;
}

/* C3: tone-map one pixel to three 8-bit codes (hue-preserving global
 * Reinhard: C_d = C_w / (1 + L) with L the scaled luminance).  FP32, fixed
 * order: t = P*l, D = 1 + t, R = 1/D, C = (P*c~) * R. */
static void tmo_pixel(const uint8_t *px, int32_t k_img, float sigma, int64_t n_lit, uint8_t *out)
{
    out[0] = out[1] = out[2] = 0;
    if (n_lit <= 0 || px[3] == 0) return;
    int kp = k_img + (int)px[3] - 136;
    if (kp < -64) return; /* C < 2^-50 < TGAM[1]: every code is 0 */
    if (kp > 40) kp = 40; /* exactly equivalent: the 1 in 1 + t is absorbed */
    float P = ldexpf(sigma, kp);
    float lf = (float)lum_y(px) * (1.0f / 65536.0f);
    float t = P * lf;
    float D = 1.0f + t;
    float R = 1.0f / D;
    for (int c = 0; c < 3; c++) {
        float ct = (float)px[c] + 0.5f;
        float C = (P * ct) * R;
        out[c] = (uint8_t)gamma_code(C);
    }
}

void oracle_tmo(const uint8_t *rgbe, int H, int W, int32_t k_img, float sigma, int64_t n_lit, uint8_t *sdr0)
{
    init_tables();
    int64_t npx = (int64_t)H * W;
    for (int64_t i = 0; i < npx; i++) tmo_pixel(rgbe + 4 * i, k_img, sigma, n_lit, sdr0 + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* C5-C9: JPEG-style 4:4:4 base layer round trip (Encoder 1 then Decoder 1) */
/* ------------------------------------------------------------------------ */
/* ITU-T T.81 Annex K, Tables K.1 (luminance) and K.2 (chrominance), natural
 * (row-major) order: row = vertical frequency v, column = horizontal u. */
static const int ANNEX_K1[64] = {
    16, 11, 10, 16, 24, 40, 51, 61,     12, 12, 14, 19, 26, 58, 60, 55,
    14, 13, 16, 24, 40, 57, 69, 56,     14, 17, 22, 29, 51, 87, 80, 62,
    18, 22, 37, 56, 68, 109, 103, 77,   24, 35, 55, 64, 81, 104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99};
static const int ANNEX_K2[64] = {
    17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
    24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
    99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99};

/* C8: quality scaling (IJG convention): s = 5000/q (q < 50) else 200 - 2q;
 * entry = clamp(floor((base * s + 50) / 100), 1, 255). */
void oracle_quant_table(int q, int chroma, int32_t *out64)
{
    int s = (q < 50) ? 5000 / q : 200 - 2 * q;
    const int *base = chroma ? ANNEX_K2 : ANNEX_K1;
    for (int i = 0; i < 64; i++) out64[i] = clampi((base[i] * s + 50) / 100, 1, 255);
}

/* C5: JFIF full-range BT.601 colour transform, 16-bit fixed point, constants
 * round(2^16 c) of Y = .299 R + .587 G + .114 B, Cb = (B - Y)/1.772 + 128,
 * Cr = (R - Y)/1.402 + 128. */
static void rgb_to_ycc(int R, int G, int B, int *Y, int *Cb, int *Cr)
{
    *Y = (19595 * R + 38470 * G + 7471 * B + 32768) >> 16;
    *Cb = (-11058 * R - 21710 * G + 32768 * B + 8388608 + 32768) >> 16;
    *Cr = (32768 * R - 27439 * G - 5329 * B + 8388608 + 32768) >> 16;
}

static void ycc_to_rgb(int Y, int Cb, int Cr, int *R, int *G, int *B)
{
    int cb = Cb - 128, cr = Cr - 128;
    *R = clampi(Y + ((91881 * cr + 32768) >> 16), 0, 255);
    *G = clampi(Y + ((-22554 * cb - 46802 * cr + 32768) >> 16), 0, 255);
    *B = clampi(Y + ((116130 * cb + 32768) >> 16), 0, 255);
}

/* C7: integer FDCT: row pass then column pass with K, rounding shifts of 11
 * and 15, giving the orthonormal 2-D DCT-II of (p - 128) to within +-1.
 * in[y][x] holds p - 128; out[v][u]. */
static void fdct8x8(const int in[8][8], int out[8][8])
{
    int T[8][8];
    for (int y = 0; y < 8; y++)
        for (int u = 0; u < 8; u++) {
            int acc = 0;
            for (int x = 0; x < 8; x++) acc += KDCT[u][x] * in[y][x];
            T[y][u] = (acc + 1024) >> 11;
        }
    for (int u = 0; u < 8; u++)
        for (int v = 0; v < 8; v++) {
            int acc = 0;
            for (int y = 0; y < 8; y++) acc += KDCT[v][y] * T[y][u];
            out[v][u] = (acc + 16384) >> 15;
        }
}

/* C7: integer IDCT: column pass then row pass with K transposed, rounding
 * shifts of 11 and 15, + 128, clamp to [0, 255].  in[v][u]; out[y][x]. */
static void idct8x8(const int in[8][8], int out[8][8])
{
    int t[8][8];
    for (int u = 0; u < 8; u++)
        for (int y = 0; y < 8; y++) {
            int acc = 0;
            for (int v = 0; v < 8; v++) acc += KDCT[v][y] * in[v][u];
            t[y][u] = (acc + 1024) >> 11;
        }
    for (int y = 0; y < 8; y++)
        for (int x = 0; x < 8; x++) {
            int acc = 0;
            for (int u = 0; u < 8; u++) acc += KDCT[u][x] * t[y][u];
            out[y][x] = clampi(((acc + 16384) >> 15) + 128, 0, 255);
        }
}

/* C9: quantise with round half away from zero, then dequantise. */
static int quant(int F, int Qt)
{
    int a = F < 0 ? -F : F;
    int q = (a + Qt / 2) / Qt;
    return F < 0 ? -q : q;
}

void oracle_fdct_block(const int32_t *in64, int32_t *out64)
{
    init_tables();
    int a[8][8], b[8][8];
    for (int i = 0; i < 64; i++) a[i / 8][i % 8] = in64[i];
    fdct8x8(a, b);
    for (int i = 0; i < 64; i++) out64[i] = b[i / 8][i % 8];
}

void oracle_idct_block(const int32_t *in64, int32_t *out64)
{
    init_tables();
    int a[8][8], b[8][8];
    for (int i = 0; i < 64; i++) a[i / 8][i % 8] = in64[i];
    idct8x8(a, b);
    for (int i = 0; i < 64; i++) out64[i] = b[i / 8][i % 8];
}

int32_t oracle_quantise(int32_t F, int32_t Qt) { return quant(F, Qt); }

/* Base layer: sdr0 (tone-mapped RGB) -> S (what Decoder 1 returns).  Blocks
 * at the right/bottom edge are completed by replicating the last column/row
 * (C6) and cropped after the inverse transform.  dctq, if not NULL, receives
 * the quantised coefficients int16 [3][H8][W8] with the 8x8 block's (v, u)
 * at row 8*by + v, column 8*bx + u. */
void oracle_base_layer(const uint8_t *sdr0, int H, int W, int q, uint8_t *S, int16_t *dctq)
{
    init_tables();
    int32_t qt[2][64];
    oracle_quant_table(q, 0, qt[0]);
    oracle_quant_table(q, 1, qt[1]);
    int H8 = (H + 7) / 8 * 8, W8 = (W + 7) / 8 * 8;
    for (int by = 0; by < H8 / 8; by++)
        for (int bx = 0; bx < W8 / 8; bx++) {
            int blk[3][8][8], F[8][8], D[8][8], rec[3][8][8];
            for (int y = 0; y < 8; y++)
                for (int x = 0; x < 8; x++) {
                    int yy = by * 8 + y, xx = bx * 8 + x;
                    if (yy > H - 1) yy = H - 1;
                    if (xx > W - 1) xx = W - 1;
                    const uint8_t *p = sdr0 + 3 * ((int64_t)yy * W + xx);
                    int Y, Cb, Cr;
                    rgb_to_ycc(p[0], p[1], p[2], &Y, &Cb, &Cr);
                    blk[0][y][x] = Y - 128;
                    blk[1][y][x] = Cb - 128;
                    blk[2][y][x] = Cr - 128;
                }
            for (int c = 0; c < 3; c++) {
                fdct8x8(blk[c], F);
                for (int v = 0; v < 8; v++)
                    for (int u = 0; u < 8; u++) {
                        int Qt = qt[c == 0 ? 0 : 1][v * 8 + u];
                        int Fq = quant(F[v][u], Qt);
                        D[v][u] = Fq * Qt;
                        if (dctq)
                            dctq[((int64_t)c * H8 + by * 8 + v) * W8 + bx * 8 + u] = (int16_t)Fq;
                    }
                idct8x8(D, rec[c]);
            }
            for (int y = 0; y < 8; y++)
                for (int x = 0; x < 8; x++) {
                    int yy = by * 8 + y, xx = bx * 8 + x;
                    if (yy >= H || xx >= W) continue;
                    int R, G, B;
                    ycc_to_rgb(rec[0][y][x], rec[1][y][x], rec[2][y][x], &R, &G, &B);
                    uint8_t *o = S + 3 * ((int64_t)yy * W + xx);
                    o[0] = (uint8_t)R;
                    o[1] = (uint8_t)G;
                    o[2] = (uint8_t)B;
                }
        }
}

/* Decoder 1 of the base layer (Sec. II.B: the JPEG decoder returns S): from
 * the quantised coefficients dctq (layout of oracle_base_layer) at quality q,
 * D = Fq * Q, inverse DCT, inverse colour transform, crop to H x W.  For the
 * coefficients oracle_base_layer writes this is the second half of that
 * function and returns the same S.  Returns -1 for bad arguments. */
int oracle_base_decode(const int16_t *dctq, int H, int W, int q, uint8_t *S)
{
    if (!dctq || !S || H < 1 || W < 1 || q < 1 || q > 100) return -1;
    init_tables();
    int32_t qt[2][64];
    oracle_quant_table(q, 0, qt[0]);
    oracle_quant_table(q, 1, qt[1]);
    int H8 = (H + 7) / 8 * 8, W8 = (W + 7) / 8 * 8;
    for (int by = 0; by < H8 / 8; by++)
        for (int bx = 0; bx < W8 / 8; bx++) {
            int D[8][8], rec[3][8][8];
            for (int c = 0; c < 3; c++) {
                for (int v = 0; v < 8; v++)
                    for (int u = 0; u < 8; u++)
                        D[v][u] = dctq[((int64_t)c * H8 + by * 8 + v) * W8 + bx * 8 + u] *
                                  qt[c == 0 ? 0 : 1][v * 8 + u];
                idct8x8(D, rec[c]);
            }
            for (int y = 0; y < 8; y++)
                for (int x = 0; x < 8; x++) {
                    int yy = by * 8 + y, xx = bx * 8 + x;
                    if (yy >= H || xx >= W) continue;
                    int R, G, B;
                    ycc_to_rgb(rec[0][y][x], rec[1][y][x], rec[2][y][x], &R, &G, &B);
                    uint8_t *o = S + 3 * ((int64_t)yy * W + xx);
                    o[0] = (uint8_t)R;
                    o[1] = (uint8_t)G;
                    o[2] = (uint8_t)B;
                }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* C10: GF restoration S* = GF(S): 3x3 binomial (1, 6, 1) x (1, 6, 1) / 64, */
/* round half up, borders replicated at the image edge, per channel.        */
/* ------------------------------------------------------------------------ */
void oracle_gf(const uint8_t *S, int H, int W, uint8_t *Sstar)
{
    static const int w[3] = {1, 6, 1};
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
            for (int c = 0; c < 3; c++) {
                int acc = 0;
                for (int i = -1; i <= 1; i++)
                    for (int j = -1; j <= 1; j++) {
                        int yy = clampi(y + i, 0, H - 1), xx = clampi(x + j, 0, W - 1);
                        acc += w[i + 1] * w[j + 1] * S[3 * ((int64_t)yy * W + xx) + c];
                    }
                Sstar[3 * ((int64_t)y * W + x) + c] = (uint8_t)((acc + 32) >> 6);
            }
}

/* ------------------------------------------------------------------------ */
/* C11: region sums.  Region (c, e) = every pixel with E == e (image-wide), */
/* channel c; s = S*_c, m = M_c.  sums[e][13] = {n, then per channel c:     */
/* sum s, sum m, sum s^2, sum s*m} at 1 + 4c + {0, 1, 2, 3}.                 */
/* ------------------------------------------------------------------------ */
void oracle_sums(const uint8_t *Sstar, const uint8_t *rgbe, int64_t npx, int64_t *sums /* [256][13] */)
{
    memset(sums, 0, sizeof(int64_t) * 256 * 13);
    for (int64_t i = 0; i < npx; i++) {
        int e = rgbe[4 * i + 3];
        int64_t *b = sums + 13 * e;
        b[0] += 1;
        for (int c = 0; c < 3; c++) {
            int64_t s = Sstar[3 * i + c], m = rgbe[4 * i + c];
            b[1 + 4 * c + 0] += s;
            b[1 + 4 * c + 1] += m;
            b[1 + 4 * c + 2] += s * s;
            b[1 + 4 * c + 3] += s * m;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* C12: least-squares slope and intercept per region (Eq. 6-7 restated for   */
/* a region as Eq. 9-10), quantised to 32-bit fixed point: a_q with 22 and  */
/* b_q with 14 fractional bits.  num = n Ssm - Ss Sm, den = n Sss - Ss^2    */
/* (exact, 128-bit).  den == 0 (one distinct s): a_q = 0.  The intercept is */
/* the least-squares intercept given the quantised slope:                   */
/* b_q = rhu((2^22 Sm - a_q Ss) / (2^8 n)).                                  */
/* ------------------------------------------------------------------------ */
void oracle_solve(const int64_t *sums, int32_t *a_q /* [3][256] */, int32_t *b_q /* [3][256] */,
                  uint8_t *present /* [256] */)
{
    for (int e = 0; e < 256; e++) {
        const int64_t *b = sums + 13 * e;
        i128 n = b[0];
        present[e] = n > 0;
        for (int c = 0; c < 3; c++) {
            a_q[c * 256 + e] = 0;
            b_q[c * 256 + e] = 0;
            if (n == 0) continue;
            i128 Ss = b[1 + 4 * c], Sm = b[2 + 4 * c], Sss = b[3 + 4 * c], Ssm = b[4 + 4 * c];
            i128 num = n * Ssm - Ss * Sm;
            i128 den = n * Sss - Ss * Ss;
            i128 a = (den == 0) ? 0 : rhu128(((i128)1 << 22) * num, den);
            i128 bb = rhu128(((i128)1 << 22) * Sm - a * Ss, ((i128)1 << 8) * n);
            a_q[c * 256 + e] = (int32_t)a;
            b_q[c * 256 + e] = (int32_t)bb;
        }
    }
}

/* C13: M* = round(a s + b) clamped to [0, 255] (Eq. 8), in fixed point:
 * clamp((a_q s + 2^8 b_q + 2^21) >> 22, 0, 255). */
static int mstar(int32_t a_q, int32_t b_q, int s)
{
    int64_t v = (int64_t)a_q * s + (int64_t)b_q * 256 + ((int64_t)1 << 21);
    v >>= 22;
    return v < 0 ? 0 : (v > 255 ? 255 : (int)v);
}

int32_t oracle_mstar(int32_t a_q, int32_t b_q, int32_t s) { return mstar(a_q, b_q, s); }

/* Residual planes r = M - M* as int16 [3][H][W], then the exponent plane
 * uint8 E[H][W] (the enhancement layer carries E losslessly). */
void oracle_resid(const uint8_t *Sstar, const uint8_t *rgbe, int64_t npx, const int32_t *a_q,
                  const int32_t *b_q, void *out_resid)
{
    int16_t *r = (int16_t *)out_resid;
    uint8_t *Ep = (uint8_t *)out_resid + 6 * npx;
    for (int64_t i = 0; i < npx; i++) {
        int e = rgbe[4 * i + 3];
        for (int c = 0; c < 3; c++) {
            int ms = mstar(a_q[c * 256 + e], b_q[c * 256 + e], Sstar[3 * i + c]);
            r[c * npx + i] = (int16_t)((int)rgbe[4 * i + c] - ms);
        }
        Ep[i] = (uint8_t)e;
    }
}

/* ------------------------------------------------------------------------ */
/* Whole encoder: RGBE -> (S, parameters, residuals).                        */
/* params_out: {Lambda, N', k_img, f_key, sigma bits} as int64[5].           */
/* ------------------------------------------------------------------------ */
int oracle_encode_enh(const uint8_t *rgbe, int H, int W, int q, uint8_t *out_sdr, int32_t *a_q,
                      int32_t *b_q, uint8_t *present, int64_t *sums, int64_t *params_out,
                      void *out_resid)
{
    if (!rgbe || !out_sdr || !a_q || !b_q || !present || !out_resid) return -1;
    if (H < 1 || W < 1 || q < 1 || q > 100) return -1;
    init_tables();
    int64_t npx = (int64_t)H * W;
    int64_t L, N;
    oracle_keystat(rgbe, npx, &L, &N);
    int32_t k, f;
    float sig;
    oracle_key_params(L, N, &k, &f, &sig);
    uint8_t *s0 = (uint8_t *)malloc(3 * npx);
    uint8_t *ss = (uint8_t *)malloc(3 * npx);
    int64_t *sm = sums ? sums : (int64_t *)malloc(sizeof(int64_t) * 256 * 13);
    if (!s0 || !ss || !sm) return -4;
    oracle_tmo(rgbe, H, W, k, sig, N, s0);
    oracle_base_layer(s0, H, W, q, out_sdr, NULL);
    oracle_gf(out_sdr, H, W, ss);
    oracle_sums(ss, rgbe, npx, sm);
    oracle_solve(sm, a_q, b_q, present);
    oracle_resid(ss, rgbe, npx, a_q, b_q, out_resid);
    if (params_out) {
        uint32_t sb;
        memcpy(&sb, &sig, 4);
        params_out[0] = L;
        params_out[1] = N;
        params_out[2] = k;
        params_out[3] = f;
        params_out[4] = sb;
    }
    free(s0);
    free(ss);
    if (!sums) free(sm);
    return 0;
}

/* Ablations of the method (the comparisons of Table I and Fig. 4): the
 * encoder with est = 0 (SLR per exponent region, as oracle_encode_enh), 2
 * (one least-squares line per channel for the whole image: every region's
 * sums pooled and solved as one region, the line written to every present
 * exponent) or 3 (no estimator: M* = S, i.e. slope 1 and intercept 0), and
 * gf = 1 (S* = GF(S), Sec. III.B) or 0 (S* = S). */
int oracle_encode_mode(const uint8_t *rgbe, int H, int W, int q, int est, int gf, uint8_t *out_sdr, int32_t *a_q,
                       int32_t *b_q, uint8_t *present, void *out_resid)
{
    if (!rgbe || !out_sdr || !a_q || !b_q || !present || !out_resid) return -1;
    if (H < 1 || W < 1 || q < 1 || q > 100 || (est != 0 && est != 2 && est != 3)) return -1;
    init_tables();
    int64_t npx = (int64_t)H * W;
    int64_t L, N;
    oracle_keystat(rgbe, npx, &L, &N);
    int32_t k, f;
    float sig;
    oracle_key_params(L, N, &k, &f, &sig);
    uint8_t *s0 = (uint8_t *)malloc(3 * npx);
    uint8_t *ss = (uint8_t *)malloc(3 * npx);
    int64_t *sm = (int64_t *)malloc(sizeof(int64_t) * 256 * 13);
    if (!s0 || !ss || !sm) return -4;
    oracle_tmo(rgbe, H, W, k, sig, N, s0);
    oracle_base_layer(s0, H, W, q, out_sdr, NULL);
    if (gf)
        oracle_gf(out_sdr, H, W, ss);
    else
        memcpy(ss, out_sdr, 3 * npx);
    oracle_sums(ss, rgbe, npx, sm);
    if (est == 2) {
        int64_t pool[13] = {0};
        for (int e = 0; e < 256; e++)
            for (int j = 0; j < 13; j++) pool[j] += sm[e * 13 + j];
        for (int e = 0; e < 256; e++)
            if (sm[e * 13] > 0)
                for (int j = 0; j < 13; j++) sm[e * 13 + j] = pool[j];
    }
    oracle_solve(sm, a_q, b_q, present);
    if (est == 3)
        for (int c = 0; c < 3; c++)
            for (int e = 0; e < 256; e++) {
                a_q[c * 256 + e] = present[e] ? 1 << 22 : 0;
                b_q[c * 256 + e] = 0;
            }
    oracle_resid(ss, rgbe, npx, a_q, b_q, out_resid);
    free(s0);
    free(ss);
    free(sm);
    return 0;
}

/* C14: decode.  The decoder rebuilds S* from S, reads (a_E, b_E) as sent
 * (never recomputes them) and adds the residual: M = M* + r. */
int oracle_decode_mode(const uint8_t *sdr, const int32_t *a_q, const int32_t *b_q, const void *resid,
                       int H, int W, int gf, uint8_t *out_rgbe);

int oracle_decode_enh(const uint8_t *sdr, const int32_t *a_q, const int32_t *b_q, const void *resid,
                      int H, int W, uint8_t *out_rgbe)
{
    return oracle_decode_mode(sdr, a_q, b_q, resid, H, W, 1, out_rgbe);
}

/* Decoder with the Gaussian filter on (gf = 1, as the method has it) or off
 * (S* = S, the ablation). */
int oracle_decode_mode(const uint8_t *sdr, const int32_t *a_q, const int32_t *b_q, const void *resid,
                       int H, int W, int gf, uint8_t *out_rgbe)
{
    if (!sdr || !a_q || !b_q || !resid || !out_rgbe || H < 1 || W < 1) return -1;
    int64_t npx = (int64_t)H * W;
    uint8_t *ss = (uint8_t *)malloc(3 * npx);
    if (!ss) return -4;
    if (gf)
        oracle_gf(sdr, H, W, ss);
    else
        memcpy(ss, sdr, 3 * npx);
    const int16_t *r = (const int16_t *)resid;
    const uint8_t *Ep = (const uint8_t *)resid + 6 * npx;
    int bad = 0;
    for (int64_t i = 0; i < npx; i++) {
        int e = Ep[i];
        for (int c = 0; c < 3; c++) {
            int m = mstar(a_q[c * 256 + e], b_q[c * 256 + e], ss[3 * i + c]) + r[c * npx + i];
            if (m < 0 || m > 255) bad = 1;
            out_rgbe[4 * i + c] = (uint8_t)m;
        }
        out_rgbe[4 * i + 3] = (uint8_t)e;
    }
    free(ss);
    return bad ? -3 : 0;
}

/* C15: residual histograms, hist[c][r + 255] for r in [-255, 255]. */
void oracle_resid_hist(const void *resid, int64_t npx, int64_t *hist /* [3][511] */)
{
    memset(hist, 0, sizeof(int64_t) * 3 * 511);
    const int16_t *r = (const int16_t *)resid;
    for (int c = 0; c < 3; c++)
        for (int64_t i = 0; i < npx; i++) hist[c * 511 + r[c * npx + i] + 255] += 1;
}

/* ------------------------------------------------------------------------ */
/* C16: learned int8 mantissa estimator (an extension, not in the paper: the */
/* paper's estimator needs no learning, Sec. I).  Model blob, little endian:  */
/*   u32 magic 'RDLM', u32 version 2, u64 hash, u32 reserved[2];            */
/*   i8  W1[32][32] (out, in)   i32 B1[32][32] (bin, out)                    */
/*   i32 m1[32], r1[32]                                                      */
/*   i8  W2[32][32]             i32 B2[32], m2[32], r2[32]                    */
/*   i8  W3[16][32]             i32 B3[16], m3[16], r3[16]                    */
/* Input features x[3k + c] = S(y + dy, x + dx)_c - 128 for the 3x3          */
/* neighbourhood k = 3(dy+1) + (dx+1) (replicated at the image border),      */
/* x[27..31] = 0.  Exponent bin b = clamp(E - 136 + k_img + 24, 0, 31): the  */
/* exponent one-hot enters as the bias row B1[b].                            */
/* Hidden layers: a = clamp((h m + 2^(r-1)) >> r, 0, 255) (64-bit product).  */
/* Output c (0..2): q8 = (o m3 + 2^(r3-1)) >> r3, M_L = clamp((q8 + 128) >> 8). */
/* ------------------------------------------------------------------------ */
#define MLP_BYTES 7512

typedef struct {
    const int8_t *W1, *W2, *W3;
    const int32_t *B1, *m1, *r1, *B2, *m2, *r2, *B3, *m3, *r3;
} mlp_view;

static int mlp_parse(const uint8_t *blob, mlp_view *v)
{
    uint32_t magic, version;
    memcpy(&magic, blob, 4);
    memcpy(&version, blob + 4, 4);
    if (magic != 0x4D4C4452u || version != 2u) return -3;
    const uint8_t *p = blob + 24;
    v->W1 = (const int8_t *)p; p += 1024;
    v->B1 = (const int32_t *)p; p += 4096;
    v->m1 = (const int32_t *)p; p += 128;
    v->r1 = (const int32_t *)p; p += 128;
    v->W2 = (const int8_t *)p; p += 1024;
    v->B2 = (const int32_t *)p; p += 128;
    v->m2 = (const int32_t *)p; p += 128;
    v->r2 = (const int32_t *)p; p += 128;
    v->W3 = (const int8_t *)p; p += 512;
    v->B3 = (const int32_t *)p; p += 64;
    v->m3 = (const int32_t *)p; p += 64;
    v->r3 = (const int32_t *)p; p += 64;
    return (p - blob) == MLP_BYTES ? 0 : -3;
}

static int64_t shr_round(int64_t v, int r) { return (v + ((int64_t)1 << (r - 1))) >> r; }

/* Learned estimate for one pixel: feat[32] int8 features, b the bin. */
static void mlp_pixel(const mlp_view *v, const int feat[32], int b, int out[3])
{
    int a1[32], a2[32];
    for (int n = 0; n < 32; n++) {
        int64_t h = v->B1[b * 32 + n];
        for (int k = 0; k < 32; k++) h += (int64_t)v->W1[n * 32 + k] * feat[k];
        int64_t q = shr_round(h * v->m1[n], v->r1[n]);
        a1[n] = q < 0 ? 0 : (q > 255 ? 255 : (int)q);
    }
    for (int n = 0; n < 32; n++) {
        int64_t h = v->B2[n];
        for (int k = 0; k < 32; k++) h += (int64_t)v->W2[n * 32 + k] * a1[k];
        int64_t q = shr_round(h * v->m2[n], v->r2[n]);
        a2[n] = q < 0 ? 0 : (q > 255 ? 255 : (int)q);
    }
    for (int c = 0; c < 3; c++) {
        int64_t o = v->B3[c];
        for (int k = 0; k < 32; k++) o += (int64_t)v->W3[c * 32 + k] * a2[k];
        int64_t q8 = shr_round(o * v->m3[c], v->r3[c]);
        int64_t m = (q8 + 128) >> 8;
        out[c] = m < 0 ? 0 : (m > 255 ? 255 : (int)m);
    }
}

/* M_L[H][W][3] for the decoded SDRI S and the exponents of rgbe (or of an
 * exponent plane Ep if rgbe is NULL). */
int oracle_mlp_estimate(const uint8_t *S, const uint8_t *rgbe, const uint8_t *Ep, int H, int W, int32_t k_img,
                        const uint8_t *blob, uint8_t *ML)
{
    mlp_view v;
    if (mlp_parse(blob, &v)) return -3;
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
            int feat[32] = {0};
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int k = 3 * (dy + 1) + (dx + 1);
                    const uint8_t *p = S + 3 * ((int64_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1));
                    for (int c = 0; c < 3; c++) feat[3 * k + c] = (int)p[c] - 128;
                }
            int64_t i = (int64_t)y * W + x;
            int E = rgbe ? rgbe[4 * i + 3] : Ep[i];
            int b = clampi(E - 136 + k_img + 24, 0, 31);
            int out[3];
            mlp_pixel(&v, feat, b, out);
            for (int c = 0; c < 3; c++) ML[3 * i + c] = (uint8_t)out[c];
        }
    return 0;
}

/* L(x) = Q16 log2 of a count x >= 1: 2^16 floor(log2 x) + LOG2F[the 12 bits
 * after the leading one, zero-filled]; L(0) = 0. */
int64_t oracle_log2q16(int64_t x)
{
    init_tables();
    if (x <= 0) return 0;
    int p = 62;
    while (!((x >> p) & 1)) p--;
    int64_t idx = p >= 12 ? (x >> (p - 12)) & 4095 : (x << (12 - p)) & 4095;
    return (int64_t)65536 * p + LOG2F[idx];
}

/* Integer entropy cost of a histogram: sum_v h_v (L(n) - L(h_v)), i.e.
 * 2^16 n H0 up to the table's rounding. */
int64_t oracle_hist_cost(const int64_t *h, int nbins)
{
    int64_t n = 0, cost = 0;
    for (int v = 0; v < nbins; v++) n += h[v];
    int64_t Ln = oracle_log2q16(n);
    for (int v = 0; v < nbins; v++)
        if (h[v]) cost += h[v] * (Ln - oracle_log2q16(h[v]));
    return cost;
}

/* Code length, in Q16 bits, of a residual histogram h (nbins bins) under the
 * distribution of the counts g (total N): sum_v h_v (L(N) - L(g_v)).  -1 when
 * some h_v > 0 has g_v = 0 (no finite code length). */
int64_t oracle_cross_cost(const int64_t *h, const int64_t *g, int64_t N, int nbins)
{
    int64_t LN = oracle_log2q16(N), cost = 0;
    for (int v = 0; v < nbins; v++)
        if (h[v]) {
            if (!g[v]) return -1;
            cost += h[v] * (LN - oracle_log2q16(g[v]));
        }
    return cost;
}

/* Learned encoder: the plain encoder, then per (c, E) region the learned
 * estimate replaces M* where its residuals cost strictly fewer bits than the
 * SLR residuals under the distribution of channel c's SLR residuals over the
 * whole image (ties and regions without a finite learned cost keep SLR);
 * flag[c][E] records the choice.  Summed over the regions, the chosen
 * residuals then cost no more under that distribution than the SLR residuals,
 * whose cost is N H0(SLR); and a histogram's own H0 is the least cost under
 * any distribution (Gibbs), so the chosen residuals' zeroth-order entropy is
 * at most SLR's, up to the rounding of the Q16 logarithms. */
int oracle_encode_learned(const uint8_t *rgbe, int H, int W, int q, const uint8_t *blob, uint8_t *out_sdr,
                          int32_t *a_q, int32_t *b_q, uint8_t *present, uint8_t *flag, int64_t *params_out,
                          void *out_resid)
{
    int rc = oracle_encode_enh(rgbe, H, W, q, out_sdr, a_q, b_q, present, NULL, params_out, out_resid);
    if (rc) return rc;
    int64_t npx = (int64_t)H * W;
    uint8_t *ss = (uint8_t *)malloc(3 * npx), *ML = (uint8_t *)malloc(3 * npx);
    int64_t *hs = (int64_t *)calloc((size_t)3 * 256 * 511, sizeof(int64_t));
    int64_t *hl = (int64_t *)calloc((size_t)3 * 256 * 511, sizeof(int64_t));
    if (!ss || !ML || !hs || !hl) return -4;
    oracle_gf(out_sdr, H, W, ss);
    rc = oracle_mlp_estimate(out_sdr, rgbe, NULL, H, W, (int32_t)params_out[2], blob, ML);
    if (rc) return rc;
    for (int64_t i = 0; i < npx; i++) {
        int e = rgbe[4 * i + 3];
        for (int c = 0; c < 3; c++) {
            int m = rgbe[4 * i + c];
            int rs = m - mstar(a_q[c * 256 + e], b_q[c * 256 + e], ss[3 * i + c]);
            int rl = m - ML[3 * i + c];
            hs[((int64_t)c * 256 + e) * 511 + rs + 255] += 1;
            hl[((int64_t)c * 256 + e) * 511 + rl + 255] += 1;
        }
    }
    int64_t g[511];
    for (int c = 0; c < 3; c++) {
        for (int v = 0; v < 511; v++) {
            g[v] = 0;
            for (int e = 0; e < 256; e++) g[v] += hs[((int64_t)c * 256 + e) * 511 + v];
        }
        for (int e = 0; e < 256; e++) {
            int64_t cs = oracle_cross_cost(hs + ((int64_t)c * 256 + e) * 511, g, npx, 511);
            int64_t cl = oracle_cross_cost(hl + ((int64_t)c * 256 + e) * 511, g, npx, 511);
            flag[c * 256 + e] = present[e] && cl >= 0 && cl < cs;
        }
    }
    int16_t *r = (int16_t *)out_resid;
    for (int64_t i = 0; i < npx; i++) {
        int e = rgbe[4 * i + 3];
        for (int c = 0; c < 3; c++)
            if (flag[c * 256 + e]) r[c * npx + i] = (int16_t)((int)rgbe[4 * i + c] - ML[3 * i + c]);
    }
    free(ss);
    free(ML);
    free(hs);
    free(hl);
    return 0;
}

/* Learned decoder: M = (flag ? M_L : M*) + r. */
int oracle_decode_learned(const uint8_t *sdr, const int32_t *a_q, const int32_t *b_q, const uint8_t *flag,
                          int32_t k_img, const uint8_t *blob, const void *resid, int H, int W, uint8_t *out_rgbe)
{
    int64_t npx = (int64_t)H * W;
    uint8_t *ss = (uint8_t *)malloc(3 * npx), *ML = (uint8_t *)malloc(3 * npx);
    if (!ss || !ML) return -4;
    oracle_gf(sdr, H, W, ss);
    const uint8_t *Ep = (const uint8_t *)resid + 6 * npx;
    int rc = oracle_mlp_estimate(sdr, NULL, Ep, H, W, k_img, blob, ML);
    if (rc) return rc;
    const int16_t *r = (const int16_t *)resid;
    int bad = 0;
    for (int64_t i = 0; i < npx; i++) {
        int e = Ep[i];
        for (int c = 0; c < 3; c++) {
            int est = flag[c * 256 + e] ? ML[3 * i + c] : mstar(a_q[c * 256 + e], b_q[c * 256 + e], ss[3 * i + c]);
            int m = est + r[c * npx + i];
            if (m < 0 || m > 255) bad = 1;
            out_rgbe[4 * i + c] = (uint8_t)m;
        }
        out_rgbe[4 * i + 3] = (uint8_t)e;
    }
    free(ss);
    free(ML);
    return bad ? -3 : 0;
}
