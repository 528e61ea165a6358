// rdl_kernels.hip -- gfx950 kernels of the dual-layer lossless Radiance
// encoder (Suzuki et al., arXiv 2309.11072) and of its enhancement-layer
// decoder.
//
// Every stage is exact integer arithmetic except the tone-mapping operator,
// which is FP32 with a fixed operation order: the file is built with
// -ffp-contract=off (and says so again below), divisions are correctly
// rounded, and no transcendental function is evaluated per pixel -- the
// logarithm and the exponentials come from frozen tables.  Integer sums are
// accumulated with integer atomics, so results do not depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>

#include "rdl_internal.h"

#pragma clang fp contract(off)

namespace rdl {

typedef short short2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Frozen tables (filled once per device by upload_tables()).
// ---------------------------------------------------------------------------
__device__ int32_t g_log2f[4096];   // round(2^16 log2(1 + (i + 0.5)/4096))
__device__ float g_exp2h[256];      // fl32(2^(j/256))
__device__ float g_exp2l[256];      // fl32(2^(j/65536))
// Gamma quantiser table, one word per float-bit bucket (see gamma_code).
__device__ __align__(16) uint32_t g_glut[GAMMA_LUT_N];

// ITU-T T.81 Annex K, Tables K.1 and K.2 (natural order).
constexpr int ANNEX_K[2][64] = {
    {16, 11, 10, 16, 24, 40, 51, 61,     12, 12, 14, 19, 26, 58, 60, 55,
     14, 13, 16, 24, 40, 57, 69, 56,     14, 17, 22, 29, 51, 87, 80, 62,
     18, 22, 37, 56, 68, 109, 103, 77,   24, 35, 55, 64, 81, 104, 113, 92,
     49, 64, 78, 87, 103, 121, 120, 101, 72, 92, 95, 98, 112, 100, 103, 99},
    {17, 18, 24, 47, 99, 99, 99, 99, 18, 21, 26, 66, 99, 99, 99, 99,
     24, 26, 56, 99, 99, 99, 99, 99, 47, 66, 99, 99, 99, 99, 99, 99,
     99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99,
     99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99, 99}};

// Quantiser constants of every quality, filled once by upload_tables():
// g_qm[q - 1][t][e] = {M | Q << 24, h, even, 0} with Q the IJG-scaled Annex K
// entry, M = ceil(2^20 / Q), h = floor(Q / 2) and even = -1 if Q is even, else 0.
__device__ uint4 g_qm[100][2][64];

// DCT basis K[u][x] = round(2^13 c_u cos((2x+1) u pi / 16)), c_0 = 1/sqrt(8),
// c_u = 1/2: the 8-point DCT-II scaled by 2^13.
constexpr int KD[8][8] = {
    {2896, 2896, 2896, 2896, 2896, 2896, 2896, 2896},
    {4017, 3406, 2276, 799, -799, -2276, -3406, -4017},
    {3784, 1567, -1567, -3784, -3784, -1567, 1567, 3784},
    {3406, -799, -4017, -2276, 2276, 4017, 799, -3406},
    {2896, -2896, -2896, 2896, 2896, -2896, -2896, 2896},
    {2276, -4017, 799, 3406, -3406, -799, 4017, -2276},
    {1567, -3784, 3784, -1567, -1567, 3784, -3784, 1567},
    {799, -2276, 3406, -4017, 4017, -3406, 2276, -799}};

__host__ __device__ constexpr int pk16(int lo, int hi) {
    return (int)(((unsigned)lo & 0xffffu) | ((unsigned)hi << 16));
}

__device__ __forceinline__ int dot2(int a, int b, int c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, a), __builtin_bit_cast(short2v, b), c, false);
}
// The same with the accumulator as a separate operand (the three-operand
// encoding): starting a chain from a shared constant then needs no copy of
// the constant into each destination.
__device__ __forceinline__ int dot2s(int a, int b, int c) {
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}
__device__ __forceinline__ int pack_i16(int lo, int hi) {
    return __builtin_bit_cast(int, __builtin_amdgcn_cvt_pk_i16(lo, hi));
}

// ---------------------------------------------------------------------------
// Helpers shared by the kernels of this file.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Every buffer a descriptor points to is device global memory.  Saying so
// once, when a kernel takes its descriptor, lets every access through it
// compile to global (not flat) memory instructions, whose waits do not
// couple with LDS operations.  The detour through an integer keeps the
// compiler from folding the two address-space casts away again.
template <class T>
__device__ __forceinline__ T *glb(T *p) {
    return (T *)((__attribute__((address_space(1))) T *)(uintptr_t)p);
}
__device__ __forceinline__ ImgDesc desc_at(const ImgDesc *__restrict__ D, int i) {
    ImgDesc d = D[i];
    d.rgbe = glb(d.rgbe);
    d.sdr0 = glb(d.sdr0);
    d.sdr = glb(d.sdr);
    d.dct = glb(d.dct);
    d.hdr = glb(d.hdr);
    d.resid = glb(d.resid);
    d.ks = glb(d.ks);
    d.sums = glb(d.sums);
    d.part = glb(d.part);
    d.status = glb(d.status);
    d.out_rgbe = glb(d.out_rgbe);
    d.hist = glb(d.hist);
    d.lres = glb(d.lres);
    d.lhist = glb(d.lhist);
    d.lrec = glb(d.lrec);
    d.lbk = glb(d.lbk);
    d.model = glb(d.model);
    return d;
}

// Image of workgroup `wg`: the last image whose first workgroup is <= wg.
__device__ __forceinline__ int find_img(const ImgDesc *__restrict__ D, int n, int wg, int which) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int w = which == 0 ? D[mid].wg_px : which == 1 ? D[mid].wg_blk : which == 2 ? D[mid].wg_tile : which == 3 ? D[mid].wg_fit : which == 4 ? D[mid].wg_res
                : which == 5 ? D[mid].wg_learn : D[mid].wg_lhist;
        if (w <= wg) lo = mid; else hi = mid - 1;
    }
    return uniform(lo);
}

// floor(a / b) for b > 0: a float64 quotient is within a few units of it
// (abs(a) < 2^55 here), and the remainder corrects it exactly.
__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {
    int64_t q = (int64_t)floor((double)a / (double)b);
    int64_t r = a - q * b;
    for (int k = 0; k < 8 && r < 0; ++k) { q -= 1; r += b; }
    for (int k = 0; k < 8 && r >= b; ++k) { q += 1; r -= b; }
    return q;
}

// Key of the global Reinhard operator: Q = floor(-Lambda / N') =
// 2^16 k_img + f, sigma = (0.18 * 2^((f >> 8) / 256)) * 2^((f & 255) / 65536).
__device__ void key_from(int64_t L, int64_t N, int &k_img, int &f_key, float &sigma) {
    if (N <= 0) { k_img = 0; f_key = 0; sigma = 0.0f; return; }
    const int64_t Q = floor_div64(-L, N);
    const int64_t k = Q >> 16;
    const int f = (int)(Q - k * 65536);
    float s = 0.18f * g_exp2h[f >> 8];
    s = s * g_exp2l[f & 255];
    k_img = (int)k;
    f_key = f;
    sigma = s;
}

// The same from nks partial (Lambda, N') pairs.
__device__ void key_params(const int64_t *ks, int nks, int &k_img, int &f_key, float &sigma, int64_t &L, int64_t &N) {
    L = 0;
    N = 0;
    for (int k = 0; k < nks; ++k) {
        L += ks[2 * k];
        N += ks[2 * k + 1];
    }
    key_from(L, N, k_img, f_key, sigma);
}

__device__ __forceinline__ uint32_t lum_y(uint32_t w) {
    return 13933u * (w & 255u) + 46871u * ((w >> 8) & 255u) + 4732u * ((w >> 16) & 255u) + 32768u;
}

// ---------------------------------------------------------------------------
// K0 zero: clear the per-image accumulators of a launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero(const ImgDesc *__restrict__ D, int n) {
    const int i = blockIdx.x;
    if (i >= n) return;
    const ImgDesc d = desc_at(D, i);
    if ((d.flags & F_ZERO_KS) && d.ks && (int)threadIdx.x < 2 * d.nks) d.ks[threadIdx.x] = 0;
    if ((d.flags & F_ZERO_SUMS) && d.part)
        for (int k = threadIdx.x; k < d.nfs * 256 * NSUM; k += 256) d.part[k] = 0;
    if ((d.flags & F_ZERO_HIST) && d.hist)
        for (int k = threadIdx.x; k < 3 * 511; k += 256) d.hist[k] = 0;
}

// ---------------------------------------------------------------------------
// K1 key statistic: Lambda = sum over E != 0 of 2^16 (E - 136) + lambda(Y),
// N' = #{E != 0}.  lambda(Y) = 2^16 (floor(log2 Y) - 16) + LOG2F[12 bits of Y
// after its leading one].  Memory bound: 4 B/px, 128-bit loads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lambda_px(uint32_t w, const uint16_t *s_log2f) {
    const uint32_t E = w >> 24;
    const uint32_t Y = lum_y(w);
    const int p = 31 - __builtin_clz(Y);
    const int idx = (int)((Y >> (p - 12)) & 4095u);
    const int v = 65536 * (p - 16 + (int)E - 136) + (int)s_log2f[idx];
    return E ? v : 0;
}

__global__ __launch_bounds__(KS_THREADS) void k_keystat(const ImgDesc *__restrict__ D, int n) {
    __shared__ uint16_t s_log2f[4096];  // every entry is below 2^16
    __shared__ int64_t s_red[2][KS_THREADS / 64];
    const int i = find_img(D, n, blockIdx.x, 0);
    const ImgDesc d = desc_at(D, i);
    const int64_t npx = (int64_t)d.H * d.W;
    const int wgl = blockIdx.x - d.wg_px;
    const int64_t base = (int64_t)wgl * KS_PX_PER_WG;
    const uint32_t *p32 = (const uint32_t *)d.rgbe;
    const bool al = (reinterpret_cast<uintptr_t>(p32) & 15) == 0;
    // The table's loads first (L2 hits), then the pixel loads; the table is
    // stored to LDS after waiting for its own loads only, so each chunk of
    // pixels can be summed as soon as it arrives.
    int32_t tl[4096 / KS_THREADS];
#pragma unroll
    for (int k = 0; k < 4096 / KS_THREADS; ++k) tl[k] = g_log2f[k * KS_THREADS + threadIdx.x];
    constexpr int NIT = KS_PX_PER_WG / (KS_THREADS * 4);
    uint4 v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int64_t px = base + (int64_t)(it * KS_THREADS + threadIdx.x) * 4;
        if (al && px + 4 <= npx) {
            v[it] = *reinterpret_cast<const uint4 *>(p32 + px);
        } else {
            v[it].x = px + 0 < npx ? p32[px + 0] : 0u;
            v[it].y = px + 1 < npx ? p32[px + 1] : 0u;
            v[it].z = px + 2 < npx ? p32[px + 2] : 0u;
            v[it].w = px + 3 < npx ? p32[px + 3] : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < 4096 / KS_THREADS; ++k) s_log2f[k * KS_THREADS + threadIdx.x] = (uint16_t)tl[k];
    __syncthreads();
    int64_t L = 0;
    int cnt = 0;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const uint32_t w[4] = {v[it].x, v[it].y, v[it].z, v[it].w};
        int part = 0;  // |part| < 4 * 2^16 * 145: no overflow
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            part += lambda_px(w[j], s_log2f);
            cnt += (w[j] >> 24) != 0;
        }
        L += part;
    }
    // wave reduction, then one atomic pair per workgroup into its stripe
    for (int off = 32; off > 0; off >>= 1) {
        L += __shfl_down(L, off, 64);
        cnt += __shfl_down(cnt, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_red[0][wv] = L; s_red[1][wv] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t a = 0, b = 0;
        for (int k = 0; k < KS_THREADS / 64; ++k) { a += s_red[0][k]; b += s_red[1][k]; }
        unsigned long long *ks = (unsigned long long *)(d.ks + 2 * (wgl % d.nks));
        atomicAdd(ks, (unsigned long long)a);
        atomicAdd(ks + 1, (unsigned long long)b);
    }
}

// Sum of the key-statistic stripes of each image into out2 (stage check);
// the scratch stripes are left zero.
__global__ void k_key_total(const ImgDesc *__restrict__ D, int n, int64_t *out2) {
    const int i = blockIdx.x;
    if (i >= n || threadIdx.x != 0) return;
    int64_t L = 0, N = 0;
    for (int k = 0; k < D[i].nks; ++k) {
        L += D[i].ks[2 * k];
        N += D[i].ks[2 * k + 1];
        if (D[i].flags & F_CLEAN_KS) D[i].ks[2 * k] = D[i].ks[2 * k + 1] = 0;
    }
    out2[2 * i] = L;
    out2[2 * i + 1] = N;
}

// ---------------------------------------------------------------------------
// K2 tone mapping + base layer, per 8x8 block:
//   RGBE -> TMO (FP32) -> 8-bit codes -> JFIF YCbCr -> FDCT (row, column)
//   -> quantise / dequantise -> IDCT (column, row) -> RGB -> S.
// Both 1-D transforms use the even/odd split of the DCT basis
// (K[u][7-x] = (-1)^u K[u][x]) on int16 pairs with v_dot2_i32_i16; this is an
// exact refactoring of the sums, so the results equal the plain matrix form.
// ---------------------------------------------------------------------------
// code = #{k : T[k] <= C} with T[k] = fl32(((k - 0.5)/255)^2.2).  A float's
// bucket is its top 16 bits (exponent + 7 mantissa bits); at most one
// threshold lies strictly inside a bucket (checked on the host when the table
// is built).  The bucket's word holds c0 2^17 + 2^17 - t, where c0 counts the
// thresholds <= the bucket start and t is the low 16 bits of the threshold
// inside it (t = 2^16 if none), so adding C's low 16 bits carries into bit 17
// exactly when C >= that threshold.  Buckets below 2^-20 and from 2 up share
// the first and last word, which hold no threshold.
constexpr uint32_t GAMMA_B0 = (127 - 20) << 7;
__device__ __forceinline__ int gamma_code(float C, const uint32_t *lut) {
    const uint32_t bits = __float_as_uint(C);
    const uint32_t b = min(max(bits >> 16, GAMMA_B0), GAMMA_B0 + GAMMA_LUT_N - 1);
    return (int)((lut[b - GAMMA_B0] + (bits & 0xFFFFu)) >> 17);
}

// Correctly rounded 1/D for D in [1, 2^47): the hardware reciprocal refined by
// one Newton step with fused multiply-adds.  Checked equal to IEEE division
// for every float in that range on gfx950 (the denominator of the operator
// below is 1 + sigma 2^(k'-16) Y with sigma < 0.36, k' <= 40 and Y < 2^24, so
// it always lies there).
__device__ __forceinline__ float recip(float D) {
    const float r0 = __builtin_amdgcn_rcpf(D);
    const float e = __builtin_fmaf(-D, r0, 1.0f);
    return __builtin_fmaf(e, r0, r0);
}

// Global Reinhard operator, hue preserving.  Per image, for each exponent E:
// P(E) = sigma 2^k', k' = k_img + E - 136 (clamped at 40: the 1 in 1 + t is
// then absorbed and the result is exactly the clamped one), and P = 0 for
// black pixels (E = 0, k' < -64, or nothing lit in the image); tmo_p fills
// that table.  Per pixel: t = P Y 2^-16, D = 1 + t, R = 1/D,
// C_c = (P (M_c + 0.5)) R, the first product as one fused multiply-add
// P M_c + P/2 whose single rounding is that of P (M_c + 0.5) (the sum is
// exact before rounding).  With P = 0 every C is 0 and every code 0.
__device__ __forceinline__ float tmo_p(int E, int kbase, float sigma) {
    const int kp = kbase + E;
    return ((E == 0) | (kp < -64)) ? 0.0f : ldexpf(sigma, min(kp, 40));
}

__device__ __forceinline__ void tmo_px(uint32_t w, const float *ptab, const uint32_t *lut, int &r, int &g, int &b) {
    // P/2 and P 2^-16 are exact: P is 0 or a normal float >= 0.18 2^-64.
    const float P = ptab[w >> 24];
    const float Ph = P * 0.5f;
    const float Pl = P * 0x1p-16f;
    const float t = Pl * (float)lum_y(w);
    const float Dn = 1.0f + t;
    const float R = recip(Dn);
    const float c0 = __builtin_fmaf(P, (float)(w & 255u), Ph) * R;
    const float c1 = __builtin_fmaf(P, (float)((w >> 8) & 255u), Ph) * R;
    const float c2 = __builtin_fmaf(P, (float)((w >> 16) & 255u), Ph) * R;
    r = gamma_code(c0, lut);
    g = gamma_code(c1, lut);
    b = gamma_code(c2, lut);
}

__device__ __forceinline__ int padd(int a, int b) {
    return __builtin_bit_cast(int, __builtin_bit_cast(short2v, a) + __builtin_bit_cast(short2v, b));
}
__device__ __forceinline__ int psub(int a, int b) {
    return __builtin_bit_cast(int, __builtin_bit_cast(short2v, a) - __builtin_bit_cast(short2v, b));
}
// Forward even/odd pairs: KF(u, 0) = (K[u][0], K[u][1]), KF(u, 1) = (K[u][2], K[u][3]).
__device__ __forceinline__ int KF(int u, int h) { return pk16(KD[u][2 * h], KD[u][2 * h + 1]); }
// Inverse pairs over the frequency index: KI(y, parity, h) =
// (K[4h + parity][y], K[4h + parity + 2][y]).
__device__ __forceinline__ int KI(int y, int par, int h) {
    return pk16(KD[4 * h + par][y], KD[4 * h + par + 2][y]);
}

// 1-D forward transform of 8 samples given as the even/odd pairs
// S01 = (x0+x7, x1+x6), S23 = (x2+x5, x3+x4), D01, D23 (differences):
// out[u] = sum_x K[u][x] x_x + bias.
__device__ __forceinline__ void fdct1(int S01, int S23, int D01, int D23, int bias, int out[8]) {
#pragma unroll
    for (int u = 0; u < 8; u += 2) out[u] = dot2(KF(u, 0), S01, dot2s(KF(u, 1), S23, bias));
#pragma unroll
    for (int u = 1; u < 8; u += 2) out[u] = dot2(KF(u, 0), D01, dot2s(KF(u, 1), D23, bias));
}

// 1-D inverse transform of 8 coefficients given as pairs E0 = (c0, c2),
// E1 = (c4, c6), O0 = (c1, c3), O1 = (c5, c7): out[y] = sum_v K[v][y] c_v + bias.
__device__ __forceinline__ void idct1(int E0, int E1, int O0, int O1, int bias, int out[8]) {
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        const int e = dot2(KI(y, 0, 0), E0, dot2s(KI(y, 0, 1), E1, bias));
        const int o = dot2(KI(y, 1, 0), O0, dot2s(KI(y, 1, 1), O1, 0));
        out[y] = e + o;
        out[7 - y] = e - o;
    }
}

// Quantise and dequantise coefficient F (before its >> 15) with the
// constants qc of its table entry: Fq = sign(f) floor((|f| + h) / Q), f = F >> 15,
// returns Fq Q.  Rounding half away from zero equals floor((f + h - e) / Q)
// for either sign, e = 1 for negative f and even Q (no ties exist for odd Q),
// and that floor is (a M + 2^11) >> 20 with a = f + h - e: the magic
// multiplier's relative error stays below 2^-9 while |a| <= 1151, and the
// 2^11 offset lifts exact multiples of Q above the truncation.  The 8x8
// transforms of 8-bit level-shifted samples keep |f| <= 1024, so every
// product fits in 31 bits.
__device__ __forceinline__ int quant_dequant(int F, uint4 qc, int &Fq) {
    const int a = (F >> 15) + (int)qc.y + ((F >> 31) & (int)qc.z);
    Fq = (__mul24(a, (int)qc.x) + 2048) >> 20;  // the low 24 bits of qc.x are M
    return __mul24(Fq, (int)(qc.x >> 24));
}

// Last phase of the base layer (shared by the encoder and the base-layer
// decoder): lane = row y of block j, whose IDCT column outputs sit in
// s_X[c][j] (two int16 per word, transposed as the column pass leaves them).
// IDCT row pass, + 128, clamp, inverse colour transform, crop, store S.
__device__ __forceinline__ void base_store_row(const ImgDesc &d, const uint32_t (*s_X)[BLK_WG][33], int j, int r,
                                               int by, int x0) {
    const int H = d.H, W = d.W;
    const int y = r;
    const int yy = by * 8 + y;
    if (yy >= H) return;
    int smp[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t *rw = &s_X[c][j][y * 4];
        int o[8];
        idct1((int)rw[0], (int)rw[1], (int)rw[2], (int)rw[3], 16384 + (128 << 15), o);
#pragma unroll
        for (int x = 0; x < 8; ++x) smp[c][x] = min(max(o[x] >> 15, 0), 255);
    }
    uint32_t ow[6];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        // JFIF inverse transform; the chroma offset of 128 is folded into the
        // rounding constants.
        const int Yv = smp[0][x], cb = smp[1][x], cr = smp[2][x];
        const int R = min(max(Yv + ((91881 * cr + 32768 - 91881 * 128) >> 16), 0), 255);
        const int G = min(max(Yv + ((-22554 * cb - 46802 * cr + 32768 + (22554 + 46802) * 128) >> 16), 0), 255);
        const int B = min(max(Yv + ((116130 * cb + 32768 - 116130 * 128) >> 16), 0), 255);
        const uint32_t rgb = (uint32_t)R | ((uint32_t)G << 8) | ((uint32_t)B << 16);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = 3 * x + k;
            const uint32_t byte = (rgb >> (8 * k)) & 255u;
            if ((p & 3) == 0) ow[p >> 2] = byte; else ow[p >> 2] |= byte << (8 * (p & 3));
        }
    }
    uint8_t *orow = d.sdr + 3 * ((int64_t)yy * W + x0);
    if (x0 + 8 <= W && ((reinterpret_cast<uintptr_t>(orow) & 3) == 0)) {
#pragma unroll
        for (int k = 0; k < 6; ++k) reinterpret_cast<uint32_t *>(orow)[k] = ow[k];
    } else {
        const int nx = min(8, W - x0);
        for (int k = 0; k < 3 * nx; ++k) orow[k] = (uint8_t)(ow[k >> 2] >> (8 * (k & 3)));
    }
}

template <bool EXTRA>
__global__ __launch_bounds__(BLK_THREADS) void k_tmo_base(const ImgDesc *__restrict__ D, int n) {
    // A workgroup owns a strip of BLK_WG horizontally adjacent 8x8 blocks of
    // one block row.  Lane t works on block j = t % BLK_WG as its row (phases
    // 1 and 3) or column (phase 2) r = t / BLK_WG; two LDS transposes join the
    // phases.  Slot stride 33 words keeps every half-wave access conflict-free.
    // EXTRA also writes the tone-mapped SDRI and the quantised coefficients.
    __shared__ __align__(16) uint32_t s_lut[GAMMA_LUT_N];
    __shared__ uint4 s_QM[2][64];
    __shared__ uint32_t s_X[3][BLK_WG][33];
    __shared__ float s_ptab[256];
    const int i = find_img(D, n, blockIdx.x, 1);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    // Prologue: the last wave derives the tone map's parameters from the key
    // statistic while the others copy the tables, so the two chains of
    // dependent loads overlap.
    if (threadIdx.x < BLK_THREADS - 64) {
        for (int k = threadIdx.x; k < GAMMA_LUT_N / 4; k += BLK_THREADS - 64)
            reinterpret_cast<uint4 *>(s_lut)[k] = reinterpret_cast<const uint4 *>(g_glut)[k];
        if (threadIdx.x < 128) (&s_QM[0][0])[threadIdx.x] = (&g_qm[d.q - 1][0][0])[threadIdx.x];
    } else {
        // The last wave: one lane derives k_img and sigma, then the wave
        // fills the per-exponent table of P.
        int kb = 0;
        float sigma = 0.0f;
        if (threadIdx.x == BLK_THREADS - 64) {
            int k_img, f_key;
            int64_t L, N;
            key_params(d.ks, d.nks, k_img, f_key, sigma, L, N);
            // No lit pixel: every pixel is black (k' below -64 for any E).
            kb = N > 0 ? k_img - 136 : -100000;
        }
        kb = __shfl(kb, 0, 64);
        sigma = __shfl(sigma, 0, 64);
        const int l = threadIdx.x & 63;
#pragma unroll
        for (int k = 0; k < 4; ++k) s_ptab[l + 64 * k] = tmo_p(l + 64 * k, kb, sigma);
    }

    const int nbx = (W + 7) >> 3, nby = (H + 7) >> 3;
    const int nstrip = (nbx + BLK_WG - 1) / BLK_WG;
    const int wgi = blockIdx.x - d.wg_blk;
    const int by = wgi / nstrip;
    const int j = threadIdx.x % BLK_WG, r = threadIdx.x / BLK_WG;
    const int bx = (wgi - by * nstrip) * BLK_WG + j;
    const bool active = bx < nbx && by < nby;
    const int x0 = bx * 8;
    __syncthreads();

    // Phase 1: lane = row r.  RGBE -> TMO -> YCbCr - 128 -> FDCT row pass; the
    // row outputs go to the slot transposed, at position r ^ (r >> 2) of
    // column u, so a column reads back as the pairs (0,1), (2,3), (5,4), (7,6).
    if (active) {
        const int yl = by * 8 + r;
        const uint32_t *row = (const uint32_t *)d.rgbe + (int64_t)min(yl, H - 1) * W;
        uint32_t px[8];
        if (x0 + 8 <= W) {
#pragma unroll
            for (int x = 0; x < 8; ++x) px[x] = row[x0 + x];
        } else {
#pragma unroll
            for (int x = 0; x < 8; ++x) px[x] = row[min(x0 + x, W - 1)];
        }
        int ch[3][8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            int cr, cg, cb;
            tmo_px(px[x], s_ptab, s_lut, cr, cg, cb);
            if (EXTRA && d.sdr0 && yl < H && x0 + x < W) {
                uint8_t *o = d.sdr0 + 3 * ((int64_t)yl * W + x0 + x);
                o[0] = (uint8_t)cr; o[1] = (uint8_t)cg; o[2] = (uint8_t)cb;
            }
            // JFIF forward transform with the level shift folded into the
            // rounding constant (a multiple of 2^16 passes through the shift).
            ch[0][x] = (19595 * cr + 38470 * cg + 7471 * cb + 32768 - (128 << 16)) >> 16;
            ch[1][x] = (-11058 * cr - 21710 * cg + 32768 * cb + 32768) >> 16;
            ch[2][x] = (32768 * cr - 27439 * cg - 5329 * cb + 32768) >> 16;
        }
        const int pos = r ^ (r >> 2);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int A01 = pack_i16(ch[c][0], ch[c][1]), A23 = pack_i16(ch[c][2], ch[c][3]);
            const int B76 = pack_i16(ch[c][7], ch[c][6]), B54 = pack_i16(ch[c][5], ch[c][4]);
            int T[8];
            fdct1(padd(A01, B76), padd(A23, B54), psub(A01, B76), psub(A23, B54), 1024, T);
            int16_t *slot = reinterpret_cast<int16_t *>(&s_X[c][j][0]);
#pragma unroll
            for (int u = 0; u < 8; ++u) slot[u * 8 + pos] = (int16_t)(T[u] >> 11);
        }
    }
    __syncthreads();

    // Phase 2: lane = column u = r.  FDCT column pass, quantise, dequantise,
    // IDCT column pass; outputs go back transposed at position
    // (u & 1) * 4 + (u >> 1) of row y, i.e. a row reads back as the pairs
    // (0,2), (4,6), (1,3), (5,7).
    const int u = r;
    int col[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) col[c][k] = (int)s_X[c][j][u * 4 + k];
    __syncthreads();
    if (active) {
        const int H8 = nby * 8, W8 = nbx * 8;
        const int pos2 = (u & 1) * 4 + (u >> 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int F[8];
            fdct1(padd(col[c][0], col[c][3]), padd(col[c][1], col[c][2]), psub(col[c][0], col[c][3]),
                  psub(col[c][1], col[c][2]), 16384, F);
            int dq[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                int Fq;
                dq[v] = quant_dequant(F[v], s_QM[c ? 1 : 0][v * 8 + u], Fq);
                if (EXTRA && d.dct) d.dct[((int64_t)c * H8 + by * 8 + v) * W8 + x0 + u] = (int16_t)Fq;
            }
            int t[8];
            idct1(pack_i16(dq[0], dq[2]), pack_i16(dq[4], dq[6]), pack_i16(dq[1], dq[3]), pack_i16(dq[5], dq[7]), 1024, t);
            int16_t *slot = reinterpret_cast<int16_t *>(&s_X[c][j][0]);
#pragma unroll
            for (int y = 0; y < 8; ++y) slot[y * 8 + pos2] = (int16_t)(t[y] >> 11);
        }
    }
    __syncthreads();

    // Phase 3: lane = row y = r.  IDCT row pass, + 128, clamp, inverse colour
    // transform, crop, store S.
    if (!active) return;
    base_store_row(d, s_X, j, r, by, x0);
}

// ---------------------------------------------------------------------------
// Base-layer decoder (Sec. II.B: the JPEG decoder of the base layer returns
// S): from the quantised coefficients int16 [3][H8][W8] (block (bx, by)'s
// (v, u) at row 8 by + v, column 8 bx + u, as the encoder writes them) and
// the header's quality: D = Fq Q, the integer IDCT and the inverse colour
// transform of the encoder's own round trip, crop, store S.  Same workgroup
// shape as k_tmo_base: lane = column (dequantise + IDCT column pass), LDS
// transpose, lane = row (base_store_row).  A header whose magic, version,
// size or quality does not fit sets *status = RDL_ECORRUPT.  Only images with
// coefficients take part.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLK_THREADS) void k_base_decode(const ImgDesc *__restrict__ D, int n) {
    __shared__ int32_t s_Q[2][64];
    __shared__ uint32_t s_X[3][BLK_WG][33];
    const int i = find_img(D, n, blockIdx.x, 1);
    const ImgDesc d = desc_at(D, i);
    if (!d.dct) return;  // uniform
    const int H = d.H, W = d.W;
    const rdl_header *h = d.hdr;
    const int q = h->q;
    if (!(h->magic == RDL_MAGIC && h->version == RDL_VERSION && h->H == H && h->W == W && q >= 1 && q <= 100)) {
        if (threadIdx.x == 0 && d.status) atomicExch(d.status, RDL_ECORRUPT);
        return;
    }
    if (threadIdx.x < 128) (&s_Q[0][0])[threadIdx.x] = (int32_t)((&g_qm[q - 1][0][0])[threadIdx.x].x >> 24);
    const int nbx = (W + 7) >> 3, nby = (H + 7) >> 3;
    const int nstrip = (nbx + BLK_WG - 1) / BLK_WG;
    const int wgi = blockIdx.x - d.wg_blk;
    const int by = wgi / nstrip;
    const int j = threadIdx.x % BLK_WG, r = threadIdx.x / BLK_WG;
    const int bx = (wgi - by * nstrip) * BLK_WG + j;
    const bool active = bx < nbx && by < nby;
    const int x0 = bx * 8;
    __syncthreads();
    // Lane = row v of its block: the row's eight coefficients (one 16-byte load
    // per channel where the array is 16-byte aligned: every row then is),
    // dequantised, go to the column slots at position (v & 1) * 4 + (v >> 1),
    // so column u reads back the pairs (0,2), (4,6), (1,3), (5,7).
    const int H8 = nby * 8, W8 = nbx * 8;
    const bool wide = (reinterpret_cast<uintptr_t>(d.dct) & 15) == 0;
    const int pos = (r & 1) * 4 + (r >> 1);
    if (active) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int16_t *row = d.dct + ((int64_t)c * H8 + by * 8 + r) * W8 + x0;
            int cf[8];
            if (wide) {
                const uint4 v = *reinterpret_cast<const uint4 *>(row);
                const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int u = 0; u < 8; ++u) cf[u] = (int)(int16_t)(w4[u >> 1] >> (16 * (u & 1)));
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) cf[u] = (int)row[u];
            }
            int16_t *slot = reinterpret_cast<int16_t *>(&s_X[c][j][0]);
#pragma unroll
            for (int u = 0; u < 8; ++u) slot[u * 8 + pos] = (int16_t)(cf[u] * s_Q[c ? 1 : 0][r * 8 + u]);
        }
    }
    __syncthreads();
    // Lane = column u: IDCT column pass; outputs back to the slot as the
    // encoder's column pass leaves them (row y at (u & 1) * 4 + (u >> 1)).
    const int u = r, pos2 = (u & 1) * 4 + (u >> 1);
    int col[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) col[c][k] = (int)s_X[c][j][u * 4 + k];
    __syncthreads();
    if (active) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int t[8];
            idct1(col[c][0], col[c][1], col[c][2], col[c][3], 1024, t);
            int16_t *slot = reinterpret_cast<int16_t *>(&s_X[c][j][0]);
#pragma unroll
            for (int y = 0; y < 8; ++y) slot[y * 8 + pos2] = (int16_t)(t[y] >> 11);
        }
    }
    __syncthreads();
    if (!active) return;
    base_store_row(d, s_X, j, r, by, x0);
}

// Every image's status word (if given) starts at RDL_OK; the decoders only
// ever replace it with RDL_ECORRUPT.
__global__ void k_status_init(const ImgDesc *__restrict__ D, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && D[i].status) glb(D[i].status)[0] = RDL_OK;
}

// ---------------------------------------------------------------------------
// GF streaming, shared by the fit, residual and decode kernels.  A wave owns a
// strip of STRIP_W = 256 px (four consecutive pixels per lane) and srh
// rows.  It walks down its rows holding S of rows y-1, y, y+1 in registers and
// takes the horizontal neighbours of its four pixels from the adjacent lanes
// (DPP wave shifts) or, at the strip ends, from one halo pixel per lane (lane
// 0: left of the strip, every other lane: right of it).  The (1,6,1) filter
// runs on two packed fields per pixel, lo = R | B << 16 and hi = G; no field
// exceeds 64 * 255 < 2^16, so packed integer adds never carry across fields.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t load_px3(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

__device__ __forceinline__ uint32_t dpp_from_left(uint32_t v) {  // lane l gets lane l-1
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t dpp_from_right(uint32_t v) {  // lane l gets lane l+1
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
}

struct GfWindow {
    uint32_t lo[3][4], hi[3][4];  // rows y-1, y, y+1 of the lane's pixels
    uint32_t hlo[3], hhi[3];      // the same rows of the lane's halo pixel
};

__device__ __forceinline__ void gf_roll(GfWindow &g) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        g.lo[0][j] = g.lo[1][j]; g.lo[1][j] = g.lo[2][j];
        g.hi[0][j] = g.hi[1][j]; g.hi[1][j] = g.hi[2][j];
    }
    g.hlo[0] = g.hlo[1]; g.hlo[1] = g.hlo[2];
    g.hhi[0] = g.hhi[1]; g.hhi[1] = g.hhi[2];
}

// The R | B << 16 words are filtered as two 16-bit lanes (packed 16-bit
// multiply-adds); G words hold one field below 2^16.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as16(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t vsum2(uint32_t a, uint32_t b, uint32_t c) {
    return as32(as16(a) + as16(c) + as16(b) * (u16x2)(6));
}
__device__ __forceinline__ uint32_t vsum(uint32_t a, uint32_t b, uint32_t c) { return a + c + __umul24(b, 6u); }

// S* of the lane's four pixels for the middle row: s[c][j], c = R, G, B.
// Must be called by the whole wave (DPP).
__device__ __forceinline__ void gf_quad(const GfWindow &g, int lane, int s[3][4]) {
    uint32_t vlo[4], vhi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        vlo[j] = vsum2(g.lo[0][j], g.lo[1][j], g.lo[2][j]);
        vhi[j] = vsum(g.hi[0][j], g.hi[1][j], g.hi[2][j]);
    }
    const uint32_t hvlo = vsum2(g.hlo[0], g.hlo[1], g.hlo[2]), hvhi = vsum(g.hhi[0], g.hhi[1], g.hhi[2]);
    uint32_t llo = dpp_from_left(vlo[3]), lhi = dpp_from_left(vhi[3]);
    uint32_t rlo = dpp_from_right(vlo[0]), rhi = dpp_from_right(vhi[0]);
    if (lane == 0) { llo = hvlo; lhi = hvhi; }
    if (lane == 63) { rlo = hvlo; rhi = hvhi; }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t Llo = j == 0 ? llo : vlo[j - 1], Lhi = j == 0 ? lhi : vhi[j - 1];
        const uint32_t Rlo = j == 3 ? rlo : vlo[j + 1], Rhi = j == 3 ? rhi : vhi[j + 1];
        const uint32_t tlo = as32((as16(Llo) + as16(Rlo) + as16(vlo[j]) * (u16x2)(6) + (u16x2)(32)) >> (u16x2)(6));
        const uint32_t thi = Lhi + Rhi + __umul24(vhi[j], 6u) + 32u;
        // Each field is at most (64 * 255 + 32) >> 6 = 255; the masks say so.
        s[0][j] = (int)(tlo & 255u);
        s[2][j] = (int)((tlo >> 16) & 255u);
        s[1][j] = (int)((thi >> 6) & 255u);
    }
}

// The lane's four pixels of the middle row unfiltered (S* = S when the
// Gaussian filter is off).
__device__ __forceinline__ void gf_centre(const GfWindow &g, int s[3][4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        s[0][j] = (int)(g.lo[1][j] & 255u);
        s[2][j] = (int)((g.lo[1][j] >> 16) & 255u);
        s[1][j] = (int)(g.hi[1][j] & 255u);
    }
}

// The strip of a workgroup and the rows of its wave.
struct StripPos {
    int lane, x, hx, ya, yb;
    uint32_t xo3, ho3, xo4;  // byte offsets in a row of S (3x, 3hx) and of RGBE (4x)
    bool fx;                 // x + 4 <= W: the lane's four pixels are all inside
};
__device__ __forceinline__ StripPos strip_pos(int wgl, int H, int W, int srh, int waves = STRIP_WAVES) {
    StripPos p;
    const int nsx = (W + STRIP_W - 1) / STRIP_W;
    const int sy = wgl / nsx, sx = wgl - sy * nsx;
    p.lane = threadIdx.x & 63;
    const int x0 = sx * STRIP_W;
    p.x = x0 + 4 * p.lane;
    p.hx = p.lane == 0 ? max(x0 - 1, 0) : min(x0 + STRIP_W, W - 1);
    // Row bounds are the same for every lane of a wave; saying so lets the
    // row addresses live in scalar registers.
    p.ya = uniform((sy * waves + (threadIdx.x >> 6)) * srh);
    p.yb = uniform(min(p.ya + srh, H));
    // W <= 2^28, so these fit 32 bits.
    p.xo3 = 3u * (uint32_t)p.x;
    p.ho3 = 3u * (uint32_t)p.hx;
    p.xo4 = 4u * (uint32_t)p.x;
    p.fx = p.x + 4 <= W;
    return p;
}

// Chunked walk: the loads of the next CH rows (S row y+1 for the window and
// the RGBE words of row y) are all issued before the first of them is used, so
// a wave waits for memory once per CH rows instead of once per row.  A raw
// S row is kept uncombined until it enters the window: the 16 bytes from the
// dword boundary at or below the lane's first byte (sh = that byte's offset),
// or, where that read would pass the row's last pixel or the buffer's end,
// the four pixels read one by one (sh = 4); the halo pixel as three bytes.
struct RowRaw {
    uint32_t d[4];
    uint32_t h[3];
    uint32_t sh;
};

// Row yy (already clamped to the image) of S.  fast: the lane may read 16
// bytes from the dword boundary at or below its first byte.
__device__ __forceinline__ void gf_row_issue(RowRaw &r, const uint8_t *__restrict__ sdr, int W, int yy, bool fast,
                                             const StripPos &sp) {
    const uint8_t *row = sdr + (int64_t)uniform(yy) * (3 * (int64_t)W);
    const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(row) + sp.xo3) & 3u;
    if (fast) {
        // The lane's first byte, minus its offset from the dword boundary
        // below it (S starts on a dword boundary, so this stays inside).
        const uint32_t *q = reinterpret_cast<const uint32_t *>((row + sp.xo3) - sh);
        r.d[0] = q[0];
        r.d[1] = q[1];
        r.d[2] = q[2];
        r.d[3] = q[3];
        r.sh = sh;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) r.d[j] = load_px3(row + 3u * (uint32_t)min(sp.x + j, W - 1));
        r.sh = 4;
    }
    const uint8_t *hp = row + sp.ho3;
    r.h[0] = hp[0];
    r.h[1] = hp[1];
    r.h[2] = hp[2];
}

// RGBE words of the lane's four pixels of row yy (pixels past W repeat W-1).
__device__ __forceinline__ void strip_rgbe4(const uint8_t *__restrict__ rgbe, int W, int yy, const StripPos &sp,
                                            uint32_t w[4]) {
    const uint8_t *row = rgbe + (int64_t)uniform(yy) * (4 * (int64_t)W);
    const uint8_t *p = row + sp.xo4;
    if (sp.fx && (((uint32_t)reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = *reinterpret_cast<const uint32_t *>(row + 4u * (uint32_t)min(sp.x + j, W - 1));
    }
}

__device__ __forceinline__ void gf_row_finish(GfWindow &g, int slot, const RowRaw &r) {
    uint32_t p[4];
    if (r.sh < 4) {
        const uint32_t e0 = __builtin_amdgcn_alignbyte(r.d[1], r.d[0], r.sh);
        const uint32_t e1 = __builtin_amdgcn_alignbyte(r.d[2], r.d[1], r.sh);
        const uint32_t e2 = __builtin_amdgcn_alignbyte(r.d[3], r.d[2], r.sh);
        p[0] = e0;
        p[1] = __builtin_amdgcn_alignbyte(e1, e0, 3);
        p[2] = __builtin_amdgcn_alignbyte(e2, e1, 2);
        p[3] = e2 >> 8;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) p[j] = r.d[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        g.lo[slot][j] = p[j] & 0x00FF00FFu;
        g.hi[slot][j] = (p[j] >> 8) & 0xFFu;
    }
    const uint32_t h = r.h[0] | (r.h[1] << 8) | (r.h[2] << 16);
    g.hlo[slot] = h & 0x00FF00FFu;
    g.hhi[slot] = (h >> 8) & 0xFFu;
}

// Calls row(y, s, w, x) for y = ya .. yb-1 in order, with s[c][j] = S*_c of
// the lane's pixels x+j of row y, w[j] their RGBE words and, if XW, x[j] their
// words of a second 4-byte-per-pixel buffer xw (loaded like the RGBE words).
// The whole wave must call it (DPP); ya < yb is uniform per wave.
constexpr int WALK_CH = 4;
template <bool XW, bool GF = true, class RowFn>
__device__ __forceinline__ void strip_walk_x(const ImgDesc &d, const StripPos &sp, const uint8_t *__restrict__ xw,
                                             RowFn &&row) {
    const int H = d.H, W = d.W;
    // The 16-byte read stays inside S on every row but the last (there the
    // lane's bytes are followed by a whole row); on the last row it must end
    // by the buffer's end.
    const uint8_t *last = d.sdr + (int64_t)(H - 1) * (3 * (int64_t)W);
    const uint32_t shl = (uint32_t)(reinterpret_cast<uintptr_t>(last) + sp.xo3) & 3u;
    const bool fast_last = sp.fx && (uint64_t)sp.xo3 - shl + 16u <= 3ull * (uint64_t)W;
    auto fast = [&](int yy) { return yy < H - 1 ? sp.fx : fast_last; };
    GfWindow g;
    {
        RowRaw r0, r1;
        const int y0 = max(sp.ya - 1, 0), y1 = sp.ya;
        gf_row_issue(r0, d.sdr, W, y0, fast(y0), sp);
        gf_row_issue(r1, d.sdr, W, y1, fast(y1), sp);
        gf_row_finish(g, 0, r0);
        gf_row_finish(g, 1, r1);
    }
    for (int y0 = sp.ya; y0 < sp.yb; y0 += WALK_CH) {
        RowRaw nr[WALK_CH];
        uint32_t w[WALK_CH][4], x[WALK_CH][4];
#pragma unroll
        for (int k = 0; k < WALK_CH; ++k) {
            // Rows past the strip repeat its last needed row (cache hits, unused).
            const int ys = min(min(y0 + k + 1, sp.yb), H - 1);
            gf_row_issue(nr[k], d.sdr, W, ys, fast(ys), sp);
            strip_rgbe4(d.rgbe, W, min(y0 + k, sp.yb - 1), sp, w[k]);
            if (XW) strip_rgbe4(xw, W, min(y0 + k, sp.yb - 1), sp, x[k]);
        }
#pragma unroll
        for (int k = 0; k < WALK_CH; ++k) {
            const int y = y0 + k;
            if (y < sp.yb) {  // uniform per wave
                gf_row_finish(g, 2, nr[k]);
                int sv[3][4];
                if (GF) gf_quad(g, sp.lane, sv);
                else gf_centre(g, sv);
                gf_roll(g);
                row(y, sv, w[k], x[k]);
            }
        }
    }
}

template <bool GF = true, class RowFn>
__device__ __forceinline__ void strip_walk(const ImgDesc &d, const StripPos &sp, RowFn &&row) {
    strip_walk_x<false, GF>(d, sp, nullptr, [&](int y, const int (&s)[3][4], const uint32_t (&w)[4],
                                                const uint32_t (&)[4]) { row(y, s, w); });
}

// The same chunked walk with other per-row data: issue(yy, side) loads the
// lane's data of row yy (issued with the S rows of the chunk), and
// row(y, s, side) receives it with S* of row y.
template <class Side, bool GF = true, class IssueFn, class RowFn>
__device__ __forceinline__ void strip_walk_side(const ImgDesc &d, const StripPos &sp, IssueFn &&issue, RowFn &&row) {
    const int H = d.H, W = d.W;
    const uint8_t *last = d.sdr + (int64_t)(H - 1) * (3 * (int64_t)W);
    const uint32_t shl = (uint32_t)(reinterpret_cast<uintptr_t>(last) + sp.xo3) & 3u;
    const bool fast_last = sp.fx && (uint64_t)sp.xo3 - shl + 16u <= 3ull * (uint64_t)W;
    auto fast = [&](int yy) { return yy < H - 1 ? sp.fx : fast_last; };
    GfWindow g;
    {
        RowRaw r0, r1;
        const int y0 = max(sp.ya - 1, 0), y1 = sp.ya;
        gf_row_issue(r0, d.sdr, W, y0, fast(y0), sp);
        gf_row_issue(r1, d.sdr, W, y1, fast(y1), sp);
        gf_row_finish(g, 0, r0);
        gf_row_finish(g, 1, r1);
    }
    for (int y0 = sp.ya; y0 < sp.yb; y0 += WALK_CH) {
        RowRaw nr[WALK_CH];
        Side sd[WALK_CH];
#pragma unroll
        for (int k = 0; k < WALK_CH; ++k) {
            const int ys = min(min(y0 + k + 1, sp.yb), H - 1);
            gf_row_issue(nr[k], d.sdr, W, ys, fast(ys), sp);
            issue(min(y0 + k, sp.yb - 1), sd[k]);
        }
#pragma unroll
        for (int k = 0; k < WALK_CH; ++k) {
            const int y = y0 + k;
            if (y < sp.yb) {  // uniform per wave
                gf_row_finish(g, 2, nr[k]);
                int sv[3][4];
                if (GF) gf_quad(g, sp.lane, sv);
                else gf_centre(g, sv);
                gf_roll(g);
                row(y, sv, sd[k]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K3 fit sums: per (channel, E) n, sum s, sum m, sum s^2, sum s m over the
// image (Eq. 9-10), s = S*_c, m = M_c.  Each lane keeps one register
// accumulator for its current exponent run and, when E changes, adds it to
// the workgroup's LDS bins (32-bit totals, added in pairs with 64-bit LDS
// atomics; a workgroup covers at most 256 px x 128 rows = 32768 px and
// 65025 x 32768 < 2^32, so no total wraps).  At the
// end the workgroup adds its present bins into one of the image's int64
// stripes with integer atomics.
// ---------------------------------------------------------------------------
// The bins are privatised R ways: lane l adds into copy l % R, so lanes of a
// wave that end runs of the same exponent at the same instant (neighbours in a
// smooth region do) hit R different addresses instead of one; the copies are
// skewed by 16 banks.  R is a tuned launch shape.
constexpr int BIN_WORDS = 256 * 14 + 16;

__device__ __forceinline__ void flush_run(uint32_t *bins, int e, uint32_t acc[NSUM]) {
    unsigned long long *b = reinterpret_cast<unsigned long long *>(bins + e * 14);
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const uint32_t lo = acc[2 * k], hi = 2 * k + 1 < NSUM ? acc[2 * k + 1] : 0u;
        atomicAdd(b + k, (unsigned long long)lo | ((unsigned long long)hi << 32));
    }
#pragma unroll
    for (int k = 0; k < NSUM; ++k) acc[k] = 0;
}

template <int R, bool GF = true>
__global__ __launch_bounds__(1024) void k_fit_sums(const ImgDesc *__restrict__ D, int n) {
    __shared__ __align__(8) uint32_t bins[R * BIN_WORDS];
    const int i = find_img(D, n, blockIdx.x, 3);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    const int wgl = blockIdx.x - d.wg_fit;
    for (int k = threadIdx.x; k < R * BIN_WORDS; k += blockDim.x) bins[k] = 0;
    __syncthreads();
    const StripPos sp = strip_pos(wgl, H, W, d.srh_fit, d.fit_waves);
    if (sp.ya < H) {  // uniform per wave
        uint32_t *mine = bins + (sp.lane % R) * BIN_WORDS;
        int cur = -1;
        uint32_t acc[NSUM];
#pragma unroll
        for (int k = 0; k < NSUM; ++k) acc[k] = 0;
        strip_walk<GF>(d, sp, [&](int, const int (&s)[3][4], const uint32_t (&w)[4]) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (sp.x + j < W) {
                    const int e = (int)(w[j] >> 24);
                    if (e != cur) {
                        if (cur >= 0) flush_run(mine, cur, acc);
                        cur = e;
                    }
                    acc[0] += 1;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const uint32_t sv = (uint32_t)s[c][j], m = (w[j] >> (8 * c)) & 255u;
                        acc[1 + 4 * c] += sv;
                        acc[2 + 4 * c] += m;
                        acc[3 + 4 * c] = __umul24(sv, sv) + acc[3 + 4 * c];
                        acc[4 + 4 * c] = __umul24(sv, m) + acc[4 + 4 * c];
                    }
                }
            }
        });
        if (cur >= 0) flush_run(mine, cur, acc);
    }
    __syncthreads();
    // Each copy's totals stay below 2^32 (see above); their sum is taken in
    // 64 bits.
    unsigned long long *gp = (unsigned long long *)(d.part + (int64_t)(wgl % d.nfs) * 256 * NSUM);
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        uint64_t cnt = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) cnt += bins[r * BIN_WORDS + e * 14];
        if (cnt == 0) continue;
#pragma unroll
        for (int k = 0; k < NSUM; ++k) {
            uint64_t v = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) v += bins[r * BIN_WORDS + e * 14 + k];
            if (v) atomicAdd(gp + k * 256 + e, (unsigned long long)v);
        }
    }
}
// ---------------------------------------------------------------------------
// K4 solve: one workgroup per image.  Three lanes per exponent value add up
// the image's sum stripes (and write the totals) while one more lane fills
// the header's key fields; then one lane per (channel, exponent) solves the
// least-squares line exactly in 128-bit integers (Eq. 6-7 / 9-10) with
// fixed-point rounding: a_q = rhu(2^22 num / den),
// b_q = rhu((2^22 Sm - a_q Ss) / (2^8 n)), while the last four waves mark the
// present exponents.
// ---------------------------------------------------------------------------
typedef __int128 i128;

__device__ __forceinline__ double i128_to_double(i128 v) {
    const int64_t hi = (int64_t)(v >> 64);
    const uint64_t lo = (uint64_t)v;
    return (double)hi * 18446744073709551616.0 + (double)lo;
}

// floor(N / D) for D > 0 when the quotient is known to be far below 2^50
// (here |quotient| < 2^32): a float64 estimate is within one of it, and is
// corrected exactly with the 128-bit remainder.
__device__ i128 floor_div128(i128 N, i128 D) {
    const double qd = floor(i128_to_double(N) / i128_to_double(D));
    int64_t q = (int64_t)qd;
    i128 r = N - (i128)q * D;
    for (int k = 0; k < 4 && r < 0; ++k) { q -= 1; r += D; }
    for (int k = 0; k < 4 && r >= D; ++k) { q += 1; r -= D; }
    return q;
}

__device__ __forceinline__ i128 rhu128(i128 x, i128 y) { return floor_div128(2 * x + y, 2 * y); }

__global__ __launch_bounds__(1024) void k_solve(const ImgDesc *__restrict__ D, int) {
    // One workgroup per image (the launch has exactly n).
    __shared__ int64_t s_b[256][NSUM];
    __shared__ int s_cnt[4];
    __shared__ uint32_t s_tot[2][4];
    const int i = blockIdx.x;
    const ImgDesc d = desc_at(D, i);
    rdl_header *h = d.hdr;
    const int t = threadIdx.x;
    // learned path: the image's SLR residual histograms start at zero
    if (d.lhist)
        for (int k = t; k < 3 * 511; k += 1024) d.lhist[LHIST_G + k] = 0;
    if (t < 3 * 256) {
        // Thread (g, e) adds values k = g, g + 3, ... of exponent e over the
        // image's stripes (all loads independent), leaves the stripes zero
        // for the next launch and keeps the totals.
        const int e = t & 255, g = t >> 8;
        int64_t v[5] = {0, 0, 0, 0, 0};
        // Stripes are laid out [stripe][value][exponent], so the lanes of a
        // wave read and clear contiguous words.  Every load is in flight
        // before the first is added: branch-free over the largest stripe
        // count, stripes past the image's count re-read its last one and are
        // masked out of the sum.
        int64_t w[FIT_STRIPES][5];
#pragma unroll
        for (int st = 0; st < FIT_STRIPES; ++st) {
            const int64_t *p = d.part + (int64_t)min(st, d.nfs - 1) * NSUM * 256 + e;
#pragma unroll
            for (int j = 0; j < 5; ++j) w[st][j] = g + 3 * j < NSUM ? p[(g + 3 * j) * 256] : 0;
        }
#pragma unroll
        for (int st = 0; st < FIT_STRIPES; ++st)
#pragma unroll
            for (int j = 0; j < 5; ++j) v[j] += st < d.nfs ? w[st][j] : 0;
#pragma unroll
        for (int st = 0; st < FIT_STRIPES; ++st) {
            if (st < d.nfs) {
                int64_t *p = d.part + (int64_t)st * NSUM * 256 + e;
#pragma unroll
                for (int j = 0; j < 5; ++j)
                    if (g + 3 * j < NSUM) p[(g + 3 * j) * 256] = 0;
            }
        }
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (g + 3 * j < NSUM) s_b[e][g + 3 * j] = v[j];
    } else if (t == 3 * 256) {
        // Meanwhile one lane of the last waves fills the key fields.
        int k_img = 0, f_key = 0;
        float sigma = 0.0f;
        int64_t L = 0, N = 0;
        if (d.ks) {
            key_params(d.ks, d.nks, k_img, f_key, sigma, L, N);
            if (d.flags & F_CLEAN_KS)
                for (int k = 0; k < 2 * d.nks; ++k) d.ks[k] = 0;
        }
        h->magic = RDL_MAGIC;
        h->version = RDL_VERSION;
        h->H = d.H;
        h->W = d.W;
        h->q = d.q;
        h->k_img = k_img;
        h->f_key = f_key;
        h->sigma = sigma;
        h->lambda_sum = L;
        h->n_lit = N;
        h->estimator = ((d.flags & F_EST_GLOBAL) ? 2 : (d.flags & F_EST_IDENT) ? 3 : 0) | ((d.flags & F_NOGF) ? 16 : 0);
        h->model_hash = 0;
    }
    __syncthreads();
    // One line per channel for the whole image: every exponent's sums pooled
    // (value k summed over exponents by thread k), then solved like a region.
    __shared__ int64_t s_g[NSUM];
    const bool global = (d.flags & F_EST_GLOBAL) != 0;  // uniform
    if (global) {
        if (t < NSUM) {
            int64_t acc = 0;
            for (int e2 = 0; e2 < 256; ++e2) acc += s_b[e2][t];
            s_g[t] = acc;
        }
        __syncthreads();
    }
    // The totals, [256][13] as the stage entry point documents them, written
    // from LDS in order.
    for (int k = t; k < 256 * NSUM; k += 1024) d.sums[k] = (&s_b[0][0])[k];
    if (t < 3 * 256) {
        // One lane per (channel, exponent): the least-squares line in exact
        // 128-bit integers with fixed-point rounding.
        const int c = t >> 8, e = t & 255;
        const int64_t *sb = global ? s_g : s_b[e];
        const i128 nn = sb[0];
        int32_t aq = 0, bq = 0;
        if (s_b[e][0] > 0 && (d.flags & F_EST_IDENT)) {
            aq = 1 << 22;  // M* = S: slope 1, intercept 0
        } else if (s_b[e][0] > 0) {
            const i128 Ss = sb[1 + 4 * c], Sm = sb[2 + 4 * c], Sss = sb[3 + 4 * c], Ssm = sb[4 + 4 * c];
            const i128 num = nn * Ssm - Ss * Sm;
            const i128 den = nn * Sss - Ss * Ss;
            const i128 a = den == 0 ? (i128)0 : rhu128(num * ((i128)1 << 22), den);
            const i128 bb = rhu128(Sm * ((i128)1 << 22) - a * Ss, nn * 256);
            aq = (int32_t)a;
            bq = (int32_t)bb;
        }
        h->a_q[c][e] = aq;
        h->b_q[c][e] = bq;
        h->flag[c][e] = 0;
    }
    // The last four waves, one lane per exponent: presence and, for the
    // learned path, inclusive scans of the region sizes and of their
    // histogram workgroup counts (ceil(n / LCH)) within each wave.
    const int e = t - 3 * 256, lane = t & 63;
    uint32_t ne = 0, nc = 0, pe = 0, pc = 0;
    if (t >= 3 * 256) {
        ne = (uint32_t)s_b[e][0];  // n <= H*W < 2^31
        nc = (ne + LCH - 1) / LCH;
        const bool present = ne > 0;
        h->present[e] = present;
        const unsigned long long bal = __ballot(present);
        if (lane == 0) s_cnt[e >> 6] = __popcll(bal);
        pe = ne;
        pc = nc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t xe = __shfl_up(pe, off, 64), xc = __shfl_up(pc, off, 64);
            if (lane >= off) { pe += xe; pc += xc; }
        }
        if (lane == 63) { s_tot[0][e >> 6] = pe; s_tot[1][e >> 6] = pc; }
    }
    __syncthreads();
    if (t == 0) h->n_regions = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    if (t >= 3 * 256 && d.lbk) {
        // Exclusive prefixes: the first record of each exponent's bucket (and
        // its write cursor for k_learn), the first histogram workgroup.
        for (int w = 0; w < (e >> 6); ++w) { pe += s_tot[0][w]; pc += s_tot[1][w]; }
        d.lbk[e] = pe - ne;
        d.lbk[256 + e] = pc - nc;
        d.lbk[513 + e] = pe - ne;
        if (e == 255) d.lbk[256 + 256] = pc;
    }
}

// ---------------------------------------------------------------------------
// K5 residuals: r = M - M*, M* = clamp((a_q s + 2^8 b_q + 2^21) >> 22, 0, 255)
// (Eq. 8), written as int16 planes, plus the exponent plane.  Same strip walk
// as the fit, with the image's coefficients in LDS.
// ---------------------------------------------------------------------------
// Bounds of valid coefficients: |a| <= 255 (a weighted mean of pairwise slopes
// (m_i - m_j)/(s_i - s_j), |s_i - s_j| >= 1), and b = mean m - a mean s, so
// -65025 <= b <= 65280; both scaled by their fixed-point units.
constexpr int32_t AQ_MAX = 255 << 22;
constexpr int32_t BQ_MIN = -65025 * 16384, BQ_MAX = 65280 * 16384;
__device__ __forceinline__ bool coef_ok(int32_t aq, int32_t bq) {
    return aq >= -AQ_MAX && aq <= AQ_MAX && bq >= BQ_MIN && bq <= BQ_MAX;
}

// A region's coefficients prepared for M* in 32-bit arithmetic: with
// a_q = 2^8 ah + al (0 <= al < 2^8), x holds ah in its low 24 bits (signed)
// and al in its top 8, y = b_q + 2^13.
__device__ __forceinline__ int2 coef_prep(int32_t aq, int32_t bq) {
    const uint32_t ah = (uint32_t)(aq >> 8) & 0xFFFFFFu, al = (uint32_t)aq & 255u;
    return make_int2((int)(ah | (al << 24)), bq + 8192);
}

// M* = clamp(floor((a_q s + 2^8 b_q + 2^21) / 2^22), 0, 255).  The numerator
// is 2^8 V + u with V = ah s + b_q + 2^13 and 0 <= u = al s < 2^16, so the
// quotient is floor((V + floor(u / 2^8)) / 2^14); for coefficients within
// the bounds above |V| < 2^31, so the 32-bit result is exact.
__device__ __forceinline__ int mstar(int2 k, int s) {
    const int v = __mul24(k.x, s) + k.y;
    const int u = (int)((((uint32_t)k.x >> 24) * (uint32_t)s) >> 8);
    return min(max((v + u) >> 14, 0), 255);
}

template <bool GF = true>
__global__ __launch_bounds__(STRIP_THREADS) void k_resid(const ImgDesc *__restrict__ D, int n) {
    __shared__ int2 s_ab[3][256];
    const int i = find_img(D, n, blockIdx.x, 4);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    const int wgl = blockIdx.x - d.wg_res;
    const rdl_header *h = d.hdr;
    for (int k = threadIdx.x; k < 3 * 256; k += STRIP_THREADS) {
        const int c = k >> 8, e = k & 255;
        s_ab[c][e] = coef_prep(h->a_q[c][e], h->b_q[c][e]);
    }
    __syncthreads();
    const StripPos sp = strip_pos(wgl, H, W, d.srh_res);
    if (sp.ya >= H) return;  // uniform per wave; no barrier follows
    const int64_t npx = (int64_t)H * W;
    int16_t *r = (int16_t *)d.resid;
    uint8_t *Ep = d.resid + 6 * npx;
    const bool al = (W & 3) == 0 && ((reinterpret_cast<uintptr_t>(d.resid) & 7) == 0);
    // Residuals of the lane's four pixels of row y.
    const auto emit = [&](int y, const int (&s)[3][4], const uint32_t (&w)[4]) {
        if (sp.x >= W) return;
        const int64_t ro = (int64_t)uniform(y) * W;  // row bases are scalar
        int rv[3][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = (int)(w[j] >> 24);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rv[c][j] = (int)((w[j] >> (8 * c)) & 255u) - mstar(s_ab[c][e], s[c][j]);
            }
        }
        int16_t *rr = r + ro;
        uint8_t *er = Ep + ro;
        if (al && sp.x + 4 <= W) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uint2 v;
                v.x = (uint32_t)pack_i16(rv[c][0], rv[c][1]);
                v.y = (uint32_t)pack_i16(rv[c][2], rv[c][3]);
                *reinterpret_cast<uint2 *>(rr + c * npx + (uint32_t)sp.x) = v;
            }
            *reinterpret_cast<uint32_t *>(er + (uint32_t)sp.x) =
                (w[0] >> 24) | ((w[1] >> 24) << 8) | ((w[2] >> 24) << 16) | ((w[3] >> 24) << 24);
        } else {
            const int nx = min(4, W - sp.x);
            for (int j = 0; j < nx; ++j) {
#pragma unroll
                for (int c = 0; c < 3; ++c) rr[c * npx + sp.x + j] = (int16_t)rv[c][j];
                er[sp.x + j] = (uint8_t)(w[j] >> 24);
            }
        }
    };
    strip_walk<GF>(d, sp, emit);
}

// Learned path, last stage: k_learn left the SLR residual planes, the
// exponent plane and every pixel's learned residuals in the outputs; in the
// regions flagged learned each channel's residual becomes the learned one.
// The key statistic's grid (KS_PX_PER_WG consecutive pixels per workgroup,
// 16 waves so that a small image still keeps enough loads in flight).  A
// step covers 8 x 1024 pixel pairs (2k, 2k + 1), lane-consecutive so that
// every plane is read and written in whole lines at any alignment; a pair's
// exponents come in one aligned 16-bit load (the exponent plane starts 6 H W
// bytes into the 2-byte aligned residual buffer).  An odd image's last pixel
// is done on its own.  An image without a flagged region returns at once.
constexpr int PATCH_THREADS = 1024, PATCH_PAIRS = 8;
static_assert(KS_PX_PER_WG % (2 * PATCH_THREADS * PATCH_PAIRS) == 0, "k_resid_patch: whole steps per workgroup");
__device__ __forceinline__ int lres_field(uint32_t w, int c) { return (int)((w >> (9 * c)) & 511u) - 255; }

__global__ __launch_bounds__(PATCH_THREADS) void k_resid_patch(const ImgDesc *__restrict__ D, int n) {
    constexpr int STEP = 2 * PATCH_THREADS * PATCH_PAIRS, NSTEP = KS_PX_PER_WG / STEP;
    __shared__ uint8_t s_fl[256];  // bit c set: channel c of exponent e is learned
    const int i = find_img(D, n, blockIdx.x, 0);
    const ImgDesc d = desc_at(D, i);
    const int64_t npx = (int64_t)d.H * d.W;
    const int64_t pe = npx & ~(int64_t)1;  // pixels in whole pairs
    const int wgl = blockIdx.x - d.wg_px;
    const int64_t base = (int64_t)wgl * KS_PX_PER_WG + 2 * (int)threadIdx.x;  // the thread's first pixel
    const uint8_t *__restrict__ ep = d.resid + 6 * npx;
    int16_t *res = reinterpret_cast<int16_t *>(d.resid);
    const uint32_t *__restrict__ lr = reinterpret_cast<const uint32_t *>(d.lres);
    // Exponents of the pairs of step it, low byte = even pixel.  The address
    // is clamped to the last whole pair (so the loads stay unconditional and
    // inside the plane); pairs past it are masked when used.
    const auto load_e = [&](int it, uint32_t (&ev)[PATCH_PAIRS]) {
#pragma unroll
        for (int j = 0; j < PATCH_PAIRS; ++j)
            ev[j] = *reinterpret_cast<const uint16_t *>(ep + min(base + it * STEP + 2 * j * PATCH_THREADS, pe - 2));
    };
    uint32_t ev[2][PATCH_PAIRS];
    if (pe >= 2) load_e(0, ev[0]);  // in flight with the flags
    int f0 = 0;
    if (threadIdx.x < 256) {  // one exponent per thread
        const int e = threadIdx.x;
        f0 = d.hdr->flag[0][e] | (d.hdr->flag[1][e] << 1) | (d.hdr->flag[2][e] << 2);
        s_fl[e] = (uint8_t)f0;
    }
    if (!__syncthreads_or(f0)) return;  // uniform
    const auto patch = [&](int64_t p, uint32_t f, uint32_t w) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if ((f >> c) & 1) res[c * npx + p] = (int16_t)lres_field(w, c);
    };
#pragma unroll
    for (int it = 0; it < NSTEP; ++it) {
        const int64_t p0 = base + it * STEP;
        if (p0 >= pe) break;
        if (it + 1 < NSTEP) load_e(it + 1, ev[(it + 1) & 1]);
        uint32_t f[2 * PATCH_PAIRS], any = 0;
#pragma unroll
        for (int j = 0; j < PATCH_PAIRS; ++j) {
            const bool in = p0 + 2 * j * PATCH_THREADS < pe;  // both pixels of the pair
            const uint32_t e2 = ev[it & 1][j];
            f[2 * j] = in ? s_fl[e2 & 255u] : 0u;
            f[2 * j + 1] = in ? s_fl[e2 >> 8] : 0u;
            any |= f[2 * j] | f[2 * j + 1];
        }
        if (!any) continue;
        uint32_t w[2 * PATCH_PAIRS];
#pragma unroll
        for (int k = 0; k < 2 * PATCH_PAIRS; ++k) w[k] = f[k] ? lr[p0 + 2 * (k >> 1) * PATCH_THREADS + (k & 1)] : 0u;
#pragma unroll
        for (int k = 0; k < 2 * PATCH_PAIRS; ++k) patch(p0 + 2 * (k >> 1) * PATCH_THREADS + (k & 1), f[k], w[k]);
    }
    // An odd image's last pixel, by the first thread of the workgroup that
    // holds it.
    if ((npx & 1) && threadIdx.x == 0 && (npx - 1) / KS_PX_PER_WG == wgl) {
        const int64_t p = npx - 1;
        const uint32_t f = s_fl[ep[p]];
        if (f) patch(p, f, lr[p]);
    }
}

// ---------------------------------------------------------------------------
// K6 decode: M = M* + r, RGBE out.  The header is checked first; a mismatch
// or a mantissa outside [0, 255] sets *status = RDL_ECORRUPT.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(STRIP_THREADS) void k_decode(const ImgDesc *__restrict__ D, int n) {
    __shared__ int2 s_ab[3][256];
    const int i = find_img(D, n, blockIdx.x, 4);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    const rdl_header *h = d.hdr;
    // estimator: bits 0-3 the estimator (0 SLR per region, 1 learned, 2 one
    // line per channel, 3 M* = S), bit 4 the Gaussian filter off.
    const int est = h->estimator & 15;
    const bool gf = (h->estimator & 16) == 0;
    const bool ok = h->magic == RDL_MAGIC && h->version == RDL_VERSION && h->H == H && h->W == W &&
                    (h->estimator & ~31) == 0 && est <= 3 && (est != 1 || (gf && d.model));
    if (!ok) {
        if (threadIdx.x == 0 && d.status) atomicExch(d.status, RDL_ECORRUPT);
        return;
    }
    if (est == 1) return;  // decoded by k_decode_learned
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < 3 * 256; k += STRIP_THREADS) {
        const int c = k >> 8, e = k & 255;
        const int32_t aq = h->a_q[c][e], bq = h->b_q[c][e];
        if (!coef_ok(aq, bq)) s_bad = 1;
        s_ab[c][e] = coef_prep(aq, bq);
    }
    __syncthreads();
    if (s_bad) {  // uniform
        if (threadIdx.x == 0 && d.status) atomicExch(d.status, RDL_ECORRUPT);
        return;
    }
    const StripPos sp = strip_pos(blockIdx.x - d.wg_res, H, W, d.srh_res);
    if (sp.ya >= H) return;
    const int64_t npx = (int64_t)H * W;
    const int16_t *r = (const int16_t *)d.resid;
    const uint8_t *Ep = d.resid + 6 * npx;
    uint32_t *out = reinterpret_cast<uint32_t *>(d.out_rgbe);
    // Wide accesses where every row starts on the boundary they need: W a
    // multiple of 4 (so y W + x is), the layer on 8 bytes and the output on
    // 16; the lane's four pixels are then inside the image or all past it.
    const bool wide = (W & 3) == 0 && (reinterpret_cast<uintptr_t>(d.resid) & 7) == 0 &&
                      (reinterpret_cast<uintptr_t>(d.out_rgbe) & 15) == 0;
    struct Side {
        uint32_t e;        // the exponents of the lane's four pixels, one byte each
        uint32_t r[3][2];  // their residuals per channel, two int16 per word
    };
    bool bad = false;
    const auto issue = [&](int yy, Side &o) {
        const int64_t off = (int64_t)yy * W + sp.x;
        if (wide && sp.fx) {
            o.e = *reinterpret_cast<const uint32_t *>(Ep + off);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint2 v = *reinterpret_cast<const uint2 *>(r + c * npx + off);
                o.r[c][0] = v.x;
                o.r[c][1] = v.y;
            }
        } else {
            o.e = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) o.r[c][0] = o.r[c][1] = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t oj = (int64_t)yy * W + min(sp.x + j, W - 1);
                o.e |= (uint32_t)Ep[oj] << (8 * j);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    o.r[c][j >> 1] |= (uint32_t)(uint16_t)r[c * npx + oj] << (16 * (j & 1));
            }
        }
    };
    const auto rowf = [&](int y, const int (&s)[3][4], const Side &o) {
        if (sp.x >= W) return;
        uint32_t wd[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = (int)((o.e >> (8 * j)) & 255u);
            uint32_t word = (uint32_t)e << 24;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int rv = (int)(int16_t)(o.r[c][j >> 1] >> (16 * (j & 1)));
                const int m = mstar(s_ab[c][e], s[c][j]) + rv;
                bad |= ((m < 0) | (m > 255)) && sp.x + j < W;
                word |= (uint32_t)(m & 255) << (8 * c);
            }
            wd[j] = word;
        }
        const int64_t o4 = (int64_t)y * W + sp.x;
        if (wide && sp.fx) {
            *reinterpret_cast<uint4 *>(out + o4) = make_uint4(wd[0], wd[1], wd[2], wd[3]);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (sp.x + j < W) out[o4 + j] = wd[j];
        }
    };
    if (gf)
        strip_walk_side<Side, true>(d, sp, issue, rowf);
    else
        strip_walk_side<Side, false>(d, sp, issue, rowf);
    if (bad && d.status) atomicExch(d.status, RDL_ECORRUPT);
}
// ---------------------------------------------------------------------------
// Learned int8 mantissa estimator (an extension beyond the paper, whose
// estimator needs no learning).  Model blob layout (little endian, 7512 B):
// 24-byte head, then W1 i8[32][32] (out, in), B1 i32[32][32] (exponent bin,
// out), m1/r1 i32[32], W2 i8[32][32], B2/m2/r2 i32[32], W3 i8[16][32],
// B3/m3/r3 i32[16].  Features: the 3x3 neighbourhood of S, 3 bytes per
// neighbour (S - 128 as int8), 27 of 32 slots; the exponent enters as the bias
// row B1[bin], bin = clamp(E - 136 + k_img + 24, 0, 31).  Hidden layers:
// a = clamp((h m + 2^(r-1)) >> r, 0, 255); output: q8 = (o m3 + 2^(r3-1)) >>
// r3, M_L = clamp((q8 + 128) >> 8, 0, 255).  The library accepts only models
// whose multipliers, shifts and biases keep every product below 2^31, so
// 32-bit arithmetic equals the exact one.
//
// The MFMA operands are signed bytes, so a hidden activation a in [0, 255]
// enters the next layer as a - 128 (a XOR 0x80), and the next layer's bias
// carries 128 sum_k W[n][k]: sum_k W[n][k] (a_k - 128) + b_n + 128 sum_k
// W[n][k] = sum_k W[n][k] a_k + b_n exactly.
//
// Each layer is an int8 MFMA D = W X with pixels along N: v_mfma_i32_16x16x32
// takes lane l's A bytes = W[l%16][k], B bytes = X[k][l%16] for the eight k of
// lane quad q = l/16, and returns D[4q + t][l%16], t = 0..3: four output
// neurons of one pixel per lane.  A 32-neuron layer is two MFMAs (neurons
// 0-15 and 16-31), so after requantisation lane (j, q) holds neurons
// 4q..4q+3 and 16+4q..16+4q+3 of pixel j.  The next layer takes exactly those
// eight as its k = 8q..8q+7 (its weight columns are read in that order), so a
// lane feeds its own bytes forward with no exchange between lanes.  The
// output layer's rows repeat R, G, B, 0 in every quad, so quad q of group g's
// result holds pixel 16g + j's estimates; lane l keeps group l/16's, which is
// pixel l.
// ---------------------------------------------------------------------------
constexpr int MB_W1 = 24, MB_B1 = 1048, MB_M1 = 5144, MB_R1 = 5272, MB_W2 = 5400, MB_B2 = 6424, MB_M2 = 6552,
              MB_R2 = 6680, MB_W3 = 6808, MB_B3 = 7320, MB_M3 = 7384, MB_R3 = 7448;
typedef int v4i __attribute__((ext_vector_type(4)));

// Requantisation paths of the hidden layers, chosen per model when it is
// set.  RQ_GENERAL: a = clamp((h m + 2^(r-1)) >> r, 0, 255), bytes packed,
// then XOR 0x80.  RQ_POW2: every hidden multiplier is 1 and every hidden
// shift at most 22, so the rounding constant and the offset ride on the
// biases (the MFMAs' C inputs) and a - 128 = clamp((h + 2^(r-1) - 2^(r+7))
// >> r, -128, 127).  RQ_PAIR: RQ_POW2 with equal shifts in every neuron pair
// (2k, 2k + 1), where one v_ashr_pk_i8_i32 shifts, saturates and packs the
// pair.
enum { RQ_GENERAL = 0, RQ_POW2 = 1, RQ_PAIR = 2 };

struct MlpLane {
    long w1a, w1b, w2a, w2b;      // this lane's A fragments of layers 1 and 2
    long w3[4];                   // output layer, one fragment per pixel group (see mlp_wave64)
    int m1[8], r1[8], c1[8];      // requantisation of this lane's eight neurons: multiplier,
    int m2[8], r2[8], c2[8];      //   shift, rounding constant 2^(r-1)
    int b2[8];                    // layer-2 C input: bias + 128 sum_k W2[n][k]
                                  //   (+ 2^(r-1) - 2^(r+7) unless RQ_GENERAL)
    int m3[3], r3[3], c3[3], b3[3];  // output: multiplier, r3 + 8, 2^(r3-1) + 2^(r3+7),
                                     //   bias + 128 sum_k W3[c][k]
};

// Eight weight bytes of row `row` at the columns lane quad q takes as its k:
// 4q..4q+3, then 16+4q..16+4q+3.
__device__ __forceinline__ long w_fwd(const uint8_t *__restrict__ w, int row, int q) {
    const uint32_t lo = *reinterpret_cast<const uint32_t *>(w + row * 32 + 4 * q);
    const uint32_t hi = *reinterpret_cast<const uint32_t *>(w + row * 32 + 16 + 4 * q);
    return (long)((uint64_t)lo | ((uint64_t)hi << 32));
}

template <int RQ>
__device__ __forceinline__ void mlp_lane_load(MlpLane &L, const uint8_t *__restrict__ blob, int lane) {
    const int j = lane & 15, q = lane >> 4;
    L.w1a = *reinterpret_cast<const long *>(blob + MB_W1 + j * 32 + 8 * q);
    L.w1b = *reinterpret_cast<const long *>(blob + MB_W1 + (16 + j) * 32 + 8 * q);
    L.w2a = w_fwd(blob + MB_W2, j, q);
    L.w2b = w_fwd(blob + MB_W2, 16 + j, q);
    // Output fragments: in group g only A rows 4g..4g+2 (channels R, G, B)
    // are non-zero, so group g's estimates land in rows 4g..4g+3 of the
    // accumulated result.
#pragma unroll
    for (int g = 0; g < 4; ++g) L.w3[g] = (j >> 2) == g && (j & 3) < 3 ? w_fwd(blob + MB_W3, j & 3, q) : 0;
    const int32_t *m1 = reinterpret_cast<const int32_t *>(blob + MB_M1), *r1 = reinterpret_cast<const int32_t *>(blob + MB_R1);
    const int32_t *m2 = reinterpret_cast<const int32_t *>(blob + MB_M2), *r2 = reinterpret_cast<const int32_t *>(blob + MB_R2);
    // the biases for offset inputs, appended to the device copy of the model
    const int32_t *b2x = reinterpret_cast<const int32_t *>(blob + MODEL_B2X);
    const int32_t *m3 = reinterpret_cast<const int32_t *>(blob + MB_M3), *r3 = reinterpret_cast<const int32_t *>(blob + MB_R3);
    const int32_t *b3x = reinterpret_cast<const int32_t *>(blob + MODEL_B3X);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int nn = t < 4 ? 4 * q + t : 16 + 4 * q + t - 4;
        L.m1[t] = m1[nn]; L.r1[t] = r1[nn]; L.c1[t] = 1 << (r1[nn] - 1);
        L.m2[t] = m2[nn]; L.r2[t] = r2[nn]; L.c2[t] = 1 << (r2[nn] - 1);
        L.b2[t] = b2x[nn] + (RQ != RQ_GENERAL ? L.c2[t] - (1 << (r2[nn] + 7)) : 0);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        L.m3[t] = m3[t];
        L.r3[t] = r3[t] + 8;
        L.c3[t] = (1 << (r3[t] - 1)) + (1 << (r3[t] + 7));
        L.b3[t] = b3x[t];
    }
}

// The bias table B1[bin][neuron] in LDS, with each neuron's rounding constant
// and offset 2^(r-1) - 2^(r+7) added unless RQ_GENERAL (256 threads).
template <int RQ>
__device__ __forceinline__ void mlp_bias_load(int32_t (*B1)[32], const uint8_t *__restrict__ blob) {
    const int32_t *b1 = reinterpret_cast<const int32_t *>(blob + MB_B1);
    const int32_t *r1 = reinterpret_cast<const int32_t *>(blob + MB_R1);
    for (int k = threadIdx.x; k < 1024; k += 256) {
        const int r = r1[k & 31];
        (&B1[0][0])[k] = b1[k] + (RQ != RQ_GENERAL ? (1 << (r - 1)) - (1 << (r + 7)) : 0);
    }
}

// One requantised neuron in the low byte: RQ_GENERAL a (XORed with 0x80 by
// the caller), RQ_POW2 a - 128.
template <int RQ>
__device__ __forceinline__ uint32_t requant_byte(int h, int m, int r, int c) {
    if (RQ != RQ_GENERAL) return (uint32_t)min(max(h >> r, -128), 127);
    return (uint32_t)min(max((__mul24(h, m) + c) >> r, 0), 255);
}

// Four neurons' MFMA input bytes a - 128, packed low to high.  RQ_PAIR: one
// shift-saturate-pack per pair and one byte permute; otherwise two byte
// permutes join pairs and a third joins the pairs.
template <int RQ>
__device__ __forceinline__ uint32_t requant4(const v4i h, const int *m, const int *r, const int *c) {
    if (RQ == RQ_PAIR) {
        typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
        const u16x2 p = {__builtin_amdgcn_ashr_pk_i8_i32(h[0], h[1], r[0]),
                         __builtin_amdgcn_ashr_pk_i8_i32(h[2], h[3], r[2])};
        return __builtin_bit_cast(uint32_t, p);
    }
    const uint32_t x01 = __builtin_amdgcn_perm(requant_byte<RQ>(h[1], m[1], r[1], c[1]),
                                               requant_byte<RQ>(h[0], m[0], r[0], c[0]), 0x0c0c0400u);
    const uint32_t x23 = __builtin_amdgcn_perm(requant_byte<RQ>(h[3], m[3], r[3], c[3]),
                                               requant_byte<RQ>(h[2], m[2], r[2], c[2]), 0x0c0c0400u);
    const uint32_t x = __builtin_amdgcn_perm(x23, x01, 0x05040100u);
    return RQ == RQ_GENERAL ? x ^ 0x80808080u : x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS of the estimator: the 64 pixels' features as four 8-byte
// chunks, chunk-major (chunk q = feature bytes 8q..8q+7), so that the 16 lanes
// reading one chunk of 16 consecutive pixels, and the 64 lanes writing one
// chunk each, touch consecutive words; and the pixels' exponent bins.
struct MlpWaveLds {
    uint64_t feat[4][64];
    int bin[64];
};

// M_L of pixel `lane` of the wave, packed R | G << 8 | B << 16 (feat and bin
// filled for all 64 pixels and made visible by the caller, every lane of the
// wave active).  B1 is the bias table in LDS.  The output layer accumulates
// the four groups in one result: group g's fragment is non-zero only in rows
// 4g..4g+2, so lane (j, q) ends with rows 4q..4q+2 of group q, the estimates
// of pixel 16q + j, which is the lane itself.  The output rounding is folded:
// floor((floor((o m3 + 2^(r3-1)) / 2^r3) + 128) / 2^8) =
// floor((o m3 + 2^(r3-1) + 2^(r3+7)) / 2^(r3+8)).
template <int RQ>
__device__ __forceinline__ uint32_t mlp_wave64(const MlpWaveLds &w, const int32_t (*B1)[32], const MlpLane &L,
                                               int lane) {
    const int j = lane & 15, q = lane >> 4;
    const v4i c2a = {L.b2[0], L.b2[1], L.b2[2], L.b2[3]};
    const v4i c2b = {L.b2[4], L.b2[5], L.b2[6], L.b2[7]};
    v4i o = {L.b3[0], L.b3[1], L.b3[2], 0};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int p = 16 * g + j;
        const long xb = (long)w.feat[q][p];
        const int b = w.bin[p];
        const v4i c1a = *reinterpret_cast<const v4i *>(&B1[b][4 * q]);
        const v4i c1b = *reinterpret_cast<const v4i *>(&B1[b][16 + 4 * q]);
        const v4i h1a = __builtin_amdgcn_mfma_i32_16x16x32_i8(L.w1a, xb, c1a, 0, 0, 0);
        const v4i h1b = __builtin_amdgcn_mfma_i32_16x16x32_i8(L.w1b, xb, c1b, 0, 0, 0);
        const long a1 = (long)((uint64_t)requant4<RQ>(h1a, L.m1, L.r1, L.c1) |
                               ((uint64_t)requant4<RQ>(h1b, L.m1 + 4, L.r1 + 4, L.c1 + 4) << 32));
        const v4i h2a = __builtin_amdgcn_mfma_i32_16x16x32_i8(L.w2a, a1, c2a, 0, 0, 0);
        const v4i h2b = __builtin_amdgcn_mfma_i32_16x16x32_i8(L.w2b, a1, c2b, 0, 0, 0);
        const long a2 = (long)((uint64_t)requant4<RQ>(h2a, L.m2, L.r2, L.c2) |
                               ((uint64_t)requant4<RQ>(h2b, L.m2 + 4, L.r2 + 4, L.c2 + 4) << 32));
        o = __builtin_amdgcn_mfma_i32_16x16x32_i8(L.w3[g], a2, o, 0, 0, 0);
    }
    uint32_t word = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t)
        word |= (uint32_t)min(max((__mul24(o[t], L.m3[t]) + L.c3[t]) >> L.r3[t], 0), 255) << (8 * t);
    return word;
}

// The 3x3 neighbourhood of a pixel as three rows of (left, centre, right) S
// words (R | G << 8 | B << 16); a wave walks down its rows and rolls it.
struct Win3 {
    uint32_t w[3][3];
    uint32_t rb[3], g[3];  // horizontal (1, 6, 1) sums of each row: R | B << 16, and G
};

__device__ __forceinline__ void win_row(Win3 &v, int slot, const uint32_t *trow, int lx) {
    const uint32_t a = trow[lx], b = trow[lx + 1], e = trow[lx + 2];
    v.w[slot][0] = a;
    v.w[slot][1] = b;
    v.w[slot][2] = e;
    // no field exceeds 8 * 255 < 2^16
    v.rb[slot] = __umul24(b & 0xFF00FFu, 6u) + (a & 0xFF00FFu) + (e & 0xFF00FFu);
    v.g[slot] = __umul24((b >> 8) & 255u, 6u) + ((a >> 8) & 255u) + ((e >> 8) & 255u);
}

__device__ __forceinline__ void win_roll(Win3 &v) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v.w[0][k] = v.w[1][k];
        v.w[1][k] = v.w[2][k];
    }
    v.rb[0] = v.rb[1];
    v.rb[1] = v.rb[2];
    v.g[0] = v.g[1];
    v.g[1] = v.g[2];
}

// S* of the window's centre pixel (no field exceeds 64 * 255 + 32 < 2^16).
__device__ __forceinline__ void win_gf(const Win3 &v, int s[3]) {
    const uint32_t L = v.rb[0] + v.rb[2] + 0x200020u + (v.rb[1] << 2) + (v.rb[1] << 1);  // B sits above bit 23
    const uint32_t G = v.g[0] + v.g[2] + 32u + __umul24(v.g[1], 6u);
    s[0] = (int)((L >> 6) & 255u);
    s[1] = (int)(G >> 6);
    s[2] = (int)(L >> 22);
}

// The window's features as the four 8-byte chunks of the MFMA operand: the
// nine neighbours' bytes (S - 128) concatenated row by row, 27 bytes, then 5
// zero bytes.
__device__ __forceinline__ void win_features(const Win3 &v, uint64_t f[4]) {
    const uint32_t *n = &v.w[0][0];  // n[k] = neighbour k, row-major
    const uint32_t f0 = __builtin_amdgcn_perm(n[1], n[0], 0x04020100u) ^ 0x80808080u;
    const uint32_t f1 = __builtin_amdgcn_perm(n[2], n[1], 0x05040201u) ^ 0x80808080u;
    const uint32_t f2 = __builtin_amdgcn_perm(n[3], n[2], 0x06050402u) ^ 0x80808080u;
    const uint32_t f3 = __builtin_amdgcn_perm(n[5], n[4], 0x04020100u) ^ 0x80808080u;
    const uint32_t f4 = __builtin_amdgcn_perm(n[6], n[5], 0x05040201u) ^ 0x80808080u;
    const uint32_t f5 = __builtin_amdgcn_perm(n[7], n[6], 0x06050402u) ^ 0x80808080u;
    const uint32_t f6 = n[8] ^ 0x808080u;
    f[0] = (uint64_t)f0 | ((uint64_t)f1 << 32);
    f[1] = (uint64_t)f2 | ((uint64_t)f3 << 32);
    f[2] = (uint64_t)f4 | ((uint64_t)f5 << 32);
    f[3] = (uint64_t)f6;
}

constexpr int LT_W = LEARN_W, LT_H = LEARN_TILE_H;  // a workgroup walks `tiles` tiles of 16 x 64 px
__device__ __forceinline__ void load_lt_tile(uint32_t (*t)[LT_W + 2], const uint8_t *__restrict__ sdr, int H, int W,
                                             int ty0, int tx0) {
    for (int k = threadIdx.x; k < (LT_H + 2) * (LT_W + 2); k += 256) {
        const int ry = k / (LT_W + 2), rx = k - ry * (LT_W + 2);
        const int yy = min(max(ty0 + ry - 1, 0), H - 1), xx = min(max(tx0 + rx - 1, 0), W - 1);
        t[ry][rx] = load_px3(sdr + 3 * ((int64_t)yy * W + xx));
    }
}

// The same tile, fetched into registers (LT_PER_THREAD words per thread) so
// that the loads of the next tile overlap the work on the current one.
constexpr int LT_WORDS = (LT_H + 2) * (LT_W + 2);
constexpr int LT_PER_THREAD = (LT_WORDS + 255) / 256;
// ry[k], xx[k]: this thread's tile row and clamped image column of word k.
__device__ __forceinline__ void lt_slots(int W, int tx0, int ry[LT_PER_THREAD], int xx[LT_PER_THREAD]) {
#pragma unroll
    for (int k = 0; k < LT_PER_THREAD; ++k) {
        const int q = min((int)threadIdx.x + 256 * k, LT_WORDS - 1);
        ry[k] = q / (LT_W + 2);
        xx[k] = min(max(tx0 + q - ry[k] * (LT_W + 2) - 1, 0), W - 1);
    }
}
__device__ __forceinline__ void fetch_lt_tile(uint32_t v[LT_PER_THREAD], const uint8_t *__restrict__ sdr, int H,
                                              int W, int ty0, const int ry[LT_PER_THREAD],
                                              const int xx[LT_PER_THREAD]) {
#pragma unroll
    for (int k = 0; k < LT_PER_THREAD; ++k) {
        const int yy = min(max(ty0 + ry[k] - 1, 0), H - 1);
        v[k] = load_px3(sdr + 3 * ((int64_t)yy * W + xx[k]));
    }
}
__device__ __forceinline__ void store_lt_tile(uint32_t (*t)[LT_W + 2], const uint32_t v[LT_PER_THREAD]) {
#pragma unroll
    for (int k = 0; k < LT_PER_THREAD; ++k) {
        const int q = threadIdx.x + 256 * k;
        if (q < LT_WORDS) (&t[0][0])[q] = v[k];
    }
}

// Row-wise fetch of a tile into registers: wave w takes tile rows w, w + 4,
// ..., lane l column l (image column tx0 - 1 + l, clamped); lanes 0-35 of
// wave 0 also take the last two columns of every row (row l / 2, column
// 64 + l % 2).  Row bases are wave-uniform, so only the column offsets are
// per lane, computed once.
constexpr int LT_ROWS_PER_WAVE = (LT_H + 2 + 3) / 4;  // 5
struct LtCols {
    uint32_t off;    // 3 * clamped image column of tile column `lane`
    uint32_t off2;   // 3 * clamped image column of tile column 64 + lane % 2
};
__device__ __forceinline__ LtCols lt_cols(int W, int tx0, int lane) {
    LtCols c;
    c.off = 3u * (uint32_t)min(max(tx0 - 1 + lane, 0), W - 1);
    c.off2 = 3u * (uint32_t)min(tx0 + 63 + (lane & 1), W - 1);
    return c;
}
__device__ __forceinline__ const uint8_t *lt_row(const uint8_t *__restrict__ sdr, int H, int W, int ty0, int ry) {
    const int yy = uniform(min(max(ty0 + ry - 1, 0), H - 1));
    return sdr + (int64_t)yy * (3 * (int64_t)W);
}
// S word of the pixel at p: two dwords from the dword boundary at or below
// p, byte-aligned (S starts on a dword boundary, which the entry points
// check), or three bytes where those 8 bytes would pass the end of S.
__device__ __forceinline__ uint32_t load_px3w(const uint8_t *p, const uint8_t *end) {
    const uint32_t sh = (uint32_t)reinterpret_cast<uintptr_t>(p) & 3u;
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p - sh);
    if (reinterpret_cast<const uint8_t *>(q) + 8 <= end)
        return __builtin_amdgcn_alignbyte(q[1], q[0], sh) & 0xFFFFFFu;
    return load_px3(p);
}
__device__ __forceinline__ void fetch_lt_rows(uint32_t v[LT_ROWS_PER_WAVE + 1], const uint8_t *__restrict__ sdr, int H,
                                              int W, int ty0, int wave, int lane, const LtCols &c) {
    const uint8_t *end = sdr + (int64_t)H * (3 * (int64_t)W);
#pragma unroll
    for (int k = 0; k < LT_ROWS_PER_WAVE; ++k) {
        const int ry = wave + 4 * k;
        v[k] = ry < LT_H + 2 ? load_px3w(lt_row(sdr, H, W, ty0, ry) + c.off, end) : 0u;
    }
    v[LT_ROWS_PER_WAVE] = 0u;
    if (wave == 0 && lane < 2 * (LT_H + 2)) {
        const int yy = min(max(ty0 + (lane >> 1) - 1, 0), H - 1);
        v[LT_ROWS_PER_WAVE] = load_px3w(sdr + (int64_t)yy * (3 * (int64_t)W) + c.off2, end);
    }
}
__device__ __forceinline__ void store_lt_rows(uint32_t (*t)[LT_W + 2], const uint32_t v[LT_ROWS_PER_WAVE + 1],
                                              int wave, int lane) {
#pragma unroll
    for (int k = 0; k < LT_ROWS_PER_WAVE; ++k) {
        const int ry = wave + 4 * k;
        if (ry < LT_H + 2) t[ry][lane] = v[k];
    }
    if (wave == 0 && lane < 2 * (LT_H + 2)) t[lane >> 1][64 + (lane & 1)] = v[LT_ROWS_PER_WAVE];
}

__device__ __forceinline__ int mlp_bin(int e, int k_img) { return min(max(e - 136 + k_img + 24, 0), 31); }

// One wave row of the estimator: the window's features and bins to LDS, then
// the three layers; returns M_L of this lane's pixel.
template <int RQ>
__device__ __forceinline__ uint32_t mlp_row(MlpWaveLds &wl, const int32_t (*B1)[32], const MlpLane &L, const Win3 &v,
                                            int e, int k_img, int lane) {
    uint64_t f[4];
    win_features(v, f);
#pragma unroll
    for (int k = 0; k < 4; ++k) wl.feat[k][lane] = f[k];
    wl.bin[lane] = mlp_bin(e, k_img);
    wave_lds_sync();
    const uint32_t ml = mlp_wave64<RQ>(wl, B1, L, lane);
    wave_lds_sync();  // feat and bin are rewritten for the next row
    return ml;
}

// Residual record of one pixel: r + 255 of the three channels for the SLR
// estimate in bits 0-26 and for the learned one in bits 32-58, 9 bits each.
__device__ __forceinline__ uint64_t lrec_pack(const int rs[3], const int rl[3]) {
    const uint32_t lo = (uint32_t)(rs[0] + 255) | ((uint32_t)(rs[1] + 255) << 9) | ((uint32_t)(rs[2] + 255) << 18);
    const uint32_t hi = (uint32_t)(rl[0] + 255) | ((uint32_t)(rl[1] + 255) << 9) | ((uint32_t)(rl[2] + 255) << 18);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Encoder side: the SLR residual planes and the exponent plane of the output
// (final wherever the region stays SLR), the learned residuals M - M_L as
// 9-bit fields (r_c + 255 at bit 9c, for the last stage), and both
// estimators' residuals as one record per pixel in the bucket of its
// exponent.  Bucket e starts at the number of pixels with a smaller exponent
// (k_solve sets the cursors there); per 16-row tile the workgroup ranks its
// pixels of each exponent with LDS atomics, reserves that many records with
// one global atomic per exponent before it computes the tile's estimates,
// and writes the records after them.  Record order within a bucket is free:
// only histograms are taken from it.  A workgroup takes a 64-px-wide column
// of `tiles` tiles (learn_tiles); each wave walks 4 consecutive rows of a
// tile with a rolling 3x3 window of S, which serves both the features and
// the Gaussian filter.
template <int RQ>
__global__ __launch_bounds__(256) void k_learn(const ImgDesc *__restrict__ D, int n, int tiles) {
    __shared__ uint32_t t[LT_H + 2][LT_W + 2];
    __shared__ int2 s_ab[3][256];
    __shared__ int32_t B1[32][32];
    __shared__ MlpWaveLds wl[4];
    __shared__ uint32_t s_cnt[256], s_base[256];
    __shared__ uint64_t s_rec[LT_H][64];   // the tile's records,
    __shared__ uint32_t s_where[LT_H][64];  // and exponent | rank << 8 (~0 outside the image)
    const int i = find_img(D, n, blockIdx.x, 5);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    const rdl_header *h = d.hdr;
    const int wgl = blockIdx.x - d.wg_learn;
    const int ntx = (W + LT_W - 1) / LT_W;
    const int ty0w = (wgl / ntx) * (LT_H * tiles), tx0 = (wgl % ntx) * LT_W;
    for (int k = threadIdx.x; k < 3 * 256; k += 256) s_ab[k >> 8][k & 255] = coef_prep(h->a_q[k >> 8][k & 255], h->b_q[k >> 8][k & 255]);
    mlp_bias_load<RQ>(B1, d.model);
    s_cnt[threadIdx.x] = 0;
    const int lane = threadIdx.x & 63, wave = uniform(threadIdx.x >> 6);
    const int x = tx0 + lane;
    const bool xin = x < W;
    const uint32_t *rgbe32 = reinterpret_cast<const uint32_t *>(d.rgbe);
    MlpLane L;
    mlp_lane_load<RQ>(L, d.model, lane);
    const int k_img = h->k_img;
    // Tile tt + 1's S words and RGBE words are in flight while tile tt is
    // worked on (every condition below is uniform for the workgroup).
    uint32_t sv[LT_ROWS_PER_WAVE + 1], wv[LT_H / 4];
    const LtCols cols = lt_cols(W, tx0, lane);
    const auto fetch_rgbe = [&](int ty, uint32_t out[LT_H / 4]) {
#pragma unroll
        for (int rr = 0; rr < LT_H / 4; ++rr) {
            const int y = uniform(ty + wave * (LT_H / 4) + rr);
            out[rr] = y < H && xin ? (rgbe32 + (int64_t)y * W)[x] : 0u;
        }
    };
    if (ty0w < H) {
        fetch_lt_rows(sv, d.sdr, H, W, ty0w, wave, lane, cols);
        fetch_rgbe(ty0w, wv);
    }
    uint32_t *lres_out = reinterpret_cast<uint32_t *>(d.lres);
    const int64_t npx = (int64_t)H * W;
    int16_t *res16 = reinterpret_cast<int16_t *>(d.resid);
    uint8_t *eplane = d.resid + 6 * npx;
    for (int tt = 0; tt < tiles; ++tt) {
        const int ty0 = ty0w + tt * LT_H;
        if (ty0 >= H) break;
        __syncthreads();
        store_lt_rows(t, sv, wave, lane);
        const int ly0 = wave * (LT_H / 4);
        uint32_t wc[LT_H / 4];
        // Rank the tile's pixels among its pixels of the same exponent (one
        // LDS atomic per pixel; a row holds about a dozen exponents).
#pragma unroll
        for (int rr = 0; rr < LT_H / 4; ++rr) {
            wc[rr] = wv[rr];
            const uint32_t e = wc[rr] >> 24;
            const bool in = xin && ty0 + ly0 + rr < H;
            s_where[ly0 + rr][lane] = in ? (e | (atomicAdd(&s_cnt[e], 1u) << 8)) : ~0u;
        }
        __syncthreads();
        // One lane per exponent reserves the tile's records of it.  The
        // atomics on the shared cursors are slow; their results are first
        // needed after the tile's estimates.
        uint32_t my_base = 0;
        {
            const uint32_t c = s_cnt[threadIdx.x];
            if (c) my_base = atomicAdd(&d.lbk[threadIdx.x], c);
            s_cnt[threadIdx.x] = 0;
        }
        if (tt + 1 < tiles && ty0 + LT_H < H) {
            fetch_lt_rows(sv, d.sdr, H, W, ty0 + LT_H, wave, lane, cols);
            fetch_rgbe(ty0 + LT_H, wv);
        }
        Win3 v;
        win_row(v, 0, t[ly0], lane);      // tile row ly0 = image row ty0 + ly0 - 1
        win_row(v, 1, t[ly0 + 1], lane);
        // One row per iteration, not unrolled: the estimator's registers are
        // then the only large live set, which keeps several waves per SIMD.
#pragma unroll 1
        for (int rr = 0; rr < LT_H / 4; ++rr) {
            const int ly = ly0 + rr, y = uniform(ty0 + ly);
            win_row(v, 2, t[ly + 2], lane);
            const bool in = xin && y < H;
            const uint32_t w = wc[0];
#pragma unroll
            for (int k = 0; k + 1 < LT_H / 4; ++k) wc[k] = wc[k + 1];
            const int e = (int)(w >> 24);
            const uint32_t ml = mlp_row<RQ>(wl[wave], B1, L, v, e, k_img, lane);
            int s[3];
            win_gf(v, s);
            win_roll(v);
            int rs[3], rl[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int m = (int)((w >> (8 * c)) & 255u);
                rs[c] = m - mstar(s_ab[c][e], s[c]);
                rl[c] = m - (int)((ml >> (8 * c)) & 255u);
            }
            s_rec[ly][lane] = lrec_pack(rs, rl);
            if (in) {
                const int64_t ro = (int64_t)y * W;
                (lres_out + ro)[x] = (uint32_t)(rl[0] + 255) | (uint32_t)(rl[1] + 255) << 9 | (uint32_t)(rl[2] + 255) << 18;
                // the SLR residuals and the exponent, final unless the region
                // is flagged learned (k_resid_patch)
#pragma unroll
                for (int c = 0; c < 3; ++c) (res16 + c * npx + ro)[x] = (int16_t)rs[c];
                (eplane + ro)[x] = (uint8_t)e;
            }
        }
        s_base[threadIdx.x] = my_base;
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < LT_H / 4; ++rr) {
            const uint32_t wh = s_where[ly0 + rr][lane];
            if (wh != ~0u) {
                // Bucket totals come from the same pixels (the fit's n_e), so
                // the index stays below H*W; the check only guards the buffer.
                const uint32_t idx = s_base[wh & 255u] + (wh >> 8);
                if (idx < (uint32_t)(H * W)) d.lrec[idx] = s_rec[ly0 + rr][lane];
            }
        }
    }
}

// Residual histograms per (estimator, channel, exponent) from the bucketed
// records.  Workgroup g of an image takes records [k LCH, (k + 1) LCH) of
// exponent e's bucket, where e is the exponent whose first histogram
// workgroup (a prefix over ceil(n_e / LCH)) is the last one <= g.  Counts go
// to LH_COPIES lane-interleaved LDS copies as 16-bit halves of 32-bit words
// (a copy counts the records of LH_THREADS / LH_COPIES threads, at most
// LCH / LH_COPIES = 2^12 per workgroup, so a half cannot carry), then
// each non-zero bin to the image's histogram with one atomic.  Residuals
// cluster near zero, so many lanes of a wave hit the same bin; the copies
// split those collisions LH_COPIES ways, and their odd word stride puts the
// copies of one bin in different LDS banks.
constexpr int LH_STRIDE = 6 * 256 + 1;
__device__ __forceinline__ void lh_inc(uint32_t *h, int hg, uint32_t v) {
    atomicAdd(&h[hg * 256 + (v >> 1)], 1u << ((v & 1u) << 4));
}

constexpr int LH_THREADS = 512;
__device__ __forceinline__ void lh_count(uint32_t *mine, uint64_t r) {
    if (r == ~0ull) return;
    const uint32_t a = (uint32_t)r, b = (uint32_t)(r >> 32);
    lh_inc(mine, 0, a & 511u);
    lh_inc(mine, 1, (a >> 9) & 511u);
    lh_inc(mine, 2, a >> 18);
    lh_inc(mine, 3, b & 511u);
    lh_inc(mine, 4, (b >> 9) & 511u);
    lh_inc(mine, 5, b >> 18);
}

static_assert(LCH / LH_COPIES < 65536, "k_lhist: a 16-bit half counts at most LCH / LH_COPIES records");
__global__ __launch_bounds__(LH_THREADS) void k_lhist(const ImgDesc *__restrict__ D, int n) {
    __shared__ uint32_t hb[LH_COPIES * LH_STRIDE];
    const int i = find_img(D, n, blockIdx.x, 6);
    const ImgDesc d = desc_at(D, i);
    const int g = blockIdx.x - d.wg_lhist;
    const uint32_t *fw = d.lbk + 256;  // first workgroup per exponent, fw[256] = total
    if ((uint32_t)g >= fw[256]) return;  // uniform
    int lo = 0, hi = 256;  // fw[lo] <= g < fw[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (fw[mid] <= (uint32_t)g) lo = mid; else hi = mid;
    }
    const int e = uniform(lo);
    const uint32_t k = (uint32_t)g - fw[e];
    const uint32_t ne = (uint32_t)d.sums[e * NSUM];
    const uint32_t first = d.lbk[513 + e] + k * LCH;
    const uint32_t cnt = min((uint32_t)LCH, ne - k * LCH);
    for (int q = threadIdx.x; q < LH_COPIES * LH_STRIDE; q += LH_THREADS) hb[q] = 0;
    __syncthreads();
    uint32_t *mine = hb + (threadIdx.x & (LH_COPIES - 1)) * LH_STRIDE;
    const uint64_t *rp = d.lrec + first;
    // Batches of U records per thread; the next batch's loads are issued
    // before the current one is counted (a valid record never has its top
    // bits set, so ~0 marks a slot past the end).
    constexpr int U = 4, STEP = LH_THREADS * U;
    uint64_t cur[U], nxt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint32_t j = LH_THREADS * u + threadIdx.x;
        cur[u] = j < cnt ? rp[j] : ~0ull;
    }
    for (uint32_t j0 = 0; j0 < cnt; j0 += STEP) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t j = j0 + STEP + LH_THREADS * u + threadIdx.x;
            nxt[u] = j < cnt ? rp[j] : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) lh_count(mine, cur[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 6 * 511; q += LH_THREADS) {
        const int hgram = q / 511, v = q - hgram * 511;  // hgram = estimator * 3 + channel
        uint32_t c = 0;
#pragma unroll
        for (int cp = 0; cp < LH_COPIES; ++cp) c += (hb[cp * LH_STRIDE + hgram * 256 + (v >> 1)] >> ((v & 1) << 4)) & 0xFFFFu;
        if (c) {
            atomicAdd(&d.lhist[((size_t)hgram * 256 + e) * 511 + v], c);
            if (hgram < 3) atomicAdd(&d.lhist[LHIST_G + hgram * 511 + v], c);  // SLR, whole image
        }
    }
}

// Q16 log2 of a count (0 for 0), from the same frozen table as the key.
__device__ __forceinline__ int64_t log2q16(uint32_t x) {
    if (x == 0) return 0;
    const int p = 31 - __builtin_clz(x);
    const uint32_t idx = p >= 12 ? (x >> (p - 12)) & 4095u : (x << (12 - p)) & 4095u;
    return (int64_t)65536 * p + g_log2f[idx];
}

// Region selection: per (channel, exponent) the learned estimate is taken
// where its residuals cost strictly fewer bits than the SLR residuals under
// the distribution g of the channel's SLR residuals over the whole image:
// cost_k = sum_v h_k[v] (L(N) - L(g_v)), and as both histograms hold the
// region's n_E residuals, cost_L < cost_S exactly when
// sum_v h_L[v] L(g_v) > sum_v h_S[v] L(g_v).  A learned residual value that
// g never takes has no finite cost and keeps SLR.  One workgroup per
// exponent; it leaves the region's six histograms zero.
__global__ __launch_bounds__(256) void k_select(const ImgDesc *__restrict__ D, int n) {
    __shared__ int64_t s_red[4][6];
    __shared__ int s_bad[3];
    const int i = blockIdx.x >> 8, e = blockIdx.x & 255;
    if (i >= n) return;
    const ImgDesc d = desc_at(D, i);
    rdl_header *h = d.hdr;
    if (e == 0 && threadIdx.x == 0) {
        h->estimator = 1;
        h->model_hash = d.model_hash;
    }
    if (!h->present[e]) {
        if (threadIdx.x < 3) h->flag[threadIdx.x][e] = 0;
        return;
    }
    if (threadIdx.x < 3) s_bad[threadIdx.x] = 0;
    // Thread t takes bins t and t + 256 of the six histograms (estimator x
    // channel) and of the three whole-image SLR histograms, all loads issued
    // before the first is used.
    uint32_t cnt[6][2], gl[3][2];
#pragma unroll
    for (int hg = 0; hg < 6; ++hg)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int v = threadIdx.x + 256 * k;
            cnt[hg][k] = v < 511 ? d.lhist[((size_t)hg * 256 + e) * 511 + v] : 0u;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int v = threadIdx.x + 256 * k;
            gl[c][k] = v < 511 ? d.lhist[LHIST_G + c * 511 + v] : 0u;
        }
#pragma unroll
    for (int hg = 0; hg < 6; ++hg)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int v = threadIdx.x + 256 * k;
            if (v < 511) d.lhist[((size_t)hg * 256 + e) * 511 + v] = 0;
        }
    __syncthreads();  // s_bad cleared
    int64_t part[6];
#pragma unroll
    for (int hg = 0; hg < 6; ++hg) {
        const int c = hg % 3;
        part[hg] = 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) part[hg] += (int64_t)cnt[hg][k] * log2q16(gl[c][k]);
        for (int off = 32; off > 0; off >>= 1) part[hg] += __shfl_down(part[hg], off, 64);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if ((cnt[3 + c][0] && !gl[c][0]) || (cnt[3 + c][1] && !gl[c][1])) s_bad[c] = 1;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int hg = 0; hg < 6; ++hg) s_red[threadIdx.x >> 6][hg] = part[hg];
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        const int64_t ps = s_red[0][c] + s_red[1][c] + s_red[2][c] + s_red[3][c];
        const int64_t pl = s_red[0][3 + c] + s_red[1][3 + c] + s_red[2][3 + c] + s_red[3][3 + c];
        h->flag[c][e] = !s_bad[c] && pl > ps ? 1 : 0;
    }
}

// Learned decoder: M = (flag ? M_L : M*) + r for headers with estimator 1.
template <int RQ>
__global__ __launch_bounds__(256) void k_decode_learned(const ImgDesc *__restrict__ D, int n, int tiles) {
    __shared__ uint32_t t[LT_H + 2][LT_W + 2];
    __shared__ int2 s_ab[3][256];
    __shared__ uint8_t s_fl[3][256];
    __shared__ int32_t B1[32][32];
    __shared__ MlpWaveLds wl[4];
    const int i = find_img(D, n, blockIdx.x, 5);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    const rdl_header *h = d.hdr;
    if (h->estimator != 1) return;  // uniform: plain headers are decoded by k_decode
    const bool ok = h->magic == RDL_MAGIC && h->version == RDL_VERSION && h->H == H && h->W == W &&
                    h->model_hash == d.model_hash;
    if (!ok) {
        if (threadIdx.x == 0 && d.status) atomicExch(d.status, RDL_ECORRUPT);
        return;
    }
    const int wgl = blockIdx.x - d.wg_learn;
    const int ntx = (W + LT_W - 1) / LT_W;
    const int ty0w = (wgl / ntx) * (LT_H * tiles), tx0 = (wgl % ntx) * LT_W;
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < 3 * 256; k += 256) {
        const int32_t aq = h->a_q[k >> 8][k & 255], bq = h->b_q[k >> 8][k & 255];
        if (!coef_ok(aq, bq)) s_bad = 1;
        s_ab[k >> 8][k & 255] = coef_prep(aq, bq);
        s_fl[k >> 8][k & 255] = h->flag[k >> 8][k & 255];
    }
    mlp_bias_load<RQ>(B1, d.model);
    __syncthreads();
    if (s_bad) {  // uniform
        if (threadIdx.x == 0 && d.status) atomicExch(d.status, RDL_ECORRUPT);
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    MlpLane L;
    mlp_lane_load<RQ>(L, d.model, lane);
    const int k_img = h->k_img;
    const int64_t npx = (int64_t)H * W;
    const int16_t *r = (const int16_t *)d.resid;
    const uint8_t *Ep = d.resid + 6 * npx;
    uint32_t *out = reinterpret_cast<uint32_t *>(d.out_rgbe);
    const int x = tx0 + lane;
    bool bad = false;
    for (int tt = 0; tt < tiles; ++tt) {
        const int ty0 = ty0w + tt * LT_H;
        __syncthreads();
        if (ty0 < H) load_lt_tile(t, d.sdr, H, W, ty0, tx0);
        __syncthreads();
        if (ty0 >= H) continue;
        const int ly0 = wave * (LT_H / 4);
        Win3 v;
        win_row(v, 0, t[ly0], lane);
        win_row(v, 1, t[ly0 + 1], lane);
#pragma unroll 1
        for (int rr = 0; rr < LT_H / 4; ++rr) {
            const int ly = ly0 + rr, y = ty0 + ly;
            win_row(v, 2, t[ly + 2], lane);
            const bool in = y < H && x < W;
            const int64_t o = (int64_t)y * W + x;
            const int e = in ? (int)Ep[o] : 0;
            const uint32_t ml = mlp_row<RQ>(wl[wave], B1, L, v, e, k_img, lane);
            int s[3];
            win_gf(v, s);
            win_roll(v);
            if (!in) continue;
            uint32_t word = (uint32_t)e << 24;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int2 ab = s_ab[c][e];
                const int est = s_fl[c][e] ? (int)((ml >> (8 * c)) & 255u) : mstar(ab, s[c]);
                const int m = est + r[c * npx + o];
                bad |= (m < 0) | (m > 255);
                word |= (uint32_t)(m & 255) << (8 * c);
            }
            out[o] = word;
        }
    }
    if (bad && d.status) atomicExch(d.status, RDL_ECORRUPT);
}

// ---------------------------------------------------------------------------
// K7 residual histograms: hist[c][r + 255].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TILE_THREADS) void k_hist(const ImgDesc *__restrict__ D, int n) {
    __shared__ uint32_t hb[3][511];
    const int i = find_img(D, n, blockIdx.x, 2);
    const ImgDesc d = desc_at(D, i);
    const int H = d.H, W = d.W;
    for (int k = threadIdx.x; k < 3 * 511; k += TILE_THREADS) (&hb[0][0])[k] = 0;
    __syncthreads();
    const int ntx = (W + TILE_W - 1) / TILE_W;
    const int tile = blockIdx.x - d.wg_tile;
    const int ty0 = (tile / ntx) * TILE_H, tx0 = (tile % ntx) * TILE_W;
    const int ly = threadIdx.x / (TILE_W / RUN), lx = (threadIdx.x % (TILE_W / RUN)) * RUN;
    const int y = ty0 + ly, x = tx0 + lx;
    if (y < H && x < W) {
        const int nx = min(RUN, W - x);
        const int64_t npx = (int64_t)H * W;
        const int16_t *r = (const int16_t *)d.resid + (int64_t)y * W + x;
        for (int c = 0; c < 3; ++c)
            for (int j = 0; j < nx; ++j) atomicAdd(&hb[c][min(max(r[c * npx + j] + 255, 0), 510)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 3 * 511; k += TILE_THREADS) {
        const uint32_t v = (&hb[0][0])[k];
        if (v) atomicAdd((unsigned long long *)&d.hist[k], (unsigned long long)v);
    }
}

// ---------------------------------------------------------------------------
// Host side: tables and launchers.
// ---------------------------------------------------------------------------
void quant_tables_host(int q, uint8_t out[2][64]) {
    const int sc = q < 50 ? 5000 / q : 200 - 2 * q;  // IJG quality scaling
    for (int t = 0; t < 2; ++t)
        for (int k = 0; k < 64; ++k) out[t][k] = (uint8_t)std::min(std::max((ANNEX_K[t][k] * sc + 50) / 100, 1), 255);
}

hipError_t upload_tables(int *bad_table) {
    *bad_table = 0;
    static int32_t log2f[4096];
    static float eh[256], el[256], thr[257];
    static uint32_t glut[GAMMA_LUT_N];
    for (int k = 0; k < 4096; ++k) log2f[k] = (int32_t)std::llround(65536.0 * std::log2(1.0 + (k + 0.5) / 4096.0));
    for (int j = 0; j < 256; ++j) {
        eh[j] = (float)std::exp2(j / 256.0);
        el[j] = (float)std::exp2(j / 65536.0);
    }
    thr[0] = 0.0f;
    for (int k = 1; k < 256; ++k) thr[k] = (float)std::pow((k - 0.5) / 255.0, 2.2);
    thr[256] = INFINITY;
    // Bucket b covers floats whose top 16 bits are b + GAMMA_B0.
    for (int b = 0; b < GAMMA_LUT_N; ++b) {
        uint32_t lo_bits = (uint32_t)(b + GAMMA_B0) << 16;
        uint32_t hi_bits = lo_bits + (1u << 16);
        float lo, hi;
        memcpy(&lo, &lo_bits, 4);
        memcpy(&hi, &hi_bits, 4);
        int cnt = 0, inside = 0;
        uint32_t t = 1u << 16;
        for (int k = 1; k < 256; ++k) {
            if (thr[k] <= lo) {
                cnt++;
            } else if (thr[k] < hi) {
                inside++;
                uint32_t tb;
                memcpy(&tb, &thr[k], 4);
                t = tb & 0xFFFFu;  // >= 1: the threshold is above the bucket start
            }
        }
        if (inside > 1) *bad_table = 1;
        // The clamped end buckets stand for every float below / above them.
        if ((b == 0 || b == GAMMA_LUT_N - 1) && inside) *bad_table = 1;
        glut[b] = ((uint32_t)cnt << 17) + (1u << 17) - t;
    }
    // Below the first bucket every code is 0, from the last one up 255.
    if (thr[1] <= ldexpf(1.0f, -20) || thr[255] >= 2.0f) *bad_table = 1;
    static uint32_t qm[100][2][64][4];
    for (int q = 1; q <= 100; ++q) {
        uint8_t qt[2][64];
        quant_tables_host(q, qt);
        for (int t = 0; t < 2; ++t)
            for (int k = 0; k < 64; ++k) {
                const uint32_t Q = qt[t][k];
                qm[q - 1][t][k][0] = (((1u << 20) + Q - 1u) / Q) | (Q << 24);
                qm[q - 1][t][k][1] = Q / 2;
                qm[q - 1][t][k][2] = (Q & 1u) ? 0u : 0xFFFFFFFFu;
                qm[q - 1][t][k][3] = 0;
            }
    }
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_qm), qm, sizeof qm)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_log2f), log2f, sizeof log2f)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_exp2h), eh, sizeof eh)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_exp2l), el, sizeof el)) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(g_glut), glut, sizeof glut)) != hipSuccess) return e;
    return hipSuccess;
}

// Self-check of recip(): compares it with IEEE division for every float whose
// bits lie in [lo, lo + count) and counts the differences.
__global__ __launch_bounds__(256) void k_check_recip(uint32_t lo, uint32_t count, unsigned long long *bad) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= count) return;
    const float D = __uint_as_float(lo + i);
    if (__float_as_uint(recip(D)) != __float_as_uint(1.0f / D)) atomicAdd(bad, 1ull);
}

void launch_check_recip(uint32_t lo, uint32_t count, unsigned long long *bad, hipStream_t s) {
    if (count) hipLaunchKernelGGL(k_check_recip, dim3((count + 255) / 256), dim3(256), 0, s, lo, count, bad);
}

void launch_zero(const ImgDesc *d, int n, hipStream_t s) { hipLaunchKernelGGL(k_zero, dim3(n), dim3(256), 0, s, d, n); }

// Descriptors passed by value (kernel arguments), written to a device table:
// the table of a launch without a host-to-device copy.
struct DescChunk {
    ImgDesc d[DESC_CHUNK];
};
__global__ void k_put_desc(ImgDesc *dst, DescChunk c, int n) {
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.d[threadIdx.x];
}
void launch_put_desc(ImgDesc *dst, const ImgDesc *host, int n, hipStream_t s) {
    for (int k = 0; k < n; k += DESC_CHUNK) {
        const int m = n - k < DESC_CHUNK ? n - k : DESC_CHUNK;
        DescChunk c;
        for (int j = 0; j < m; ++j) c.d[j] = host[k + j];
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, dst + k, c, m);
    }
}
void launch_keystat(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_keystat, dim3(wgs), dim3(KS_THREADS), 0, s, d, n);
}
void launch_tmo_base(const ImgDesc *d, int n, int wgs, bool extra, hipStream_t s) {
    if (extra)
        hipLaunchKernelGGL(k_tmo_base<true>, dim3(wgs), dim3(BLK_THREADS), 0, s, d, n);
    else
        hipLaunchKernelGGL(k_tmo_base<false>, dim3(wgs), dim3(BLK_THREADS), 0, s, d, n);
}
void launch_fit_sums(const ImgDesc *d, int n, int wgs, int bins, int waves, hipStream_t s, bool gf) {
    const dim3 block(64 * waves);
    if (!gf)
        hipLaunchKernelGGL((k_fit_sums<2, false>), dim3(wgs), block, 0, s, d, n);
    else if (bins >= 4)
        hipLaunchKernelGGL(k_fit_sums<4>, dim3(wgs), block, 0, s, d, n);
    else if (bins == 2)
        hipLaunchKernelGGL(k_fit_sums<2>, dim3(wgs), block, 0, s, d, n);
    else
        hipLaunchKernelGGL(k_fit_sums<1>, dim3(wgs), block, 0, s, d, n);
}
void launch_solve(const ImgDesc *d, int n, hipStream_t s) { hipLaunchKernelGGL(k_solve, dim3(n), dim3(1024), 0, s, d, n); }
void launch_key_total(const ImgDesc *d, int n, int64_t *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_key_total, dim3(n), dim3(64), 0, s, d, n, out2);
}
void launch_resid(const ImgDesc *d, int n, int wgs, hipStream_t s, bool gf) {
    if (gf)
        hipLaunchKernelGGL(k_resid<true>, dim3(wgs), dim3(STRIP_THREADS), 0, s, d, n);
    else
        hipLaunchKernelGGL(k_resid<false>, dim3(wgs), dim3(STRIP_THREADS), 0, s, d, n);
}
void launch_resid_patch(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_resid_patch, dim3(wgs), dim3(PATCH_THREADS), 0, s, d, n);
}
void launch_base_decode(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_base_decode, dim3(wgs), dim3(BLK_THREADS), 0, s, d, n);
}
void launch_status_init(const ImgDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_status_init, dim3((n + 255) / 256), dim3(256), 0, s, d, n);
}
void launch_decode(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_decode, dim3(wgs), dim3(STRIP_THREADS), 0, s, d, n);
}
void launch_learn(const ImgDesc *d, int n, int wgs, int rq, int tiles, hipStream_t s) {
    if (rq == RQ_PAIR)
        hipLaunchKernelGGL(k_learn<RQ_PAIR>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
    else if (rq == RQ_POW2)
        hipLaunchKernelGGL(k_learn<RQ_POW2>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
    else
        hipLaunchKernelGGL(k_learn<RQ_GENERAL>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
}
void launch_lhist(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_lhist, dim3(wgs), dim3(LH_THREADS), 0, s, d, n);
}
void launch_select(const ImgDesc *d, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(256 * n), dim3(256), 0, s, d, n);
}
void launch_decode_learned(const ImgDesc *d, int n, int wgs, int rq, int tiles, hipStream_t s) {
    if (rq == RQ_PAIR)
        hipLaunchKernelGGL(k_decode_learned<RQ_PAIR>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
    else if (rq == RQ_POW2)
        hipLaunchKernelGGL(k_decode_learned<RQ_POW2>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
    else
        hipLaunchKernelGGL(k_decode_learned<RQ_GENERAL>, dim3(wgs), dim3(256), 0, s, d, n, tiles);
}
void launch_hist(const ImgDesc *d, int n, int wgs, hipStream_t s) {
    hipLaunchKernelGGL(k_hist, dim3(wgs), dim3(TILE_THREADS), 0, s, d, n);
}

}  // namespace rdl
