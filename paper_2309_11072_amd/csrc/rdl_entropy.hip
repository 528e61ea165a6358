// rdl_entropy.hip -- gfx950 kernels of the entropy code of the enhancement
// layer: a static rANS coder (Duda, "Asymmetric numeral systems", 2013, the
// range variant) over the three residual planes and the exponent plane, with
// 64 interleaved coder states per group of symbols, one wave per group.  The
// paper hands these planes to an off-the-shelf lossless coder (JPEG 2000,
// Sec. IV); this coder stands in for it.  The stream format is described in
// rdl.h.
//
// Encoder: [k_ent_ediff (left differences of the exponents)] -> k_ent_hist
// (plane histograms) -> k_ent_freq (frequencies, header) -> k_ent_enc (one
// wave per group, words in emission order into a workspace) -> k_ent_scan
// (group offsets) -> k_ent_pack (each group's words reversed into place).
// Decoder: k_ent_dec (tables in LDS, one wave per group) [-> (k_ent_eseg,
// k_ent_ecarry: rows wider than a tile) -> k_ent_eundo: the differences
// summed back along each row, a segmented prefix sum].
// Everything is integer arithmetic except the encoder's division by a
// frequency, which takes a float reciprocal estimate and corrects it to the
// exact quotient.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "rdl_internal.h"

namespace rdl {

namespace {

constexpr int ENT_HC = 4;                  // privatised LDS copies of the histograms
constexpr bool ENT_PACK16 = false;         // 16-bit counters, two per word
constexpr bool ENT_CMINOR = true;          // copies of a bin in adjacent words (else one block per copy)
constexpr int ENT_HWORDS = ENT_PACK16 ? 1024 : 2048;   // words per copy
constexpr int ENT_HSTRIDE = ENT_HWORDS + 1;            // odd stride between copy blocks
constexpr int ENT_HTOTAL = ENT_CMINOR ? ENT_HC * ENT_HWORDS : ENT_HC * ENT_HSTRIDE;
constexpr int ENT_HIST_THREADS = 512;

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over a block of NW waves (every thread receives it).
template <int NW>
__device__ uint32_t block_sum(uint32_t v, uint32_t *sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += sh[k];
    return t;
}

template <int NW>
__device__ unsigned long long block_max64(unsigned long long v, unsigned long long *sh) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, off, 64), hi = __shfl_xor((uint32_t)(v >> 32), off, 64);
        const unsigned long long o = (unsigned long long)hi << 32 | lo;
        v = o > v ? o : v;
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t = sh[k] > t ? sh[k] : t;
    return t;
}

// Exclusive prefix maximum over a block of NW waves (0 before lane 0).
template <int NW>
__device__ uint32_t block_excl_max(uint32_t v, uint32_t *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc = max(inc, y);
    }
    __syncthreads();
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) before = k < w ? max(before, sh[k]) : before;
    const uint32_t ex = __shfl_up(inc, 1, 64);
    return max(before, lane == 0 ? 0u : ex);
}

// Exclusive prefix sum over a block of NW waves; total receives the sum.
template <int NW>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    __syncthreads();
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t before = 0, t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t x = sh[k];
        before += k < w ? x : 0u;
        t += x;
    }
    total = t;
    return before + inc - v;
}

// Plane histograms: residual symbols r + 255 (511 for a value outside
// [-255, 255], never a legal symbol) and exponents.  Counters are 16-bit
// halves of LDS words in ENT_HC copies (lane l counts into copy l mod ENT_HC);
// a bin of one workgroup never exceeds ENT_HIST_PX = 16384 < 2^16, so halves
// cannot carry.  Exponents are smooth across neighbouring pixels, so a wave
// adds each run of equal exponents over consecutive lanes with one atomic (the
// run's first lane adds its length).  The copies are then added into the
// image's histograms with integer atomics.
__device__ __forceinline__ uint32_t ent_word(uint32_t c, uint32_t bin) {
    const uint32_t wb = ENT_PACK16 ? bin >> 1 : bin;
    return ENT_CMINOR ? wb * ENT_HC + c : c * ENT_HSTRIDE + wb;
}

__device__ __forceinline__ void ent_count(uint32_t *h, uint32_t c, uint32_t bin, uint32_t k) {
    atomicAdd(h + ent_word(c, bin), ENT_PACK16 ? k << ((bin & 1) * 16) : k);
}

__global__ __launch_bounds__(ENT_HIST_THREADS) void k_ent_hist(EntArgs a) {
    __shared__ uint32_t h[ENT_HTOTAL];
    for (int k = threadIdx.x; k < ENT_HTOTAL; k += ENT_HIST_THREADS) h[k] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t mine = (uint32_t)lane & (ENT_HC - 1);
    const int64_t i0 = (int64_t)blockIdx.x * ENT_HIST_PX;
    const int n = (int)(a.N - i0 < ENT_HIST_PX ? a.N - i0 : ENT_HIST_PX);
    constexpr int PER = ENT_HIST_PX / ENT_HIST_THREADS;  // 32 px per thread and plane
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int16_t *rp = (const int16_t *)a.resid + p * a.N + i0;
        int v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = j * ENT_HIST_THREADS + threadIdx.x;
            v[j] = (int)rp[min(i, n - 1)];  // clamped: every load is valid, counted below only if i < n
        }
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if (j * ENT_HIST_THREADS + (int)threadIdx.x < n)
                ent_count(h, mine, p * 512 + min((uint32_t)(v[j] + 255), 511u), 1u);
    }
    const uint8_t *e8 = a.eplane + i0;
    int ev[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = j * ENT_HIST_THREADS + threadIdx.x;
        const int v = (int)e8[min(i, n - 1)];
        ev[j] = i < n ? v : -1;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int v = ev[j];
        const int left = __shfl_up(v, 1, 64);
        const bool head = lane == 0 || v != left;
        const unsigned long long m = __ballot(head);
        // the run ends at the next head (a lane past the end has v = -1, a head of its own)
        const unsigned long long after = lane == 63 ? 0ull : m >> (lane + 1);
        const int len = after ? (int)__builtin_ctzll(after) + 1 : 64 - lane;
        if (head && v >= 0) ent_count(h, mine, 3 * 512 + v, (uint32_t)len);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2048; b += ENT_HIST_THREADS) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < ENT_HC; ++k) {
            const uint32_t wv = h[ent_word(k, b)];
            v += ENT_PACK16 ? (wv >> ((b & 1) * 16)) & 0xFFFFu : wv;
        }
        if (v) atomicAdd(&a.ws->hist[blockIdx.x % ENT_HSTRIPES][b >> 9][b & 511], v);
    }
}

// The same histograms from 16-byte loads, for a layer at a 16-byte aligned
// address with at least 16 pixels.  Workgroups [0, nr) read the residual
// planes as one array of 3N int16 values (element e is in plane
// (e >= N) + (e >= 2N)), 8 per lane and load; the rest read the exponent
// bytes, 16 per lane and load, and count each run of equal exponents within
// the lane's 16 bytes with one atomic.  Loads cover whole aligned 16-byte
// chunks: the residual chunks end at most 14 bytes past the residuals, inside
// the exponent plane (N >= 16); the exponent chunks stop at the last chunk
// that ends inside the layer, and the remaining bytes (fewer than 16) are
// counted one per lane by the last workgroup.
constexpr int ENT_VEC_CHUNKS = 8;  // 16-byte chunks per lane and workgroup
constexpr int ENT_VEC_SPAN = ENT_HIST_THREADS * ENT_VEC_CHUNKS * 16;  // bytes per workgroup

__global__ __launch_bounds__(ENT_HIST_THREADS) void k_ent_hist_vec(EntArgs a, int nr) {
    __shared__ uint32_t h[ENT_HTOTAL];
    for (int k = threadIdx.x; k < ENT_HTOTAL; k += ENT_HIST_THREADS) h[k] = 0;
    __syncthreads();
    const uint32_t mine = threadIdx.x & (ENT_HC - 1);
    const int64_t N = a.N;
    if ((int)blockIdx.x < nr) {
        const int64_t nchunk = (6 * N + 15) >> 4;
        const uint4 *src = reinterpret_cast<const uint4 *>(a.resid);
        uint4 q[ENT_VEC_CHUNKS];
        int64_t ch[ENT_VEC_CHUNKS];
#pragma unroll
        for (int j = 0; j < ENT_VEC_CHUNKS; ++j) {
            ch[j] = ((int64_t)blockIdx.x * ENT_VEC_CHUNKS + j) * ENT_HIST_THREADS + threadIdx.x;
            q[j] = src[ch[j] < nchunk ? ch[j] : nchunk - 1];
        }
#pragma unroll
        for (int j = 0; j < ENT_VEC_CHUNKS; ++j) {
            const uint32_t w4[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t e = ch[j] * 8 + k;
                if (ch[j] < nchunk && e < 3 * N) {
                    const int r = (int)(int16_t)(w4[k >> 1] >> (16 * (k & 1)));
                    const uint32_t p = (e >= N) + (e >= 2 * N);
                    ent_count(h, mine, p * 512 + min((uint32_t)(r + 255), 511u), 1u);
                }
            }
        }
    } else {
        const uintptr_t e_lo = reinterpret_cast<uintptr_t>(a.eplane), e_hi = e_lo + N;
        const uintptr_t c_lo = e_lo & ~(uintptr_t)15;
        const int64_t nchunk = (int64_t)((e_hi & ~(uintptr_t)15) - c_lo) >> 4;  // whole chunks inside the layer
        const int wb = (int)blockIdx.x - nr;
        uint4 q[ENT_VEC_CHUNKS];
        int64_t ch[ENT_VEC_CHUNKS];
#pragma unroll
        for (int j = 0; j < ENT_VEC_CHUNKS; ++j) {
            ch[j] = ((int64_t)wb * ENT_VEC_CHUNKS + j) * ENT_HIST_THREADS + threadIdx.x;
            const int64_t cc = ch[j] < nchunk ? ch[j] : (nchunk > 0 ? nchunk - 1 : 0);
            q[j] = nchunk > 0 ? reinterpret_cast<const uint4 *>(c_lo)[cc] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < ENT_VEC_CHUNKS; ++j) {
            if (ch[j] >= nchunk) continue;
            const uint32_t w4[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
            const uintptr_t at = c_lo + (uintptr_t)ch[j] * 16;
            int cur = -1;
            uint32_t len = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int v = (int)((w4[k >> 2] >> (8 * (k & 3))) & 255u);
                const int key = at + k >= e_lo ? v : -1;  // bytes before the plane are residuals
                if (key != cur) {
                    if (cur >= 0) ent_count(h, mine, 3 * 512 + cur, len);
                    cur = key;
                    len = 0;
                }
                ++len;
            }
            if (cur >= 0) ent_count(h, mine, 3 * 512 + cur, len);
        }
        if (wb == (int)gridDim.x - nr - 1) {  // bytes after the last whole chunk
            const uintptr_t t0 = c_lo + (uintptr_t)nchunk * 16;
            const uintptr_t b = (t0 > e_lo ? t0 : e_lo) + threadIdx.x;
            if (b < e_hi) ent_count(h, mine, 3 * 512 + *reinterpret_cast<const uint8_t *>(b), 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 2048; b += ENT_HIST_THREADS) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < ENT_HC; ++k) {
            const uint32_t wv = h[ent_word(k, b)];
            v += ENT_PACK16 ? (wv >> ((b & 1) * 16)) & 0xFFFFu : wv;
        }
        if (v) atomicAdd(&a.ws->hist[blockIdx.x % ENT_HSTRIPES][b >> 9][b & 511], v);
    }
}

// Histograms of a stream with residual contexts: workgroup (x, 0) counts
// ENT_HIST_PX pixels of the three residual planes, reading each pixel's three
// context bytes once (S >> 5, kept packed in a register per pixel) and
// counting the planes one after another in the same LDS bins (8 x 512 per
// plane, ENT_HC copies), which it flushes between planes; workgroup (x, 1)
// counts the exponent symbols' runs as k_ent_hist does.
__global__ __launch_bounds__(ENT_HIST_THREADS) void k_ent_hist_ctx(EntArgs a) {
    __shared__ uint32_t h[ENT_NCTX * 512 * ENT_HC];
    static_assert(ENT_CMINOR && !ENT_PACK16, "k_ent_hist_ctx: one 32-bit counter per bin and copy");
    const int lane = threadIdx.x & 63;
    const uint32_t mine = (uint32_t)lane & (ENT_HC - 1);
    const int64_t i0 = (int64_t)blockIdx.x * ENT_HIST_PX;
    const int n = (int)(a.N - i0 < ENT_HIST_PX ? a.N - i0 : ENT_HIST_PX);
    constexpr int PER = ENT_HIST_PX / ENT_HIST_THREADS;  // 32 px per thread
    auto clear = [&]() {
        for (int k = threadIdx.x; k < ENT_NCTX * 512 * ENT_HC; k += ENT_HIST_THREADS) h[k] = 0;
    };
    auto flush = [&](int t0, int nb) {
        for (int b = threadIdx.x; b < nb; b += ENT_HIST_THREADS) {
            uint32_t v = 0;
#pragma unroll
            for (int k = 0; k < ENT_HC; ++k) v += h[ent_word(k, b)];
            if (v) atomicAdd(&a.ws->hist[blockIdx.x % ENT_HSTRIPES][t0 + (b >> 9)][b & 511], v);
        }
    };
    clear();
    if (blockIdx.y == 0) {
        const uint8_t *sp = a.sdr + 3 * i0;
        // pixel j's contexts at bits 9 (j mod 3) + 3c of cx[j / 3], channel c
        uint32_t cx[(PER + 2) / 3];
#pragma unroll
        for (int k = 0; k < (PER + 2) / 3; ++k) cx[k] = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = min(j * ENT_HIST_THREADS + (int)threadIdx.x, n - 1);  // clamped: every load valid
            cx[j / 3] |= (((uint32_t)sp[3 * i] >> 5) | (((uint32_t)sp[3 * i + 1] >> 5) << 3) |
                          (((uint32_t)sp[3 * i + 2] >> 5) << 6)) << (9 * (j % 3));
        }
        __syncthreads();  // bins cleared
#pragma unroll 1
        for (int p = 0; p < 3; ++p) {
            const int16_t *rp = (const int16_t *)a.resid + p * a.N + i0;
            int v[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) v[j] = (int)rp[min(j * ENT_HIST_THREADS + (int)threadIdx.x, n - 1)];
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if (j * ENT_HIST_THREADS + (int)threadIdx.x < n)
                    ent_count(h, mine, ((cx[j / 3] >> (9 * (j % 3) + 3 * p)) & 7u) * 512 +
                                           min((uint32_t)(v[j] + 255), 511u), 1u);
            __syncthreads();
            flush(ENT_NCTX * p, ENT_NCTX * 512);
            if (p < 2) {
                __syncthreads();  // every copy read before the clear
                clear();
                __syncthreads();
            }
        }
    } else {
        __syncthreads();
        const uint8_t *e8 = a.eplane + i0;
        int ev[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = j * ENT_HIST_THREADS + threadIdx.x;
            const int v = (int)e8[min(i, n - 1)];
            ev[j] = i < n ? v : -1;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int v = ev[j];
            const int left = __shfl_up(v, 1, 64);
            const bool head = lane == 0 || v != left;
            const unsigned long long m = __ballot(head);
            const unsigned long long after = lane == 63 ? 0ull : m >> (lane + 1);
            const int len = after ? (int)__builtin_ctzll(after) + 1 : 64 - lane;
            if (head && v >= 0) ent_count(h, mine, (uint32_t)v, (uint32_t)len);
        }
        __syncthreads();
        flush(ENT_NTAB_CTX - 1, 512);
    }
}

// Frequencies of table blockIdx.x (512 threads, one per symbol):
// f = 1 + floor(h (M - P) / N) for the P present symbols, N their total
// count, the remainder to the smallest symbol of the largest count;
// c = exclusive prefix sum.  A table with no symbol (a context no pixel
// falls in) stays all zero.  Writes the stream's frequency table and the
// encoder's table, clears the histogram; table 0's workgroup writes the fixed
// header words.  The last table is the exponents' (256 symbols).
__global__ __launch_bounds__(512) void k_ent_freq(EntArgs a) {
    __shared__ uint32_t sh[8];
    __shared__ unsigned long long shm[8];
    const int p = blockIdx.x, s = threadIdx.x, nsym = p < a.ntab - 1 ? 511 : 256;
    uint32_t h = 0;
#pragma unroll
    for (int k = 0; k < ENT_HSTRIPES; ++k) {
        h += a.ws->hist[k][p][s];
        a.ws->hist[k][p][s] = 0;
    }
    const bool pres = s < nsym && h > 0;
    const uint32_t nbad = block_sum<8>(s >= nsym && h > 0 ? 1u : 0u, sh);
    const uint32_t P = block_sum<8>(pres ? 1u : 0u, sh);
    const uint32_t ntot = block_sum<8>(pres ? h : 0u, sh);  // <= N < 2^31
    uint32_t f = pres ? 1u + (uint32_t)(((uint64_t)h * (ENT_M - P)) / (uint64_t)ntot) : 0u;
    const uint32_t sum = block_sum<8>(f, sh);
    const unsigned long long key = pres ? ((unsigned long long)h << 16 | (0xFFFFu - (uint32_t)s)) : 0ull;
    const unsigned long long best = block_max64<8>(key, shm);
    if (pres && key == best) f += ENT_M - sum;
    uint32_t tot;
    const uint32_t c = block_excl_scan<8>(f, sh, tot);
    const bool bad = nbad != 0;
    reinterpret_cast<uint16_t *>(a.out + 40)[512 * p + s] = bad ? 0 : (uint16_t)f;
    // fl(1/f) lowered by 4 ulps: x fl(.) then stays below x / f (see enc_group)
    a.ws->tab[p][s] = make_uint2(f | c << 16, f ? __float_as_uint(1.0f / (float)f) - 4u : 0u);
    if (s == 0) a.ws->bad[p] = bad ? 1u : 0u;
    if (p == 0 && s < 8) {
        const uint32_t v = s == 0 ? 0x454C4452u
                         : s == 1 ? 1u
                         : s == 2 ? (uint32_t)a.H
                         : s == 3 ? (uint32_t)a.W
                         : s == 4 ? (uint32_t)a.log2_k
                         : s == 5 ? (uint32_t)ENT_PB
                         : s == 6 ? (uint32_t)a.G
                                  : (uint32_t)a.flags;
        reinterpret_cast<uint32_t *>(a.out)[s] = v;
    }
}

// One wave per group: lane l codes symbols l, l + 64, ... of the group from
// the last step to the first.  A lane renormalises (emits its low 16 bits)
// when x >= 2^17 f; the words of a step go out in descending lane order, so
// that the stored (reversed) stream lists them in ascending order.  Then
// x = (x div f) M + (x mod f) + c, with the quotient from a float reciprocal
// r' = fl(1/f) lowered by 4 ulps (relative decrease between 2^-22 and 2^-21):
// fl(fl(x) r') <= x/f (1 + 2^-24)^3 (1 - 2^-22) < x / f, and x < 2^17 f
// bounds its shortfall by 2^17 (2^-21 + 3 2^-24) < 0.11, so the truncated
// estimate is x div f or one less and one upward correction makes it exact.
// Finally every
// lane's state, lanes 63 down to 0, low half first.  RES: a residual plane
// (int16 values, symbol r + 255), else the exponent plane (bytes).  CTX: the
// table of symbol i is its context ctx[3 i] >> 5 (the base layer's byte of the
// plane's channel), entry (context << 9) + symbol of tb.
template <bool RES, bool CTX, typename V>
__device__ __forceinline__ void enc_group(const V *src, const uint8_t *ctx, int n, const uint2 *tb, uint16_t *out,
                                          uint32_t *cnt_out, int lane, uint32_t dummy) {
    const int T = (n + 63) >> 6;
    const int tfull = (n >> 6) - 1;  // steps 0..tfull hold a symbol in every lane
    // Symbols of steps t0, t0 - 1, ..., t0 - 7 and a mask of the lane's valid
    // ones.  Every load reads a valid address (the index is clamped) and its
    // value is used unconditionally, so the loads stay free of branches; the
    // next block's loads are issued before the current block is coded.  Steps
    // before the first (t < 0) have no symbol in any lane and change nothing.
    auto sym_of = [](int v) -> uint32_t { return RES ? min((uint32_t)(v + 255), 511u) : (uint32_t)v; };
    auto tab_of = [](uint32_t sdr_byte) -> uint32_t { return CTX ? (sdr_byte >> 5) << 9 : 0u; };
    auto load_block = [&](int t0, uint32_t (&sv)[8]) -> uint32_t {
        if (t0 - 7 >= 0 && t0 <= tfull) {  // whole block inside the group: fixed offsets
            const V *q = src + t0 * 64 + lane;
#pragma unroll
            for (int k = 0; k < 8; ++k) sv[k] = sym_of((int)q[-64 * k]);
            if (CTX) {
                const uint8_t *qc = ctx + 3 * (t0 * 64 + lane);
#pragma unroll
                for (int k = 0; k < 8; ++k) sv[k] |= tab_of(qc[-192 * k]);
            }
            return 0xFFu;
        }
        uint32_t vm = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int t = t0 - k, i = t * 64 + lane, ic = min(max(i, 0), n - 1);
            sv[k] = sym_of((int)src[ic]) | (CTX ? tab_of(ctx[3 * ic]) : 0u);
            vm |= (t >= 0 && i < n ? 1u : 0u) << k;
        }
        return vm;
    };
    uint32_t x = ENT_L, wpos = 0;
    uint32_t cur[8], nxt[8];
    // One step.  ALL: every lane has a symbol (a block inside the full steps).
    // The quotient estimate never exceeds x div f (the table holds fl(1/f)
    // lowered by 4 ulps) and falls short by less than 1, so one upward
    // correction makes it exact.  A lane that renormalises writes at
    // wpos + (number of renormalising lanes above it).
    auto step = [&](auto all, uint32_t s, bool valid) {
        constexpr bool ALL = decltype(all)::value;
        const bool have = ALL || valid;
        const uint2 e = tb[s];
        const uint32_t f = e.x & 0xFFFFu, c = e.x >> 16;
        const bool ren = have && (x >> 17) >= f;
        const uint64_t m = __builtin_amdgcn_ballot_w64(ren);
        const uint32_t tot = (uint32_t)__builtin_popcountll(m);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // every lane stores (no branch): lanes without a word write their dummy slot
        const uint32_t keep = 0u - (uint32_t)ren;  // all ones where the lane writes a word
        out[((wpos + tot - 1u - below) & keep) | (dummy & ~keep)] = (uint16_t)x;
        wpos += tot;
        const uint32_t xr = ren ? x >> 16 : x;
        uint32_t q = (uint32_t)((float)xr * __uint_as_float(e.y));
        uint32_t r = xr - __umul24(q, f);  // q < 2^18, f <= 2^15: 24-bit product exact
        const bool up = r >= f;
        q = up ? q + 1 : q;
        r = up ? r - f : r;
        const uint32_t xn = (q << ENT_PB) + r + c;
        x = ALL ? xn : (have ? xn : xr);
    };
    uint32_t vcur = load_block(T - 1, cur);
    for (int t0 = T - 1; t0 >= 0; t0 -= 8) {
        const uint32_t vnxt = load_block(t0 - 8, nxt);
        if (t0 - 7 >= 0 && t0 <= tfull) {  // wave-uniform
#pragma unroll
            for (int k = 0; k < 8; ++k) step(std::true_type{}, cur[k], true);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) step(std::false_type{}, cur[k], (vcur >> k) & 1u);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
        vcur = vnxt;
    }
    const uint32_t fp = wpos + 2 * (63 - lane);
    out[fp] = (uint16_t)x;
    out[fp + 1] = (uint16_t)(x >> 16);
    if (lane == 0) *cnt_out = wpos + 128;
}

__global__ __launch_bounds__(256) void k_ent_enc(EntArgs a) {
    __shared__ uint2 stab[4][512];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = a.G;
    const int64_t gi = (int64_t)blockIdx.x * 4 + w;
    const bool live = gi < 4 * (int64_t)G;
    const int p = live ? (int)(gi / G) : 0;
    for (int k = lane; k < 512; k += 64) stab[w][k] = a.ws->tab[p][k];
    __syncthreads();
    if (!live) return;
    if (a.ws->bad[p]) {
        if (lane == 0) a.cnt[gi] = 0;
        return;
    }
    const int64_t Z = (int64_t)64 << a.log2_k, g = gi - (int64_t)p * G, base = g * Z;
    const int n = (int)(a.N - base < Z ? a.N - base : Z);
    uint16_t *out = a.tmp + gi * ent_slot(a.log2_k);
    const uint32_t dummy = (uint32_t)(Z + 128 + lane);
    if (p < 3)
        enc_group<true, false>((const int16_t *)a.resid + p * a.N + base, nullptr, n, stab[w], out, a.cnt + gi, lane,
                               dummy);
    else
        enc_group<false, false>(a.eplane + base, nullptr, n, stab[w], out, a.cnt + gi, lane, dummy);
}

// Encoder with residual contexts: the groups of plane blockIdx.y, four per
// workgroup, which holds the plane's tables (8 contexts x 512 entries for a
// residual plane, the exponents' one table for plane 3).
__global__ __launch_bounds__(256) void k_ent_enc_ctx(EntArgs a) {
    __shared__ uint2 stab[ENT_NCTX * 512];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int p = blockIdx.y, G = a.G, g = blockIdx.x * 4 + w;
    const int t0 = p < 3 ? ENT_NCTX * p : ENT_NTAB_CTX - 1, nt = p < 3 ? ENT_NCTX : 1;
    for (int k = threadIdx.x; k < nt * 512; k += 256) stab[k] = a.ws->tab[t0 + (k >> 9)][k & 511];
    uint32_t bad = 0;
    for (int k = 0; k < nt; ++k) bad |= a.ws->bad[t0 + k];
    __syncthreads();
    if (g >= G) return;
    const int64_t gi = (int64_t)p * G + g;
    if (bad) {
        if (lane == 0) a.cnt[gi] = 0;
        return;
    }
    const int64_t Z = (int64_t)64 << a.log2_k, base = (int64_t)g * Z;
    const int n = (int)(a.N - base < Z ? a.N - base : Z);
    uint16_t *out = a.tmp + gi * ent_slot(a.log2_k);
    const uint32_t dummy = (uint32_t)(Z + 128 + lane);
    if (p < 3)
        enc_group<true, true>((const int16_t *)a.resid + p * a.N + base, a.sdr + 3 * base + p, n, stab, out,
                              a.cnt + gi, lane, dummy);
    else
        enc_group<false, false>(a.eplane + base, nullptr, n, stab, out, a.cnt + gi, lane, dummy);
}

// Group offsets (exclusive prefix sum of the word counts) into the stream's
// table, the total length into the header and *out_len; an invalid layer
// (a residual outside [-255, 255]) yields magic 0 and length 0.
__global__ __launch_bounds__(1024) void k_ent_scan(EntArgs a) {
    __shared__ uint32_t sh[16];
    uint32_t anybad = 0;
    for (int t = 0; t < a.ntab; ++t) anybad |= a.ws->bad[t];
    const bool ok = anybad == 0;
    const int64_t n = 4 * (int64_t)a.G;
    uint64_t *start = reinterpret_cast<uint64_t *>(a.out + a.hdr);
    uint64_t carry = 0;
    for (int64_t b = 0; b < n; b += 1024) {
        const int64_t k = b + threadIdx.x;
        const uint32_t v = k < n ? a.cnt[k] : 0u;
        uint32_t tot;
        const uint32_t e = block_excl_scan<16>(v, sh, tot);
        if (k < n) start[k] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        const uint64_t total = (uint64_t)a.hdr + 32 * (uint64_t)a.G + 2 * carry;
        reinterpret_cast<uint64_t *>(a.out)[4] = ok ? total : 0ull;
        if (!ok) reinterpret_cast<uint32_t *>(a.out)[0] = 0u;
        *a.out_len = ok ? total : 0ull;
        a.ws->ok = ok ? 1u : 0u;
    }
}

// Each group's words, reversed, at its offset in the payload.
__global__ __launch_bounds__(256) void k_ent_pack(EntArgs a) {
    if (!a.ws->ok) return;
    const int64_t gi = blockIdx.x;
    const uint32_t n = a.cnt[gi];
    const uint64_t st = reinterpret_cast<const uint64_t *>(a.out + a.hdr)[gi];
    const uint16_t *__restrict__ src = a.tmp + gi * ent_slot(a.log2_k);
    uint16_t *__restrict__ dst = reinterpret_cast<uint16_t *>(a.out + a.hdr + 32 * (int64_t)a.G) + st;
    // 8 loads in flight per lane (indices clamped: a group has n >= 128 words)
    for (uint32_t k0 = 0; k0 < n; k0 += 8 * 256) {
        uint16_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t k = k0 + j * 256 + threadIdx.x;
            v[j] = src[k < n ? n - 1 - k : 0];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t k = k0 + j * 256 + threadIdx.x;
            if (k < n) dst[k] = v[j];
        }
    }
}

__global__ void k_ent_status(int32_t *st) {
    if (threadIdx.x == 0) st[0] = RDL_OK;
}

// Decodes one group into dst (RES: int16 residuals, else exponent bytes);
// returns whether it failed to end exactly at its last word with every state
// back at L.  Word positions count from the group's first word; pos and b
// are wave-uniform.  Steps where every lane has a symbol run without the
// lane mask; only the group's last, partial step keeps it.
template <bool RES, typename V, typename LD>
__device__ __forceinline__ bool dec_group(V *dst, int n, const uint2 *dtab, const uint16_t *slot_sym, uint16_t *rg,
                                          uint32_t (&R)[4], uint32_t b, uint32_t pos, uint32_t x, uint32_t nw,
                                          const LD &ld, int lane) {
    bool bad = false;
    auto step = [&](auto all, int t) {
        constexpr bool ALL = decltype(all)::value;
        if (pos >= b + 256) {
#pragma unroll
            for (int k = 0; k < 4; ++k) rg[(b + 512 + k * 64 + lane) & 511] = (uint16_t)R[k];
            b += 256;
#pragma unroll
            for (int k = 0; k < 4; ++k) R[k] = ld(b + 512 + k * 64 + lane);
        }
        const int i = t * 64 + lane;
        const bool have = ALL || i < n;
        const uint32_t slot = x & (ENT_M - 1);
        const uint2 e = dtab[slot_sym[slot]];
        const uint32_t xn = (e.x >> 16) * (x >> ENT_PB) + slot - (e.x & 0xFFFFu);
        x = ALL ? xn : (have ? xn : x);
        const bool ren = have && x < ENT_L;
        const uint64_t m = __builtin_amdgcn_ballot_w64(ren);
        const uint32_t idx = pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const bool inside = idx < nw;
        const uint32_t wv = rg[idx & 511];
        bad = bad || (ren && !inside);
        x = ren ? x << 16 | (inside ? wv : 0u) : x;
        pos += (uint32_t)__builtin_popcountll(m);
        if (ALL || have) dst[i] = RES ? (V)((int)e.y - 255) : (V)e.y;
    };
    const int tfull = n >> 6;
    for (int t = 0; t < tfull; ++t) step(std::true_type{}, t);
    if (n & 63) step(std::false_type{}, tfull);
    return bad || pos != nw || x != ENT_L;
}

// Decoder: ENT_DEC_WAVES groups of one plane per workgroup.  The workgroup
// builds the plane's tables from the stream's frequencies: the present
// symbols in order, {c | f << 16, symbol}, and for every one of the M slots
// the index of the present symbol holding it (64 KB of LDS).  Each wave reads
// its lanes' states, and per step: slot = x mod M, the symbol in two LDS
// reads, x = f (x div M) + slot - c, and the lanes with x < L read the next
// words in lane order.  A group must end exactly at its last word with every state
// back at L; a frequency table, group offset or word count that does not fit
// sets *status = RDL_ECORRUPT (reads stay inside the group).
__global__ __launch_bounds__(256) void k_ent_dec(EntArgs a) {
    __shared__ uint2 dtab[512];
    __shared__ __align__(16) uint16_t slot_sym[ENT_M];
    __shared__ uint32_t sh[4];
    __shared__ uint16_t ring[ENT_DEC_WAVES][512];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = a.G, gpp = (G + ENT_DEC_WAVES - 1) / ENT_DEC_WAVES;
    // with residual contexts only plane 3 comes here (k_ent_dec_ctx takes the others)
    const int p = a.ntab == 4 ? blockIdx.x / gpp : 3, g = (blockIdx.x % gpp) * ENT_DEC_WAVES + w;
    const int nsym = p < 3 ? 511 : 256, tix = p < 3 ? p : a.ntab - 1;
    const uint32_t fw = reinterpret_cast<const uint32_t *>(a.code + 40 + 1024 * tix)[threadIdx.x];
    const uint32_t s0 = 2 * threadIdx.x, f0 = fw & 0xFFFFu, f1 = fw >> 16;
    uint32_t tot, P;
    const uint32_t c0 = block_excl_scan<4>(f0 + f1, sh, tot);
    const uint32_t j0 = block_excl_scan<4>((f0 > 0) + (f1 > 0), sh, P);
    const uint32_t nbad = block_sum<4>(((int)s0 >= nsym && f0) + ((int)s0 + 1 >= nsym && f1), sh);
    if (tot != ENT_M || nbad) {
        if (threadIdx.x == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
        return;
    }
    if (f0) dtab[j0] = make_uint2(c0 | f0 << 16, s0);
    if (f1) dtab[j0 + (f0 > 0)] = make_uint2((c0 + f0) | f1 << 16, s0 + 1);
    // The slot table: each present symbol's index marked at its first slot
    // (the slots in between left 0), then a prefix maximum over the M slots
    // (indices grow with c), lane t owning slots [128 t, 128 t + 128).
    uint4 *st4 = reinterpret_cast<uint4 *>(slot_sym) + 16 * threadIdx.x;
#pragma unroll
    for (int k = 0; k < 16; ++k) st4[k] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    if (f0) slot_sym[c0] = (uint16_t)j0;
    if (f1) slot_sym[c0 + f0] = (uint16_t)(j0 + (f0 > 0));
    __syncthreads();
    uint4 sv[16];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) sv[k] = st4[k];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        uint32_t *w = reinterpret_cast<uint32_t *>(&sv[k]);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const uint32_t lo = max(run, w[h] & 0xFFFFu);
            run = max(lo, w[h] >> 16);
            w[h] = lo | run << 16;
        }
    }
    const uint32_t before = block_excl_max<4>(run, sh);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t *w = reinterpret_cast<const uint32_t *>(&sv[k]);
        uint32_t o[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) o[h] = max(w[h] & 0xFFFFu, before) | max(w[h] >> 16, before) << 16;
        st4[k] = make_uint4(o[0], o[1], o[2], o[3]);
    }
    __syncthreads();
    if (g >= G) return;
    const int64_t gi = (int64_t)p * G + g;
    const uint64_t *start = reinterpret_cast<const uint64_t *>(a.code + a.hdr);
    const uint16_t *words = reinterpret_cast<const uint16_t *>(a.code + a.hdr + 32 * (int64_t)G);
    const uint64_t u0 = start[gi], u1 = gi + 1 < 4 * (int64_t)G ? start[gi + 1] : (uint64_t)a.nwords;
    // a group holds its 128 state words and at most one word per symbol
    if (!(u0 <= u1 && u1 <= (uint64_t)a.nwords && u1 - u0 >= 128 && u1 - u0 <= (uint64_t)ent_slot(a.log2_k))) {
        if (lane == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
        return;
    }
    const uint16_t *gw = words + u0;  // the group's words
    const uint32_t nw = (uint32_t)(u1 - u0);
    uint32_t x = (uint32_t)gw[2 * lane] << 16 | gw[2 * lane + 1];
    // The wave's words [b, b + 512) sit in an LDS ring (slot = position mod 512)
    // and the next 256 in registers; once the first half is consumed the
    // registers refill it and load the following 256.  A step consumes at
    // most 64 words and starts below b + 256, so its reads stay in the ring.
    // Words past the group's end read as 0 and are never consumed by a
    // well-formed group.
    uint16_t *rg = ring[w];
    const uint32_t pos = 128, b = 128;
    auto ld = [&](uint32_t q) -> uint32_t {
        const uint32_t v = gw[q < nw ? q : nw - 1];  // clamped: nw - 1 >= 127
        return q < nw ? v : 0u;
    };
#pragma unroll
    for (int k = 0; k < 8; ++k) rg[(b + k * 64 + lane) & 511] = (uint16_t)ld(b + k * 64 + lane);
    uint32_t R[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) R[k] = ld(b + 512 + k * 64 + lane);
    const int64_t Z = (int64_t)64 << a.log2_k, base = (int64_t)g * Z;
    const int n = (int)(a.N - base < Z ? a.N - base : Z);
    bool bad;
    if (p < 3)
        bad = dec_group<true>(reinterpret_cast<int16_t *>(a.dst) + p * a.N + base, n, dtab, slot_sym, rg, R, b, pos,
                              x, nw, ld, lane);
    else
        bad = dec_group<false>(a.dplane + base, n, dtab, slot_sym, rg, R, b, pos, x, nw, ld, lane);
    if (__ballot(bad) && lane == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
}

// Decoder of a residual plane with contexts: one group per wave, four groups
// of plane blockIdx.y per workgroup.  The workgroup holds the plane's 8
// context tables in 16-bit arrays: per table the present symbols' first slots
// c (with M after the last) and symbols, and per bucket of 16 slots the index
// of the symbol holding the bucket's first slot (the number of symbols with
// c <= 16 b, less one: the last symbol whose first slot rounds up to bucket b
// marks it, then a prefix maximum).  A step reads its lanes' contexts (the
// base layer's bytes, loaded a block of 8 steps ahead), takes slot = x mod M,
// and finds the symbol holding it by a binary search between the bucket's
// entry and the next bucket's (at most 17 candidates, 5 halvings); the rest
// is dec_group's step.  A table that sums to neither 0 nor M, a symbol 511,
// or a symbol whose context table is empty sets *status = RDL_ECORRUPT.
constexpr int ENT_CB = 2048;  // buckets per context table (16 slots each)

template <typename LD>
__device__ __forceinline__ bool dec_group_ctx(int16_t *dst, const uint8_t *ctx, int n, const uint16_t (*pc)[513],
                                              const uint16_t (*ps)[512], const uint16_t (*bk)[ENT_CB],
                                              const uint32_t *np, uint16_t *rg, uint32_t (&R)[4], uint32_t b,
                                              uint32_t pos, uint32_t x, uint32_t nw, const LD &ld, int lane) {
    bool bad = false;
    auto load_ctx = [&](int t0, uint32_t (&cv)[8]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = min((t0 + k) * 64 + lane, n - 1);  // clamped: every load valid
            cv[k] = (uint32_t)ctx[3 * i] >> 5;
        }
    };
    auto step = [&](int t, uint32_t k) {
        if (pos >= b + 256) {
#pragma unroll
            for (int q = 0; q < 4; ++q) rg[(b + 512 + q * 64 + lane) & 511] = (uint16_t)R[q];
            b += 256;
#pragma unroll
            for (int q = 0; q < 4; ++q) R[q] = ld(b + 512 + q * 64 + lane);
        }
        const int i = t * 64 + lane;
        const bool have = i < n;
        const uint32_t slot = x & (ENT_M - 1), bb = slot >> 4, P = np[k];
        bad = bad || (have && P == 0);
        uint32_t lo = P ? bk[k][bb] : 0u, hi = P ? (bb < ENT_CB - 1 ? bk[k][bb + 1] : P - 1) : 0u;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (pc[k][mid] <= slot) lo = mid; else hi = mid - 1;
        }
        const uint32_t c = pc[k][lo], f = pc[k][lo + 1] - c, sym = ps[k][lo];
        const uint32_t xn = f * (x >> ENT_PB) + slot - c;
        x = have ? xn : x;
        const bool ren = have && x < ENT_L;
        const uint64_t m = __builtin_amdgcn_ballot_w64(ren);
        const uint32_t idx = pos + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const bool inside = idx < nw;
        const uint32_t wv = rg[idx & 511];
        bad = bad || (ren && !inside);
        x = ren ? x << 16 | (inside ? wv : 0u) : x;
        pos += (uint32_t)__builtin_popcountll(m);
        if (have) dst[i] = (int16_t)((int)sym - 255);
    };
    const int T = (n + 63) >> 6;
    uint32_t cur[8], nxt[8];
    load_ctx(0, cur);
    for (int t0 = 0; t0 < T; t0 += 8) {
        load_ctx(t0 + 8, nxt);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (t0 + k < T) step(t0 + k, cur[k]);  // wave-uniform
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
    }
    return bad || pos != nw || x != ENT_L;
}

__global__ __launch_bounds__(256) void k_ent_dec_ctx(EntArgs a) {
    __shared__ uint16_t pc[ENT_NCTX][513];
    __shared__ uint16_t ps[ENT_NCTX][512];
    __shared__ __align__(16) uint16_t bk[ENT_NCTX][ENT_CB];
    __shared__ uint32_t np[ENT_NCTX];
    __shared__ uint32_t sh[4];
    __shared__ uint16_t ring[ENT_DEC_WAVES][512];
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = a.G, p = blockIdx.y, g = blockIdx.x * ENT_DEC_WAVES + w;
    bool corrupt = false;
    for (int k = 0; k < ENT_NCTX; ++k) {
        uint4 *bq = reinterpret_cast<uint4 *>(&bk[k][0]) + threadIdx.x;  // this thread's 8 buckets
        *bq = make_uint4(0u, 0u, 0u, 0u);
        const uint32_t fw = reinterpret_cast<const uint32_t *>(a.code + 40 + 1024 * (ENT_NCTX * p + k))[threadIdx.x];
        const uint32_t s0 = 2 * threadIdx.x, f0 = fw & 0xFFFFu, f1 = fw >> 16;
        uint32_t tot, P;
        const uint32_t c0 = block_excl_scan<4>(f0 + f1, sh, tot);  // its barriers also order the clears
        const uint32_t j0 = block_excl_scan<4>((f0 > 0) + (f1 > 0), sh, P);
        const uint32_t nbad = block_sum<4>(s0 + 1 >= 511 && f1 ? 1u : 0u, sh);
        corrupt = corrupt || (tot != ENT_M && tot != 0) || nbad;  // uniform
        const bool use = tot == ENT_M && !nbad;
        // a present symbol at c marks bucket ceil(c / 16) unless the next
        // present symbol (at c + f) rounds up to the same bucket
        auto put = [&](uint32_t j, uint32_t c, uint32_t f, uint32_t sym) {
            pc[k][j] = (uint16_t)c;
            ps[k][j] = (uint16_t)sym;
            const uint32_t bb = (c + 15) >> 4;
            if (bb < ENT_CB && ((c + f + 15) >> 4) != bb) bk[k][bb] = (uint16_t)j;
        };
        if (use && f0) put(j0, c0, f0, s0);
        if (use && f1) put(j0 + (f0 > 0), c0 + f0, f1, s0 + 1);
        if (threadIdx.x == 0) {
            np[k] = use ? P : 0u;
            if (use) pc[k][P] = (uint16_t)ENT_M;
        }
        __syncthreads();
        // prefix maximum over the 2048 marks, 8 per thread
        uint4 v = *bq;
        uint32_t e[8] = {v.x & 0xFFFFu, v.x >> 16, v.y & 0xFFFFu, v.y >> 16,
                         v.z & 0xFFFFu, v.z >> 16, v.w & 0xFFFFu, v.w >> 16};
#pragma unroll
        for (int q = 1; q < 8; ++q) e[q] = max(e[q], e[q - 1]);
        const uint32_t before = block_excl_max<4>(e[7], sh);
        // (its barriers also keep the next table's clear after these reads)
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = max(e[q], before);
        *bq = make_uint4(e[0] | e[1] << 16, e[2] | e[3] << 16, e[4] | e[5] << 16, e[6] | e[7] << 16);
    }
    __syncthreads();
    if (corrupt) {
        if (threadIdx.x == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
        return;
    }
    if (g >= G) return;
    const int64_t gi = (int64_t)p * G + g;
    const uint64_t *start = reinterpret_cast<const uint64_t *>(a.code + a.hdr);
    const uint16_t *words = reinterpret_cast<const uint16_t *>(a.code + a.hdr + 32 * (int64_t)G);
    const uint64_t u0 = start[gi], u1 = gi + 1 < 4 * (int64_t)G ? start[gi + 1] : (uint64_t)a.nwords;
    if (!(u0 <= u1 && u1 <= (uint64_t)a.nwords && u1 - u0 >= 128 && u1 - u0 <= (uint64_t)ent_slot(a.log2_k))) {
        if (lane == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
        return;
    }
    const uint16_t *gw = words + u0;
    const uint32_t nw = (uint32_t)(u1 - u0);
    uint32_t x = (uint32_t)gw[2 * lane] << 16 | gw[2 * lane + 1];
    uint16_t *rg = ring[w];
    const uint32_t pos = 128, b = 128;
    auto ld = [&](uint32_t q) -> uint32_t {
        const uint32_t v = gw[q < nw ? q : nw - 1];  // clamped: nw - 1 >= 127
        return q < nw ? v : 0u;
    };
#pragma unroll
    for (int k = 0; k < 8; ++k) rg[(b + k * 64 + lane) & 511] = (uint16_t)ld(b + k * 64 + lane);
    uint32_t R[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) R[k] = ld(b + 512 + k * 64 + lane);
    const int64_t Z = (int64_t)64 << a.log2_k, base = (int64_t)g * Z;
    const int n = (int)(a.N - base < Z ? a.N - base : Z);
    const bool bad = dec_group_ctx(reinterpret_cast<int16_t *>(a.dst) + p * a.N + base, a.sdr + 3 * base + p, n,
                                   pc, ps, bk, np, rg, R, b, pos, x, nw, ld, lane);
    if (__ballot(bad) && lane == 0 && a.status) atomicExch(a.status, RDL_ECORRUPT);
}

// ---- Left differences of the exponent plane (stream flag bit 0) ----------
// Plane 3 may hold d = (E[i] - E[i-1]) mod 256, with d = E[i] at the first
// pixel of a row.  The encoder writes d into its workspace; the decoder sums
// d back along each row.  The plane is cut into the 16-byte aligned chunks
// that cover it, one per lane (256 lanes per tile): with lead = the plane's
// address mod 16, chunk t holds pixels [16 t - lead, + 16).  A chunk wholly
// inside the plane moves with one 16-byte load or store, the (at most two)
// others byte by byte, so no access leaves the plane.

// Decoder.  A run of pixels is summarised by a segment value: the sum mod 256
// of its d since the last row start inside it (or of all of them), in bits
// 0-7, and bit 8 set when a row starts inside.  Joining run a then run b is
// associative: b if a row starts in b, else the sums added with a's bit.  The
// exponent before pixel i is then the value of the join of all runs before
// it (its own row started inside them).
__device__ __forceinline__ uint32_t seg_join(uint32_t a, uint32_t b) {
    return (b & 256u) ? b : (((a + b) & 255u) | (a & 256u));
}

struct EChunk {
    uint32_t v[16];  // the chunk's bytes (0 outside the plane)
    int64_t i0;      // pixel index of byte 0 (negative in a leading partial chunk)
    uint32_t col0;   // column of byte 0, as if the rows continued before pixel 0
    bool full;       // all 16 bytes inside the plane
};

__device__ __forceinline__ void echunk_load(const uint8_t *e, int64_t N, int W, int64_t t, EChunk &c) {
    const int lead = (int)(reinterpret_cast<uintptr_t>(e) & 15);
    c.i0 = 16 * t - lead;
    c.full = c.i0 >= 0 && c.i0 + 16 <= N;
    // |i0| < 2^31: one 32-bit modulo; byte -i0 (pixel 0) then falls on column 0
    const uint32_t m = (uint32_t)(c.i0 < 0 ? -c.i0 : c.i0) % (uint32_t)W;
    c.col0 = c.i0 < 0 && m ? (uint32_t)W - m : m;
    if (c.full) {
        const uint4 q = *reinterpret_cast<const uint4 *>(e + c.i0);
        const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) c.v[k] = (w4[k >> 2] >> (8 * (k & 3))) & 255u;
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t i = c.i0 + k;
            c.v[k] = i >= 0 && i < N ? (uint32_t)e[i] : 0u;
        }
    }
}

__device__ __forceinline__ void echunk_store(uint8_t *e, int64_t N, const EChunk &c, const uint32_t (&o)[16]) {
    if (c.full) {
        uint32_t w4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < 16; ++k) w4[k >> 2] |= (o[k] & 255u) << (8 * (k & 3));
        *reinterpret_cast<uint4 *>(e + c.i0) = make_uint4(w4[0], w4[1], w4[2], w4[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t i = c.i0 + k;
            if (i >= 0 && i < N) e[i] = (uint8_t)o[k];
        }
    }
}

__device__ __forceinline__ uint32_t echunk_seg(const EChunk &c, int64_t N, int W) {
    uint32_t seg = 0, col = c.col0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t i = c.i0 + k;
        if (i >= 0 && i < N) seg = col == 0 ? (c.v[k] | 256u) : seg_join(seg, c.v[k]);
        col = col + 1 == (uint32_t)W ? 0u : col + 1;
    }
    return seg;
}

// Encoder: d of chunk t into out, which has the plane's lead (a workspace).
__global__ __launch_bounds__(256) void k_ent_ediff(const uint8_t *__restrict__ e, uint8_t *__restrict__ out,
                                                   int64_t N, int W) {
    EChunk c;
    echunk_load(e, N, W, (int64_t)blockIdx.x * 256 + threadIdx.x, c);
    if (c.i0 >= N) return;
    uint32_t prev = c.i0 >= 1 ? (uint32_t)e[c.i0 - 1] : 0u;  // used only past a row's first pixel
    uint32_t o[16], col = c.col0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        o[k] = (col == 0 ? c.v[k] : c.v[k] - prev) & 255u;
        prev = c.v[k];
        col = col + 1 == (uint32_t)W ? 0u : col + 1;
    }
    echunk_store(out, N, c, o);
}

// Exclusive scan of segment values over a workgroup of NW waves (0 is the
// identity); total receives the join of all of them.
template <int NW>
__device__ uint32_t seg_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc = seg_join(y, inc);
    }
    __syncthreads();
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint32_t before = 0, t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        if (k < w) before = seg_join(before, sh[k]);
        t = seg_join(t, sh[k]);
    }
    uint32_t ex = __shfl_up(inc, 1, 64);
    ex = lane == 0 ? 0u : ex;
    total = t;
    return seg_join(before, ex);
}

// Segment value of each tile of 256 chunks.
__global__ __launch_bounds__(256) void k_ent_eseg(const uint8_t *__restrict__ e, int64_t N, int W,
                                                  uint32_t *__restrict__ seg) {
    __shared__ uint32_t sh[4];
    EChunk c;
    echunk_load(e, N, W, (int64_t)blockIdx.x * 256 + threadIdx.x, c);
    uint32_t tot;
    seg_excl_scan<4>(echunk_seg(c, N, W), sh, tot);
    if (threadIdx.x == 0) seg[blockIdx.x] = tot;
}

// Exclusive scan of the tiles' values (one workgroup).
__global__ __launch_bounds__(1024) void k_ent_ecarry(const uint32_t *__restrict__ seg, uint32_t *__restrict__ carry,
                                                     int64_t ntiles) {
    __shared__ uint32_t sh[16];
    uint32_t run = 0;
    for (int64_t b = 0; b < ntiles; b += 1024) {
        const int64_t k = b + threadIdx.x;
        uint32_t tot;
        const uint32_t ex = seg_excl_scan<16>(k < ntiles ? seg[k] : 0u, sh, tot);
        if (k < ntiles) carry[k] = seg_join(run, ex);
        run = seg_join(run, tot);
    }
}

// E along each row from d (src, in the workspace) into the layer's plane
// (dst, at the same address mod 16).  The value carried into tile b is the
// join of the tiles before it.  When rows are at most ENT_ETILE pixels wide
// (direct), tile b - 1 holds a row start (tile 0 holds pixel 0, any other is
// ENT_ETILE consecutive pixels), so that join is tile b - 1's own value: the
// workgroup reads tile b - 1 as well and no separate pass is needed.
// Otherwise the carry comes from k_ent_eseg and k_ent_ecarry.
__global__ __launch_bounds__(256) void k_ent_eundo(const uint8_t *__restrict__ src, uint8_t *__restrict__ dst,
                                                   int64_t N, int W, const uint32_t *__restrict__ carry, int direct) {
    __shared__ uint32_t sh[4];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    EChunk c;
    echunk_load(src, N, W, t, c);
    uint32_t cin = 0, tot;
    if (!direct) {
        cin = carry[blockIdx.x];
    } else if (blockIdx.x > 0) {
        EChunk pc;
        echunk_load(src, N, W, t - 256, pc);
        seg_excl_scan<4>(echunk_seg(pc, N, W), sh, cin);
    }
    const uint32_t ex = seg_excl_scan<4>(echunk_seg(c, N, W), sh, tot);
    uint32_t acc = seg_join(cin, ex) & 255u, col = c.col0, o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        acc = (col == 0 ? c.v[k] : acc + c.v[k]) & 255u;
        o[k] = acc;
        col = col + 1 == (uint32_t)W ? 0u : col + 1;
    }
    echunk_store(dst, N, c, o);
}

}  // namespace

void launch_ent_encode(const EntArgs &a, hipStream_t s) {
    const int64_t ng = 4 * (int64_t)a.G;
    if (a.flags & 1) {
        const uint8_t *e = a.resid + 6 * a.N;
        const int lead = (int)(reinterpret_cast<uintptr_t>(e) & 15);
        hipLaunchKernelGGL(k_ent_ediff, dim3((unsigned)ent_etiles(a.N, lead)), dim3(256), 0, s, e, a.ediff, a.N, a.W);
    }
    if (a.flags & 2) {
        hipLaunchKernelGGL(k_ent_hist_ctx, dim3((unsigned)((a.N + ENT_HIST_PX - 1) / ENT_HIST_PX), 2),
                           dim3(ENT_HIST_THREADS), 0, s, a);
        hipLaunchKernelGGL(k_ent_freq, dim3(ENT_NTAB_CTX), dim3(512), 0, s, a);
        hipLaunchKernelGGL(k_ent_enc_ctx, dim3((unsigned)((a.G + 3) / 4), 4), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_ent_scan, dim3(1), dim3(1024), 0, s, a);
        hipLaunchKernelGGL(k_ent_pack, dim3((unsigned)ng), dim3(256), 0, s, a);
        return;
    }
    if ((reinterpret_cast<uintptr_t>(a.resid) & 15) == 0 && a.N >= 16) {
        const int64_t nr = ((6 * a.N + 15) / 16 + ENT_VEC_SPAN / 16 - 1) / (ENT_VEC_SPAN / 16);
        const int64_t ne = (a.N + 16 + ENT_VEC_SPAN - 1) / ENT_VEC_SPAN;
        hipLaunchKernelGGL(k_ent_hist_vec, dim3((unsigned)(nr + ne)), dim3(ENT_HIST_THREADS), 0, s, a, (int)nr);
    } else {
        hipLaunchKernelGGL(k_ent_hist, dim3((unsigned)((a.N + ENT_HIST_PX - 1) / ENT_HIST_PX)), dim3(ENT_HIST_THREADS),
                           0, s, a);
    }
    hipLaunchKernelGGL(k_ent_freq, dim3(4), dim3(512), 0, s, a);
    hipLaunchKernelGGL(k_ent_enc, dim3((unsigned)((ng + 3) / 4)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_ent_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_ent_pack, dim3((unsigned)ng), dim3(256), 0, s, a);
}

void launch_ent_decode(const EntArgs &a, hipStream_t s) {
    if (a.status) hipLaunchKernelGGL(k_ent_status, dim3(1), dim3(64), 0, s, a.status);
    const int gpp = (a.G + ENT_DEC_WAVES - 1) / ENT_DEC_WAVES;
    if (a.flags & 2) {
        hipLaunchKernelGGL(k_ent_dec_ctx, dim3((unsigned)gpp, 3), dim3(64 * ENT_DEC_WAVES), 0, s, a);
        hipLaunchKernelGGL(k_ent_dec, dim3((unsigned)gpp), dim3(64 * ENT_DEC_WAVES), 0, s, a);  // plane 3
    } else {
        hipLaunchKernelGGL(k_ent_dec, dim3((unsigned)(4 * gpp)), dim3(64 * ENT_DEC_WAVES), 0, s, a);
    }
    if (a.flags & 1) {
        uint8_t *e = a.dst + 6 * a.N;
        const int64_t nt = ent_etiles(a.N, (int)(reinterpret_cast<uintptr_t>(e) & 15));
        const int direct = a.W <= ENT_ETILE;
        if (!direct) {
            hipLaunchKernelGGL(k_ent_eseg, dim3((unsigned)nt), dim3(256), 0, s, a.dplane, a.N, a.W, a.eagg);
            hipLaunchKernelGGL(k_ent_ecarry, dim3(1), dim3(1024), 0, s, a.eagg, a.eagg + nt, nt);
        }
        hipLaunchKernelGGL(k_ent_eundo, dim3((unsigned)nt), dim3(256), 0, s, a.dplane, e, a.N, a.W, a.eagg + nt,
                           direct);
    }
}

}  // namespace rdl
