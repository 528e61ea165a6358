// rdl_jpeg.hip -- gfx950 kernels that write the base layer's quantised
// coefficients as a baseline sequential JPEG file (ITU-T T.81) in JFIF: the
// file a viewer shows (the paper's base layer is a JPEG file, Sec. II.B and
// Sec. IV).  One scan per component, Huffman tables optimised for the image
// (Annex K.2), codes as Annex C assigns them.  The file layout is described in
// rdl.h; every byte equals what a plain sequential writer produces.
//
// k_jpg_count (symbol counts per table) -> k_jpg_tables (four Huffman tables,
// the file header) -> k_jpg_bits (bit length of every 8x8 block, sums per
// workgroup) -> k_jpg_offsets (bit offset of every workgroup's blocks, scan
// sizes) -> k_jpg_zero (raw bit buffer) -> k_jpg_emit (every block's bits at
// its offset) -> k_jpg_ffcount (0xFF bytes per chunk) -> k_jpg_layout
// (where every chunk goes, SOS headers, EOI, length) -> k_jpg_stuff (bytes
// with a 0x00 after each 0xFF).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rdl_internal.h"

namespace rdl {

namespace {

// Zig-zag order (Figure A.6): the anti-diagonals s = u + v from the top left,
// downwards on odd s, upwards on even s; zz[k] = natural index of the k-th.
struct ZigZag {
    int zz[64];
    constexpr ZigZag() : zz() {
        int k = 0;
        for (int s = 0; s <= 14; ++s) {
            const int lo = s > 7 ? s - 7 : 0, hi = s < 7 ? s : 7;
            if (s & 1)
                for (int r = lo; r <= hi; ++r) zz[k++] = r * 8 + (s - r);
            else
                for (int r = hi; r >= lo; --r) zz[k++] = r * 8 + (s - r);
        }
    }
};
__constant__ ZigZag c_zz = ZigZag();

__device__ __forceinline__ int ssss(int v) {
    const uint32_t a = (uint32_t)(v < 0 ? -v : v);
    return a ? 32 - __clz(a) : 0;
}

struct Geo {
    int nbx, nby, nblk, wpc;  // blocks per row / column / component, workgroups per component
    int64_t H8, W8;
};
__device__ __forceinline__ Geo geo(const JpgArgs &a) {
    Geo g;
    g.nbx = (a.W + 7) >> 3;
    g.nby = (a.H + 7) >> 3;
    g.nblk = g.nbx * g.nby;
    g.wpc = (g.nblk + JPG_BLK_WG - 1) / JPG_BLK_WG;
    g.H8 = (int64_t)g.nby * 8;
    g.W8 = (int64_t)g.nbx * 8;
    return g;
}

// The coefficients of block k of component c, in zig-zag order, and the DC of
// the block before it in raster order (0 for the first).
__device__ __forceinline__ void load_block(const JpgArgs &a, const Geo &g, int c, int k, int v[64], int &pred) {
    const int by = k / g.nbx, bx = k - by * g.nbx;
    const int16_t *base = a.dct + (int64_t)c * g.H8 * g.W8 + (int64_t)by * 8 * g.W8 + bx * 8;
    int nat[64];
    if ((reinterpret_cast<uintptr_t>(a.dct) & 15) == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint4 q = *reinterpret_cast<const uint4 *>(base + r * g.W8);
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int u = 0; u < 8; ++u) nat[r * 8 + u] = (int)(int16_t)(w4[u >> 1] >> (16 * (u & 1)));
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int u = 0; u < 8; ++u) nat[r * 8 + u] = base[r * g.W8 + u];
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) v[i] = nat[c_zz.zz[i]];
    pred = 0;
    if (k > 0) {
        const int pk = k - 1, pby = pk / g.nbx, pbx = pk - pby * g.nbx;
        pred = a.dct[(int64_t)c * g.H8 * g.W8 + (int64_t)pby * 8 * g.W8 + pbx * 8];
    }
}

// Calls f(ac, symbol, extra, n) for the block's symbols (Annex F.1.2).  An AC
// size above 15 (a coefficient of 2^15 in magnitude, which baseline JPEG does
// not allow and the encoder never makes) is clamped into the symbol so that
// every symbol stays below 256.
template <class F>
__device__ __forceinline__ void block_symbols(const int v[64], int pred, F &&f) {
    const int diff = v[0] - pred;
    int s = ssss(diff);
    f(0, s, (uint32_t)(diff < 0 ? diff - 1 : diff) & ((1u << s) - 1u), s);
    int run = 0;
#pragma unroll
    for (int k = 1; k < 64; ++k) {
        if (v[k] == 0) {
            ++run;
            continue;
        }
        while (run > 15) {
            f(1, 0xF0, 0u, 0);
            run -= 16;
        }
        s = ssss(v[k]);
        f(1, run * 16 + min(s, 15), (uint32_t)(v[k] < 0 ? v[k] - 1 : v[k]) & ((1u << s) - 1u), s);
        run = 0;
    }
    if (run > 0) f(1, 0x00, 0u, 0);
}

// ---------------------------------------------------------------------------
// Symbol counts: one thread per block; table 0 = Y, 1 = Cb and Cr.  A few
// symbols (EOB, the small sizes) take most counts, so lane l counts into copy
// l mod JPG_HC, the copies of a bin in adjacent words (different banks).
constexpr int JPG_HC = 8;
__global__ __launch_bounds__(JPG_BLK_WG) void k_jpg_count(JpgArgs a) {
    __shared__ uint32_t h[2][2][256][JPG_HC];
    for (int k = threadIdx.x; k < 2 * 2 * 256 * JPG_HC; k += JPG_BLK_WG) (&h[0][0][0][0])[k] = 0;
    __syncthreads();
    const Geo g = geo(a);
    const int c = blockIdx.x / g.wpc, k = (blockIdx.x - c * g.wpc) * JPG_BLK_WG + threadIdx.x;
    const int t = c ? 1 : 0;
    const int cp = threadIdx.x & (JPG_HC - 1);
    if (k < g.nblk) {
        int v[64], pred;
        load_block(a, g, c, k, v, pred);
        block_symbols(v, pred, [&](int ac, int sym, uint32_t, int) { atomicAdd(&h[t][ac][sym][cp], 1u); });
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * 2 * 256; i += JPG_BLK_WG) {
        uint32_t x = 0;
#pragma unroll
        for (int q = 0; q < JPG_HC; ++q) x += (&h[0][0][0][0])[i * JPG_HC + q];
        if (x) atomicAdd(&a.ws->cnt[0][0][0] + i, x);
    }
}

// ---------------------------------------------------------------------------
// Huffman tables (Annex K.2) and the file header: one wave per table
// (t = Y / chroma, ac), 4 waves.
//   Figure K.1: while two symbols with a count remain, merge the least (ties:
//   the larger value) into the next least; every symbol of the two merged
//   groups gains one bit.  Groups are tracked by a label per symbol, so a
//   merge is one pass over the 257 symbols (256 + the reserved point).
//   Figure K.3: sizes above 16 are cut; K.4: symbols listed by size, then value;
//   Annex C: canonical codes.  Then the waves write SOI, APP0, DQT, SOF0, DHT.
}  // namespace
}  // namespace rdl
// The device library's wave reduction (DPP; every lane must be active).
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_min_u64(unsigned long long);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_min_u32(unsigned int);
namespace rdl {
namespace {
__device__ __forceinline__ unsigned long long wave_min(unsigned long long v) { return __ockl_wfred_min_u64(v); }
__device__ __forceinline__ unsigned int wave_min(unsigned int v) { return __ockl_wfred_min_u32(v); }

__device__ __forceinline__ void put_be16(uint8_t *p, int v) {
    p[0] = (uint8_t)(v >> 8);
    p[1] = (uint8_t)v;
}

__global__ __launch_bounds__(256) void k_jpg_tables(JpgArgs a) {
    __shared__ int s_nb[4][258];
    __shared__ uint8_t s_hv[4][256];
    __shared__ int s_n[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;  // table w: t = w >> 1, ac = w & 1
    const int t = w >> 1, ac = w & 1;
    // Lane l holds symbols l + 64 j (j < 5; symbol 256 is the reserved point):
    // count, group label and code size in registers.
    uint64_t f[5];
    int grp[5], cs[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const int i = lane + 64 * j;
        f[j] = i < 256 ? a.ws->cnt[t][ac][i] : (i == 256 ? 1u : 0u);
        grp[j] = i;
        cs[j] = 0;
    }
    for (int i = lane; i < 258; i += 64) s_nb[w][i] = 0;
    // Figure K.1.  A group's key is (count, 511 - representative): the least
    // key is the least count, ties to the larger symbol.  Keys fit 32 bits
    // when the table's total count is below 2^22 (every group count is then
    // below it, and no key reaches the all-ones "none"), else 64.
    uint64_t total = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) total += f[j];
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)total, off, 64), hi = __shfl_xor((uint32_t)(total >> 32), off, 64);
        total += (uint64_t)hi << 32 | lo;
    }
    auto merge_all = [&](auto key_type) {
        using KT = decltype(key_type);
        constexpr KT NONE = (KT)~(KT)0;
        for (;;) {
            // the lane's least and second least keys; the second least of the
            // wave is the owner lane's second or another lane's least (keys
            // are distinct)
            KT m1 = NONE, m2 = NONE;
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const KT key = (KT)f[j] << 9 | (KT)(511 - (lane + 64 * j));
                const bool lt1 = f[j] && key < m1, lt2 = f[j] && !lt1 && key < m2;
                m2 = lt1 ? m1 : (lt2 ? key : m2);
                m1 = lt1 ? key : m1;
            }
            const KT k1 = wave_min(m1);
            const int v1 = 511 - (int)(k1 & 511);
            const KT k2 = wave_min(m1 == k1 ? m2 : m1);
            if (k2 == NONE) break;  // uniform
            const int v2 = 511 - (int)(k2 & 511);
            // Only a group's representative (the symbol holding its count) has
            // a count, and a group's label is its representative: true at the
            // start, and a merge relabels v2's group to v1.  So v1 and v2 are
            // the labels of the two groups.
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const int i = lane + 64 * j;
                if (grp[j] == v1 || grp[j] == v2) {
                    cs[j] += 1;
                    grp[j] = v1;
                }
                if (i == v1) f[j] += (uint64_t)(k2 >> 9);
                if (i == v2) f[j] = 0;
            }
        }
    };
    if (total < (1u << 22))
        merge_all(0u);
    else
        merge_all(0ull);
    // Figure K.2's size histogram and Figure K.4's list, by ballots over the
    // 64-symbol chunks, up to the longest size (at most 256: cut at 32, as
    // the figure's arrays are, sizes above would no longer pair up and
    // Figure K.3 would not yield a code); the reserved point (symbol 256,
    // lane 0's fifth entry) is counted, not listed.
    int maxlen = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) maxlen = max(maxlen, cs[j]);
    for (int off = 32; off > 0; off >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, off, 64));
    int nsym = 0;
    for (int len = 1; len <= maxlen; ++len) {
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const bool in = cs[j] == len;
            const unsigned long long m = __ballot(in);
            if (j < 4) {
                if (in) s_hv[w][nsym + __popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)(lane + 64 * j);
                nsym += __popcll(m);
            }
            cnt += __popcll(m);
        }
        if (lane == 0) s_nb[w][len] = cnt;
    }
    // Figure K.3 (sizes above 16 cut), then the reserved point dropped
    if (lane == 0) {
        int *nb = s_nb[w];
        for (int i = maxlen; i > 16; --i)
            while (nb[i] > 0) {
                int j = i - 2;
                while (nb[j] == 0) --j;
                nb[i] -= 2;
                nb[i - 1] += 1;
                nb[j + 1] += 2;
                nb[j] -= 1;
            }
        int i = 16;
        while (i > 1 && nb[i] == 0) --i;
        if (nb[i] > 0) nb[i] -= 1;
        s_n[w] = nsym;
    }
    __syncthreads();
    // Annex C: canonical codes by rank, code | size << 16 per symbol; the
    // rank-r symbol of size len takes the first code of that size + its place
    {
        uint32_t code = 0;
        int r0 = 0;
        for (int len = 1; len <= 16; ++len) {
            const int nl = s_nb[w][len];
            for (int r = r0 + lane; r < r0 + nl; r += 64)
                if (r < nsym) a.ws->code[t][ac][s_hv[w][r]] = (code + (uint32_t)(r - r0)) | (uint32_t)len << 16;
            code = (code + (uint32_t)nl) << 1;
            r0 += nl;
        }
    }
    // File header: SOI, APP0, DQT, SOF0, DHT (wave 0 writes the fixed part,
    // each wave its DHT table)
    uint8_t *o = a.out;
    if (w == 0 && lane == 0) {
        put_be16(o + 0, 0xFFD8);
        put_be16(o + 2, 0xFFE0);
        put_be16(o + 4, 16);
        const uint8_t jfif[14] = {'J', 'F', 'I', 'F', 0, 1, 1, 0, 0, 1, 0, 1, 0, 0};
        for (int k = 0; k < 14; ++k) o[6 + k] = jfif[k];
        put_be16(o + 20, 0xFFDB);
        put_be16(o + 22, 2 + 2 * 65);
        for (int tt = 0; tt < 2; ++tt) {
            o[24 + 65 * tt] = (uint8_t)tt;
            for (int k = 0; k < 64; ++k) o[25 + 65 * tt + k] = a.qt[tt][c_zz.zz[k]];
        }
        uint8_t *sf = o + 154;
        put_be16(sf, 0xFFC0);
        put_be16(sf + 2, 17);
        sf[4] = 8;
        put_be16(sf + 5, a.H);
        put_be16(sf + 7, a.W);
        sf[9] = 3;
        for (int c = 0; c < 3; ++c) {
            sf[10 + 3 * c] = (uint8_t)(c + 1);
            sf[11 + 3 * c] = 0x11;
            sf[12 + 3 * c] = (uint8_t)(c ? 1 : 0);
        }
        int dl = 2;
        for (int k = 0; k < 4; ++k) dl += 17 + s_n[k];
        put_be16(o + 173, 0xFFC4);
        put_be16(o + 175, dl);
        a.ws->hdr_len = 175 + dl;
    }
    // DHT tables in the order (Y DC, Y AC, chroma DC, chroma AC) = waves 0..3
    if (lane == 0) {
        int at = 177;
        for (int k = 0; k < w; ++k) at += 17 + s_n[k];
        o[at] = (uint8_t)(ac * 16 + t);
        for (int len = 1; len <= 16; ++len) o[at + len] = (uint8_t)s_nb[w][len];
        for (int r = 0; r < nsym; ++r) o[at + 17 + r] = s_hv[w][r];
    }
    // counts back to zero for the next call
    for (int i = lane; i < 256; i += 64) a.ws->cnt[t][ac][i] = 0;
}

// ---------------------------------------------------------------------------
// Bit length of every block; sums per workgroup.
__global__ __launch_bounds__(JPG_BLK_WG) void k_jpg_bits(JpgArgs a) {
    __shared__ uint8_t s_sz[2][256];
    __shared__ uint32_t s_red[JPG_BLK_WG / 64];
    const Geo g = geo(a);
    const int c = blockIdx.x / g.wpc, k = (blockIdx.x - c * g.wpc) * JPG_BLK_WG + threadIdx.x;
    const int t = c ? 1 : 0;
    for (int i = threadIdx.x; i < 512; i += JPG_BLK_WG) (&s_sz[0][0])[i] = (uint8_t)(a.ws->code[t][i >> 8][i & 255] >> 16);
    __syncthreads();
    uint32_t bits = 0;
    if (k < g.nblk) {
        int v[64], pred;
        load_block(a, g, c, k, v, pred);
        block_symbols(v, pred, [&](int ac, int sym, uint32_t, int n) { bits += s_sz[ac][sym] + n; });
        a.blen[(int64_t)c * g.nblk + k] = bits;
    }
    for (int off = 32; off > 0; off >>= 1) bits += __shfl_xor(bits, off, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < JPG_BLK_WG / 64; ++i) s += s_red[i];
        a.wsum[blockIdx.x] = s;
    }
}

// Exclusive scan of the workgroup sums per component (bit offsets within the
// component's scan), the scans' bit counts and their raw-buffer word offsets.
__global__ __launch_bounds__(1024) void k_jpg_offsets(JpgArgs a) {
    __shared__ uint32_t sh[16];
    __shared__ uint64_t s_carry;
    const Geo g = geo(a);
    for (int c = 0; c < 3; ++c) {
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (int b = 0; b < g.wpc; b += 1024) {
            const int i = b + threadIdx.x;
            const uint32_t v = i < g.wpc ? a.wsum[c * g.wpc + i] : 0u;
            // block exclusive scan
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            uint32_t inc = v;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            if (lane == 63) sh[wv] = inc;
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int k = 0; k < 16; ++k) {
                before += k < wv ? sh[k] : 0u;
                tot += sh[k];
            }
            if (i < g.wpc) a.woff[c * g.wpc + i] = s_carry + before + inc - v;
            __syncthreads();
            if (threadIdx.x == 0) s_carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) a.ws->bits[c] = s_carry;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint64_t wo = 0;
        for (int c = 0; c < 3; ++c) {
            a.ws->raw_word[c] = wo;
            wo += (a.ws->bits[c] + 31) / 32;
        }
        a.ws->raw_words = wo;
    }
}

__global__ void k_jpg_zero(JpgArgs a) {
    const uint64_t n = a.ws->raw_words;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        a.raw[i] = 0;
}

// Every block's bits at its offset: bit p of a scan is bit 7 - (p mod 8) of its
// byte p / 8, so a 32-bit word of the raw buffer holds 4 bytes in memory order
// (written byte-swapped).  A block builds its words in a register and stores
// them; its first and last words may hold bits of the neighbouring blocks and
// are ORed in instead.  The last block of a scan pads the last byte with 1-bits.
struct WordOut {
    uint32_t *raw;
    uint64_t w;        // next word to write
    uint64_t first;    // the block's first word (shared with the block before)
    uint64_t acc;      // pending bits, the oldest at the top of the nacc low bits
    int nacc;
    __device__ __forceinline__ void put(uint32_t v, int n) {
        if (n == 0) return;
        acc = (acc << n) | v;
        nacc += n;
        if (nacc >= 32) {
            const uint32_t word = (uint32_t)(acc >> (nacc - 32));
            nacc -= 32;
            if (w == first) atomicOr(raw + w, __builtin_bswap32(word));
            else raw[w] = __builtin_bswap32(word);
            ++w;
        }
    }
    __device__ __forceinline__ void finish() {  // the last, partial word is shared with the next block
        if (nacc > 0) atomicOr(raw + w, __builtin_bswap32((uint32_t)(acc << (32 - nacc))));
    }
};

__global__ __launch_bounds__(JPG_BLK_WG) void k_jpg_emit(JpgArgs a) {
    __shared__ uint32_t s_code[2][256];
    __shared__ uint32_t sh[JPG_BLK_WG / 64];
    const Geo g = geo(a);
    const int c = blockIdx.x / g.wpc, k = (blockIdx.x - c * g.wpc) * JPG_BLK_WG + threadIdx.x;
    const int t = c ? 1 : 0;
    for (int i = threadIdx.x; i < 512; i += JPG_BLK_WG) (&s_code[0][0])[i] = a.ws->code[t][i >> 8][i & 255];
    const uint32_t len = k < g.nblk ? a.blen[(int64_t)c * g.nblk + k] : 0u;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = len;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) sh[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < wv; ++i) before += sh[i];
    if (k >= g.nblk) return;
    const uint64_t pos = a.woff[blockIdx.x] + before + inc - len;
    WordOut o;
    o.raw = a.raw + a.ws->raw_word[c];
    o.w = o.first = pos >> 5;
    o.acc = 0;
    o.nacc = (int)(pos & 31);  // the block starts inside its first word: leading zero bits
    int v[64], pred;
    load_block(a, g, c, k, v, pred);
    block_symbols(v, pred, [&](int ac, int sym, uint32_t extra, int n) {
        const uint32_t cs = s_code[ac][sym];
        o.put(cs & 0xFFFFu, (int)(cs >> 16));
        o.put(extra, n);
    });
    if (k == g.nblk - 1 && ((pos + len) & 7)) {
        const int pad = 8 - (int)((pos + len) & 7);
        o.put((1u << pad) - 1u, pad);
    }
    o.finish();
}

// 0xFF bytes per chunk of JPG_CHUNK raw bytes of each scan.
// (A fixed grid walks the chunks that hold data.)
// Bytes [b0, b0 + 16) of a scan's raw bits (nbytes > 0), from four word
// loads whose indices are clamped to the scan's last word, so every load is
// issued unconditionally; bytes past the scan read as 0.
__device__ __forceinline__ void raw16(const uint32_t *w, uint64_t nbytes, uint64_t b0, uint32_t (&by)[16]) {
    const uint64_t last = (nbytes + 3) / 4 - 1;
    uint32_t x[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint64_t q = b0 / 4 + m;
        x[m] = w[q < last ? q : last];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) by[i] = b0 + i < nbytes ? (x[i >> 2] >> (8 * (i & 3))) & 255u : 0u;
}

__global__ __launch_bounds__(256) void k_jpg_ffcount(JpgArgs a) {
    static_assert(JPG_CHUNK == 256 * 16, "one 16-byte piece per lane and chunk");
    __shared__ uint32_t sh[4];
    for (int c = 0; c < 3; ++c) {
        const uint64_t nbytes = (a.ws->bits[c] + 7) / 8;
        const int64_t nch = (int64_t)((nbytes + JPG_CHUNK - 1) / JPG_CHUNK);
        const uint32_t *raw = a.raw + a.ws->raw_word[c];
        for (int64_t j = blockIdx.x; j < nch; j += gridDim.x) {
            uint32_t n = 0, by[16];
            raw16(raw, nbytes, (uint64_t)j * JPG_CHUNK + (uint64_t)threadIdx.x * 16, by);
#pragma unroll
            for (int i = 0; i < 16; ++i) n += by[i] == 0xFFu ? 1u : 0u;
            for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
            __syncthreads();
            if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = n;
            __syncthreads();
            if (threadIdx.x == 0) a.ffcnt[c * a.cpc + j] = sh[0] + sh[1] + sh[2] + sh[3];
        }
    }
}

// Where every chunk's bytes go in the file; SOS headers, EOI, the length.
__global__ __launch_bounds__(1024) void k_jpg_layout(JpgArgs a) {
    __shared__ uint32_t sh[16];
    __shared__ uint64_t s_carry, s_at;
    if (threadIdx.x == 0) s_at = a.ws->hdr_len;
    __syncthreads();
    for (int c = 0; c < 3; ++c) {
        const uint64_t nbytes = (a.ws->bits[c] + 7) / 8;
        if (threadIdx.x == 0) {
            uint8_t *sos = a.out + s_at;
            put_be16(sos, 0xFFDA);
            put_be16(sos + 2, 8);
            sos[4] = 1;
            sos[5] = (uint8_t)(c + 1);
            sos[6] = (uint8_t)(c ? 0x11 : 0x00);
            sos[7] = 0;
            sos[8] = 63;
            sos[9] = 0;
            s_at += 10;
            s_carry = 0;
        }
        __syncthreads();
        const int nch = (int)((nbytes + JPG_CHUNK - 1) / JPG_CHUNK);
        for (int b = 0; b < nch; b += 1024) {
            const int i = b + threadIdx.x;
            const uint32_t v = i < nch ? a.ffcnt[c * a.cpc + i] : 0u;
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            uint32_t inc = v;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            if (lane == 63) sh[wv] = inc;
            __syncthreads();
            uint32_t before = 0, tot = 0;
            for (int k = 0; k < 16; ++k) {
                before += k < wv ? sh[k] : 0u;
                tot += sh[k];
            }
            // file position of chunk i's first byte: scan start + bytes before + stuffed zeros before
            if (i < nch) a.cpos[c * a.cpc + i] = s_at + (uint64_t)i * JPG_CHUNK + s_carry + before + inc - v;
            __syncthreads();
            if (threadIdx.x == 0) s_carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) s_at += nbytes + s_carry;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        put_be16(a.out + s_at, 0xFFD9);
        *a.out_len = s_at + 2;
    }
}

// Raw bytes of a chunk into the file, a 0x00 after each 0xFF (16 per thread;
// a fixed grid walks the chunks that hold data).
__global__ __launch_bounds__(256) void k_jpg_stuff(JpgArgs a) {
    __shared__ uint32_t sh[4];
    for (int c = 0; c < 3; ++c) {
        const uint64_t nbytes = (a.ws->bits[c] + 7) / 8;
        const int64_t nch = (int64_t)((nbytes + JPG_CHUNK - 1) / JPG_CHUNK);
        const uint32_t *raw = a.raw + a.ws->raw_word[c];
        for (int64_t j = blockIdx.x; j < nch; j += gridDim.x) {
            const uint64_t b0 = (uint64_t)j * JPG_CHUNK + (uint64_t)threadIdx.x * 16;
            uint32_t by[16];
            uint32_t n = 0;
            if (b0 < nbytes) raw16(raw, nbytes, b0, by);
            else
#pragma unroll
                for (int i = 0; i < 16; ++i) by[i] = 0u;
#pragma unroll
            for (int i = 0; i < 16; ++i) n += by[i] == 0xFFu ? 1u : 0u;
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            uint32_t inc = n;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(inc, off, 64);
                if (lane >= off) inc += y;
            }
            __syncthreads();
            if (lane == 63) sh[wv] = inc;
            __syncthreads();
            uint32_t before = 0;
            for (int i = 0; i < wv; ++i) before += sh[i];
            uint64_t at = a.cpos[c * a.cpc + j] + (uint64_t)threadIdx.x * 16 + before + inc - n;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (b0 + i < nbytes) {
                    a.out[at++] = (uint8_t)by[i];
                    if (by[i] == 0xFFu) a.out[at++] = 0;
                }
            }
        }
    }
}

}  // namespace

void launch_jpeg(const JpgArgs &a, hipStream_t s) {
    const int nbx = (a.W + 7) >> 3, nby = (a.H + 7) >> 3, nblk = nbx * nby;
    const int wpc = (nblk + JPG_BLK_WG - 1) / JPG_BLK_WG;
    hipLaunchKernelGGL(k_jpg_count, dim3(3 * wpc), dim3(JPG_BLK_WG), 0, s, a);
    hipLaunchKernelGGL(k_jpg_tables, dim3(1), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_jpg_bits, dim3(3 * wpc), dim3(JPG_BLK_WG), 0, s, a);
    hipLaunchKernelGGL(k_jpg_offsets, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_jpg_zero, dim3(1024), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_jpg_emit, dim3(3 * wpc), dim3(JPG_BLK_WG), 0, s, a);
    const int sgrid = (int)std::min<int64_t>(a.cpc, 1024);
    hipLaunchKernelGGL(k_jpg_ffcount, dim3(sgrid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_jpg_layout, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_jpg_stuff, dim3(sgrid), dim3(256), 0, s, a);
}

}  // namespace rdl
