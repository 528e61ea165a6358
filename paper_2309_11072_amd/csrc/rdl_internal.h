// rdl_internal.h -- shared between the HIP kernels and the host C-ABI layer
// of the MI355X encoder (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rdl.h"

namespace rdl {

// Work decomposition, fixed for every stage kernel.
constexpr int KS_THREADS = 1024;   // key statistic: 1024 lanes x 32 px
constexpr int KS_PX_PER_WG = 32768;
constexpr int KS_STRIPES = 16;     // partial-sum copies per image, so that no
constexpr int FIT_STRIPES = 4;     //   address takes more than a few atomics
constexpr int BLK_WG = 32;        // tone map + base layer: 32 blocks of one block row,
constexpr int BLK_THREADS = 256;   //   8 lanes per block
constexpr int STRIP_W = 256;       // GF-based stages (fit, residual, decode): a wave
constexpr int STRIP_WAVES = 4;     //   walks srh rows of a 256-px strip, 4 px per
constexpr int STRIP_THREADS = 64 * STRIP_WAVES;  // lane; 4 waves stacked per workgroup
constexpr int SRH_MIN = 2, SRH_MAX = 32;  // srh: a power of two in [2, 32], tuned per
constexpr int SRH_FIT_DEFAULT = 16;       //   kernel and image size
constexpr int SRH_RES_DEFAULT = 8;
constexpr int FIT_BINS_DEFAULT = 2;       // privatised copies of the fit's LDS bins: 1, 2 or 4
constexpr int FIT_WG_ROWS_MAX = 128;      // waves x rows per fit workgroup: <= 32768 px, so
                                          //   the workgroup's 32-bit bin totals cannot wrap
constexpr int LCH = 32768;         // learned path: residual records per histogram workgroup
constexpr int LH_COPIES = 8;       //   and its lane-interleaved LDS histogram copies
// Learned path: a workgroup takes a 64-px-wide column of `tiles` tiles of 16
// rows.  More tiles spread a workgroup's set-up (model fragments, bias table,
// coefficients) over more pixels; fewer keep a small launch at several
// workgroups per CU.  Chosen per launch from its pixel count.
constexpr int LEARN_W = 64, LEARN_TILE_H = 16;
inline int learn_tiles(size_t launch_px) { return launch_px >= ((size_t)1 << 25) ? 12 : 8; }
constexpr int MODEL_BYTES = 7512;
// The device copy of a model appends biases derived on the host when it is
// set: B2[n] + 128 sum_k W2[n][k] (32 x i32) and B3[c] + 128 sum_k W3[c][k]
// (16 x i32), the biases for hidden activations offset by -128.
constexpr int MODEL_B2X = MODEL_BYTES, MODEL_B3X = MODEL_BYTES + 128, MODEL_DEV_BYTES = MODEL_BYTES + 192;
constexpr int TILE_H = 16;         // residual histogram: 16 x 128 px tiles,
constexpr int TILE_W = 128;        //   256 lanes x 8 consecutive px
constexpr int TILE_THREADS = 256;
constexpr int RUN = 8;
constexpr int NSUM = 13;           // n, then (sum s, sum m, sum s^2, sum s m) x 3
// Per-image scratch (int64): key-statistic stripes, final sums, sum stripes.
constexpr int SCR_KS = 0;
constexpr int SCR_SUMS = SCR_KS + 2 * KS_STRIPES;
constexpr int SCR_PART = SCR_SUMS + 256 * NSUM;
constexpr int SCR_LBK = SCR_PART + FIT_STRIPES * 256 * NSUM;
constexpr int LBK_WORDS = 256 + 257 + 256;  // learned path: uint32 bucket table (see ImgDesc::lbk)
constexpr int SCRATCH_I64 = SCR_LBK + (LBK_WORDS + 1) / 2;
constexpr int GAMMA_LUT_N = 21 * 128;             // float-bit buckets 2^-20 .. 2^1

// One image of a launch.  Every kernel walks a flattened workgroup space over
// all images of the launch; wg_* is this image's first workgroup.
struct ImgDesc {
    const uint8_t *rgbe;   // [H][W][4]
    uint8_t *sdr0;         // optional [H][W][3] tone-mapped SDRI
    uint8_t *sdr;          // [H][W][3]
    int16_t *dct;          // optional [3][H8][W8]
    rdl_header *hdr;
    uint8_t *resid;        // 7*H*W
    int64_t *ks;           // [nks][2] partial (Lambda, N'), summed by readers
    int64_t *sums;         // [256][13] regression sums (written by k_solve)
    int64_t *part;         // [nfs][13][256] partial regression sums (value-major)
    int32_t *status;       // decode only, optional
    uint8_t *out_rgbe;     // decode only
    int64_t *hist;         // [3][511] residual histograms
    uint8_t *lres;         // learned path: [H][W] learned residuals, (r_c + 255) << 9c words
    uint32_t *lhist;       // learned path: [2][3][256][511] residual histograms (estimator, channel),
                           //   then [3][511] of the SLR residuals over the image
    uint64_t *lrec;        // learned path: [H*W] residual records, grouped by exponent
    uint32_t *lbk;         // learned path: [256] record cursors, [257] first histogram
                           //   workgroup of each exponent, [256] first record of each exponent
    const uint8_t *model;  // learned path: model blob (device)
    uint64_t model_hash;
    int32_t H, W, q, flags;
    int32_t nks, nfs, srh_fit, srh_res;  // rows per wave of the fit / residual+decode strip walks
    int32_t wg_px, wg_blk, wg_tile, wg_fit, wg_res, wg_learn, wg_lhist;
    int32_t fit_bins, fit_waves;  // the fit launch's bin copies and waves per workgroup
};

// Accumulator hygiene: scratch stripes are all-zero between launch sequences
// (zeroed at allocation; k_solve and k_key_total zero what they consume).
// F_ZERO_* ask k_zero to clear a caller's buffer; F_CLEAN_KS lets the last
// consumer zero the key-statistic stripes (set only when they are scratch).
// F_EST_GLOBAL / F_EST_IDENT / F_NOGF select the ablation estimators of the
// encoder (one line per channel for the whole image; M* = S; S* = S).
enum : int32_t { F_ZERO_KS = 1, F_ZERO_SUMS = 2, F_ZERO_HIST = 4, F_CLEAN_KS = 8, F_EST_GLOBAL = 16, F_EST_IDENT = 32,
                 F_NOGF = 64 };

inline int wgs_px(int H, int W) { return (int)(((int64_t)H * W + KS_PX_PER_WG - 1) / KS_PX_PER_WG); }
inline int wgs_blk(int H, int W) { return ((H + 7) / 8) * (((W + 7) / 8 + BLK_WG - 1) / BLK_WG); }
inline int wgs_tile(int H, int W) { return ((H + TILE_H - 1) / TILE_H) * ((W + TILE_W - 1) / TILE_W); }
inline int wgs_strip(int H, int W, int srh, int waves = STRIP_WAVES) {
    const int sh = srh * waves;
    return ((H + sh - 1) / sh) * ((W + STRIP_W - 1) / STRIP_W);
}
inline int wgs_learn(int H, int W, int tiles) {
    const int rows = LEARN_TILE_H * tiles;
    return ((H + rows - 1) / rows) * ((W + LEARN_W - 1) / LEARN_W);
}
// Learned path, per image: residual histograms [2][3][256][511] (estimator,
// channel, exponent), then the SLR residual histogram of each channel over
// the whole image [3][511] (at LHIST_G).
constexpr size_t LHIST_G = (size_t)2 * 3 * 256 * 511;
inline size_t lhist_words() { return LHIST_G + 3 * 511; }
// Histogram workgroups of an image: one per LCH records of each exponent,
// at most H*W / LCH + 1 per present exponent.
inline int wgs_lhist(int H, int W) { return (int)(((int64_t)H * W + LCH - 1) / LCH) + 256; }

// Kernel launchers (defined in rdl_kernels.hip).
hipError_t upload_tables(int *bad_table);
void launch_zero(const ImgDesc *d, int n, hipStream_t s);
constexpr int DESC_CHUNK = 4;  // descriptors per k_put_desc launch (kernel-argument bytes)
void launch_put_desc(ImgDesc *dst, const ImgDesc *host, int n, hipStream_t s);
void launch_check_recip(uint32_t lo, uint32_t count, unsigned long long *bad, hipStream_t s);
void launch_keystat(const ImgDesc *d, int n, int wgs, hipStream_t s);
void launch_tmo_base(const ImgDesc *d, int n, int wgs, bool extra, hipStream_t s);
void launch_fit_sums(const ImgDesc *d, int n, int wgs, int bins, int waves, hipStream_t s, bool gf = true);
void launch_solve(const ImgDesc *d, int n, hipStream_t s);
void launch_key_total(const ImgDesc *d, int n, int64_t *out2, hipStream_t s);
void launch_resid(const ImgDesc *d, int n, int wgs, hipStream_t s, bool gf = true);
void launch_resid_patch(const ImgDesc *d, int n, int wgs, hipStream_t s);  // learned path; wgs = wgs_px
void launch_decode(const ImgDesc *d, int n, int wgs, hipStream_t s);
void launch_base_decode(const ImgDesc *d, int n, int wgs, hipStream_t s);
void launch_status_init(const ImgDesc *d, int n, hipStream_t s);
void launch_hist(const ImgDesc *d, int n, int wgs, hipStream_t s);
void launch_learn(const ImgDesc *d, int n, int wgs, int rq, int tiles, hipStream_t s);  // rq: RQ_* path
void launch_lhist(const ImgDesc *d, int n, int wgs, hipStream_t s);
void launch_select(const ImgDesc *d, int n, hipStream_t s);
void launch_decode_learned(const ImgDesc *d, int n, int wgs, int rq, int tiles, hipStream_t s);

// Entropy code of the enhancement layer (static rANS with 64 interleaved
// states per group; kernels in rdl_entropy.hip, format in rdl.h).
constexpr int ENT_PB = 15;                 // probability scale M = 2^15
constexpr uint32_t ENT_M = 1u << ENT_PB;
constexpr uint32_t ENT_L = 1u << 16;       // states lie in [2^16, 2^32)
constexpr int ENT_HDR = 4136;              // fixed header bytes before the group table (4 tables)
constexpr int ENT_NCTX = 8;                // residual contexts per channel (S >> 5)
constexpr int ENT_NTAB_CTX = 3 * ENT_NCTX + 1;  // tables of a stream with contexts (the exponents' last)
constexpr int ENT_HDR_CTX = 40 + 1024 * ENT_NTAB_CTX;  // 25640
constexpr int ENT_HIST_PX = 16384;         // histogram workgroup: pixels per workgroup
constexpr int ENT_DEC_WAVES = 4;           // decoder: groups (waves) per workgroup
constexpr int ENT_HSTRIPES = 16;           // copies of the image's histograms (workgroup w adds
                                           //   into copy w mod 16, so hot bins take few atomics)
struct EntWs {
    uint32_t hist[ENT_HSTRIPES][ENT_NTAB_CTX][512];  // table histograms; zero between calls (k_ent_freq clears)
    uint2 tab[ENT_NTAB_CTX][512];  // encoder tables: {f | c << 16, bits of fl(1/f)}
    uint32_t bad[ENT_NTAB_CTX];    // table counted a residual outside [-255, 255]
    uint32_t ok;                   // the stream is valid (set by k_ent_scan)
    uint32_t pad[2];
};
struct EntArgs {
    const uint8_t *resid;   // encoder input / decoder output: 7*H*W bytes
    const uint8_t *eplane;  // encoder: plane 3's symbols (the exponents, or their left differences)
    uint8_t *ediff;         // encoder: where the left differences go (workspace, 16-byte aligned)
    uint32_t *eagg;         // decoder: [2][tiles] segment values of the inverse (workspace)
    uint8_t *dplane;        // decoder: where plane 3's symbols go (the layer, or the workspace)
    int32_t flags;          // bit 0: plane 3 holds left differences; bit 1: residual contexts
    const uint8_t *sdr;     // flags bit 1: the decoded base layer (H*W*3 bytes), the contexts
    int32_t ntab;           // tables in the stream: 4, or ENT_NTAB_CTX with contexts
    int32_t hdr;            // header bytes before the group table: ENT_HDR or ENT_HDR_CTX
    uint8_t *out;           // encoder: the code stream
    const uint8_t *code;    // decoder: the code stream
    uint8_t *dst;           // decoder: the enhancement layer
    uint64_t *out_len;
    int32_t *status;
    EntWs *ws;
    uint32_t *cnt;          // [4 G] words of each group
    uint16_t *tmp;          // [4 G][ent_slot] each group's words in emission order
    int64_t N;
    int64_t nwords;         // decoder: payload words
    int32_t H, W, log2_k, G;
};
inline int64_t ent_groups(int H, int W, int log2_k) {
    const int64_t z = (int64_t)64 << log2_k;
    return ((int64_t)H * W + z - 1) / z;
}
// Workspace words per group: at most one word per symbol plus the 128 state
// words, then 64 words that lanes without a word to emit write instead.
__host__ __device__ inline int64_t ent_slot(int log2_k) { return ((int64_t)64 << log2_k) + 128 + 64; }
inline size_t ent_cnt_off() { return (sizeof(EntWs) + 255) & ~(size_t)255; }
inline size_t ent_tmp_off(int64_t G) { return (ent_cnt_off() + 4 * (size_t)G * 4 + 255) & ~(size_t)255; }
inline size_t ent_ediff_off(int H, int W, int log2_k) {
    const int64_t G = ent_groups(H, W, log2_k);
    return (ent_tmp_off(G) + 4 * (size_t)G * (size_t)ent_slot(log2_k) * 2 + 255) & ~(size_t)255;
}
// The exponents' differences sit at the workspace offset + the plane's
// address mod 16 (lead), so that both share their 16-byte chunks.
inline size_t ent_ws_bytes(int H, int W, int log2_k) {
    return ent_ediff_off(H, W, log2_k) + (((size_t)H * W + 16 + 255) & ~(size_t)255);
}
// Workgroups of the left-difference kernels: 256 lanes of one 16-byte chunk.
constexpr int ENT_ETILE = 4096;
inline int64_t ent_etiles(int64_t N, int lead) { return (N + lead + ENT_ETILE - 1) / ENT_ETILE; }
// The decoder's workspace: the segment values of the inverse after EntWs,
// then the exponents' differences (at the plane's lead, as in the encoder).
inline size_t ent_dplane_off(int64_t N) { return (ent_cnt_off() + 8 * (size_t)ent_etiles(N, 15) + 255) & ~(size_t)255; }
inline size_t ent_dec_ws_bytes(int64_t N) { return ent_dplane_off(N) + (((size_t)N + 16 + 255) & ~(size_t)255); }
void launch_ent_encode(const EntArgs &a, hipStream_t s);
void launch_ent_decode(const EntArgs &a, hipStream_t s);

// Base-layer JPEG file (kernels in rdl_jpeg.hip, format in rdl.h).
constexpr int JPG_BLK_WG = 256;        // blocks (threads) per workgroup
constexpr int JPG_CHUNK = 4096;        // raw bytes per stuffing workgroup
constexpr int JPG_BLOCK_BITS = 2048;   // most bits of one block for any int16 input: DC 16 + 17,
                                       //   at most 63 AC symbols of 16 + 15 bits, ZRLs and EOB
struct JpgWs {
    uint32_t cnt[2][2][256];   // symbol counts per (table, DC/AC); zero between calls
    uint32_t code[2][2][256];  // code | size << 16
    uint64_t bits[3];          // bits of each scan
    uint64_t raw_word[3];      // first raw-buffer word of each scan
    uint64_t raw_words;
    uint64_t hdr_len;          // bytes before the first SOS
};
struct JpgArgs {
    const int16_t *dct;        // quantised coefficients [3][H8][W8]
    uint8_t *out;
    uint64_t *out_len;
    JpgWs *ws;
    uint32_t *blen;            // [3][nblk] bits of each block
    uint32_t *wsum;            // [3][wpc] bits of each workgroup's blocks
    uint64_t *woff;            // [3][wpc] their first bit within the scan
    uint32_t *raw;             // scans' bits, MSB first, bytes in memory order
    uint32_t *ffcnt;           // [3][cpc] 0xFF bytes per chunk
    uint64_t *cpos;            // [3][cpc] file position of each chunk
    int32_t H, W, q, cpc;
    uint8_t qt[2][64];         // quantisation tables, natural order
};
void quant_tables_host(int q, uint8_t out[2][64]);
void launch_jpeg(const JpgArgs &a, hipStream_t s);
inline int64_t jpg_blocks(int H, int W) { return (int64_t)((H + 7) / 8) * ((W + 7) / 8); }
inline int64_t jpg_raw_words(int H, int W) { return 3 * (jpg_blocks(H, W) * JPG_BLOCK_BITS / 32 + 2); }
inline int jpg_cpc(int H, int W) { return (int)((jpg_blocks(H, W) * JPG_BLOCK_BITS / 8 + 1) / JPG_CHUNK + 1); }

// Training kernels (defined in rdl_train.hip).
void launch_train_samples(const uint8_t *rgbe, const uint8_t *sdr, int H, int W, int k_img, const int64_t *idx,
                          int64_t n, void *out, hipStream_t s);
void launch_train_step(float *prm, float *m1, float *m2, const void *smp, int64_t base, int64_t nsamp, int batch,
                       float *part, float *ploss, float lr, int step, float *loss_out, hipStream_t s);
int train_nparam();
int train_sample_bytes();

}  // namespace rdl
