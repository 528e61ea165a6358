/*
 * rdl.h -- C ABI of the MI355X (gfx950) encoder for dual-layer lossless coding
 * of Radiance (RGBE) HDR images, after Suzuki et al., "Lightning-Fast
 * Dual-Layer Lossless Coding for Radiance Format High Dynamic Range Images"
 * (arXiv 2309.11072).
 *
 * Plain C99.  No C++ or torch type crosses this boundary and no function
 * throws.  Every data pointer is a DEVICE pointer unless the comment says
 * "host"; the caller owns every data buffer.  `stream` is a hipStream_t
 * passed as void* (NULL = the null stream).  Calls only enqueue work on
 * `stream` and never synchronise it; an argument error is returned before
 * anything is enqueued.  One rdl_ctx must not be used from two host threads
 * or on two streams at the same time.
 *
 * Layouts (all row-major, pixel (y, x) at index y*W + x):
 *   rgbe   uint8 [H][W][4]  R, G, B mantissas then the shared exponent E
 *                           (Sec. II.A, Fig. 1).  Any 32-bit word is accepted.
 *   sdr    uint8 [H][W][3]  the base-layer SDR image S exactly as a JPEG
 *                           decoder returns it (Sec. III.A: "encoded-decoded
 *                           SDRI").
 *   resid  7*H*W bytes      int16 r[3][H][W] = M - M* (Eq. 8), then uint8
 *                           E[H][W]: the enhancement layer's two planes.
 *   header rdl_header       side information of Sec. III.C: one fixed-point
 *                           (a_E, b_E) per channel and exponent value.
 */
#ifndef RDL_H
#define RDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RDL_MAGIC 0x314C4452u /* "RDL1" little-endian */
#define RDL_VERSION 1u

/* Status codes.  RDL_EHIP: the HIP runtime reported an error (rdl_strerror
 * then names it).  RDL_ECORRUPT: a header failed validation. */
enum {
    RDL_OK = 0,
    RDL_EINVAL = -1,
    RDL_EHIP = -2,
    RDL_ECORRUPT = -3,
    RDL_ENOMEM = -4,
    RDL_EUNSUPPORTED = -5
};

/* Side information (Sec. III.C: each parameter is a 32-bit value; the decoder
 * reads them and never recomputes them).  a_q has 22 and b_q 14 fractional
 * bits: a_E = a_q / 2^22, b_E = b_q / 2^14.  Written in device memory by the
 * encoder so that a whole encode can be captured in a graph.  7232 bytes. */
typedef struct rdl_header {
    uint32_t magic;      /* RDL_MAGIC */
    uint32_t version;    /* RDL_VERSION */
    int32_t H, W, q;     /* image size and base-layer JPEG quality */
    int32_t k_img;       /* tone-mapping key: Q = 2^16 k_img + f_key */
    int32_t f_key;       /* (Q is minus the Q16 mean log2 luminance)  */
    float sigma;         /* 0.18 * 2^(f_key / 2^16)                    */
    int64_t lambda_sum;  /* Q16 sum of log2 luminance over lit pixels  */
    int64_t n_lit;       /* number of pixels with E != 0               */
    int32_t estimator;   /* bits 0-3: 0 SLR per region, 1 flag[][]      */
                         /* chooses SLR or learned, 2 one SLR line per  */
                         /* channel (ablation), 3 M* = S (ablation: no  */
                         /* estimator); bit 4: Gaussian filter off      */
    int32_t n_regions;   /* number of exponent values present          */
    uint64_t model_hash; /* learned estimator in use (0 if none)       */
    int32_t a_q[3][256]; /* slope per (channel, E), Q22                */
    int32_t b_q[3][256]; /* intercept per (channel, E), Q14            */
    uint8_t present[256];  /* 1 if some pixel has exponent E            */
    uint8_t flag[3][256];  /* 0 = SLR estimate, 1 = learned estimate    */
} rdl_header;

typedef struct rdl_ctx rdl_ctx;

/* Create a context on HIP device `device`: uploads the frozen tables and
 * allocates a small scratch area (grown on demand).  Host pointer out. */
int rdl_create(rdl_ctx **out, int device);
void rdl_destroy(rdl_ctx *ctx);
const char *rdl_strerror(int code);

/* Bytes of the residual buffer for an H x W image: 7*H*W. 0 if invalid. */
size_t rdl_resid_bytes(int H, int W);
size_t rdl_header_bytes(void);

/* Host-side validation of a header copied to the host: magic, version, size
 * and parameter bounds (|a_q| <= 255*2^22, -65025*2^14 <= b_q <= 65280*2^14,
 * the ranges every least-squares line through 8-bit data stays in).  RDL_OK
 * or RDL_ECORRUPT. */
int rdl_header_validate(const rdl_header *host_hdr, int H, int W);

/* Encoder (Sec. III, Fig. 2 bottom; all four steps on the GPU):
 *   (a) RGBE unpack + global Reinhard tone mapping to an 8-bit SDRI (Sec. IV);
 *   (b) JPEG-style 4:4:4 8x8 integer FDCT, quantise (Annex K tables scaled by
 *       q), dequantise, integer IDCT: out_sdr = S, what Decoder 1 returns;
 *   (c) S* = GF(S) and, per (channel, E), exact sums of Eq. 9-10, then the
 *       fixed-point slope and intercept -> out_coeffs;
 *   (d) out_resid = M - M* with M* = round(a_E S* + b_E) in [0, 255] (Eq. 8).
 * rgbe: H*W*4 bytes; out_sdr: H*W*3; out_coeffs: one rdl_header; out_resid:
 * rdl_resid_bytes(H, W).  1 <= H, W; W <= 2^28; H*W < 2^31; 1 <= q <= 100.
 * rgbe, out_sdr and out_coeffs start on 4-byte boundaries, out_resid on a
 * 2-byte one.  Buffers must not overlap.  RDL_EINVAL on a bad argument.
 * This is rdl_encode_batch with one image: plans and launch modes (below)
 * apply to it the same way. */
int rdl_encode_enh(rdl_ctx *ctx, const uint8_t *rgbe, int H, int W, int q, uint8_t *out_sdr,
                   rdl_header *out_coeffs, void *out_resid, void *stream);

/* Decoder of the enhancement layer (Sec. I: the HDR image is recovered by
 * adding the residuals; Sec. III.C: parameters are read, not recomputed):
 * S* = GF(sdr), M = M*(a_E, b_E, S*) + r, out_rgbe = (M, E).  coeffs is a
 * DEVICE header (as written by rdl_encode_enh); sdr, coeffs and out_rgbe
 * start on 4-byte boundaries, resid on a 2-byte one.  If status (device int32,
 * may be NULL) is given it is set to RDL_OK first, then to RDL_ECORRUPT if the
 * header's magic, version or size do not match, a coefficient is outside the
 * bounds rdl_header_validate checks, or a decoded mantissa leaves [0, 255]. */
int rdl_decode_enh(rdl_ctx *ctx, const uint8_t *sdr, const rdl_header *coeffs, const void *resid,
                   int H, int W, uint8_t *out_rgbe, int32_t *status, void *stream);

/* Decoder of the base layer (Sec. II.B: the base layer's JPEG decoder returns
 * S; Sec. IV: quality Q): from the quantised coefficients dct (device, int16
 * [3][H8][W8], H8 and W8 rounded up to 8, block (bx, by)'s coefficient (v, u)
 * at row 8 by + v, column 8 bx + u, as rdl_stage_tmo_base writes them) and
 * the quality in the DEVICE header coeffs: D = Fq Q, the normative integer
 * IDCT, + 128, clamp, JFIF inverse colour transform, crop -> out_sdr (device,
 * H*W*3).  For coefficients the encoder wrote this returns exactly the
 * encoder's S (the decoded values of any other coefficients whose products
 * Fq Q exceed 16 bits are unspecified, but stay in [0, 255]).  dct on a
 * 2-byte boundary, coeffs and out_sdr on 4-byte ones.  status (device int32,
 * may be NULL): RDL_OK, or RDL_ECORRUPT when the header's magic, version or
 * size do not match or its quality is outside [1, 100]. */
int rdl_base_decode(rdl_ctx *ctx, const int16_t *dct, const rdl_header *coeffs, int H, int W, uint8_t *out_sdr,
                    int32_t *status, void *stream);

/* Batched decoder: n images of any sizes in one pass per stage.  imgs is a
 * HOST array.  For an image with dct (may be NULL) the base layer is first
 * decoded from its coefficients into sdr (as rdl_base_decode); otherwise sdr
 * holds S.  Then every image is decoded as rdl_decode_enh would decode it,
 * the learned ones with the context's model.  Alignments and status as for
 * those two calls.  The context's descriptor table is shared with the other
 * single-call entry points: calls on one context must not overlap. */
typedef struct rdl_dimage {
    const int16_t *dct;
    uint8_t *sdr;
    const rdl_header *hdr;
    const void *resid;
    int32_t H, W;
    uint8_t *out_rgbe;
    int32_t *status;
} rdl_dimage;
int rdl_decode_batch(rdl_ctx *ctx, const rdl_dimage *imgs, int n, void *stream);

/* Batched encoder: n images of any sizes and qualities in one pass per stage
 * (every stage kernel walks a flattened tile space over all images).  imgs is
 * a HOST array of n descriptors.  Each image is encoded exactly as
 * rdl_encode_enh would encode it.
 *
 * The first call for a given set of descriptors (buffers, sizes, qualities,
 * launch shapes, model) builds a plan for it: a device copy of the descriptor
 * table and scratch accumulators of its own (hipMalloc, synchronous).  Later
 * calls with the same descriptors reuse it and only enqueue the stage
 * kernels.  The context keeps the 8 most recent plans; building a ninth
 * waits for the oldest plan's last call to finish (an event recorded after
 * it on its stream) and hands that plan's buffers to the new plan where they
 * are large enough, so that a caller cycling through new image sets does not
 * allocate per call once its sizes have been seen.  Calls that share a plan
 * share its scratch, so they must not overlap (same stream, or ordered). */
typedef struct rdl_image {
    const uint8_t *rgbe;
    int32_t H, W, q;
    uint8_t *sdr;
    rdl_header *hdr;
    void *resid;
    int16_t *dct;  /* optional (may be NULL): also the base layer's quantised
                      coefficients, int16 [3][H8][W8] as rdl_stage_tmo_base
                      writes them (for rdl_jpeg_encode); 2-byte aligned */
} rdl_image;
int rdl_encode_batch(rdl_ctx *ctx, const rdl_image *imgs, int n, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the batched
 * encoder above with no allocation of any kind.  Its scratch (the descriptor
 * table and the per-image accumulators, about 136 KB per image) lives in a
 * static device array of the library sized for RDL_NOALLOC_MAX_IMAGES images
 * (2.2 MB), one copy per GPU, held until the process ends; the descriptors
 * are written there by a kernel (no host-to-device copy) and the
 * accumulators are cleared by a kernel at the start of every call.  Inputs,
 * outputs, layouts, alignments and the result are those of
 * rdl_encode_batch; launch shapes come from the context's tuning table; the
 * stages are always launched directly on `stream` (a caller may capture
 * them).  Every call on one GPU, from any context, shares that GPU's array:
 * calls that overlap on one GPU race (order them on one stream).  Errors:
 * RDL_ENOMEM if n > RDL_NOALLOC_MAX_IMAGES (rdl_strerror names the limit),
 * RDL_EUNSUPPORTED if the context's estimator is the learned one (it needs
 * per-pixel buffers), otherwise as rdl_encode_batch.  Nothing is enqueued on
 * an error. */
#define RDL_NOALLOC_MAX_IMAGES 16
int rdl_encode_batch_noalloc(rdl_ctx *ctx, const rdl_image *imgs, int n, void *stream);

/* How the encoder's stage kernels are enqueued.  RDL_LAUNCH_DIRECT (the
 * default): one launch per stage on the caller's stream.  RDL_LAUNCH_GRAPH:
 * the stages of a plan are captured in a HIP graph at its first use and the
 * graph is launched on every call.  With five stage kernels per encode the
 * direct launches are the faster choice (a graph launch costs more host time
 * than the five launches it replaces); the graph mode is for callers that
 * prefer one launch per encode.  Returns RDL_EINVAL for any other mode. */
enum { RDL_LAUNCH_DIRECT = 0, RDL_LAUNCH_GRAPH = 1 };
int rdl_set_launch_mode(rdl_ctx *ctx, int mode);

/* ---- Learned mantissa estimator (an extension beyond the paper, whose
 * estimator needs no learning, Sec. I) ----
 * A model is an int8 MLP over each pixel's 3x3 x 3-channel neighbourhood of S
 * (bytes S - 128) plus a 32-bin exponent one-hot (entering as a bias row),
 * two hidden layers of 32 (ReLU, int32 accumulate, requantised to unsigned
 * bytes) and a Q8 output per channel.  Blob: RDL_MODEL_BYTES bytes, little
 * endian:
 *   u32 magic 'RDLM', u32 version 2, u64 FNV-1a-64 hash of bytes 24..end,
 *   u32 reserved[2], i8 W1[32][32] (out, in), i32 B1[32][32] (bin, out),
 *   i32 m1[32], r1[32], i8 W2[32][32], i32 B2[32], m2[32], r2[32],
 *   i8 W3[16][32], i32 B3[16], m3[16], r3[16];
 * bin = clamp(E - 136 + k_img + 24, 0, 31); hidden a = clamp((h m + 2^(r-1))
 * >> r, 0, 255); output q8 = (o m3 + 2^(r3-1)) >> r3, estimate
 * clamp((q8 + 128) >> 8, 0, 255).  Accepted only with m in [1, 2^10),
 * r in [1, 28] (r3 in [1, 22]) and |B| <= 2^18.  Fastest: every hidden m = 1,
 * hidden r <= 22 and equal r in each neuron pair (2k, 2k + 1).
 *
 * rdl_set_model copies a HOST blob to the device (NULL clears it); RDL_ECORRUPT
 * for a bad magic, hash or value limit.  rdl_set_estimator(ctx, 1) makes the
 * encoders compute, per (channel, E) region, the code length of both
 * estimators' residuals under the image's SLR residual histogram of that
 * channel (Q16 integer log2; a learned residual value absent from that
 * histogram rules the learned estimate out) and use the learned estimate only
 * where it is strictly shorter (flag[c][E] = 1, estimator = 1, model_hash
 * set), so that, up to the rounding of the Q16 logarithms, the image's
 * zeroth-order entropy never exceeds plain SLR's (Gibbs' inequality); 0
 * restores plain SLR.  The decoder uses the context's model for headers with
 * estimator 1 (status RDL_ECORRUPT if the hash differs or no model is set). */
#define RDL_MODEL_BYTES 7512
int rdl_set_model(rdl_ctx *ctx, const void *blob, size_t nbytes);
int rdl_set_estimator(rdl_ctx *ctx, int mode);

/* ---- Ablations of the paper's method (Sec. III, the comparisons of Table I
 * and Fig. 4), as encoder settings of a context ----
 * rdl_set_estimator(ctx, 2): one least-squares line per channel for the whole
 * image (every exponent's sums pooled, Eq. 9-10 over all pixels; written to
 * every present exponent's a_q, b_q).  rdl_set_estimator(ctx, 3): no
 * estimator, M* = S (a_q = 2^22, b_q = 0 for every present exponent), the
 * plain residual of a layer without SLRME.  rdl_set_gf(ctx, 0): S* = S, no
 * Gaussian-filter restoration (Sec. III.B); 1 restores it.  The header's
 * estimator field records both (bit 4 = filter off), so rdl_decode_enh and
 * rdl_decode_batch decode every mode.  The learned estimator needs the filter:
 * encoding with mode 1 and the filter off gives RDL_EUNSUPPORTED.
 * RDL_EINVAL for another mode or switch value. */
int rdl_set_gf(rdl_ctx *ctx, int on);

/* ---- Training of the learned estimator (FP32, off the encoder's path) ----
 * Float model: x = (S - 128)/128 over the 3x3 x 3 neighbourhood, h1 =
 * W1 x + B1[bin], a1 = ReLU(h1), h2 = W2 a1 + B2, a2 = ReLU(h2), o = W3 a2 +
 * B3 predicting M/256; mean squared error; Adam (0.9, 0.999, 1e-8).  The
 * parameter vector holds rdl_train_nparam() floats: W1[32][27], B1[32][32]
 * (bin, out), W2[32][32], B2[32], W3[3][32], B3[3].
 * rdl_train_samples builds n sample records (rdl_train_sample_bytes() bytes
 * each: 27 feature bytes S - 128, bin, M_R, M_G, M_B, pad) for the pixel
 * indices idx (device int64, y*W + x) of an encoded image (rgbe, its decoded
 * SDRI sdr, and k_img from its header).  rdl_train_step runs one Adam step on
 * samples [base, base + batch) (clipped at n_samples), step >= 1; loss_out
 * (device float, may be NULL) receives the summed squared error of the batch.
 * Gradient sums are reduced in a fixed order: a step is deterministic. */
int rdl_train_sample_bytes(void);
int rdl_train_nparam(void);
int rdl_train_samples(rdl_ctx *ctx, const uint8_t *rgbe, const uint8_t *sdr, int H, int W, int k_img,
                      const int64_t *idx, int64_t n, void *out_samples, void *stream);
int rdl_train_step(rdl_ctx *ctx, float *params, float *adam_m, float *adam_v, const void *samples, int64_t base,
                   int64_t n_samples, int batch, float lr, int step, float *loss_out, void *stream);

/* Residual histograms for the zeroth-order-entropy metric: hist int64
 * [3][511], hist[c][r + 255] counts residual value r of channel c. */
int rdl_resid_hist(rdl_ctx *ctx, const void *resid, int H, int W, int64_t *hist, void *stream);

/* ---- The base layer as a JPEG file (Sec. II.B and Sec. IV: the base layer
 * is a JPEG file that any viewer shows) ----
 * rdl_jpeg_encode writes the quantised coefficients dct (device, int16
 * [3][H8][W8] as rdl_stage_tmo_base writes them, 2-byte aligned) at quality q
 * as a baseline sequential JPEG (ITU-T T.81) in a JFIF file -> out (device,
 * cap >= rdl_jpeg_bound(H, W) bytes); the file's length goes to *out_len
 * (DEVICE u64, 8-byte aligned).  Layout: SOI; APP0 "JFIF" 1.01, no thumbnail;
 * DQT with the two tables of quality q in zig-zag order; SOF0 (8 bits, H x W,
 * components 1, 2, 3 = Y, Cb, Cr, 1x1 sampling, tables 0, 1, 1); DHT with the
 * four Huffman tables (Y DC, Y AC, chroma DC, chroma AC), each optimised for
 * this image by Annex K.2 (Figure K.1 takes the larger symbol on equal
 * counts) with codes as Annex C assigns them; then one scan per component
 * (SOS: one component, tables 0/0 for Y and 1/1 for Cb and Cr, Ss 0, Se 63),
 * blocks in raster order, the DC predicted from the previous block of the
 * scan, each scan's last byte padded with 1-bits and every 0xFF data byte
 * followed by 0x00; EOI.  A decoder's IDCT gives S to within its own rounding
 * (rdl_base_decode gives it exactly).  1 <= H, W <= 65535 (RDL_EINVAL
 * otherwise).  The context keeps a workspace for the largest image seen
 * (about 800 bytes per 8x8 block; allocated synchronously when it grows), so
 * calls on one context must not overlap.  rdl_jpeg_bound is 0 for bad sizes. */
size_t rdl_jpeg_bound(int H, int W);
int rdl_jpeg_encode(rdl_ctx *ctx, const int16_t *dct, int H, int W, int q, uint8_t *out, size_t cap,
                    uint64_t *out_len, void *stream);

/* ---- Entropy code of the enhancement layer (an extension: the paper codes
 * the residual and exponent planes with JPEG 2000, Sec. IV) ----
 * A static rANS coder (J. Duda, "Asymmetric numeral systems", 2013, the range
 * variant): probability scale M = 2^15, states in [2^16, 2^32), 16-bit
 * renormalisation.  Encoding s: if x >= 2^17 f[s], emit x mod 2^16 and
 * x = x div 2^16; then x = (x div f[s]) M + (x mod f[s]) + c[s], with
 * c[s] = sum of f[t] for t < s.  Decoding reverses it.
 *
 * Planes p = 0, 1, 2: the residuals of channel R, G, B as symbols r + 255
 * (511 symbols); p = 3: the exponents (256 symbols); each N = H W symbols in
 * raster order.  With flags bit 0 set, plane 3 holds the exponents' left
 * differences instead, (E[y][x] - E[y][x-1]) mod 256 with E[y][0] itself:
 * the shared exponent is smooth, so these are mostly 0 (the residuals, close
 * to white, are never differenced).  Frequencies of a plane from its counts h (P symbols present):
 * f[s] = 1 + floor(h[s] (M - P) / N) where h[s] > 0, else 0; the smallest
 * symbol of the largest count takes the remainder M - sum f.
 *
 * Groups: K = 2^log2_k steps (4 <= log2_k <= 12); a plane is cut into
 * G = ceil(N / 64K) groups of 64K consecutive symbols (the last one shorter),
 * symbol i of a group going to lane i mod 64 at step i div 64.  The encoder
 * starts each lane at 2^16, runs the steps last to first and the lanes 63 to
 * 0 (skipping lanes without a symbol), then emits each lane's state, lanes 63
 * to 0, low half first.  A group's stored words are its emitted words in
 * reverse: lane states 0..63 (high, low), then per step from the first the
 * words of the lanes that renormalise, in lane order.  Each group costs
 * 64 x 32 bits of states, i.e. 32 / K bits per symbol.
 *
 * Stream, little-endian: u32 magic 0x454C4452 ("RDLE"), u32 version 1,
 * i32 H, i32 W, i32 log2_k, i32 prob_bits (15), u32 G, u32 flags (0 or 1), u64 total bytes,
 * u16 freq[4][512] (entries past a plane's alphabet 0) -- RDL_ENT_HEADER_BYTES
 * in all -- then u64 start[4][G] (first word of each group, counted from the
 * payload), then the payload of u16 words, groups in plane-major order.
 *
 * rdl_ent_encode: resid (device, rdl_resid_bytes(H, W), 2-byte aligned) ->
 * out (device, 8-byte aligned, cap >= rdl_ent_bound bytes); the stream length
 * goes to *out_len (DEVICE u64, 8-byte aligned).  A residual outside
 * [-255, 255] yields a stream with magic 0 and *out_len = 0.  The context
 * keeps a workspace sized for the largest layer seen (the plane histograms,
 * the coder tables, every group's words before they are put in order and the
 * exponents' differences, about 9 bytes per pixel; allocated synchronously
 * when it grows), so calls on one context must not overlap.  rdl_ent_bound is
 * 0 for bad sizes.  rdl_set_ent_predict(ctx, 1) (the default) makes the
 * encoder set flags bit 0; 0 codes the exponents as they are; RDL_EINVAL for
 * another value.
 *
 * rdl_ent_decode: code (device, 8-byte aligned, len bytes) and a HOST copy of
 * its first RDL_ENT_HEADER_BYTES bytes, which is validated first (magic,
 * version, sizes, log2_k, G, frequency sums, total <= len: RDL_ECORRUPT) ->
 * out_resid (device, rdl_resid_bytes(H, W), 2-byte aligned); a stream with
 * flags bit 0 uses the context's workspace (about one byte per pixel: the
 * differences, summed back along each row into out_resid), so it must not
 * overlap other calls on the context either.  If status
 * (device int32, may be NULL) is given it receives RDL_OK, or RDL_ECORRUPT
 * when the device copy's tables or a group's offsets or words do not decode
 * exactly (every read stays inside the stream). */
#define RDL_ENT_HEADER_BYTES 4136
size_t rdl_ent_bound(int H, int W, int log2_k);
int rdl_ent_encode(rdl_ctx *ctx, const void *resid, int H, int W, int log2_k, void *out, size_t cap,
                   uint64_t *out_len, void *stream);
int rdl_ent_decode(rdl_ctx *ctx, const void *code, size_t len, const void *header, int H, int W,
                   void *out_resid, int32_t *status, void *stream);
int rdl_set_ent_predict(rdl_ctx *ctx, int on);

/* Residual contexts (stream flags bit 1; an extension like the coder
 * itself).  The residual of channel p at pixel i is coded with the table of
 * its context k = sdr[3 i + p] >> 5 (k = 0..7), sdr being the decoded base
 * layer (the encoder's out_sdr, H x W x 3 bytes, channel-interleaved), which
 * a decoder holds before it reads this layer: the residuals' spread follows
 * where the tone curve put the pixel, so 8 tables per channel fit it better
 * than one.  Symbols stay in the same groups and lanes; only the table of
 * each symbol changes.  The stream is the format above with T = 25 tables in
 * place of 4: u16 freq[25][512] at byte 40 (channel p, context k at table
 * 8 p + k; the exponents' at 24; a table whose context no pixel has is all
 * zero, the others sum to M, with N = the symbols coded with that table in
 * the frequency rule), so the group table starts at RDL_ENT_CTX_HEADER_BYTES.
 * The encoder's exponent plane follows rdl_set_ent_predict as above.
 * rdl_ent_encode_ctx / rdl_ent_decode_ctx take the same arguments as
 * rdl_ent_encode / rdl_ent_decode plus sdr (device, 3 H W bytes; RDL_EINVAL
 * if NULL), and the decoder's header copy holds RDL_ENT_CTX_HEADER_BYTES
 * bytes; each decoder rejects the other's streams (RDL_ECORRUPT), and a
 * symbol whose context table is empty (a decode against another sdr) sets
 * *status = RDL_ECORRUPT.  The larger header (21.5 KB more) pays for itself
 * above about 0.3 Mpx. */
#define RDL_ENT_CTX_HEADER_BYTES 25640
size_t rdl_ent_bound_ctx(int H, int W, int log2_k);
int rdl_ent_encode_ctx(rdl_ctx *ctx, const void *resid, const uint8_t *sdr, int H, int W, int log2_k, void *out,
                       size_t cap, uint64_t *out_len, void *stream);
int rdl_ent_decode_ctx(rdl_ctx *ctx, const void *code, size_t len, const void *header, const uint8_t *sdr, int H,
                       int W, void *out_resid, int32_t *status, void *stream);

/* ---- Stage entry points (each is one step of rdl_encode_enh, for checks) ---- */

/* Key statistic (Sec. IV, Reinhard's operator needs the log-average
 * luminance): out2 int64[2] = {Lambda, N'}: the Q16 sum of log2 luminance over
 * pixels with E != 0, and their number. */
int rdl_stage_keystat(rdl_ctx *ctx, const uint8_t *rgbe, int H, int W, int64_t *out2, void *stream);

/* Tone mapping + base layer from a key statistic (int64[2] from
 * rdl_stage_keystat).  out_sdr0 (may be NULL) receives the tone-mapped SDRI
 * before JPEG (H*W*3); out_sdr receives S; out_dct (may be NULL) receives the
 * quantised coefficients int16 [3][H8][W8] (H8, W8 rounded up to 8). */
int rdl_stage_tmo_base(rdl_ctx *ctx, const uint8_t *rgbe, int H, int W, int q, const int64_t *keystat,
                       uint8_t *out_sdr0, uint8_t *out_sdr, int16_t *out_dct, void *stream);

/* Regression fit (Sec. III.B, Eq. 9-10): sums int64 [256][13] per exponent:
 * {n, then per channel c at 1+4c: sum s, sum m, sum s^2, sum s m} with
 * s = GF(sdr)_c and m = M_c; then the header's coefficients.  keystat may
 * be NULL (the header's key fields are then zero). */
int rdl_stage_fit(rdl_ctx *ctx, const uint8_t *rgbe, const uint8_t *sdr, int H, int W, int q,
                  const int64_t *keystat, int64_t *out_sums, rdl_header *out_coeffs, void *stream);

/* Residuals from given coefficients (Eq. 8). */
int rdl_stage_resid(rdl_ctx *ctx, const uint8_t *rgbe, const uint8_t *sdr, const rdl_header *coeffs,
                    int H, int W, void *out_resid, void *stream);

/* ---- Instrumentation ---- */

/* Stage kernels of rdl_encode_enh in launch order; the index into ms[] of
 * rdl_profile_encode. */
enum {
    RDL_STAGE_KEYSTAT = 0,  /* key statistic                           */
    RDL_STAGE_TMO_BASE = 1, /* tone map + JPEG-style base layer -> S   */
    RDL_STAGE_FIT = 2,      /* GF + per-(channel, E) regression sums   */
    RDL_STAGE_SOLVE = 3,    /* fixed-point coefficients -> header      */
    RDL_STAGE_RESID = 4,    /* GF + estimate + residual planes (learned */
                            /* path: the learned regions' residuals    */
    RDL_NSTAGES = 5
};

/* Stages of the encoder with the learned estimator, in launch order: the
 * five above, then (learned path only) the learned inference with the
 * records by exponent, their histograms and the region selection, after the
 * solve and before the residuals.  Index into ms[] of rdl_stage_times. */
enum {
    RDL_STAGE_LEARN = 5,    /* learned estimate + residual records     */
    RDL_STAGE_LHIST = 6,    /* residual histograms per (est, ch, E)    */
    RDL_STAGE_SELECT = 7,   /* per-region estimator flags              */
    RDL_NSTAGES_ALL = 8
};

/* Stage timing of ordinary encodes (instrumentation).  With on = 1, every
 * later rdl_encode_enh / rdl_encode_batch call that launches its stages
 * directly records a HIP event on its stream before the first stage kernel
 * and after each one (library-owned events, reused; the calls of at most
 * RDL_TIMING_MAX_CALLS encodes are kept, later ones are not recorded).
 * Calls in graph launch mode record nothing.  rdl_stage_times waits for the
 * recorded events, writes to the HOST array ms[RDL_NSTAGES_ALL] the mean
 * duration in milliseconds of each stage over the recorded calls (the time
 * between the events around its kernel on the stream; stages that did not
 * run: 0), writes the number of recorded calls to *calls (host, may be
 * NULL) and starts a new recording.  on = 0 stops recording and drops what
 * was recorded. */
#define RDL_TIMING_MAX_CALLS 64
int rdl_set_stage_timing(rdl_ctx *ctx, int on);
int rdl_stage_times(rdl_ctx *ctx, float *ms, int *calls);

/* Runs the same kernels as rdl_encode_enh (same arguments and outputs) for
 * timing: each stage kernel is launched `reps` times back to back between a
 * pair of HIP events on `stream`, and the mean duration of one launch, in
 * milliseconds, goes to the HOST array ms[RDL_NSTAGES].  Repeated stages see
 * scaled sums or cleaned scratch, which leaves their cost unchanged; one
 * ordinary encode at the end leaves correct outputs.  Synchronises `stream`;
 * not capturable. */
int rdl_profile_encode(rdl_ctx *ctx, const uint8_t *rgbe, int H, int W, int q, uint8_t *out_sdr,
                       rdl_header *out_coeffs, void *out_resid, int reps, float *ms, void *stream);

/* ---- Launch-shape tuning ----
 *
 * The GF-based stages give each wave a strip of 256 pixels and some rows,
 * waves stacked per workgroup.  Tall strips leave SIMDs idle on small images;
 * short ones re-read more halo rows of S.  In the fit every workgroup ends by
 * adding its per-(channel, E) totals to the image's global sums, so fewer,
 * larger workgroups (more waves each) cost fewer global atomics.  The fit's
 * LDS bins can be kept in 1, 2 or 4 copies that neighbouring lanes alternate
 * between.  The context keeps one value per tuning parameter and size class
 * floor(log2(H * W)) (0..31), initially: fit 16 waves x 8 rows from 4 Mpx
 * up, 8 x 16 from 1 Mpx, else 4 x 16, with 2 bin copies; residual/decode 8
 * rows (4 waves).  A batch uses each image's own class for
 * the rows; the fit's waves and bin copies are one per launch, its largest
 * image's, and a fit workgroup spans at most 128 rows (waves x rows; larger
 * row counts are clamped).  Encoder plans are keyed on the shapes, so a
 * change takes effect at the next call. */
enum {
    RDL_TUNE_FIT_ROWS = 0,   /* rows per wave of the fit (k_fit_sums)         */
    RDL_TUNE_RESID_ROWS = 1, /* rows per wave of the residual/decode walks    */
    RDL_TUNE_FIT_BINS = 2,   /* privatised copies of the fit's LDS bins       */
    RDL_TUNE_FIT_WAVES = 3,  /* waves per fit workgroup                       */
    RDL_NTUNE = 4
};

/* Encodes the caller's image once (same arguments and outputs as
 * rdl_encode_enh, plain estimator), then, for each parameter, launches its
 * kernel `reps` times back to back for each value (rows: 2, 4, 8, 16, 32;
 * bin copies: 1, 2, 4; waves: 4, 8, 16), one parameter after the other, timed
 * with HIP events on `stream`, and keeps the fastest for the image's size
 * class; the HOST array best[RDL_NTUNE] (may be NULL) receives the choices.
 * Outputs hold a correct encode on return.  Synchronises `stream`; not
 * capturable.  RDL_EINVAL for the argument errors of rdl_encode_enh or
 * reps < 1. */
int rdl_autotune(rdl_ctx *ctx, const uint8_t *rgbe, int H, int W, int q, uint8_t *out_sdr,
                 rdl_header *out_coeffs, void *out_resid, int reps, int *best, void *stream);

/* Read / write one entry (for saving and restoring a tuned table).  Rows are
 * powers of two in [2, 32], bin copies 1, 2 or 4, waves 4, 8 or 16; anything
 * else, or a parameter or class out of range, gives RDL_EINVAL. */
int rdl_get_tuning(rdl_ctx *ctx, int param, int size_class, int *value);
int rdl_set_tuning(rdl_ctx *ctx, int param, int size_class, int value);

/* Self-check of the reciprocal the tone-mapping kernel uses (the hardware
 * estimate refined by one fused Newton step, in place of IEEE division, whose
 * result it must equal for every denominator the operator can produce, the
 * floats in [1, 2^47)).  Compares the two for every float whose bit pattern
 * lies in [lo_bits, hi_bits) and writes the number of differences to the HOST
 * *mismatches.  Allocates a few bytes of device memory; synchronises
 * `stream`.  RDL_EINVAL if hi_bits < lo_bits. */
int rdl_check_recip(rdl_ctx *ctx, uint32_t lo_bits, uint32_t hi_bits, uint64_t *mismatches, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* RDL_H */
