/*
 * rdl_jpeg_oracle.c -- CPU oracle for the base layer's JPEG bitstream.
 *
 * TEST INFRASTRUCTURE ONLY, under the same rules as rdl_oracle.c.
 *
 * The paper's base layer is a JPEG file (Sec. II.B, Sec. IV: MATLAB's JPEG
 * writer at quality Q) that any viewer shows.  This writes the encoder's
 * quantised coefficients as a baseline sequential JPEG (ITU-T T.81) in a JFIF
 * file, step by step in the standard's terms:
 *   - SOI, APP0 (JFIF 1.01, no thumbnail), DQT (the two quantisation tables of
 *     quality q, in zig-zag order), SOF0 (8-bit, H x W, components 1, 2, 3 =
 *     Y, Cb, Cr, all 1x1 sampling, tables 0, 1, 1), DHT (four tables), then
 *     one non-interleaved scan per component (SOS: Ns = 1, DC/AC tables 0/0
 *     for Y and 1/1 for Cb and Cr, Ss = 0, Se = 63, Ah = Al = 0), EOI;
 *   - blocks of a scan in raster order, ceil(W/8) x ceil(H/8) of them; the DC
 *     difference to the previous block of the scan (0 before the first) and
 *     the AC run/size symbols in zig-zag order with ZRL and EOB (Annex F.1.2);
 *     magnitude bits: the value, or for a negative value the value minus one,
 *     in SSSS bits (F.1.2.1);
 *   - Huffman tables optimised for the image: the symbol counts of each table
 *     (DC and AC of Y; DC and AC of Cb and Cr together) go through Annex K.2
 *     (Figures K.1 to K.4: code sizes with a reserved code point, sizes
 *     limited to 16 bits, symbols ordered by size), codes assigned as in
 *     Annex C (Figures C.1 to C.3);
 *   - bytes of the entropy-coded data are written MSB first, each 0xFF byte
 *     followed by a stuffed 0x00, and a scan's last byte padded with 1-bits.
 * Readings where the standard leaves a choice: when Figure K.1 meets two
 * symbols of equal least count it takes the one with the larger value; where
 * Figure K.1 gives code sizes above 32 (a chain of counts each about twice
 * the one before, totals above 2^32), the size histogram and Figure K.3's
 * loop extend to the longest size instead of stopping at 32.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void oracle_quant_table(int q, int chroma, int32_t *out64);

/* Zig-zag order: the k-th coefficient of the scan is natural index zz[k],
 * walking the anti-diagonals s = u + v from the top left, downwards on odd
 * diagonals and upwards on even ones (Figure A.6). */
static void zigzag(int zz[64])
{
    int k = 0;
    for (int s = 0; s <= 14; s++) {
        int lo = s > 7 ? s - 7 : 0, hi = s < 7 ? s : 7;
        if (s & 1)
            for (int r = lo; r <= hi; r++) zz[k++] = r * 8 + (s - r);
        else
            for (int r = hi; r >= lo; r--) zz[k++] = r * 8 + (s - r);
    }
}

/* SSSS: the number of bits of |v| (0 for v = 0). */
static int ssss(int v)
{
    int a = v < 0 ? -v : v, n = 0;
    while (a) {
        n++;
        a >>= 1;
    }
    return n;
}

/* Annex K.2: code lengths from symbol counts freq[0..255] (a copy is made),
 * with a reserved symbol 256 of count 1 so that no code is all ones; then
 * sizes limited to 16 bits and the symbols listed by size.  bits[1..16]
 * counts the codes of each length, huffval[] the symbols in code order;
 * returns their number. */
int oracle_jpeg_huff_table(const int64_t *freq_in, uint8_t bits[17], uint8_t huffval[256])
{
    int64_t freq[257];
    int codesize[257], others[257], nb[258];
    for (int i = 0; i < 256; i++) freq[i] = freq_in[i];
    freq[256] = 1;
    for (int i = 0; i < 257; i++) {
        codesize[i] = 0;
        others[i] = -1;
    }
    for (;;) {
        int v1 = -1, v2 = -1;
        for (int i = 0; i < 257; i++)  /* least count, ties to the larger value */
            if (freq[i] > 0 && (v1 < 0 || freq[i] <= freq[v1])) v1 = i;
        for (int i = 0; i < 257; i++)
            if (i != v1 && freq[i] > 0 && (v2 < 0 || freq[i] <= freq[v2])) v2 = i;
        if (v2 < 0) break;
        freq[v1] += freq[v2];
        freq[v2] = 0;
        codesize[v1]++;
        while (others[v1] >= 0) {
            v1 = others[v1];
            codesize[v1]++;
        }
        others[v1] = v2;
        codesize[v2]++;
        while (others[v2] >= 0) {
            v2 = others[v2];
            codesize[v2]++;
        }
    }
    /* Figure K.2's size histogram runs to the longest size K.1 gave (at most
     * 256): cut at 32, as the figure's arrays are, the sizes above would no
     * longer pair up as siblings and Figure K.3 would not yield a code */
    memset(nb, 0, sizeof nb);
    int maxlen = 0;
    for (int i = 0; i < 257; i++) {
        if (codesize[i]) nb[codesize[i]]++;
        if (codesize[i] > maxlen) maxlen = codesize[i];
    }
    for (int i = maxlen; i > 16; i--)  /* Figure K.3 */
        while (nb[i] > 0) {
            int j = i - 2;
            while (nb[j] == 0) j--;
            nb[i] -= 2;
            nb[i - 1]++;
            nb[j + 1] += 2;
            nb[j]--;
        }
    int i = 16;
    while (i > 1 && nb[i] == 0) i--;
    if (nb[i] > 0) nb[i]--;  /* drop the reserved code point */
    memset(bits, 0, 17);
    for (int k = 1; k <= 16; k++) bits[k] = (uint8_t)nb[k];
    int n = 0;
    for (int len = 1; len <= maxlen; len++)  /* Figure K.4 */
        for (int s = 0; s < 256; s++)
            if (codesize[s] == len) huffval[n++] = (uint8_t)s;
    int total = 0;
    for (int k = 1; k <= 16; k++) total += bits[k];
    return total < n ? total : n;
}

/* Annex C: code of each symbol from bits/huffval (canonical codes). */
static void huff_codes(const uint8_t bits[17], const uint8_t *huffval, int n, uint16_t code[256], uint8_t size[256])
{
    memset(size, 0, 256);
    memset(code, 0, 512);
    uint32_t c = 0;
    int k = 0;
    for (int len = 1; len <= 16; len++) {
        for (int j = 0; j < bits[len]; j++, k++) {
            if (k >= n) return;
            code[huffval[k]] = (uint16_t)c;
            size[huffval[k]] = (uint8_t)len;
            c++;
        }
        c <<= 1;
    }
}

/* Bit writer with byte stuffing. */
typedef struct {
    uint8_t *out;
    int64_t cap, pos;
    uint32_t acc;
    int nacc;
    int overflow;
} bitw;

static void put_byte(bitw *w, uint8_t b)
{
    if (w->pos < w->cap) w->out[w->pos] = b; else w->overflow = 1;
    w->pos++;
}

static void put_bits(bitw *w, uint32_t v, int n)
{
    for (int i = n - 1; i >= 0; i--) {
        w->acc = (w->acc << 1) | ((v >> i) & 1u);
        if (++w->nacc == 8) {
            put_byte(w, (uint8_t)w->acc);
            if ((w->acc & 0xFF) == 0xFF) put_byte(w, 0);
            w->acc = 0;
            w->nacc = 0;
        }
    }
}

static void flush_bits(bitw *w)
{
    while (w->nacc) put_bits(w, 1, 1);
}

static void put16(bitw *w, int v)
{
    put_byte(w, (uint8_t)(v >> 8));
    put_byte(w, (uint8_t)v);
}

/* The symbols of one block: calls sym(table, symbol, value bits, n) in order. */
typedef void (*sym_fn)(void *ctx, int ac, int symbol, uint32_t extra, int n);

static void block_symbols(const int16_t *dct, int64_t W8, int by, int bx, int *pred, const int zz[64], sym_fn f,
                          void *ctx)
{
    int v[64];
    for (int k = 0; k < 64; k++) {
        int n = zz[k];
        v[k] = dct[(int64_t)(by * 8 + n / 8) * W8 + bx * 8 + n % 8];
    }
    int diff = v[0] - *pred;
    *pred = v[0];
    int s = ssss(diff);
    f(ctx, 0, s, (uint32_t)(diff < 0 ? diff - 1 : diff) & ((1u << s) - 1u), s);
    int run = 0;
    for (int k = 1; k < 64; k++) {
        if (v[k] == 0) {
            run++;
            continue;
        }
        while (run > 15) {
            f(ctx, 1, 0xF0, 0, 0);
            run -= 16;
        }
        s = ssss(v[k]);
        /* a size above 15 is outside baseline JPEG (never made by the
           encoder); clamped so that the symbol stays a byte */
        f(ctx, 1, run * 16 + (s > 15 ? 15 : s), (uint32_t)(v[k] < 0 ? v[k] - 1 : v[k]) & ((1u << s) - 1u), s);
        run = 0;
    }
    if (run > 0) f(ctx, 1, 0x00, 0, 0);
}

typedef struct {
    int64_t freq[2][256];  /* DC, AC */
} count_ctx;

static void count_sym(void *ctx, int ac, int symbol, uint32_t extra, int n)
{
    (void)extra;
    (void)n;
    ((count_ctx *)ctx)->freq[ac][symbol]++;
}

typedef struct {
    bitw *w;
    uint16_t code[2][256];
    uint8_t size[2][256];
} emit_ctx;

static void emit_sym(void *ctx, int ac, int symbol, uint32_t extra, int n)
{
    emit_ctx *e = (emit_ctx *)ctx;
    put_bits(e->w, e->code[ac][symbol], e->size[ac][symbol]);
    if (n) put_bits(e->w, extra, n);
}

/* The JFIF file of quantised coefficients dctq int16 [3][H8][W8] (block
 * (bx, by)'s (v, u) at row 8 by + v, column 8 bx + u) at quality q.  Returns
 * its length, -1 for bad arguments, -2 when cap is too small. */
int64_t oracle_jpeg_write(const int16_t *dctq, int H, int W, int q, uint8_t *out, int64_t cap)
{
    if (!dctq || !out || H < 1 || W < 1 || H > 65535 || W > 65535 || q < 1 || q > 100) return -1;
    int zz[64];
    zigzag(zz);
    const int nbx = (W + 7) / 8, nby = (H + 7) / 8;
    const int64_t H8 = (int64_t)nby * 8, W8 = (int64_t)nbx * 8;
    /* symbol counts: table 0 = Y, table 1 = Cb and Cr */
    count_ctx cnt[2];
    memset(cnt, 0, sizeof cnt);
    for (int c = 0; c < 3; c++) {
        int pred = 0;
        for (int by = 0; by < nby; by++)
            for (int bx = 0; bx < nbx; bx++)
                block_symbols(dctq + c * H8 * W8, W8, by, bx, &pred, zz, count_sym, &cnt[c ? 1 : 0]);
    }
    uint8_t bits[2][2][17], hval[2][2][256];
    int nval[2][2];
    for (int t = 0; t < 2; t++)
        for (int ac = 0; ac < 2; ac++) nval[t][ac] = oracle_jpeg_huff_table(cnt[t].freq[ac], bits[t][ac], hval[t][ac]);
    bitw w = {out, cap, 0, 0, 0, 0};
    put16(&w, 0xFFD8);
    put16(&w, 0xFFE0);
    put16(&w, 16);
    const uint8_t jfif[14] = {'J', 'F', 'I', 'F', 0, 1, 1, 0, 0, 1, 0, 1, 0, 0};
    for (int k = 0; k < 14; k++) put_byte(&w, jfif[k]);
    put16(&w, 0xFFDB);
    put16(&w, 2 + 2 * 65);
    for (int t = 0; t < 2; t++) {
        int32_t qt[64];
        oracle_quant_table(q, t, qt);
        put_byte(&w, (uint8_t)t);
        for (int k = 0; k < 64; k++) put_byte(&w, (uint8_t)qt[zz[k]]);
    }
    put16(&w, 0xFFC0);
    put16(&w, 17);
    put_byte(&w, 8);
    put16(&w, H);
    put16(&w, W);
    put_byte(&w, 3);
    for (int c = 0; c < 3; c++) {
        put_byte(&w, (uint8_t)(c + 1));
        put_byte(&w, 0x11);
        put_byte(&w, (uint8_t)(c ? 1 : 0));
    }
    int dht_len = 2;
    for (int t = 0; t < 2; t++)
        for (int ac = 0; ac < 2; ac++) dht_len += 17 + nval[t][ac];
    put16(&w, 0xFFC4);
    put16(&w, dht_len);
    for (int t = 0; t < 2; t++)
        for (int ac = 0; ac < 2; ac++) {
            put_byte(&w, (uint8_t)(ac * 16 + t));
            for (int k = 1; k <= 16; k++) put_byte(&w, bits[t][ac][k]);
            for (int k = 0; k < nval[t][ac]; k++) put_byte(&w, hval[t][ac][k]);
        }
    for (int c = 0; c < 3; c++) {
        const int t = c ? 1 : 0;
        put16(&w, 0xFFDA);
        put16(&w, 8);
        put_byte(&w, 1);
        put_byte(&w, (uint8_t)(c + 1));
        put_byte(&w, (uint8_t)(t * 16 + t));
        put_byte(&w, 0);
        put_byte(&w, 63);
        put_byte(&w, 0);
        emit_ctx e;
        e.w = &w;
        for (int ac = 0; ac < 2; ac++) huff_codes(bits[t][ac], hval[t][ac], nval[t][ac], e.code[ac], e.size[ac]);
        int pred = 0;
        for (int by = 0; by < nby; by++)
            for (int bx = 0; bx < nbx; bx++) block_symbols(dctq + c * H8 * W8, W8, by, bx, &pred, zz, emit_sym, &e);
        flush_bits(&w);
    }
    put16(&w, 0xFFD9);
    return w.overflow ? -2 : w.pos;
}
