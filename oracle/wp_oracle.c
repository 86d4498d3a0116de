/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, scalar, deliberately slow implementation of what the decoder
 * computes, written from Lemire & Boytsov, "Decoding billions of integers
 * per second through vectorization" (arXiv:1209.2137). Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it. It shares
 * no source, header, table or helper with the GPU library; both follow the
 * stream layout written out in the design document (re-stated below).
 *
 * Every function cites the passage of the paper it follows. Arithmetic on
 * array values is uint32 modulo 2^32 throughout.
 *
 * Stream layout (little-endian 32-bit words):
 *   header  (8 words) magic, n_lo, n_hi, stride, n_units, tail_bytes,
 *                     tail_off, total_words
 *   directory         ndir = n_units (+1 for the tail when present)
 *                     entries: first the ndir word offsets of the units
 *                     (and tail), then the ndir groups of S bases,
 *                     S = stride, base_s = x[start - S + s] (0 before the
 *                     array start); zero-padded to a multiple of 4 words
 *   units             binary packing: 4-word width descriptor (byte j = b_j)
 *                     then 16 blocks of 128 values, block j in 4*b_j words.
 *                     BP32: 16 meta-blocks, each a descriptor word (byte j =
 *                     width of its block j) then its four blocks of 32
 *                     values, block j in b_j words; zero-padded to a
 *                     multiple of 4 words (see oracle_bp32_encode)
 *                     patched (FastPFOR) page of up to 512 blocks: see
 *                     oracle_fp_encode; exception arrays padded to 128
 *                     values (SIMD-FastPFOR) or to 32 (FastPFOR,
 *                     oracle_fp32_encode); SimplePFOR pages hold one
 *                     Simple-8b array instead (oracle_sp_encode);
 *                     codec 6 keeps the page in the paper's own layout
 *                     (oracle_fpi_encode)
 *   tail              Variable Byte of the last n mod 128 deltas,
 *                     zero-padded to a word
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OB 128u                /* block length: 128 integers (Section 6.2) */
#define OBP_BLOCKS 16u         /* SIMD-BP128 meta-block: 16 blocks (Section 6.2) */
#define OFP_BLOCKS 512u        /* patched page: 2^16 integers (Section 5) */
#define OMAGIC_BP 0x31425057u  /* "WPB1" */
#define OMAGIC_FP 0x31465057u  /* "WPF1" */
#define OMAGIC_BP32 0x32335057u /* "WP32" */
#define OMAGIC_FP32 0x33465057u /* "WPF3" */
#define OMAGIC_BPV 0x31565057u  /* "WPV1" */
#define OMAGIC_SP 0x31535057u   /* "WPS1" */
#define OMAGIC_FPI 0x31495057u  /* "WPI1" */
#define OB32 32u               /* BP32 block: 32 integers (Section 6.2) */
#define OSEG_BLOCKS 64u        /* patched-page segment: 64 blocks (8192 integers) */

enum { O_OK = 0, O_ERR_ARG = -1, O_ERR_CAP = -2, O_ERR_CORRUPT = -3 };

/* ---- Section 2 (binary notation): a positive integer x needs
 * ceil(log2(x+1)) binary digits; zero needs none. Counted digit by digit. */
uint32_t oracle_bits(uint32_t x)
{
    uint32_t b = 0;
    while (x != 0) {
        b++;
        x >>= 1;
    }
    return b;
}

/* ---- Section 4, Figs. 4-5: fields of b bits laid end to end, field i
 * occupying bits [i*b, i*b+b) of the word sequence, word w holding bits
 * [32w, 32w+32), least significant bit first; a field may straddle two
 * words. Written bit by bit. Only the low b bits of each value are kept
 * (the 2^b-1 mask of Section 4). `words` must hold ceil(count*b/32) words;
 * they are cleared first. */
void oracle_pack(const uint32_t *vals, uint64_t count, uint32_t b, uint32_t *words)
{
    uint64_t nwords = (count * b + 31) / 32;
    memset(words, 0, nwords * sizeof(uint32_t));
    for (uint64_t i = 0; i < count; i++) {
        for (uint32_t j = 0; j < b; j++) {
            if ((vals[i] >> j) & 1u) {
                uint64_t bit = i * b + j;
                words[bit / 32] |= 1u << (bit % 32);
            }
        }
    }
}

void oracle_unpack(const uint32_t *words, uint64_t count, uint32_t b, uint32_t *vals)
{
    for (uint64_t i = 0; i < count; i++) {
        uint32_t v = 0;
        for (uint32_t j = 0; j < b; j++) {
            uint64_t bit = i * b + j;
            if ((words[bit / 32] >> (bit % 32)) & 1u)
                v |= 1u << j;
        }
        vals[i] = v;
    }
}

/* ---- Section 4, vectorized layout (the 4 x 32-bit figure for b = 5):
 * values go round-robin to four 32-bit lanes -- value i to lane i mod 4,
 * as that lane's field i div 4 -- each lane lays its fields end to end,
 * least significant bit first, and the lanes' words interleave: bit q of
 * lane l is bit q mod 32 of word 4 (q div 32) + l. count must be a
 * multiple of 4 (128 in a block). Written bit by bit; `words` (4 words per
 * 32 bits of a lane) are cleared first. */
void oracle_pack_vertical(const uint32_t *vals, uint64_t count, uint32_t b, uint32_t *words)
{
    uint64_t nwords = 4 * ((count / 4 * b + 31) / 32);
    memset(words, 0, nwords * sizeof(uint32_t));
    for (uint64_t i = 0; i < count; i++) {
        uint64_t lane = i % 4, field = i / 4;
        for (uint32_t j = 0; j < b; j++) {
            if ((vals[i] >> j) & 1u) {
                uint64_t q = field * b + j; /* bit q of the lane */
                words[4 * (q / 32) + lane] |= 1u << (q % 32);
            }
        }
    }
}

void oracle_unpack_vertical(const uint32_t *words, uint64_t count, uint32_t b, uint32_t *vals)
{
    for (uint64_t i = 0; i < count; i++) {
        uint64_t lane = i % 4, field = i / 4;
        uint32_t v = 0;
        for (uint32_t j = 0; j < b; j++) {
            uint64_t q = field * b + j;
            if ((words[4 * (q / 32) + lane] >> (q % 32)) & 1u)
                v |= 1u << j;
        }
        vals[i] = v;
    }
}

/* ---- Section 3: differential coding. stride 1: d_i = x_i - x_{i-1};
 * stride 4 (the vectorised form): d_i = x_i - x_{i-4}, the first four
 * values kept; stride 0: no differencing. Values before the array start
 * count as `init` (0 for the codecs). Computed in place from the largest
 * index down, as the section's worked example (1,4,13 -> 1,3,9) does. */
int oracle_delta_encode_inplace(uint32_t *data, uint64_t n, uint32_t init, int stride)
{
    if (stride != 0 && stride != 1 && stride != 4)
        return O_ERR_ARG;
    if (stride == 0)
        return O_OK;
    for (uint64_t i = n; i-- > 0;) {
        uint32_t prev = (i >= (uint64_t)stride) ? data[i - stride] : init;
        data[i] = data[i] - prev;
    }
    return O_OK;
}

/* Section 3: decoding is the prefix sum x_i = d_i + x_{i-S}, computed in
 * place in increasing index order (worked example 1,3,9 -> 1,4,13). */
int oracle_delta_decode_inplace(uint32_t *data, uint64_t n, uint32_t init, int stride)
{
    if (stride != 0 && stride != 1 && stride != 4)
        return O_ERR_ARG;
    if (stride == 0)
        return O_OK;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t prev = (i >= (uint64_t)stride) ? data[i - stride] : init;
        data[i] = data[i] + prev;
    }
    return O_OK;
}

/* ---- Section 2 (Variable Byte): seven data bits per byte, low-order group
 * first; the eighth bit is 1 only on the last byte of an integer (the
 * section's example: 200 becomes the bytes 0x48, 0x81). Returns bytes written. */
uint32_t oracle_vbyte_encode(const uint32_t *vals, uint32_t count, uint8_t *out)
{
    uint32_t p = 0;
    for (uint32_t i = 0; i < count; i++) {
        uint32_t v = vals[i];
        while (v >= 128u) {
            out[p++] = (uint8_t)(v & 127u);
            v >>= 7;
        }
        out[p++] = (uint8_t)(v | 128u);
    }
    return p;
}

/* Decodes `count` integers from at most `nbytes` bytes. Returns the number
 * of bytes consumed, or -1 if the bytes run out or an integer is longer
 * than five bytes or overflows 32 bits. */
int64_t oracle_vbyte_decode(const uint8_t *in, uint64_t nbytes, uint32_t count, uint32_t *vals)
{
    uint64_t p = 0;
    for (uint32_t i = 0; i < count; i++) {
        uint64_t v = 0;
        uint32_t shift = 0;
        for (;;) {
            if (p >= nbytes || shift > 28)
                return -1;
            uint8_t byte = in[p++];
            v |= (uint64_t)(byte & 127u) << shift;
            shift += 7;
            if (byte & 128u)
                break;
        }
        if (v > 0xFFFFFFFFull)
            return -1;
        vals[i] = (uint32_t)v;
    }
    return (int64_t)p;
}

/* ---- Section 5: width choice of the patched schemes for one block of
 * `count` values. A histogram of bit widths 0..32; maxb the largest width;
 * for each candidate b in [0, maxb] the exceptions are the c(b) values
 * wider than b, each costed at 8 bits of position plus maxb-b high bits;
 * the block costs count*b + c(b)*(8 + maxb - b) bits. The smallest cost
 * wins; equal costs keep the wider b (fewer exceptions). Writes b, maxb and
 * the exception count c. */
void oracle_fp_choose(const uint32_t *vals, uint32_t count, uint32_t *b_out,
                      uint32_t *maxb_out, uint32_t *c_out)
{
    uint64_t hist[33];
    memset(hist, 0, sizeof hist);
    for (uint32_t i = 0; i < count; i++)
        hist[oracle_bits(vals[i])]++;
    uint32_t maxb = 0;
    for (uint32_t w = 0; w <= 32; w++)
        if (hist[w] != 0)
            maxb = w;
    uint32_t best_b = maxb;
    uint64_t best_cost = (uint64_t)count * maxb;
    uint64_t best_c = 0;
    for (int b = (int)maxb - 1; b >= 0; b--) {
        uint64_t c = 0;
        for (uint32_t w = (uint32_t)b + 1; w <= 32; w++)
            c += hist[w];
        uint64_t cost = (uint64_t)count * (uint64_t)b + c * (8u + maxb - (uint32_t)b);
        if (cost < best_cost) {
            best_cost = cost;
            best_b = (uint32_t)b;
            best_c = c;
        }
    }
    *b_out = best_b;
    *maxb_out = maxb;
    *c_out = (uint32_t)best_c;
}

/* ---------------------------------------------------------------------- */
/* Stream assembly shared by both codecs (header, directory, tail).        */

static uint64_t o_pad4(uint64_t w) { return (w + 3u) & ~(uint64_t)3u; }

static uint64_t o_units(int codec, uint64_t n)
{
    uint64_t nfull = n / OB;
    uint64_t per = (codec == 1 || codec == 3 || codec == 5 || codec == 6) ? OFP_BLOCKS : OBP_BLOCKS;
    return (nfull + per - 1) / per;
}

static uint32_t o_magic(int codec)
{
    return codec == 0   ? OMAGIC_BP
           : codec == 1 ? OMAGIC_FP
           : codec == 2 ? OMAGIC_BP32
           : codec == 3 ? OMAGIC_FP32
           : codec == 4 ? OMAGIC_BPV
           : codec == 5 ? OMAGIC_SP
                              : OMAGIC_FPI;
}

/* Worst-case stream size in words, computed from the layout. */
uint64_t oracle_max_words(int codec, uint64_t n)
{
    uint64_t nfull = n / OB;
    uint64_t tail = n % OB;
    uint64_t units = o_units(codec, n);
    uint64_t words = 8 + o_pad4((1 + 4) * (units + 1));
    if (codec == 0 || codec == 4) {
        words += units * 4 + nfull * OB;
    } else if (codec == 2) {
        /* a descriptor word per 128 values, every block at 32 bits, and at
         * most 3 words of padding per unit */
        words += units * 3 + nfull * (1 + OB);
    } else if (codec == 6) {
        /* per page: offset word, byte counter, bitset, 32 array counts and
         * 3 words of padding; packed <= 128 words per block; byte array <=
         * (3 + 127) bytes per block + 3 bytes of padding; exception bits of
         * a block <= 127 * 32 and at most 31 values of padding per array */
        words += units * (1 + 1 + 1 + 32 + 3 + 1 + 32 * 31) + nfull * (OB + (3 + 127) / 4 + 1 + 127);
    } else if (codec == 5) {
        /* per page: header <= 39 words (4, 7 segment bases of up to 4
         * words, 7 segment entries) and 3 words of padding; packed <= 128
         * words per block; metadata <= (3 + 128) bytes per block (+16 B
         * padding); at most one 64-bit Simple-8b word per exception */
        words += units * (39 + 3 + 4) + nfull * (OB + (3 + OB) / 4 + 1 + 2 * OB);
    } else {
        /* per page: header <= 64 words (4 + 32 counts + 7 segment bases of
         * up to 4 words); packed <= 128 words per block;
         * metadata <= (3 + 127) bytes per block (+16 B padding); every array
         * k holds at most one group of padding, and the exception bits of a
         * block never exceed 32*127 */
        words += units * (64 + 4 + 32 * 4 * 32) + nfull * (OB + (3 + 127) / 4 + 1 + 127);
    }
    words += (tail * 5 + 3) / 4;
    return words;
}

/* ---- Section 6.2, SIMD-BP128: blocks of 128 deltas, each stored in
 * b = bits(max) bits (computed, as the section suggests, from one OR over
 * the block: the width of the OR equals the largest width), 16 blocks per
 * meta-block behind a 128-bit descriptor of 8-bit widths. The remainder
 * after the last full block is Variable Byte (Section 6.2).
 * codec 0 = binary packing, 1 = patched pages (oracle_fp_encode).
 * Returns the stream length in words or a negative error. */
static int64_t o_encode(int codec, const uint32_t *x, uint64_t n, int stride,
                        uint32_t *out, uint64_t cap);

int64_t oracle_bp_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(0, x, n, stride, out, cap);
}

int64_t oracle_fp_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(1, x, n, stride, out, cap);
}

/* ---- Section 6.2, BP32: blocks of 32 deltas, each at b = bits(max) bits
 * in the plain (horizontal) layout of Section 4, four blocks per meta-block
 * behind one 32-bit word of four 8-bit widths, so every block starts on a
 * 32-bit boundary. Meta-blocks hold 128 values, so the header, directory
 * (units of 16 meta-blocks) and Variable Byte remainder are those of the
 * SIMD-BP128 stream. */
int64_t oracle_bp32_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(2, x, n, stride, out, cap);
}

/* ---- Section 5, FastPFOR: the same pages as SIMD-FastPFOR except that
 * each exception array is padded to a multiple of 32 values (packed at k
 * bits, 32 values in k words) instead of 128. The regular values need no
 * change: 128 values packed one after the other at b bits are the same
 * words as four groups of 32. The page is zero-padded to 4 words (units
 * start on 16-byte boundaries). */
int64_t oracle_fp32_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(3, x, n, stride, out, cap);
}

/* ---- Section 6.2 with the vectorized layout of Section 4: the SIMD-BP128
 * stream as the paper's own code lays it out, each block packed across
 * four interleaved 32-bit lanes (oracle_pack_vertical); widths,
 * descriptors, sizes and everything around the blocks as in
 * oracle_bp_encode. */
int64_t oracle_bpv_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(4, x, n, stride, out, cap);
}

/* Binary-packing meta-block: the descriptor then each block's packed words
 * (vertical: the four-lane layout). */
static uint64_t o_bp_unit(const uint32_t *d, uint64_t nblocks, uint32_t *out, int vertical)
{
    uint32_t desc[4] = {0, 0, 0, 0};
    uint64_t pos = 4;
    for (uint64_t j = 0; j < nblocks; j++) {
        uint32_t all = 0;
        for (uint32_t i = 0; i < OB; i++)
            all |= d[j * OB + i];
        uint32_t b = oracle_bits(all);
        desc[j / 4] |= b << (8 * (j % 4));
        if (vertical)
            oracle_pack_vertical(d + j * OB, OB, b, out + pos);
        else
            oracle_pack(d + j * OB, OB, b, out + pos);
        pos += (uint64_t)OB * b / 32;
    }
    memcpy(out, desc, sizeof desc);
    return pos;
}

/* BP32 unit: nmeta meta-blocks, each [descriptor][block 0]..[block 3],
 * then zero words up to a multiple of 4. */
static uint64_t o_bp32_unit(const uint32_t *d, uint64_t nmeta, uint32_t *out)
{
    uint64_t pos = 0;
    for (uint64_t m = 0; m < nmeta; m++) {
        uint64_t at = pos++;
        uint32_t desc = 0;
        for (uint32_t j = 0; j < 4; j++) {
            const uint32_t *blk = d + (m * 4 + j) * OB32;
            uint32_t all = 0;
            for (uint32_t i = 0; i < OB32; i++)
                all |= blk[i];
            uint32_t b = oracle_bits(all);
            desc |= b << (8 * j);
            oracle_pack(blk, OB32, b, out + pos);
            pos += b; /* 32 values of b bits fill b words */
        }
        out[at] = desc;
    }
    while (pos % 4)
        out[pos++] = 0;
    return pos;
}

/* ---- Section 5, FastPFOR page, re-arranged for parallel parsing:
 *   [nblocks, packed_words, meta_bytes, bitset] + count_k for every set k
 *       (ascending) + the segment bases, zero-padded to 4 words.  bitset bit
 *       k-1 <=> array k non-empty, k = 1..32 (the 32-bit bitset of Section
 *       5). Segment bases (an addition to the paper's page, for decoding
 *       one page by several independent parallel workers): the page's
 *       blocks form segments of 64 (8192 integers); for every segment g >= 1
 *       the S values just before its first integer, x[start_g - S + s],
 *       s = 0..S-1 (S = stride; none for stride 0). Section 3's prefix sum
 *       is the only dependency between the blocks of a page that the
 *       metadata does not settle: with these values each segment's sums
 *       start on their own. Cost: S words per 8192 integers.
 *   packed: block t's low b_t bits of its 128 values, 4*b_t words each,
 *       blocks back to back
 *   metadata bytes: b[nblocks], maxb[nblocks], c[nblocks], then every
 *       block's exception positions (0..127) in block order -- the same
 *       bytes as the section's per-block byte array, grouped by kind;
 *       zero-padded to 16 bytes
 *   exception arrays, for each set k ascending: the high parts (value >> b)
 *       of exceptions of blocks with maxb - b = k, in block order, packed
 *       at k bits in groups of 128 (SIMD-FastPFOR pads to a multiple of 128
 *       values; the padding values are 0), 4*k words per group. */
static uint64_t o_fp_page(const uint32_t *d, uint64_t nblocks, uint32_t *out, uint64_t pad,
                          const uint32_t *x, uint64_t start, int stride)
{
    uint32_t *bw = malloc(nblocks * sizeof(uint32_t));
    uint32_t *mb = malloc(nblocks * sizeof(uint32_t));
    uint32_t *cc = malloc(nblocks * sizeof(uint32_t));
    uint32_t *arr[33];
    uint64_t cnt[33];
    uint64_t need[33];
    memset(need, 0, sizeof need);
    for (uint64_t t = 0; t < nblocks; t++) {
        oracle_fp_choose(d + t * OB, OB, &bw[t], &mb[t], &cc[t]);
        need[mb[t] - bw[t]] += cc[t];
    }
    for (int k = 0; k <= 32; k++) {
        arr[k] = malloc((need[k] + OB) * sizeof(uint32_t));
        cnt[k] = 0;
    }
    uint8_t *pos_bytes = malloc(nblocks * OB + 1);
    uint64_t npos = 0;
    uint64_t packed_words = 0;
    for (uint64_t t = 0; t < nblocks; t++) {
        const uint32_t *blk = d + t * OB;
        packed_words += (uint64_t)OB * bw[t] / 32;
        uint32_t k = mb[t] - bw[t];
        for (uint32_t i = 0; i < OB; i++) {
            if (oracle_bits(blk[i]) > bw[t]) {
                pos_bytes[npos++] = (uint8_t)i;
                arr[k][cnt[k]++] = blk[i] >> bw[t];
            }
        }
    }
    uint32_t bitset = 0;
    uint32_t nset = 0;
    for (uint32_t k = 1; k <= 32; k++)
        if (cnt[k] != 0) {
            bitset |= 1u << (k - 1);
            nset++;
        }
    uint64_t meta_bytes = 3 * nblocks + npos;
    uint64_t nseg = (nblocks + OSEG_BLOCKS - 1) / OSEG_BLOCKS;
    uint64_t hdr_words = o_pad4(4 + nset + (uint64_t)stride * (nseg - 1));
    memset(out, 0, hdr_words * sizeof(uint32_t));
    out[0] = (uint32_t)nblocks;
    out[1] = (uint32_t)packed_words;
    out[2] = (uint32_t)meta_bytes;
    out[3] = bitset;
    uint32_t hi = 4;
    for (uint32_t k = 1; k <= 32; k++)
        if (cnt[k] != 0)
            out[hi++] = (uint32_t)cnt[k];
    for (uint64_t g = 1; g < nseg; g++) {
        uint64_t sg = start + g * OSEG_BLOCKS * OB; /* first integer of segment g */
        for (int t = 0; t < stride; t++)
            out[hi++] = x[sg - (uint64_t)stride + (uint64_t)t];
    }
    uint64_t p = hdr_words;
    /* packed truncated values (oracle_pack keeps the low b bits) */
    for (uint64_t t = 0; t < nblocks; t++) {
        oracle_pack(d + t * OB, OB, bw[t], out + p);
        p += (uint64_t)OB * bw[t] / 32;
    }
    /* metadata bytes */
    uint64_t meta_words = ((meta_bytes + 15) / 16) * 4;
    uint8_t *mbytes = (uint8_t *)(out + p);
    memset(mbytes, 0, meta_words * 4);
    for (uint64_t t = 0; t < nblocks; t++) {
        mbytes[t] = (uint8_t)bw[t];
        mbytes[nblocks + t] = (uint8_t)mb[t];
        mbytes[2 * nblocks + t] = (uint8_t)cc[t];
    }
    for (uint64_t e = 0; e < npos; e++)
        mbytes[3 * nblocks + e] = pos_bytes[e];
    p += meta_words;
    /* exception arrays */
    for (uint32_t k = 1; k <= 32; k++) {
        if (cnt[k] == 0)
            continue;
        uint64_t padded = ((cnt[k] + pad - 1) / pad) * pad;
        for (uint64_t e = cnt[k]; e < padded; e++)
            arr[k][e] = 0;
        oracle_pack(arr[k], padded, k, out + p);
        p += padded * k / 32;
    }
    /* with 32-value padding the arrays may end inside a 16-byte group: the
     * page is zero-padded to 4 words so that every unit starts on 16 bytes */
    while (p % 4)
        out[p++] = 0;
    for (int k = 0; k <= 32; k++)
        free(arr[k]);
    free(bw);
    free(mb);
    free(cc);
    free(pos_bytes);
    return p;
}

/* ---- Section 2 (the Simple family), Simple-8b: 64-bit words, a 4-bit
 * selector and 60 data bits holding `count` integers of `bits` bits each,
 * the modes of the paper's Simple-8b table (selectors 0 and 1: runs of 240
 * and 120 zeros, no data bits). Encoding is greedy: for the next word the
 * selectors are tried from 0 upward and the first one whose count of
 * integers is still available and fits in its bits is taken (selector 15,
 * one integer of up to 60 bits, always fits a 32-bit value). Readings:
 * the selector is the word's top four bits, integer j of a word sits at
 * bits [j*bits, (j+1)*bits), and a selector needs `count` integers left
 * (no padding of the last word). */
static const uint32_t O_S8_COUNT[16] = {240, 120, 60, 30, 20, 15, 12, 10, 8, 7, 6, 5, 4, 3, 2, 1};
static const uint32_t O_S8_BITS[16] = {0, 0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 15, 20, 30, 60};

void oracle_s8_mode(uint32_t sel, uint32_t *count, uint32_t *bits)
{
    *count = O_S8_COUNT[sel & 15u];
    *bits = O_S8_BITS[sel & 15u];
}

uint64_t oracle_s8_encode(const uint32_t *v, uint64_t n, uint64_t *out)
{
    uint64_t i = 0, w = 0;
    while (i < n) {
        uint32_t sel = 0;
        for (; sel < 16; sel++) {
            uint64_t cnt = O_S8_COUNT[sel];
            uint32_t bits = O_S8_BITS[sel];
            if (cnt > n - i)
                continue;
            int fits = 1;
            for (uint64_t j = 0; j < cnt && fits; j++)
                fits = bits >= 32 || (v[i + j] >> bits) == 0;
            if (fits)
                break;
        }
        uint64_t word = (uint64_t)sel << 60;
        for (uint64_t j = 0; j < O_S8_COUNT[sel] && O_S8_BITS[sel] > 0; j++)
            word |= (uint64_t)v[i + j] << (j * O_S8_BITS[sel]);
        out[w++] = word;
        i += O_S8_COUNT[sel];
    }
    return w;
}

/* Decodes nwords words into at most n integers; returns the number of
 * integers, or O_ERR_CORRUPT if they exceed n or a value exceeds 32 bits. */
int64_t oracle_s8_decode(const uint64_t *in, uint64_t nwords, uint32_t *v, uint64_t n)
{
    uint64_t k = 0;
    for (uint64_t w = 0; w < nwords; w++) {
        uint32_t sel = (uint32_t)(in[w] >> 60), cnt = O_S8_COUNT[sel], bits = O_S8_BITS[sel];
        if (cnt > n - k)
            return O_ERR_CORRUPT;
        for (uint32_t j = 0; j < cnt; j++) {
            uint64_t x = bits ? (in[w] >> (j * bits)) & ((1ull << bits) - 1u) : 0u;
            if (x >> 32)
                return O_ERR_CORRUPT;
            v[k++] = (uint32_t)x;
        }
    }
    return (int64_t)k;
}

/* Where high part number e of a page sits in its Simple-8b words: the index
 * of the word holding it | the number of that word's values before it
 * << 24; e equal to the page's exception count gives the word count. */
static uint32_t o_sp_entry(const uint64_t *s8, uint64_t ns8, uint64_t e)
{
    uint64_t v = 0;
    for (uint64_t w = 0; w < ns8; w++) {
        uint64_t cnt = O_S8_COUNT[s8[w] >> 60];
        if (e < v + cnt)
            return (uint32_t)w | ((uint32_t)(e - v) << 24);
        v += cnt;
    }
    return (uint32_t)ns8;
}

/* ---- Section 5, SimplePFOR: the pages of FastPFOR (the same widths by
 * the same cost rule, the same packed values, positions and metadata),
 * with the exceptions' high parts (value >> b) collected over the whole
 * page in block order and coded once with Simple-8b instead of one packed
 * array per width. Page: [nblocks, packed_words, meta_bytes, s8_words]
 * (s8_words: 32-bit words of the Simple-8b array, two per 64-bit word, low
 * half first), then, as in the FastPFOR pages, for each 64-block segment
 * after the first the S values before it, then for each such segment its
 * entry into the Simple-8b words (o_sp_entry of the exceptions before it;
 * both additions to the paper's page that let segments decode
 * independently), padded to 4 words; packed values, metadata (b, maxb, c
 * per block, then the positions; zero-padded to 16 bytes), the Simple-8b
 * words, zero-padded to 4 words. */
static uint64_t o_sp_page(const uint32_t *d, uint64_t nblocks, uint32_t *out, const uint32_t *x, uint64_t start,
                          int stride)
{
    uint32_t *bw = malloc(nblocks * sizeof(uint32_t));
    uint32_t *mb = malloc(nblocks * sizeof(uint32_t));
    uint32_t *cc = malloc(nblocks * sizeof(uint32_t));
    uint32_t *hv = malloc((nblocks * OB + 1) * sizeof(uint32_t));
    uint8_t *pos_bytes = malloc(nblocks * OB + 1);
    uint64_t nexc = 0, packed_words = 0;
    for (uint64_t t = 0; t < nblocks; t++) {
        const uint32_t *blk = d + t * OB;
        oracle_fp_choose(blk, OB, &bw[t], &mb[t], &cc[t]);
        packed_words += (uint64_t)OB * bw[t] / 32;
        for (uint32_t i = 0; i < OB; i++)
            if (oracle_bits(blk[i]) > bw[t]) {
                pos_bytes[nexc] = (uint8_t)i;
                hv[nexc++] = blk[i] >> bw[t];
            }
    }
    uint64_t *s8 = malloc((nexc + 1) * sizeof(uint64_t));
    uint64_t ns8 = oracle_s8_encode(hv, nexc, s8);
    uint64_t meta_bytes = 3 * nblocks + nexc;
    uint64_t nseg = (nblocks + OSEG_BLOCKS - 1) / OSEG_BLOCKS;
    uint64_t hdr_words = o_pad4(4 + ((uint64_t)stride + 1) * (nseg - 1));
    memset(out, 0, hdr_words * sizeof(uint32_t));
    out[0] = (uint32_t)nblocks;
    out[1] = (uint32_t)packed_words;
    out[2] = (uint32_t)meta_bytes;
    out[3] = (uint32_t)(2 * ns8);
    uint64_t hi = 4;
    for (uint64_t g = 1; g < nseg; g++) {
        uint64_t sg = start + g * OSEG_BLOCKS * OB; /* first integer of segment g */
        for (int t = 0; t < stride; t++)
            out[hi++] = x[sg - (uint64_t)stride + (uint64_t)t];
    }
    uint64_t before = 0; /* exceptions of the blocks before segment g */
    for (uint64_t g = 1; g < nseg; g++) {
        for (uint64_t t = (g - 1) * OSEG_BLOCKS; t < g * OSEG_BLOCKS; t++)
            before += cc[t];
        out[hi++] = o_sp_entry(s8, ns8, before);
    }
    uint64_t p = hdr_words;
    for (uint64_t t = 0; t < nblocks; t++) {
        oracle_pack(d + t * OB, OB, bw[t], out + p);
        p += (uint64_t)OB * bw[t] / 32;
    }
    uint64_t meta_words = ((meta_bytes + 15) / 16) * 4;
    uint8_t *mbytes = (uint8_t *)(out + p);
    memset(mbytes, 0, meta_words * 4);
    for (uint64_t t = 0; t < nblocks; t++) {
        mbytes[t] = (uint8_t)bw[t];
        mbytes[nblocks + t] = (uint8_t)mb[t];
        mbytes[2 * nblocks + t] = (uint8_t)cc[t];
    }
    for (uint64_t e = 0; e < nexc; e++)
        mbytes[3 * nblocks + e] = pos_bytes[e];
    p += meta_words;
    for (uint64_t w = 0; w < ns8; w++) {
        out[p++] = (uint32_t)(s8[w] & 0xFFFFFFFFu);
        out[p++] = (uint32_t)(s8[w] >> 32);
    }
    while (p % 4)
        out[p++] = 0;
    free(bw);
    free(mb);
    free(cc);
    free(hv);
    free(pos_bytes);
    free(s8);
    return p;
}

/* SimplePFOR (codec 5): see o_sp_page. */
static int64_t o_encode(int codec, const uint32_t *x, uint64_t n, int stride,
                        uint32_t *out, uint64_t cap);

int64_t oracle_sp_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(5, x, n, stride, out, cap);
}

/* ---- Section 5, FastPFOR page in the paper's own layout (the page-layout
 * figure and the text around it), the byte array read serially:
 *   word 0: the word offset, from the page start, of the byte array's
 *       32-bit length counter (the offset "of the byte array": the counter
 *       opens it)
 *   the blocks' truncated values: block t's low b_t bits, 4*b_t words
 *   the counter: the byte array's length in bytes
 *   the byte array, zero-padded to a multiple of 4 bytes: per block in
 *       order b, maxb, and, only when maxb > b, the exception count c and
 *       the c positions (0..127), one byte each
 *   a 32-bit bitset (bit k-1: array k is not empty), then for each
 *       non-empty array k ascending its 32-bit length counter and its
 *       values' high parts packed at k bits, padded to a multiple of 32
 *       values (FastPFOR)
 *   zero words up to a multiple of 4 (units start on 16 bytes). */
static uint64_t o_fpi_page(const uint32_t *d, uint64_t nblocks, uint32_t *out)
{
    uint32_t *bw = malloc(nblocks * sizeof(uint32_t));
    uint32_t *mb = malloc(nblocks * sizeof(uint32_t));
    uint32_t *cc = malloc(nblocks * sizeof(uint32_t));
    uint8_t *ba = malloc(nblocks * (3 + OB) + 4);
    uint32_t *arr[33];
    uint64_t cnt[33];
    for (int k = 0; k <= 32; k++) {
        arr[k] = malloc((nblocks * OB + 32) * sizeof(uint32_t));
        cnt[k] = 0;
    }
    uint64_t p = 1, nba = 0;
    for (uint64_t t = 0; t < nblocks; t++) {
        const uint32_t *blk = d + t * OB;
        oracle_fp_choose(blk, OB, &bw[t], &mb[t], &cc[t]);
        oracle_pack(blk, OB, bw[t], out + p);
        p += (uint64_t)OB * bw[t] / 32;
        ba[nba++] = (uint8_t)bw[t];
        ba[nba++] = (uint8_t)mb[t];
        if (mb[t] > bw[t]) {
            uint32_t k = mb[t] - bw[t];
            ba[nba++] = (uint8_t)cc[t];
            for (uint32_t i = 0; i < OB; i++)
                if (oracle_bits(blk[i]) > bw[t]) {
                    ba[nba++] = (uint8_t)i;
                    arr[k][cnt[k]++] = blk[i] >> bw[t];
                }
        }
    }
    out[0] = (uint32_t)p;
    out[p++] = (uint32_t)nba;
    uint64_t baw = (nba + 3) / 4;
    memset(out + p, 0, baw * 4);
    memcpy(out + p, ba, nba);
    p += baw;
    uint32_t bitset = 0;
    for (uint32_t k = 1; k <= 32; k++)
        if (cnt[k] != 0)
            bitset |= 1u << (k - 1);
    out[p++] = bitset;
    for (uint32_t k = 1; k <= 32; k++) {
        if (cnt[k] == 0)
            continue;
        out[p++] = (uint32_t)cnt[k];
        uint64_t padded = ((cnt[k] + 31) / 32) * 32;
        for (uint64_t e = cnt[k]; e < padded; e++)
            arr[k][e] = 0;
        oracle_pack(arr[k], padded, k, out + p);
        p += padded * k / 32;
    }
    while (p % 4)
        out[p++] = 0;
    for (int k = 0; k <= 32; k++)
        free(arr[k]);
    free(bw);
    free(mb);
    free(cc);
    free(ba);
    return p;
}

/* The paper's layout (codec 6): see o_fpi_page. */
int64_t oracle_fpi_encode(const uint32_t *x, uint64_t n, int stride, uint32_t *out, uint64_t cap)
{
    return o_encode(6, x, n, stride, out, cap);
}

static int64_t o_encode(int codec, const uint32_t *x, uint64_t n, int stride,
                        uint32_t *out, uint64_t cap)
{
    if (stride != 0 && stride != 1 && stride != 4)
        return O_ERR_ARG;
    if (cap < oracle_max_words(codec, n))
        return O_ERR_CAP;
    if (oracle_max_words(codec, n) >= 0xFFFFFFFFull)
        return O_ERR_ARG;
    uint32_t *d = malloc((n + 1) * sizeof(uint32_t));
    memcpy(d, x, n * sizeof(uint32_t));
    oracle_delta_encode_inplace(d, n, 0, stride);

    uint64_t nfull = n / OB;
    uint64_t tail = n % OB;
    uint64_t units = o_units(codec, n);
    uint64_t per = (codec == 1 || codec == 3 || codec == 5 || codec == 6) ? OFP_BLOCKS : OBP_BLOCKS;
    uint64_t E = 1 + (uint64_t)stride;
    uint64_t ndir = units + (tail ? 1 : 0);
    uint64_t dir_words = o_pad4(E * ndir);
    memset(out, 0, (8 + dir_words) * sizeof(uint32_t));
    uint64_t p = 8 + dir_words;
    for (uint64_t u = 0; u < ndir; u++) {
        uint64_t start = u * per * OB; /* first value of the unit (or tail) */
        if (u == units)
            start = nfull * OB;
        out[8 + u] = (uint32_t)p;
        uint32_t *bases = out + 8 + ndir + u * (uint64_t)stride;
        for (uint64_t s = 0; s < (uint64_t)stride; s++) {
            /* base_s = x[start - S + s], 0 before the array start */
            bases[s] = (start + s >= (uint64_t)stride) ? x[start + s - stride] : 0u;
        }
        if (u < units) {
            uint64_t nb = nfull - u * per;
            if (nb > per)
                nb = per;
            p += (codec == 0 || codec == 4) ? o_bp_unit(d + start, nb, out + p, codec == 4)
                 : codec == 2 ? o_bp32_unit(d + start, nb, out + p)
                 : codec == 5 ? o_sp_page(d + start, nb, out + p, x, start, stride)
                 : codec == 6 ? o_fpi_page(d + start, nb, out + p)
                              : o_fp_page(d + start, nb, out + p, codec == 3 ? 32 : OB, x, start, stride);
        }
    }
    uint64_t tail_off = p;
    uint32_t tail_bytes = 0;
    if (tail) {
        uint8_t buf[OB * 5];
        tail_bytes = oracle_vbyte_encode(d + nfull * OB, (uint32_t)tail, buf);
        uint64_t tw = (tail_bytes + 3) / 4;
        memset(out + p, 0, tw * 4);
        memcpy(out + p, buf, tail_bytes);
        p += tw;
    }
    out[0] = o_magic(codec);
    out[1] = (uint32_t)(n & 0xFFFFFFFFu);
    out[2] = (uint32_t)(n >> 32);
    out[3] = (uint32_t)stride;
    out[4] = (uint32_t)units;
    out[5] = tail_bytes;
    out[6] = (uint32_t)tail_off;
    out[7] = (uint32_t)p;
    free(d);
    return (int64_t)p;
}

/* ---------------------------------------------------------------------- */
/* Decoding: the exact inverse, with every field checked against the       */
/* stream's bounds; a bad stream returns O_ERR_CORRUPT.                     */

static int o_bp_unit_decode(const uint32_t *w, uint64_t avail, uint64_t nblocks, uint32_t *d, int vertical)
{
    if (avail < 4)
        return O_ERR_CORRUPT;
    uint64_t pos = 4;
    for (uint64_t j = 0; j < OBP_BLOCKS; j++) {
        uint32_t b = (w[j / 4] >> (8 * (j % 4))) & 255u;
        if (j >= nblocks) {
            if (b != 0)
                return O_ERR_CORRUPT;
            continue;
        }
        if (b > 32 || pos + (uint64_t)OB * b / 32 > avail)
            return O_ERR_CORRUPT;
        if (vertical)
            oracle_unpack_vertical(w + pos, OB, b, d + j * OB);
        else
            oracle_unpack(w + pos, OB, b, d + j * OB);
        pos += (uint64_t)OB * b / 32;
    }
    if (pos != avail)
        return O_ERR_CORRUPT;
    return O_OK;
}

static int o_bp32_unit_decode(const uint32_t *w, uint64_t avail, uint64_t nmeta, uint32_t *d)
{
    uint64_t pos = 0;
    for (uint64_t m = 0; m < nmeta; m++) {
        if (pos >= avail)
            return O_ERR_CORRUPT;
        uint32_t desc = w[pos++];
        for (uint32_t j = 0; j < 4; j++) {
            uint32_t b = (desc >> (8 * j)) & 255u;
            if (b > 32 || pos + b > avail)
                return O_ERR_CORRUPT;
            oracle_unpack(w + pos, OB32, b, d + (m * 4 + j) * OB32);
            pos += b;
        }
    }
    if (o_pad4(pos) != avail)
        return O_ERR_CORRUPT;
    return O_OK;
}

/* Section 5: exceptions are first decoded in bulk for the whole page, then
 * each block is unpacked and its exceptions patched in: the value at each
 * listed position gains the next high part of array k = maxb - b, shifted
 * left by b. */
static int o_fp_page_decode(const uint32_t *w, uint64_t avail, uint64_t nblocks_expected,
                            uint32_t *d, uint64_t pad, int stride, uint32_t *segb)
{
    if (avail < 4)
        return O_ERR_CORRUPT;
    uint64_t nblocks = w[0], packed_words = w[1], meta_bytes = w[2];
    uint32_t bitset = w[3];
    if (nblocks != nblocks_expected)
        return O_ERR_CORRUPT;
    uint32_t nset = 0;
    for (uint32_t k = 1; k <= 32; k++)
        if (bitset & (1u << (k - 1)))
            nset++;
    uint64_t nseg = (nblocks + OSEG_BLOCKS - 1) / OSEG_BLOCKS;
    uint64_t hdr_words = o_pad4(4 + nset + (uint64_t)stride * (nseg - 1));
    if (hdr_words > avail)
        return O_ERR_CORRUPT;
    uint64_t cnt[33] = {0};
    uint32_t hi = 4;
    for (uint32_t k = 1; k <= 32; k++)
        if (bitset & (1u << (k - 1))) {
            cnt[k] = w[hi++];
            if (cnt[k] == 0 || cnt[k] > nblocks * OB)
                return O_ERR_CORRUPT;
        }
    /* the segment bases, checked by the caller against the decoded values */
    for (uint64_t i = 0; i < (uint64_t)stride * (nseg - 1); i++)
        segb[i] = w[hi++];
    uint64_t p = hdr_words;
    uint64_t packed_at = p;
    if (packed_words > avail - p)
        return O_ERR_CORRUPT;
    p += packed_words;
    uint64_t meta_words = ((meta_bytes + 15) / 16) * 4;
    if (meta_bytes < 3 * nblocks || meta_words > avail - p)
        return O_ERR_CORRUPT;
    const uint8_t *mbytes = (const uint8_t *)(w + p);
    p += meta_words;
    /* bulk-decode every exception array */
    uint32_t *arr[33] = {0};
    uint64_t used[33] = {0};
    int rc = O_OK;
    for (uint32_t k = 1; k <= 32; k++) {
        if (cnt[k] == 0)
            continue;
        uint64_t padded = ((cnt[k] + pad - 1) / pad) * pad;
        if (padded * k / 32 > avail - p) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        arr[k] = malloc(padded * sizeof(uint32_t));
        oracle_unpack(w + p, padded, k, arr[k]);
        p += padded * k / 32;
    }
    if (o_pad4(p) != avail) {
        rc = O_ERR_CORRUPT;
        goto done;
    }
    uint64_t bitpos_words = 0;
    uint64_t epos = 3 * nblocks;
    for (uint64_t t = 0; t < nblocks; t++) {
        uint32_t b = mbytes[t], maxb = mbytes[nblocks + t], c = mbytes[2 * nblocks + t];
        if (b > 32 || maxb > 32 || maxb < b || c > OB || (c == 0) != (maxb == b)) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        if (bitpos_words + (uint64_t)OB * b / 32 > packed_words) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        oracle_unpack(w + packed_at + bitpos_words, OB, b, d + t * OB);
        bitpos_words += (uint64_t)OB * b / 32;
        uint32_t k = maxb - b;
        for (uint32_t e = 0; e < c; e++) {
            if (epos >= meta_bytes || arr[k] == NULL || used[k] >= cnt[k]) {
                rc = O_ERR_CORRUPT;
                goto done;
            }
            uint32_t at = mbytes[epos++];
            /* positions lie in [0, 127], ascending inside a block */
            if (at >= OB || (e > 0 && at <= mbytes[epos - 2])) {
                rc = O_ERR_CORRUPT;
                goto done;
            }
            d[t * OB + at] |= arr[k][used[k]++] << b;
        }
    }
    if (bitpos_words != packed_words || epos != meta_bytes) {
        rc = O_ERR_CORRUPT;
        goto done;
    }
    for (uint32_t k = 1; k <= 32; k++)
        if (used[k] != cnt[k])
            rc = O_ERR_CORRUPT;
done:
    for (uint32_t k = 1; k <= 32; k++)
        free(arr[k]);
    return rc;
}

/* The segment bases go to segb (checked by the caller against the decoded
 * values); every segment entry must be where the page's Simple-8b words
 * put the segment's first high part. */
static int o_sp_page_decode(const uint32_t *w, uint64_t avail, uint64_t nblocks_expected, uint32_t *d, int stride,
                            uint32_t *segb)
{
    if (avail < 4)
        return O_ERR_CORRUPT;
    uint64_t nblocks = w[0], packed_words = w[1], meta_bytes = w[2], s8_words = w[3];
    if (nblocks != nblocks_expected || (s8_words & 1u))
        return O_ERR_CORRUPT;
    uint64_t nseg = (nblocks + OSEG_BLOCKS - 1) / OSEG_BLOCKS;
    uint64_t hdr_words = o_pad4(4 + ((uint64_t)stride + 1) * (nseg - 1));
    if (hdr_words > avail)
        return O_ERR_CORRUPT;
    for (uint64_t i = 0; i < (uint64_t)stride * (nseg - 1); i++)
        segb[i] = w[4 + i];
    const uint32_t *entry = w + 4 + (uint64_t)stride * (nseg - 1);
    uint64_t p = hdr_words, packed_at = hdr_words;
    if (packed_words > avail - p)
        return O_ERR_CORRUPT;
    p += packed_words;
    uint64_t meta_words = ((meta_bytes + 15) / 16) * 4;
    if (meta_bytes < 3 * nblocks || meta_words > avail - p)
        return O_ERR_CORRUPT;
    const uint8_t *mbytes = (const uint8_t *)(w + p);
    p += meta_words;
    if (s8_words > avail - p || o_pad4(p + s8_words) != avail)
        return O_ERR_CORRUPT;
    uint64_t nexc = meta_bytes - 3 * nblocks;
    uint64_t ns8 = s8_words / 2;
    uint64_t *s8 = malloc((ns8 + 1) * sizeof(uint64_t));
    uint32_t *hv = malloc((nexc + 1) * sizeof(uint32_t));
    for (uint64_t k = 0; k < ns8; k++)
        s8[k] = (uint64_t)w[p + 2 * k] | ((uint64_t)w[p + 2 * k + 1] << 32);
    int rc = O_OK;
    if (oracle_s8_decode(s8, ns8, hv, nexc) != (int64_t)nexc) {
        rc = O_ERR_CORRUPT;
        goto done;
    }
    uint64_t bitpos_words = 0, epos = 3 * nblocks, e_at = 0;
    for (uint64_t t = 0; t < nblocks; t++) {
        uint32_t b = mbytes[t], maxb = mbytes[nblocks + t], c = mbytes[2 * nblocks + t];
        if (b > 32 || maxb > 32 || maxb < b || c > OB || (c == 0) != (maxb == b) ||
            bitpos_words + (uint64_t)OB * b / 32 > packed_words) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        if (t > 0 && t % OSEG_BLOCKS == 0 && entry[t / OSEG_BLOCKS - 1] != o_sp_entry(s8, ns8, e_at)) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        oracle_unpack(w + packed_at + bitpos_words, OB, b, d + t * OB);
        bitpos_words += (uint64_t)OB * b / 32;
        uint32_t k = maxb - b;
        for (uint32_t e = 0; e < c; e++) {
            if (epos >= meta_bytes) {
                rc = O_ERR_CORRUPT;
                goto done;
            }
            uint32_t at = mbytes[epos++];
            uint32_t h = hv[e_at++];
            /* positions in [0, 127], ascending inside a block; a high part
             * of at most maxb - b bits */
            if (at >= OB || (e > 0 && at <= mbytes[epos - 2]) || (k < 32 && (h >> k) != 0)) {
                rc = O_ERR_CORRUPT;
                goto done;
            }
            d[t * OB + at] |= h << b;
        }
    }
    if (bitpos_words != packed_words || epos != meta_bytes)
        rc = O_ERR_CORRUPT;
done:
    free(s8);
    free(hv);
    return rc;
}

/* The paper's layout, parsed the way the page is written: the offset word
 * locates the byte array, the byte array is read record by record (b,
 * maxb, then c and the positions only when maxb > b), the exception
 * arrays are found one after the other behind the bitset; exceptions are
 * unpacked in bulk, then each block is unpacked and patched. */
static int o_fpi_page_decode(const uint32_t *w, uint64_t avail, uint64_t nblocks, uint32_t *d)
{
    if (avail < 1)
        return O_ERR_CORRUPT;
    uint64_t cpos = w[0];
    if (cpos < 1 || cpos >= avail)
        return O_ERR_CORRUPT;
    uint64_t nba = w[cpos];
    uint64_t baw = (nba + 3) / 4;
    if (baw > avail - cpos - 1)
        return O_ERR_CORRUPT;
    const uint8_t *ba = (const uint8_t *)(w + cpos + 1);
    uint64_t xp = cpos + 1 + baw; /* the bitset */
    if (xp >= avail)
        return O_ERR_CORRUPT;
    uint32_t bitset = w[xp++];
    uint64_t cnt[33] = {0};
    uint32_t *arr[33] = {0};
    uint64_t used[33] = {0};
    int rc = O_OK;
    for (uint32_t k = 1; k <= 32; k++) {
        if (!(bitset & (1u << (k - 1))))
            continue;
        if (xp >= avail) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        cnt[k] = w[xp++];
        uint64_t padded = ((cnt[k] + 31) / 32) * 32;
        if (cnt[k] == 0 || cnt[k] > nblocks * OB || padded * k / 32 > avail - xp) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        arr[k] = malloc(padded * sizeof(uint32_t));
        oracle_unpack(w + xp, padded, k, arr[k]);
        xp += padded * k / 32;
    }
    if (o_pad4(xp) != avail) {
        rc = O_ERR_CORRUPT;
        goto done;
    }
    uint64_t at = 0, pk = 1;
    for (uint64_t t = 0; t < nblocks; t++) {
        if (at + 2 > nba) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        uint32_t b = ba[at], maxb = ba[at + 1];
        at += 2;
        if (b > 32 || maxb > 32 || maxb < b || pk + (uint64_t)OB * b / 32 > cpos) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        oracle_unpack(w + pk, OB, b, d + t * OB);
        pk += (uint64_t)OB * b / 32;
        if (maxb == b)
            continue;
        uint32_t k = maxb - b;
        if (at + 1 > nba) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        uint32_t c = ba[at++];
        if (c == 0 || c >= OB || at + c > nba) {
            rc = O_ERR_CORRUPT;
            goto done;
        }
        for (uint32_t e = 0; e < c; e++) {
            uint32_t pos = ba[at + e];
            if (pos >= OB || (e > 0 && pos <= ba[at + e - 1]) || arr[k] == NULL || used[k] >= cnt[k]) {
                rc = O_ERR_CORRUPT;
                goto done;
            }
            d[t * OB + pos] |= arr[k][used[k]++] << b;
        }
        at += c;
    }
    if (pk != cpos || at != nba) {
        rc = O_ERR_CORRUPT;
        goto done;
    }
    for (uint32_t k = 1; k <= 32; k++)
        if (used[k] != cnt[k])
            rc = O_ERR_CORRUPT;
    /* the byte array's padding is zero */
    for (uint64_t i = nba; i < 4 * baw; i++)
        if (ba[i] != 0)
            rc = O_ERR_CORRUPT;
done:
    for (uint32_t k = 1; k <= 32; k++)
        free(arr[k]);
    return rc;
}

static int o_decode(int codec, const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    if (in_words < 8)
        return O_ERR_CORRUPT;
    if (in[0] != o_magic(codec))
        return O_ERR_CORRUPT;
    uint64_t hn = (uint64_t)in[1] | ((uint64_t)in[2] << 32);
    int stride = (int)in[3];
    if (hn != n || (stride != 0 && stride != 1 && stride != 4))
        return O_ERR_CORRUPT;
    uint64_t nfull = n / OB, tail = n % OB;
    uint64_t units = o_units(codec, n);
    uint64_t per = (codec == 1 || codec == 3 || codec == 5 || codec == 6) ? OFP_BLOCKS : OBP_BLOCKS;
    uint64_t total = in[7], tail_off = in[6], tail_bytes = in[5];
    if (in[4] != units || total > in_words || (tail == 0) != (tail_bytes == 0))
        return O_ERR_CORRUPT;
    uint64_t E = 1 + (uint64_t)stride;
    uint64_t ndir = units + (tail ? 1 : 0);
    uint64_t dir_end = 8 + o_pad4(E * ndir);
    if (dir_end > total || tail_off > total)
        return O_ERR_CORRUPT;
    for (uint64_t u = 0; u < ndir; u++) {
        uint64_t off = in[8 + u];
        const uint32_t *bases = in + 8 + ndir + u * (uint64_t)stride;
        uint64_t end = (u + 1 < units) ? in[8 + u + 1] : tail_off;
        uint64_t start = (u == units) ? nfull * OB : u * per * OB;
        uint64_t count;
        uint64_t nsegb = 0;      /* stored segment bases of a patched page */
        uint32_t segb[4 * (OFP_BLOCKS / OSEG_BLOCKS)];
        int rc;
        if (u < units) {
            uint64_t nb = nfull - u * per;
            if (nb > per)
                nb = per;
            count = nb * OB;
            if (off < dir_end || end < off || end > total)
                return O_ERR_CORRUPT;
            rc = (codec == 0 || codec == 4) ? o_bp_unit_decode(in + off, end - off, nb, out + start, codec == 4)
                 : codec == 2 ? o_bp32_unit_decode(in + off, end - off, nb, out + start)
                 : codec == 5 ? o_sp_page_decode(in + off, end - off, nb, out + start, stride, segb)
                 : codec == 6 ? o_fpi_page_decode(in + off, end - off, nb, out + start)
                              : o_fp_page_decode(in + off, end - off, nb, out + start, codec == 3 ? 32 : OB,
                                                 stride, segb);
            if (codec == 1 || codec == 3 || codec == 5)
                nsegb = (uint64_t)stride * ((nb + OSEG_BLOCKS - 1) / OSEG_BLOCKS - 1);
        } else {
            count = tail;
            if (off != tail_off || off + (tail_bytes + 3) / 4 != total)
                return O_ERR_CORRUPT;
            int64_t used = oracle_vbyte_decode((const uint8_t *)(in + off), tail_bytes,
                                               (uint32_t)tail, out + start);
            rc = (used == (int64_t)tail_bytes) ? O_OK : O_ERR_CORRUPT;
        }
        if (rc != O_OK)
            return rc;
        /* prefix sum of the unit from its stored bases (Section 3) */
        for (uint64_t i = 0; i < count && stride != 0; i++) {
            uint32_t prev = (i >= (uint64_t)stride) ? out[start + i - stride] : bases[i];
            out[start + i] = out[start + i] + prev;
        }
        /* a patched page's segment bases are the values just before each
         * segment */
        for (uint64_t i = 0; i < nsegb; i++) {
            uint64_t g = 1 + i / (uint64_t)stride, t = i % (uint64_t)stride;
            if (out[start + g * OSEG_BLOCKS * OB - (uint64_t)stride + t] != segb[i])
                return O_ERR_CORRUPT;
        }
    }
    if (ndir == 0 && total != dir_end)
        return O_ERR_CORRUPT;
    return O_OK;
}

int oracle_bp_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(0, in, in_words, out, n);
}

int oracle_fp_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(1, in, in_words, out, n);
}

int oracle_bp32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(2, in, in_words, out, n);
}

int oracle_fp32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(3, in, in_words, out, n);
}

int oracle_bpv_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(4, in, in_words, out, n);
}

int oracle_sp_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(5, in, in_words, out, n);
}

int oracle_fpi_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n)
{
    return o_decode(6, in, in_words, out, n);
}

/* ------------------------------------------------------------------------
 * Intersection of two posting lists (the consumer of decoded lists that the
 * paper's conclusion discusses: conjunctive queries intersect sorted lists).
 * Definition: the values present in both a and b, ascending. a and b must be
 * strictly increasing. A two-pointer walk: advance whichever side holds the
 * smaller value, emit on equality. Returns the number of values written to
 * out (room for min(na, nb) values). */
uint64_t oracle_intersect(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out)
{
    uint64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) {
            i++;
        } else if (b[j] < a[i]) {
            j++;
        } else {
            out[k++] = a[i];
            i++;
            j++;
        }
    }
    return k;
}
