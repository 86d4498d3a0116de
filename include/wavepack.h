/*
 * wavepack -- MI355X (gfx950) decoder for binary-packed and patched
 * (SIMD-BP128 / SIMD-FastPFOR style) compressed uint32 arrays, after
 * Lemire & Boytsov, "Decoding billions of integers per second through
 * vectorization" (arXiv:1209.2137).
 *
 * C ABI. Plain pointers and sizes only.
 *
 * Conventions for every call below
 *   - Pointers are DEVICE pointers (memory of the current HIP device) unless
 *     the name starts with h_ (host memory).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on `stream`: they enqueue work and return.
 *   - Compressed streams (`in`, `out` of the encoders) and decoded outputs
 *     must be 16-byte aligned (hipMalloc and torch allocations are).
 *   - The caller owns every buffer and keeps it alive until the stream work
 *     has completed. The library never frees caller memory.
 *   - Return value: WP_OK (0) or a negative WP_ERR_* code. Problems the host
 *     can see (null pointers, bad stride, capacity, misalignment) return at
 *     once and enqueue nothing. Problems inside a compressed stream are
 *     found by the kernels: they record WP_ERR_CORRUPT in a per-device
 *     error word (a static device variable of the library, read and cleared
 *     by wp_check; it is shared by all streams of the device), skip the bad
 *     unit, and never write outside [out, out + n).
 *   - Allocation and synchronisation: the decoders, wp_batch_decode and
 *     wp_decode_range neither allocate nor synchronise. The encoders, delta_decode_inplace, wp_intersect and
 *     wp_intersect_compressed use a library-owned scratch area per (device,
 *     stream); when a call needs more than that stream's area holds, it
 *     synchronises the stream, frees the area and allocates a larger one
 *     (so such a first call must not happen under stream capture).
 *   - All arithmetic on values is uint32 modulo 2^32 (sums wrap).
 *
 * Stream layout (32-bit little-endian words; both codecs)
 *   header, 8 words: magic ('WPB1' binary packing, 'WPF1' patched), n low,
 *       n high, stride S (0, 1 or 4), n_units, tail_bytes, tail_off,
 *       total_words
 *   directory: ndir entries, one per unit plus one for the tail when
 *       n % 128 != 0: first the ndir word offsets (from the stream start),
 *       then ndir groups of S bases, base_s = x[start - S + s] (0 before the
 *       array start), so every unit decodes on its own; zero-padded to a
 *       multiple of 4 words
 *   units: binary packing -- a meta-block of up to 16 blocks of 128 values
 *       (2048 values): a 16-byte descriptor whose byte j is block j's width
 *       b_j, then each block's 128 deltas packed at b_j bits in 4*b_j words
 *       (field i at bits [i*b, i*b+b) of the block's words, least
 *       significant bit first). Section 4 (bit layout) and Section 6.2
 *       (SIMD-BP128: 16 blocks of 128 integers behind a 128-bit descriptor).
 *       WP_CODEC_BPV (magic 'WPV1'): the same, with each block in the
 *       paper's vectorized layout (Section 4): value i is field i / 4 of
 *       32-bit lane i % 4, each lane's fields end to end from its least
 *       significant bit, word w of lane l at word 4w + l of the block.
 *       BP32 -- 16 meta-blocks of four 32-value blocks (2048 values):
 *       each meta-block is a descriptor word whose byte j is the width b_j
 *       of its block j, then its four blocks, block j in b_j words (32
 *       fields of b_j bits, same bit order); the unit is zero-padded to a
 *       multiple of 4 words. Section 6.2 (BP32: four blocks of 32 integers
 *       behind a 32-bit descriptor of 8-bit widths, blocks 32-bit aligned).
 *       patched -- a page of up to 512 blocks (2^16 values), Section 5:
 *       [nblocks, packed_words, meta_bytes, bitset] + one count per
 *       non-empty exception array k (bit k-1 of bitset) + the segment
 *       bases: for each 64-block segment of the page but the first, the S
 *       values just before its first integer (x[start - S + s]; an addition
 *       to the paper's page that lets the segments decode independently),
 *       padded to 4 words;
 *       the blocks' low b bits (4*b words each); the metadata bytes
 *       b[nblocks], maxb[nblocks], c[nblocks] and all exception positions,
 *       padded to 16 bytes; then for each k ascending the high parts
 *       (delta >> b) of the exceptions of blocks with maxb - b = k, packed
 *       at k bits in groups of 128 (zero padded). FastPFOR (WP_CODEC_FP32,
 *       magic 'WPF3'): the same page with each array padded to a multiple
 *       of 32 values (k words per 32) instead of 128, and the page
 *       zero-padded to 4 words.
 *   tail: Variable Byte (Section 2.4; 7 data bits per byte, low group
 *       first, top bit set on the last byte) of the last n % 128 deltas,
 *       zero-padded to a word.
 *   Deltas: Section 3. S = 1: d_i = x_i - x_{i-1}; S = 4: d_i = x_i - x_{i-4};
 *   S = 0: the values themselves. Decoding is the prefix sum.
 */
#ifndef WAVEPACK_H
#define WAVEPACK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WP_OK 0
#define WP_ERR_INVALID_ARG (-1) /* null pointer, bad stride, misaligned, n too large */
#define WP_ERR_CAPACITY (-2)    /* out_cap_words below wp_max_compressed_words(codec, n) */
#define WP_ERR_CORRUPT (-3)     /* reported by wp_check: a stream failed validation */
#define WP_ERR_HIP (-4)         /* a HIP runtime call failed */

#define WP_CODEC_BP 0 /* binary packing, 16 x 128-integer blocks per unit */
#define WP_CODEC_FP 1 /* patched pages of 2^16 integers */
#define WP_CODEC_BP32 2 /* binary packing, 64 x 32-integer blocks per unit */
#define WP_CODEC_FP32 3 /* patched pages, exception arrays padded to 32 values */
#define WP_CODEC_BPV 4  /* binary packing as WP_CODEC_BP, four-lane block layout */
#define WP_CODEC_SP 5   /* patched pages, exception high parts in one Simple-8b array per page */
#define WP_CODEC_FPI 6  /* patched pages in the paper's own page layout (counted byte array) */

/* Largest stream any input of n integers can produce, in 32-bit words.
 * Host only, pure. Returns 0 when n is beyond the format (streams are
 * addressed with 32-bit word offsets). */
uint64_t wp_max_compressed_words(int32_t codec, uint64_t n);

/* Binary-packing encoder (Section 6.2, SIMD-BP128; widths as in Section 6.2:
 * b = bits of the OR of a block's deltas; remainder in Variable Byte).
 *   in[n]            values to compress (any uint32; sorted input compresses best)
 *   delta_stride     0 (no differencing), 1 (standard) or 4 (vectorised), Section 3
 *   out[out_cap_words]  receives the stream; out_cap_words must be at least
 *                    wp_max_compressed_words(WP_CODEC_BP, n)
 *   out_words        device uint64: receives the stream length in words
 *                    (written on the stream, no implicit synchronisation)
 * Uses a library-owned scratch area per (device, stream), grown on demand
 * (growing synchronises the stream and allocates). */
int32_t bp_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                  uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* Binary-packing decoder: writes out[0..n) from the stream in[0..in_words).
 * Unpacks each 128-integer block at its width (Section 4), then runs the
 * prefix sum of Section 3 from the unit's stored base. n must equal the n
 * recorded in the stream header (checked on the device). Allocates nothing. */
int32_t bp_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                  void *stream);

/* SIMD-BP128 encoder with the paper's own four-lane (vectorized) block
 * layout (Section 4 figure of 32 integers of 5 bits; Section 6.2): widths,
 * descriptors, sizes and everything around the blocks as bp_encode, only
 * the order of the bits inside each block differs. Arguments as bp_encode,
 * with WP_CODEC_BPV for the capacity. */
int32_t bp_vertical_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                           uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* Decoder for bp_vertical_encode's streams: as bp_decode. Allocates
 * nothing. */
int32_t bp_vertical_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                           void *stream);

/* BP32 encoder (Section 6.2, BP32: 32-integer blocks at b = bits of the OR
 * of their deltas, four per meta-block behind a word of widths). Arguments
 * as bp_encode, with WP_CODEC_BP32 for the capacity. Narrower blocks adapt
 * better to local gaps than 128-integer ones, for a descriptor word per 128
 * integers instead of a quarter. */
int32_t bp32_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                    uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* BP32 decoder: unpacks each 32-integer block at its width (Section 4),
 * then the prefix sum of Section 3 from the unit's stored base. Arguments
 * and errors as bp_decode. Allocates nothing. */
int32_t bp32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                    void *stream);

/* Patched encoder (Section 5, FastPFOR with SIMD-FastPFOR padding): per
 * 128-integer block the width b minimising 128*b + c*(8 + maxb - b) (c =
 * values wider than b; equal costs keep the larger b); exceptions' high bits
 * go to page-wide arrays by k = maxb - b. Arguments as bp_encode, with
 * WP_CODEC_FP for the capacity. */
int32_t fastpfor_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                        uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* FastPFOR encoder (Section 5: as fastpfor_encode, but each page's
 * exception arrays are padded to a multiple of 32 values, not 128, which
 * saves up to 96 values of padding per array). Arguments as bp_encode,
 * with WP_CODEC_FP32 for the capacity. */
int32_t fastpfor32_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                          uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* FastPFOR decoder for fastpfor32_encode's streams: as fastpfor_decode.
 * Allocates nothing. */
int32_t fastpfor32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                          void *stream);

/* SimplePFOR pages (Section 5, SimplePFOR; Section 2, Simple-8b): the
 * pages of fastpfor_encode (same widths by the same cost rule, same packed
 * values, metadata and positions), with the high parts of a page's
 * exceptions collected in block order into one array coded with Simple-8b
 * (64-bit words: a 4-bit selector, the word's top four bits, and 60 data
 * bits holding the mode's count of equal-width integers, integer j at bits
 * [j*bits, (j+1)*bits); greedy: the first selector, from 0 up, whose count
 * is still available and whose width fits them). Page: [nblocks,
 * packed_words, meta_bytes, Simple-8b words (32-bit words, two per 64-bit
 * word, low half first)] + the segment bases (as in the patched pages: for
 * each 64-block segment after the first, the S values just before it) +
 * for each such segment its entry into the Simple-8b words (the index of
 * the 64-bit word holding the high part of the segment's first exception
 * | the number of that word's values before it << 24; the word count when
 * no exception follows), padded to 4 words; packed values, metadata, the
 * Simple-8b words, zero-padded to 4 words (magic 'WPS1'). The bases and
 * entries are additions to the paper's page that let segments decode
 * independently. */

/* SimplePFOR encoder: the pages described above (widths, metadata and
 * positions as fastpfor_encode; the high parts of each page's exceptions,
 * in block order, coded greedily with Simple-8b). Arguments as bp_encode,
 * with WP_CODEC_SP for the capacity; scratch as bp_encode, plus about
 * 169 KB per 65536 integers (each page's Simple-8b word starts, 105 KB,
 * and its blocks' exception widths, 64 KB). */
int32_t simplepfor_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                          uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* SimplePFOR decoder: as fastpfor_decode (one wavefront per 64-block
 * segment), the high parts taken from the page's Simple-8b words, decoded
 * from the segment's entry on as its blocks need them. A page whose blocks
 * hold more exceptions than the cost rule ever keeps (over 102 in a block,
 * in passes that would overfill the segment's ring of high parts) is
 * reported as corrupt. Allocates nothing. */
int32_t simplepfor_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                          void *stream);

/* FastPFOR pages in the paper's own layout (Section 5 and its page-layout
 * figure), magic 'WPI1', header, directory and tail as everywhere: a page
 * is [offset word][the blocks' truncated values, 4*b words each][byte
 * counter][byte array][bitset][for each non-empty array k ascending: its
 * length counter, its high parts packed at k bits, padded to 32 values],
 * zero-padded to 4 words. The offset word holds the word offset of the
 * byte counter; the byte array (zero-padded to 4 bytes) holds per block b,
 * maxb and, only when maxb > b, the count c and the c positions. Widths,
 * exceptions and arrays are those of fastpfor32_encode. The byte array
 * can only be read record by record; the decoder walks it. */

/* Encoder for that layout. Arguments as bp_encode, with WP_CODEC_FPI for
 * the capacity; scratch as bp_encode (it also holds the FastPFOR stream
 * that the pages are rearranged from). */
int32_t fastpfor_inline_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                               uint64_t out_cap_words, uint64_t *out_words, void *stream);

/* Decoder for that layout: as fastpfor_decode. One wavefront per page
 * copies the page's byte array into LDS (when it fits in 12 KB; otherwise
 * it reads it from the page), walks its records for every block's widths,
 * count and positions, walks the counted exception arrays, then decodes
 * the page pass by pass. Allocates nothing. */
int32_t fastpfor_inline_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                               void *stream);

/* Patched decoder (Section 5): unpack each block's low bits, patch each
 * exception with its high part from array k shifted left by b, then the
 * prefix sum. Arguments as bp_decode. Allocates nothing. */
int32_t fastpfor_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                        void *stream);

/* In-place differential decoding (Section 3): data[i] += data[i - stride]
 * in increasing index order, values before index 0 taken as `init`:
 *   stride 1: data[i] = init + d_0 + ... + d_i
 *   stride 4: data[i] = init + sum of d_j, j <= i, j = i (mod 4)
 * One pass over the data (8 bytes of traffic per integer) with a
 * decoupled look-back across tiles. Uses a library-owned scratch area per
 * (device, stream) of 64 bytes per 32768 integers, grown on demand
 * (growing synchronises the stream and allocates). Returns
 * WP_ERR_INVALID_ARG for a stride other than 1 or 4, a null or misaligned
 * `data` (n > 0), WP_ERR_HIP if the scratch allocation or a launch fails. */
int32_t delta_decode_inplace(uint32_t *data, uint64_t n, uint32_t init, int32_t stride,
                             void *stream);

/* delta_decode_inplace without any allocation, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, result and errors as
 * delta_decode_inplace, for n <= 2^28 integers (2^28 + 1 and more return
 * WP_ERR_CAPACITY and enqueue nothing). Its scan status words live in a
 * fixed array of about 512 KiB in the library's code object, one per device, held
 * until the process ends; each call first clears the part it uses with a
 * fill kernel (no memset node). Every call on a device shares that array:
 * calls that overlap on one device (on different streams, or from several
 * threads) race and give wrong sums; enqueue them on one stream or
 * serialise them. The first call on a device looks the array's address up
 * (no allocation). */
int32_t delta_decode_inplace_noalloc(uint32_t *data, uint64_t n, uint32_t init, int32_t stride,
                                     void *stream);

/* Intersection of two decoded posting lists (the conjunctive-query step
 * that consumes decoded lists, discussed with the paper's conclusions):
 * writes the values present in both `a` (na values) and `b` (nb values),
 * ascending, to out[0..k) and k to *out_count (device uint64, 8-byte
 * aligned), asynchronously on `stream`. a and b are device arrays that must
 * be strictly increasing (otherwise the result is unspecified but stays in
 * out[0..na)); out must hold na values. Each element of a is looked up in b
 * by binary search, so pass the shorter list as a. Uses the library's
 * per-stream scratch (one byte per element of a). Returns
 * WP_ERR_INVALID_ARG for null pointers or na >= 2^32, WP_ERR_HIP if a
 * launch or the scratch allocation fails. */
int32_t wp_intersect(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out,
                     uint64_t *out_count, void *stream);

/* As wp_intersect, with the second list still compressed (`b_comp`,
 * b_words words, nb integers, any WP_CODEC_* but WP_CODEC_FPI; 16-byte
 * aligned): the directory serves as a skip list. A strictly increasing
 * list's unit holds values between the value stored as its base (the value
 * just before the unit) and the next unit's, so only the units (and the
 * tail) that some element of `a` falls in are decoded, into b_work
 * (device, nb integers, 16-byte aligned, caller-owned; every other element
 * of b_work is left as it was). A stream without differential coding
 * (stride 0) gives no such bounds: all of it is decoded. A corrupt stream is
 * reported through wp_check. Same result, output and errors as
 * wp_intersect. */
int32_t wp_intersect_compressed(const uint32_t *a, uint64_t na, const uint32_t *b_comp, uint64_t b_words,
                                uint64_t nb, int32_t codec, uint32_t *b_work, uint32_t *out,
                                uint64_t *out_count, void *stream);

/* Random access by key (the directory's bases as a skip list, Section 3
 * differential coding): the index range [i0, i1) of the values v with
 * key_lo <= v <= key_hi in a non-decreasing list held as the stream `in`
 * (in_words words, n integers, any WP_CODEC_* but WP_CODEC_FPI, 16-byte aligned). Only the
 * units (and the tail) whose values can lie in the key range, or in which
 * the range's ends fall, are decoded into `out` (device, n integers,
 * 16-byte aligned, caller-owned), each at its place in the whole list:
 * out[i0..i1) then holds the values in the key range and every element of
 * out outside the decoded units is left as it was. range (device, two
 * uint64, 8-byte aligned) receives i0 and i1. A stream without
 * differential coding (stride 0) gives no bounds: all of it is decoded.
 * For a list that is not non-decreasing the range is unspecified (but lies
 * in [0, n]). Asynchronous on `stream`; a corrupt stream is reported
 * through wp_check (range then reads 0, 0). Returns WP_ERR_INVALID_ARG for
 * null or misaligned pointers, an unknown codec or key_lo > key_hi,
 * WP_ERR_HIP if a launch fails. Allocates nothing: two launches, the
 * decoding (each unit checks its own stored bases) and the two searches. */
int32_t wp_decode_range(const uint32_t *in, uint64_t in_words, uint64_t n, int32_t codec, uint32_t key_lo,
                        uint32_t key_hi, uint32_t *out, uint64_t *range, void *stream);

/* Timing hook (host): the calling thread's next bp_decode,
 * fastpfor_decode or delta_decode_inplace records `start_event` when its
 * main kernel starts and `stop_event` when that kernel ends (hipEvent_t,
 * created by the caller with timing enabled; either may be NULL). The
 * events bracket the kernel alone, not the launch path before it; they
 * are consumed by that one call. Always returns WP_OK. */
int32_t wp_time_next_launch(void *start_event, void *stop_event);

/* Workgroup shape of the single-list decoders (set by the autotuner;
 * process-wide; WP_CODEC_BPV shares WP_CODEC_BP's setting and
 * WP_CODEC_FP32 WP_CODEC_FP's). Binary packing (WP_CODEC_BP, _BPV and
 * _BP32): every wavefront decodes its own run of
 * consecutive meta-blocks, streaming the run's compressed words through a
 * private LDS ring; waves: wavefronts per workgroup (1, 2, 4 or 8); vpl
 * must be 4 (each lane unpacks four integers of a block per pass); depth:
 * 16-byte loads per lane in flight (2, 3 or 4; 0 = 2); wg_per_cu: runs
 * per compute unit, 0..1024, which sets the run length (0 = 128; many
 * short runs let the hardware balance the load). Patched pages: one
 * wavefront per page (four blocks per pass), waves = pages per workgroup
 * (1, 2, 4 or 8), vpl 4; depth and wg_per_cu are ignored. Returns
 * WP_ERR_INVALID_ARG for anything else. */
int32_t wp_set_decode_tune(int32_t codec, int32_t waves, int32_t vpl, int32_t depth, int32_t wg_per_cu);

/* Synchronises `stream`, then returns and clears this device's error word:
 * WP_OK, WP_ERR_CORRUPT, or WP_ERR_HIP if the synchronisation failed. The
 * word is device-wide: it reports a corrupt stream met by work on any
 * stream of the device since the last wp_check, and work still running on
 * other streams may set it after this call has read it. */
int32_t wp_check(void *stream);

/* Static description of a code. */
const char *wp_strerror(int32_t code);

/* ---------------------------------------------------------------------- */
/* Batched decoding of many lists in one launch (not in the paper: the GPU
 * counterpart of decoding many posting lists). A plan turns a list
 * registry into work items -- 64-block segments of patched pages, runs of
 * meta-blocks and tails of lists without full blocks -- and one kernel
 * launch covers them all, a wavefront for each item, the largest and the
 * smallest items alternately (the longest start first): by
 * default a grid of one wavefront per item (the hardware dispatcher
 * balances the load), or, with wp_tune.wg_per_cu > 0, a persistent grid
 * whose wavefronts pull the items from a work queue (a device counter).
 * The item holding a list's last unit also decodes the list's tail. */

typedef struct wp_list {
    uint64_t comp_off_words; /* stream start, in words from `pool` (multiple of 4) */
    uint64_t comp_words;     /* stream length in words */
    uint64_t out_off;        /* first output element, from `out_base` (multiple of 4) */
    uint64_t n;              /* integers in the list */
    int32_t codec;           /* WP_CODEC_BP or WP_CODEC_FP */
    int32_t reserved;        /* must be 0 */
    uint32_t *out;           /* if not NULL: the list's own destination (device,
                                16-byte aligned, n integers, caller-owned), used
                                instead of out_base + out_off (out_off ignored) */
} wp_list;

typedef struct wp_tune {
    int32_t waves;     /* wavefronts per workgroup: 2, 4 or 8 (0 = 4) */
    int32_t vpl;       /* integers per lane and pass: 4 (0 = 4) */
    int32_t depth;     /* binary packing: 16-byte loads per lane in flight, 2, 3 or 4 (0 = 2) */
    int32_t run_units; /* meta-blocks per binary-packing work item (one wavefront), 1..63 (0 = 8) */
    int32_t wg_per_cu; /* 0: one workgroup per `waves` items (the one-shot grid);
                          1..64: the persistent form, wg_per_cu workgroups per
                          compute unit whose wavefronts take items from a
                          device counter (cleared by a kernel launched, or a
                          graph node placed, before the decoder) */
    int32_t use_graph; /* 1 = replay a hipGraph built at plan time, 0 = plain launches */
} wp_tune;

/* Builds a plan: validates the registry on the host (codec, alignment of
 * comp_off_words and out_off (or of the list's own `out`) to 4 words,
 * comp_words >= 8), cuts every list
 * into work items (runs of run_units meta-blocks, page segments, tails
 * of lists without full blocks; largest and smallest alternately), uploads the list and item arrays (it synchronises
 * `stream` once), and, when tune->use_graph, builds and instantiates a
 * hipGraph holding the decoder's kernel node. `pool` and
 * `out_base` (device, 16-byte aligned) are kept; out_base may be NULL when
 * every list names its own `out`; h_lists may be freed on return. `tune`
 * (an addition to the plan call of the design: the workgroup shape and
 * the size of a binary-packing work item are chosen by the autotuner,
 * which must be able to try them) may be NULL (defaults, graph on). The plan allocates its
 * own device arrays; *h_plan is released with wp_batch_free. Output ranges
 * of different lists must not overlap. Returns WP_ERR_INVALID_ARG for a bad
 * registry or tune, WP_ERR_HIP if an allocation or copy fails. */
int32_t wp_batch_plan(const uint32_t *pool, uint32_t *out_base, const wp_list *h_lists,
                      uint64_t nlists, const wp_tune *tune, void **h_plan, void *stream);

/* Decodes every list of the plan on `stream` (asynchronous): one kernel
 * launch, or one hipGraph launch when the plan has a graph. Stream
 * contents are validated as in bp_decode; a bad list is reported through
 * wp_check. Launches of the same plan may overlap only if the caller
 * accepts both writing the same outputs. Allocates nothing. */
int32_t wp_batch_decode(void *h_plan, void *stream);

/* Re-targets an existing plan at a new registry (same meaning as in
 * wp_batch_plan) for callers that plan many small batches, such as a
 * serving loop: the list and item arrays are staged in plan-owned pinned
 * host memory and copied on `stream` without synchronising it, reusing the
 * plan's device arrays (they only grow, with a synchronisation, when the
 * new registry is larger than any before). The plan then uses plain
 * launches (a graph would hold the old item count). The caller enqueues
 * the previous decode of this plan on the same stream or has waited for it. */
int32_t wp_batch_replan(void *h_plan, const uint32_t *pool, uint32_t *out_base, const wp_list *h_lists,
                        uint64_t nlists, void *stream);

/* Number of work items in a plan (host). */
uint64_t wp_batch_items(const void *h_plan);

/* Releases a plan (synchronises the device first, then frees the plan's
 * device arrays and graph). */
int32_t wp_batch_free(void *h_plan);

#ifdef __cplusplus
}
#endif

#endif /* WAVEPACK_H */
