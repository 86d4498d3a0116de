// Encoders: bp_encode, bp_vertical_encode, bp32_encode, fastpfor_encode
// and fastpfor32_encode, producing the stream layout the decoders read (see
// wavepack.h).
//
// SIMD-BP128 and its four-lane layout: one fused launch (k_bp_encode below)
// that reads the input once, then the tail and header. The other codecs,
// four stream-ordered launches:
//   1. analyze: one workgroup per unit computes every block's width(s) and
//      the unit's length in words;
//   2. an in-place inclusive scan of the unit lengths (the chained scan of
//      delta_decode_inplace) gives every unit its offset;
//   3. pack: one workgroup per unit writes its directory entry and data;
//   4. finish: the Variable Byte tail, the header and the stream length.
// Bits are OR-ed into place (LDS atomics for a block's packed words,
// device atomics for a page's exception arrays, after the region has been
// cleared), so the order in which lanes write never matters.
#include <cstddef>
#include <type_traits>

#include "wp_device.hpp"
#include "wp_host.hpp"
#include "wp_lookback.hpp"

namespace wp {

// binary digits of x, ceil(log2(x + 1)) (Section 2); 0 for x = 0
__device__ __forceinline__ uint32_t nbits(uint32_t x) { return 32u - (uint32_t)__clz((int)x); }

// delta of Section 3 at index i (values before the array start count as 0)
__device__ __forceinline__ uint32_t delta_at(const uint32_t *__restrict__ x, uint64_t i, uint32_t S)
{
    const uint32_t v = x[i];
    if (S == 0)
        return v;
    return i >= S ? v - x[i - S] : v;
}

// ORs the low b bits of value i of a block into the block's word string
__device__ __forceinline__ void or_field(uint32_t *w, uint32_t i, uint32_t b, uint32_t v)
{
    if (b == 0)
        return;
    const uint32_t pos = i * b, s = pos & 31u;
    v &= width_mask(b);
    atomicOr(&w[pos >> 5], v << s);
    if (s + b > 32u)
        atomicOr(&w[(pos >> 5) + 1], v >> (32u - s));
}

// A thread's eight consecutive values of a block at b bits are b whole
// bytes of the block's bit string (fields end to end, least significant bit
// first), starting on byte `byte0` of `wb` because the thread's first field
// starts on bit 8 * b * (its index in the block): written with byte stores,
// and no other thread writes those bytes, so no atomics and no clearing.
__device__ __forceinline__ void put_bytes8(uint8_t *wb, uint32_t byte0, uint32_t b, const uint32_t (&d)[8])
{
    const uint32_t m = width_mask(b);
    uint64_t acc = 0;
    uint32_t nbits = 0, o = byte0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        acc |= (uint64_t)(d[r] & m) << nbits;
        nbits += b;
        while (nbits >= 8) {
            wb[o++] = (uint8_t)acc;
            acc >>= 8;
            nbits -= 8;
        }
    }
}

// The same for the four-lane layout of Section 4: value i is field i / 4 of
// 32-bit lane i % 4, the lanes' words interleaved (word w of lane l at 4w + l)
__device__ __forceinline__ void or_field_vertical(uint32_t *w, uint32_t i, uint32_t b, uint32_t v)
{
    if (b == 0)
        return;
    const uint32_t lane = i & 3u, pos = (i >> 2) * b, s = pos & 31u;
    v &= width_mask(b);
    atomicOr(&w[4 * (pos >> 5) + lane], v << s);
    if (s + b > 32u)
        atomicOr(&w[4 * ((pos >> 5) + 1) + lane], v >> (32u - s));
}

// ------------------------------------------------------------------------
// Binary packing (Section 6.2): block width = bits of the OR of its deltas.
//
// One workgroup of 256 threads per meta-block: thread t holds integers
// 8t .. 8t+7 (two 16-byte loads), so block j is the 16 threads of row j of
// the workgroup's wavefronts; the deltas' predecessors come from the
// neighbouring lane, and from memory for a wavefront's first lane.

// Deltas of integers i0 .. i0+7 of the unit starting at integer u0 (full
// blocks only: integers at or beyond `lim` read as 0).
__device__ __forceinline__ void unit_deltas8(const uint32_t *__restrict__ x, uint64_t u0, uint64_t lim, uint32_t S,
                                             uint32_t (&d)[8])
{
    const uint32_t tid = threadIdx.x;
    const uint64_t i0 = u0 + 8ull * tid;
    const uint64_t have = lim > u0 ? lim - u0 : 0;
    const BufRsrc rs = make_rsrc(x + u0, (uint32_t)((have < kBpUnitInts ? have : kBpUnitInts) * 4u));
    const uint4 a = buf_load_u4(rs, tid * 32u), c = buf_load_u4(rs, tid * 32u + 16u);
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
    if (S == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
            d[r] = v[r];
        return;
    }
    // the four integers before i0: the previous lane's last four, or from
    // memory for lane 0 (0 before the array start)
    uint32_t pv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        pv[r] = (uint32_t)__shfl_up((int)v[4 + r], 1, 64);
    if (lane_id() == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            pv[r] = (i0 >= (uint64_t)(4 - r) && i0 - 4 + r < lim) ? x[i0 - 4 + r] : 0u;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint32_t before = S == 1 ? (r == 0 ? pv[3] : v[r - 1]) : (r < 4 ? pv[r] : v[r - 4]);
        d[r] = v[r] - before;
    }
}

// ------------------------------------------------------------------------
// Binary packing in one pass over the input (SIMD-BP128 and its four-lane
// layout). A workgroup of kEncGroups groups of 256 threads takes kEncTile
// consecutive meta-blocks, its tile index from the launch's counter (so a
// tile's predecessors always started first). Thread t of group h = t / 256
// holds integers 8 (t mod 256) .. +7 of the group's kEncHalf meta-blocks in
// registers, all read at once; the widths give every meta-block's length,
// the tile's total goes through the decoupled look-back for the tile's
// offset in the stream, and the tile is assembled in LDS (the descriptor,
// then the blocks' words: byte stores, or fields OR-ed in by LDS atomics
// for the four-lane layout) and written with 16-byte stores (unit offsets
// are multiples of 4 words). The input is read once.
// Tiles of 8 meta-blocks in two groups: the chained scan completes at most
// about 64 tiles per device-scope round trip, which caps smaller tiles;
// larger ones need more registers per thread or more threads per
// workgroup, and leave fewer workgroups per compute unit to overlap one
// tile's loads with another's look-back and writes.
#ifndef WP_ENC_TILE
#define WP_ENC_TILE 8
#endif
constexpr uint32_t kEncTile = WP_ENC_TILE;  // meta-blocks per workgroup
#ifndef WP_ENC_GROUPS
#define WP_ENC_GROUPS 2
#endif
#ifndef WP_ENC_MIN_WAVES
#define WP_ENC_MIN_WAVES 4
#endif
constexpr uint32_t kEncGroups = WP_ENC_GROUPS;     // groups of 256 threads per workgroup
constexpr uint32_t kEncThreads = 256 * kEncGroups;
constexpr uint32_t kEncHalf = kEncTile / kEncGroups;  // meta-blocks per group
// LDS words for the tile's compressed stream (the tiles of compressible
// lists fit; the others are assembled a meta-block per group at a time)
constexpr uint32_t kEncLdsWords = 8192 > kEncGroups * (4 + kBpUnitInts) ? 8192 : kEncGroups * (4 + kBpUnitInts);
static_assert(kEncTile % kEncGroups == 0 && kEncTile <= 64, "whole groups; one look-back lane per meta-block");

template <bool V>
__global__ __launch_bounds__(kEncThreads, WP_ENC_MIN_WAVES) void k_bp_encode(const uint32_t *__restrict__ x, uint64_t n, uint32_t S,
                                                   uint64_t units, uint32_t dir_end, uint32_t *__restrict__ out,
                                                   uint64_t *__restrict__ status, uint32_t *__restrict__ total)
{
    __shared__ __align__(16) uint32_t s_u[kEncLdsWords];  // the tile's stream, or one meta-block per group
    __shared__ uint32_t s_b[kEncTile][kBpBlocks];     // widths
    __shared__ uint32_t s_boff[kEncTile][kBpBlocks];  // a block's first word in its meta-block
    __shared__ uint32_t s_off[kEncTile + 1];          // a meta-block's first word in the tile
    __shared__ uint32_t s_tile, s_pre;
    const uint32_t tid = threadIdx.x;
    const uint32_t h = tid >> 8, t = tid & 255u;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    if (tid == 0)
        s_tile = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long *>(status), 1ull);
    __syncthreads();
    const uint32_t tile = uniform(s_tile);
    const uint64_t u0 = (uint64_t)tile * kEncTile;
    const uint32_t nu = (uint32_t)(units - u0 < kEncTile ? units - u0 : kEncTile);
    const uint64_t lim = (n / kBlock) * kBlock;  // full blocks only
    // every load of the group's meta-blocks first: the thread's eight values
    // and, for the wavefront's first lane, the four before them
    uint32_t d[kEncHalf][8];
    uint32_t pw[kEncHalf][4];  // uniform: the four values before the wavefront's first
    const uint64_t i0w = 512ull * (wave & 3u);  // the wavefront's first integer in its meta-block
    const uint32_t hw = uniform(h);
#pragma unroll
    for (uint32_t m = 0; m < kEncHalf; ++m) {
        const uint64_t base = (u0 + kEncHalf * hw + m) * kBpUnitInts;
        const uint64_t have = lim > base ? lim - base : 0;
        const BufRsrc rs = make_rsrc(x + base, (uint32_t)((have < kBpUnitInts ? have : kBpUnitInts) * 4u));
        const uint4 a = buf_load_u4(rs, t * 32u), c = buf_load_u4(rs, t * 32u + 16u);
        d[m][0] = a.x, d[m][1] = a.y, d[m][2] = a.z, d[m][3] = a.w;
        d[m][4] = c.x, d[m][5] = c.y, d[m][6] = c.z, d[m][7] = c.w;
        const uint64_t iw = base + i0w;
        const bool prev = S != 0 && iw >= 4 && iw <= lim;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            pw[m][r] = prev ? uniform(x[iw - 4 + r]) : 0u;
    }
    if (S != 0) {
#pragma unroll
        for (uint32_t m = 0; m < kEncHalf; ++m) {
            // the four integers before the thread's first: the previous
            // lane's last four (0 before the array start)
            uint32_t pv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                pv[r] = (uint32_t)__shfl_up((int)d[m][4 + r], 1, 64);
            if (lane == 0)
                pv[0] = pw[m][0], pv[1] = pw[m][1], pv[2] = pw[m][2], pv[3] = pw[m][3];
            uint32_t v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                v[r] = d[m][r];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const uint32_t before = S == 1 ? (r == 0 ? pv[3] : v[r - 1]) : (r < 4 ? pv[r] : v[r - 4]);
                d[m][r] = v[r] - before;
            }
        }
    }
    // block widths: OR over the block's 16 threads (one row of 16 lanes)
    const uint32_t j = t >> 4;
#pragma unroll
    for (uint32_t m = 0; m < kEncHalf; ++m) {
        uint32_t o = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            o |= d[m][r];
#pragma unroll
        for (int k = 1; k < 16; k <<= 1)
            o |= (uint32_t)__shfl_xor((int)o, k, 64);
        const uint64_t u = u0 + kEncHalf * hw + m;
        const uint64_t left = lim / kBlock > u * kBpBlocks ? lim / kBlock - u * kBpBlocks : 0;
        const uint32_t nb = (uint32_t)(left < kBpBlocks ? left : kBpBlocks);
        if ((t & 15u) == 0)
            s_b[kEncHalf * h + m][j] = j < nb ? nbits(o) : 0u;
    }
    __syncthreads();
    // each block's first word inside its meta-block (threads 0..255), each
    // meta-block's length, the tile's offset (wavefront 0)
    if (tid < kEncTile * kBpBlocks) {
        const uint32_t mb = tid >> 4, jj = tid & 15u;
        uint32_t pre = 0;
        for (uint32_t q = 0; q < jj; ++q)
            pre += s_b[mb][q];
        s_boff[mb][jj] = 4 + 4 * pre;
    }
    if (wave == 0) {
        uint32_t sz = 0;
        if (lane < nu)
            for (uint32_t q = 0; q < kBpBlocks; ++q)
                sz += s_b[lane][q];
        sz = lane < nu ? 4 + 4 * sz : 0u;
        const uint32_t incl = wave_scan_incl(sz);
        if (lane < kEncTile)
            s_off[lane + 1] = incl;
        if (lane == 0)
            s_off[0] = 0;
        const uint32_t agg[4] = {wave_read(incl, 63), 0, 0, 0};
        uint32_t pre[4];
        wave_lookback<1>(status, tile, agg, 0u, pre);
        if (lane == 0) {
            s_pre = pre[0];
            if (u0 + nu == units)
                *total = pre[0] + agg[0];
        }
    }
    __syncthreads();
    const uint32_t pre = s_pre;
    // directory entries of the tile's meta-blocks: offset, then S bases
    const uint64_t ndir = dir_entries(n, kBpBlocks);
    if (tid < nu * (1 + S)) {
        const uint32_t mb = tid / (1 + S), k = tid % (1 + S);
        const uint64_t u = u0 + mb, start = u * kBpUnitInts;
        if (k == 0)
            out[kHdrWords + u] = dir_end + pre + s_off[mb];
        else
            out[kHdrWords + ndir + u * S + (k - 1)] = (start + (k - 1) >= S) ? x[start + (k - 1) - S] : 0u;
    }
    // meta-block m of the group into `dst` (its descriptor, then its blocks'
    // words: each thread's eight fields are b whole bytes of its block, or
    // are OR-ed into the cleared words in the four-lane layout)
    auto assemble = [&](uint32_t m, uint32_t *dst) __attribute__((always_inline)) {
        const uint32_t mb = kEncHalf * hw + m;
        if (t < 4)
            dst[t] = s_b[mb][4 * t] | (s_b[mb][4 * t + 1] << 8) | (s_b[mb][4 * t + 2] << 16) |
                     (s_b[mb][4 * t + 3] << 24);
        const uint32_t b = s_b[mb][j];
        if (b) {
            uint32_t *const w = dst + s_boff[mb][j];
            if constexpr (V) {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    or_field_vertical(w, 8 * (t & 15u) + r, b, d[m][r]);
            } else {
                put_bytes8(reinterpret_cast<uint8_t *>(w), (t & 15u) * b, b, d[m]);
            }
        }
    };
    const uint32_t tile_words = s_off[nu];
    if (tile_words <= kEncLdsWords) {
        // the whole tile in LDS at once, then one contiguous copy
        if constexpr (V) {
            for (uint32_t i = tid; i < tile_words; i += kEncThreads)
                s_u[i] = 0;
            __syncthreads();
        }
#pragma unroll
        for (uint32_t m = 0; m < kEncHalf; ++m)
            if (kEncHalf * hw + m < nu)
                assemble(m, s_u + s_off[kEncHalf * hw + m]);
        __syncthreads();
        uint4 *const dst = reinterpret_cast<uint4 *>(out + dir_end + pre);
        const uint4 *const src = reinterpret_cast<const uint4 *>(s_u);
        for (uint32_t i = tid; i < tile_words / 4; i += kEncThreads)
            dst[i] = src[i];
        return;
    }
    uint32_t *const su = s_u + hw * (4 + kBpUnitInts);
#pragma unroll
    for (uint32_t m = 0; m < kEncHalf; ++m) {
        const uint32_t mb = kEncHalf * hw + m;
        const bool live = mb < nu;
        const uint32_t size = live ? s_off[mb + 1] - s_off[mb] : 0u;
        if constexpr (V) {
            for (uint32_t i = t; i < size; i += 256)
                su[i] = 0;
            __syncthreads();
        }
        if (live)
            assemble(m, su);
        __syncthreads();
        if (live) {
            uint4 *const dst = reinterpret_cast<uint4 *>(out + dir_end + pre + s_off[mb]);
            const uint4 *const src = reinterpret_cast<const uint4 *>(su);
            for (uint32_t i = t; i < size / 4; i += 256)
                dst[i] = src[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// BP32 (Section 6.2): 32-integer blocks, four per meta-block behind a
// descriptor word of their widths. Same thread layout as above: block k of
// the unit is the four threads 4k .. 4k+3.

__global__ __launch_bounds__(256) void k_bp32_analyze(const uint32_t *__restrict__ x, uint64_t n, uint32_t S,
                                                      uint8_t *__restrict__ widths, uint32_t *__restrict__ sizes)
{
    constexpr uint32_t NB = kBpUnitInts / kB32;
    __shared__ uint32_t s_b[NB];
    const uint64_t u = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint64_t nfull = n / kBlock;
    uint32_t d[8];
    unit_deltas8(x, u * kBpUnitInts, nfull * kBlock, S, d);
    uint32_t o = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r)
        o |= d[r];
    o |= (uint32_t)__shfl_xor((int)o, 1, 64);
    o |= (uint32_t)__shfl_xor((int)o, 2, 64);
    const uint64_t left = nfull - u * kBpBlocks;
    const uint32_t nm = (uint32_t)(left < kBpBlocks ? left : kBpBlocks);  // meta-blocks of the unit
    const uint32_t k = tid >> 2;
    if ((tid & 3u) == 0)
        s_b[k] = k < 4 * nm ? nbits(o) : 0u;
    __syncthreads();
    if (tid < NB)
        widths[u * NB + tid] = (uint8_t)s_b[tid];
    if (tid == 0) {
        uint32_t sum = 0;
        for (uint32_t j = 0; j < NB; ++j)
            sum += s_b[j];
        sizes[u] = (nm + sum + 3u) & ~3u;
    }
}

// The unit is assembled in LDS (each meta-block's descriptor word, then its
// blocks' words, fields OR-ed in by LDS atomics) and written with 16-byte
// stores.
__global__ __launch_bounds__(256) void k_bp32_pack(const uint32_t *__restrict__ x, uint64_t n, uint32_t S,
                                                   const uint8_t *__restrict__ widths,
                                                   const uint32_t *__restrict__ incl, uint32_t dir_end,
                                                   uint32_t *__restrict__ out)
{
    constexpr uint32_t NB = kBpUnitInts / kB32;
    __shared__ __align__(16) uint32_t s_u[kBpBlocks + kBpUnitInts];
    __shared__ uint32_t s_b[NB], s_off[NB];
    const uint64_t u = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - u * kBpBlocks;
    const uint32_t nm = (uint32_t)(left < kBpBlocks ? left : kBpBlocks);
    uint32_t d[8];
    unit_deltas8(x, u * kBpUnitInts, nfull * kBlock, S, d);
    if (tid < NB)
        s_b[tid] = widths[u * NB + tid];
    __syncthreads();
    if (tid < NB) {
        // block k's first word: the descriptors of meta-blocks 0..k/4 and
        // the words of blocks 0..k-1 come before it
        uint32_t pre = 0;
        for (uint32_t j = 0; j < tid; ++j)
            pre += s_b[j];
        s_off[tid] = (tid >> 2) + 1u + pre;
    }
    __syncthreads();
    const uint32_t used = nm ? s_off[4 * nm - 1] + s_b[4 * nm - 1] : 0u;
    const uint32_t size = (used + 3u) & ~3u;
    if (tid < size - used)  // the unit's zero padding
        s_u[used + tid] = 0;
    if (tid < nm)
        s_u[s_off[4 * tid] - 1] =
            s_b[4 * tid] | (s_b[4 * tid + 1] << 8) | (s_b[4 * tid + 2] << 16) | (s_b[4 * tid + 3] << 24);
    const uint32_t k = tid >> 2, b = s_b[k];
    if (b)
        put_bytes8(reinterpret_cast<uint8_t *>(s_u + s_off[k]), (tid & 3u) * b, b, d);
    const uint32_t off = dir_end + incl[u] - size;
    write_dir_entry(out, u, dir_entries(n, kBpBlocks), S, off, x, u * kBpUnitInts);
    __syncthreads();
    uint4 *const dst = reinterpret_cast<uint4 *>(out + off);
    const uint4 *const src = reinterpret_cast<const uint4 *>(s_u);
    for (uint32_t i = tid; i < size / 4; i += 256)
        dst[i] = src[i];
}

// ------------------------------------------------------------------------
// Patched pages (Section 5): per block, the width b minimising
// 128*b + c(b)*(8 + maxb - b) over b in [0, maxb], c(b) = values wider than
// b; among equal costs the largest b (the rule scans b downward from maxb
// and only a strictly smaller cost replaces the current choice).
//
// One wavefront per pair of blocks, four values per lane, each half of the
// wavefront one block: the block's 128 widths go into its own 33-bin LDS
// histogram (eight copies, one per 16-lane row and value slot, so that an
// atomic add meets at most 16 lanes on one bin; a bin's eight copies are
// adjacent, so the wavefront clears both histograms with 16-byte stores and
// lane b of a half reads its bin with two 16-byte loads); lane b of a half
// then holds c(b) (values minus the inclusive prefix of the bins up to b),
// its cost, and one minimum over the half of (cost << 6 | 63 - b) picks the
// width; b = 32 (no exceptions) is the one candidate outside the half's
// lanes, rated when the block has a 32-bit value.

constexpr int kEncDepth = 4;  // block pairs in flight per wavefront in the patched encoder

// Deltas of a pair of consecutive blocks of a page for a wavefront: lane l
// holds integers 4l..4l+3 of the pair (lanes 0..31 the first block, 32..63
// the second), D pairs' loads in flight. Loads go through a buffer
// resource over the page's full blocks, so a block past the page reads as
// zeros; lane 0 takes the four integers before the pair from memory.
template <int D>
struct PairRing {
    uint4 v[D], pv[D];

    template <uint32_t S>
    __device__ __forceinline__ void issue(int d, BufRsrc rs, const uint32_t *__restrict__ x, uint64_t pstart,
                                          uint32_t q, uint32_t lane)
    {
        v[d] = buf_load_u4(rs, (2u * q * kBlock + 4u * lane) * 4u);
        pv[d] = make_uint4(0, 0, 0, 0);
        if (S != 0 && lane == 0) {
            if (q != 0)
                pv[d] = buf_load_u4(rs, (2u * q * kBlock - 4u) * 4u);
            else if (pstart >= 4)
                pv[d] = make_uint4(x[pstart - 4], x[pstart - 3], x[pstart - 2], x[pstart - 1]);
        }
    }

    template <uint32_t S>
    __device__ __forceinline__ void take(int d, uint32_t lane, uint32_t (&dl)[4]) const
    {
        const uint4 a = v[d];
        if constexpr (S == 0) {
            dl[0] = a.x, dl[1] = a.y, dl[2] = a.z, dl[3] = a.w;
        } else if constexpr (S == 1) {
            uint32_t prev = (uint32_t)__shfl_up((int)a.w, 1, 64);
            if (lane == 0)
                prev = pv[d].w;
            dl[0] = a.x - prev, dl[1] = a.y - a.x, dl[2] = a.z - a.y, dl[3] = a.w - a.z;
        } else {
            uint32_t p0 = (uint32_t)__shfl_up((int)a.x, 1, 64), p1 = (uint32_t)__shfl_up((int)a.y, 1, 64);
            uint32_t p2 = (uint32_t)__shfl_up((int)a.z, 1, 64), p3 = (uint32_t)__shfl_up((int)a.w, 1, 64);
            if (lane == 0)
                p0 = pv[d].x, p1 = pv[d].y, p2 = pv[d].z, p3 = pv[d].w;
            dl[0] = a.x - p0, dl[1] = a.y - p1, dl[2] = a.z - p2, dl[3] = a.w - p3;
        }
    }
};

// Page tables of a patched page for the packer. The per-block tables are
// dead once the block records are built; `room` sizes the union so that
// the packer's metadata and exception area, which runs on over the tables,
// holds 32 KB.
template <int WAVES>
struct FpLds {
    union {
        uint32_t room[WAVES][4 * kBlock + 4];
        struct {
            uint8_t b[kFpBlocks];
            uint8_t mb[kFpBlocks];
            uint8_t c[kFpBlocks];
            uint32_t blkoff[kFpBlocks + 1];  // word offset of each block in the packed region
            uint32_t posoff[kFpBlocks + 1];  // offset of each block's positions
            uint32_t rank[kFpBlocks];        // index of the block's first exception in its array
        };
    };
    // per block: {b | k << 8, packed word offset, bit offset of its first
    // exception's high part, position offset}
    uint4 rec[kFpBlocks + 8 * WAVES];
    uint32_t ktot[WAVES][33];
    uint32_t kcar[33];
    uint32_t excbase[33];            // word offset of array k from the page start
    uint32_t kcnt[33];
    uint32_t stot[WAVES][2];
};

// Tables of a patched page from its per-block metadata L.b, L.mb, L.c
// (entries from nb to the end of its last round of T blocks hold 0): block
// offsets in the packed region (exclusive sum of 4*b), offsets into the position bytes
// (exclusive sum of c) and, per block, the index of its first exception in
// array k = maxb - b -- exceptions are appended to their array in block
// order (Section 5), so this is the number of exceptions of earlier blocks
// with the same k. Per-k totals accumulate in L.kcar (zeroed by the caller,
// as is L.ktot). Rounds of T blocks; within a wavefront the same-k ranks
// come from one masked scan per distinct k (ballot loop).
template <int WAVES>
__device__ __forceinline__ void fp_tables(FpLds<WAVES> &L, uint32_t nb, uint32_t &tot_words, uint32_t &tot_pos)
{
    constexpr int T = 64 * WAVES;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    uint32_t carry_w = 0, carry_p = 0;
    for (uint32_t r0 = 0; r0 < nb; r0 += T) {
        const uint32_t t = r0 + tid;
        const uint32_t bw = 4u * L.b[t];
        const uint32_t cc = L.c[t];
        const uint32_t kk = (uint32_t)L.mb[t] - (uint32_t)L.b[t];
        const uint32_t iw = wave_scan_incl(bw);
        const uint32_t ip = wave_scan_incl(cc);
        if (lane == 63) {
            L.stot[wave][0] = iw;
            L.stot[wave][1] = ip;
        }
        // rank among the wave's earlier blocks of the same k
        uint32_t rk = 0;
        uint64_t todo = ballot(cc > 0);
        while (todo) {
            const uint32_t lead = (uint32_t)__builtin_ctzll(todo);
            const uint32_t k0 = wave_read(kk, lead);
            const bool mine = cc > 0 && kk == k0;
            const uint64_t mm = ballot(mine);
            const uint32_t x = mine ? cc : 0u;
            const uint32_t incl = wave_scan_incl(x);
            if (mine)
                rk = incl - x;
            if (lane == 0)
                L.ktot[wave][k0 > 32 ? 0 : k0] = wave_read(incl, 63);
            todo &= ~mm;
        }
        __syncthreads();
        uint32_t bw_before = carry_w, p_before = carry_p, all_w = 0, all_p = 0, k_before = 0;
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t a = L.stot[w][0], c2 = L.stot[w][1];
            if (w < (int)wave) {
                bw_before += a;
                p_before += c2;
            }
            all_w += a;
            all_p += c2;
        }
        if (cc > 0 && kk <= 32) {
            k_before = L.kcar[kk];
            for (int w = 0; w < (int)wave; ++w)
                k_before += L.ktot[w][kk];
        }
        L.blkoff[t] = bw_before + iw - bw;
        L.posoff[t] = p_before + ip - cc;
        L.rank[t] = k_before + rk;
        carry_w += all_w;
        carry_p += all_p;
        __syncthreads();
        if (tid < 33) {
            uint32_t s = 0;
            for (int w = 0; w < WAVES; ++w) {
                s += L.ktot[w][tid];
                L.ktot[w][tid] = 0;
            }
            L.kcar[tid] += s;
        }
        __syncthreads();
    }
    tot_words = carry_w;
    tot_pos = carry_p;
}

// Inclusive sum and minimum over each half of the wavefront (lanes 0..31,
// 32..63): row steps, then row 1 (3) takes row 0's (2's) last lane.
__device__ __forceinline__ uint32_t half_scan_incl(uint32_t v)
{
    v = row_scan_incl(v);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    return v;
}

__device__ __forceinline__ uint32_t half_min_at_ends(uint32_t v)  // lane 31: min of 0..31, lane 63: of 32..63
{
    constexpr uint32_t kId = 0xffffffffu;
    auto step = [&](uint32_t o) __attribute__((always_inline)) { v = o < v ? o : v; };
    step(__builtin_amdgcn_update_dpp(kId, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    step(__builtin_amdgcn_update_dpp(kId, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    step(__builtin_amdgcn_update_dpp(kId, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    step(__builtin_amdgcn_update_dpp(kId, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    step(__builtin_amdgcn_update_dpp(kId, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    return v;
}

// With SPW (SimplePFOR pages), block k's exceptions' high-part widths also
// go to spx[k * kSpWidthSlot ...], in position order.
template <bool P32, uint32_t S, bool SPW>
__device__ __forceinline__ void fp_analyze(const uint32_t *__restrict__ x, uint64_t n, uint8_t *__restrict__ meta,
                                           uint64_t nblk, uint32_t *__restrict__ sizes, uint8_t *__restrict__ spx)
{
    __shared__ uint32_t s_cnt[33];
    // per wavefront and block of the pair: bin w's eight copies at 8w .. 8w + 7
    __shared__ __align__(16) uint32_t s_hist[8][2][8 * 33];
    __shared__ uint32_t s_pw, s_pc;
    const uint64_t p = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - p * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    if (tid < 33)
        s_cnt[tid] = 0;
    if (tid == 0)
        s_pw = 0, s_pc = 0;
    __syncthreads();
    const uint32_t half = lane >> 5, b_l = lane & 31u;  // the lane's block of the pair; the width it rates
    uint32_t *const h = s_hist[wave][half];
    uint4 *const h4all = reinterpret_cast<uint4 *>(s_hist[wave][0]);  // both histograms, 132 groups of four
    const uint4 *const h4 = reinterpret_cast<const uint4 *>(h);
    // per-wavefront sums, added to the page's once at the end: packed
    // words, exceptions, and (lane k) exceptions of width difference k
    uint32_t acc_pw = 0, acc_pc = 0, acc_k = 0;
    const uint64_t pstart = p * kFpUnitInts;
    const BufRsrc rs = make_rsrc(x + pstart, nb * kBlock * 4u);
    const uint32_t npair = (nb + 1) / 2;
    // the wavefront takes pairs wave, wave + 8, ...; kEncDepth of them in flight
    constexpr int D = kEncDepth;
    PairRing<D> ring;
#pragma unroll
    for (int d = 0; d < D; ++d)
        ring.template issue<S>(d, rs, x, pstart, wave + 8u * d, lane);
    for (uint32_t q0 = wave; q0 < npair; q0 += 8u * D)
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t q = q0 + 8u * d;
        if (q >= npair)
            break;
        uint32_t dl[4];
        ring.template take<S>(d, lane, dl);
        ring.template issue<S>(d, rs, x, pstart, q + 8u * D, lane);
        h4all[lane] = make_uint4(0, 0, 0, 0);
        h4all[64 + lane] = make_uint4(0, 0, 0, 0);
        if (lane < 4)
            h4all[128 + lane] = make_uint4(0, 0, 0, 0);
        wave_lds_order();
        const uint32_t copy = 4u * ((lane >> 4) & 1u);
        bool w32 = false;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t w = nbits(dl[c]);
            w32 = w32 || w == 32u;
            atomicAdd(&h[8 * w + copy + c], 1u);
        }
        wave_lds_order();
        const uint4 g0 = h4[2 * b_l], g1 = h4[2 * b_l + 1];
        const uint32_t hb = (g0.x + g0.y) + (g0.z + g0.w) + (g1.x + g1.y) + (g1.z + g1.w);  // values of width b_l
        const uint64_t used = ballot(hb != 0), wide = ballot(w32);
        // widest value of each block: 32 if some value needs 32 bits
        const uint32_t uA = (uint32_t)used, uB = (uint32_t)(used >> 32);
        const uint32_t mA = (uint32_t)wide ? 32u : 31u - (uint32_t)__builtin_clz(uA | 1u);
        const uint32_t mB = (uint32_t)(wide >> 32) ? 32u : 31u - (uint32_t)__builtin_clz(uB | 1u);
        const uint32_t maxb = half ? mB : mA;
        const uint32_t c = kBlock - half_scan_incl(hb);  // values wider than b_l
        const uint32_t cost = kBlock * b_l + c * (8u + maxb - b_l);
        const uint32_t key = half_min_at_ends(b_l <= maxb ? (cost << 6) | (63u - b_l) : 0xffffffffu);
        constexpr uint32_t kKey32 = ((kBlock * 32u) << 6) | (63u - 32u);  // b = 32: no exceptions
        uint32_t kA = wave_read(key, 31), kB = wave_read(key, 63);
        kA = mA == 32u && kKey32 < kA ? kKey32 : kA;
        kB = mB == 32u && kKey32 < kB ? kKey32 : kB;
        const uint32_t bA = 63u - (kA & 63u), bB = 63u - (kB & 63u);
        const uint32_t cA = bA == 32u ? 0u : wave_read(c, (int)bA);
        const uint32_t cB = bB == 32u ? 0u : wave_read(c, 32 + (int)(bB & 31u));
        const uint32_t t = 2u * q;
        const bool liveB = t + 1 < nb;
        const uint64_t blk = p * kFpBlocks + t;
        if (lane == 0 || (lane == 32 && liveB)) {
            const uint64_t bk = blk + half;
            meta[bk] = (uint8_t)(half ? bB : bA);
            meta[nblk + bk] = (uint8_t)(half ? mB : mA);
            meta[2 * nblk + bk] = (uint8_t)(half ? cB : cA);
        }
        if constexpr (SPW) {
            // the lane's exceptions, ranked within its block (lanes of a half
            // hold the block's values in order)
            const uint32_t b = half ? bB : bA;
            uint32_t em = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                em |= (nbits(dl[k]) > b ? 1u : 0u) << k;
            if (half && !liveB)
                em = 0;
            const uint32_t ce = (uint32_t)__builtin_popcount(em);
            uint32_t at = half_scan_incl(ce) - ce;  // < 102: the cost rule's bound
            uint8_t *const slot = spx + (blk + half) * kSpWidthSlot;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((em >> k) & 1u)
                    slot[at++] = (uint8_t)(nbits(dl[k]) - b);
        }
        acc_pw += 4 * bA + (liveB ? 4 * bB : 0u);
        acc_pc += cA + (liveB ? cB : 0u);
        acc_k += (lane == mA - bA ? cA : 0u) + (liveB && lane == mB - bB ? cB : 0u);
        wave_lds_order();
    }
    if (lane == 0) {
        atomicAdd(&s_pw, acc_pw);
        atomicAdd(&s_pc, acc_pc);
    }
    if (lane < 33 && acc_k)
        atomicAdd(&s_cnt[lane], acc_k);
    __syncthreads();
    if (tid == 0) {
        uint32_t nset = 0, exc_w = 0;
        for (uint32_t k = 1; k <= 32; ++k)
            if (s_cnt[k]) {
                ++nset;
                exc_w += exc_array_words<P32>(s_cnt[k], k);
            }
        const uint32_t meta_bytes = 3 * nb + s_pc;
        const uint32_t nsb = S * (page_items<kPageFp>(nb) - 1);  // segment bases
        sizes[p] = pad4(pad4(4 + nset + nsb) + s_pw + ((meta_bytes + 15) / 16) * 4 + exc_w);
    }
}

template <bool P32, uint32_t S>
__global__ __launch_bounds__(512) void k_fp_analyze(const uint32_t *__restrict__ x, uint64_t n,
                                                    uint8_t *__restrict__ meta, uint64_t nblk,
                                                    uint32_t *__restrict__ sizes)
{
    fp_analyze<P32, S, false>(x, n, meta, nblk, sizes, nullptr);
}

// The SimplePFOR form; strides 0 and 1 fit eight wavefronts per SIMD
// without spilling (stride 4 does not).
template <uint32_t S>
__global__ __launch_bounds__(512) void k_sp_analyze(const uint32_t *__restrict__ x, uint64_t n,
                                                    uint8_t *__restrict__ meta, uint64_t nblk,
                                                    uint32_t *__restrict__ sizes, uint8_t *__restrict__ spx)
{
    fp_analyze<false, S, true>(x, n, meta, nblk, sizes, spx);
}
template <uint32_t S>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8))) void k_sp_analyze8(
    const uint32_t *__restrict__ x, uint64_t n, uint8_t *__restrict__ meta, uint64_t nblk,
    uint32_t *__restrict__ sizes, uint8_t *__restrict__ spx)
{
    fp_analyze<false, S, true>(x, n, meta, nblk, sizes, spx);
}

// LDS staging of a page's metadata and exception arrays in k_fp_pack
// k_fp_pack's LDS, one buffer: the wavefronts' block areas (8 KB), then the
// page's metadata and exception arrays, whose area runs on over the page
// tables of FpLds (dead once the block records exist) up to the records:
// 51 KB in all, three workgroups per compute unit
constexpr uint32_t kPackSwBytes = 8u * 2u * kBlock * 4u;
constexpr uint32_t kPackTailLead = 16384;
constexpr uint32_t kPackTailWords = (kPackTailLead + (uint32_t)offsetof(FpLds<8>, rec)) / 4u;
static_assert(kPackTailWords >= 8192, "the metadata and exception area holds 32 KB");
static_assert((kPackSwBytes + kPackTailLead) % 16 == 0, "the page tables stay 16-byte aligned");

template <bool P32, uint32_t S>
__global__ __launch_bounds__(512) void k_fp_pack(const uint32_t *__restrict__ x, uint64_t n,
                                                 const uint8_t *__restrict__ meta, uint64_t nblk,
                                                 const uint32_t *__restrict__ incl, uint32_t dir_end,
                                                 uint32_t *__restrict__ out)
{
    __shared__ __align__(16) uint8_t s_raw[kPackSwBytes + kPackTailLead + sizeof(FpLds<8>)];
    uint32_t *const sw_all = reinterpret_cast<uint32_t *>(s_raw);  // 2 * kBlock words per wavefront
    uint32_t *const s_tail = reinterpret_cast<uint32_t *>(s_raw + kPackSwBytes);
    FpLds<8> &L = *reinterpret_cast<FpLds<8> *>(s_raw + kPackSwBytes + kPackTailLead);
    constexpr int T = 512;
    static_assert(T == kFpBlocks, "one block's metadata per thread");
    const uint64_t p = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - p * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    // block tid's metadata, kept in registers for the metadata bytes
    const bool my_in = tid < nb;
    const uint8_t my_b = my_in ? meta[p * kFpBlocks + tid] : 0;
    const uint8_t my_mb = my_in ? meta[nblk + p * kFpBlocks + tid] : 0;
    const uint8_t my_c = my_in ? meta[2 * nblk + p * kFpBlocks + tid] : 0;
    L.b[tid] = my_b;
    L.mb[tid] = my_mb;
    L.c[tid] = my_c;
    for (uint32_t i = tid; i < 8 * 33; i += T)
        (&L.ktot[0][0])[i] = 0;
    if (tid < 33)
        L.kcar[tid] = 0;
    __syncthreads();
    uint32_t packed_words = 0, npos = 0;
    fp_tables<8>(L, nb, packed_words, npos);
    // per-k counts are in L.kcar; exception array offsets from the page start
    uint32_t bitset = 0;
    for (uint32_t k = 1; k <= 32; ++k)
        bitset |= L.kcar[k] ? (1u << (k - 1)) : 0u;
    const uint32_t nset = __builtin_popcount(bitset);
    const uint32_t nsb = S * (page_items<kPageFp>(nb) - 1);  // segment bases after the counts
    const uint32_t hdr_w = pad4(4 + nset + nsb);
    const uint32_t meta_bytes = 3 * nb + npos;
    const uint32_t meta_w = ((meta_bytes + 15) / 16) * 4;
    const uint32_t exc_at = hdr_w + packed_words + meta_w;
    if (wave == 0) {
        const uint32_t k = lane + 1;
        const uint32_t cnt = lane < 32 ? L.kcar[k] : 0u;
        const uint32_t wk = exc_array_words<P32>(cnt, k);
        const uint32_t incl_k = wave_scan_incl(wk);
        if (lane < 32)
            L.excbase[k] = exc_at + incl_k - wk;
        if (lane == 63)
            L.kcnt[0] = pad4(exc_at + incl_k);  // page length in words
    }
    __syncthreads();
    const uint32_t size = L.kcnt[0];
    // one record per block, read by the packing wavefront with one load:
    // {b | k << 8, word offset in the packed region, bit offset of its first
    // exception's high part from the end of the packed region, offset of its
    // positions}; visible after the barrier that opens the assembly below
    for (uint32_t t = tid; t < nb; t += T) {
        const uint32_t b = L.b[t], k = (uint32_t)L.mb[t] - b;
        const uint32_t ebit = k ? (L.excbase[k <= 32 ? k : 0] - (hdr_w + packed_words)) * 32u + L.rank[t] * k : 0u;
        L.rec[t] = make_uint4(b | (k << 8), L.blkoff[t], ebit, L.posoff[t]);
    }
    const uint32_t off = dir_end + incl[p] - size;
    write_dir_entry(out, p, dir_entries(n, kFpBlocks), S, off, x, p * kFpUnitInts);
    uint32_t *page = out + off;
    if (tid == 0) {
        page[0] = nb;
        page[1] = packed_words;
        page[2] = meta_bytes;
        page[3] = bitset;
    }
    if (tid >= 32 && tid < 64) {  // counts of the non-empty arrays, k ascending
        const uint32_t k = tid - 31;
        if ((bitset >> (k - 1)) & 1u)
            page[4 + __builtin_popcount(bitset & ((1u << (k - 1)) - 1u))] = L.kcar[k];
    }
    if constexpr (S > 0) {
        // segment g >= 1: the S input values just before its first integer
        if (tid >= 128 && tid - 128 < nsb) {
            const uint32_t i = tid - 128, g = 1 + i / S, t = i % S;
            page[4 + nset + i] = x[p * kFpUnitInts + g * kSegInts - S + t];
        }
    }
    if (tid >= 64 && tid - 64 >= 4 + nset + nsb && tid - 64 < hdr_w)
        page[tid - 64] = 0;
    // The metadata bytes and exception arrays (words tail0 .. size of the
    // page) are assembled with byte stores and ORs: in LDS when they fit,
    // then written out with 16-byte stores; otherwise in place in HBM after
    // clearing it (device atomics).
    const uint32_t tail0 = hdr_w + packed_words;  // a multiple of 4
    const uint32_t tail_w = size - tail0;         // a multiple of 4
    uint32_t *const sw = sw_all + wave * (2 * kBlock);
    // the wavefront takes blocks wave, wave + 8, ...; kEncDepth of them in flight
    constexpr int D = kEncDepth;
    auto assemble = [&](auto in_lds_tag) __attribute__((always_inline)) {
        constexpr bool IN_LDS = decltype(in_lds_tag)::value;
        uint32_t *const tw = IN_LDS ? s_tail : page + tail0;
        for (uint32_t i = tid; i < tail_w; i += T)
            tw[i] = 0;
        if constexpr (!IN_LDS)
            __threadfence();
        __syncthreads();
        uint8_t *const mbytes = reinterpret_cast<uint8_t *>(tw);
        if (my_in) {
            mbytes[tid] = my_b;
            mbytes[nb + tid] = my_mb;
            mbytes[2 * nb + tid] = my_c;
        }
        // a wavefront packs two blocks per pass, four integers per lane, each
        // half of the wavefront one block into its half of the block area
        const uint64_t pstart = p * kFpUnitInts;
        const BufRsrc rs = make_rsrc(x + pstart, nb * kBlock * 4u);
        const uint32_t npair = (nb + 1) / 2;
        const uint32_t half = lane >> 5, ql = lane & 31u;
        PairRing<D> ring;
#pragma unroll
        for (int d = 0; d < D; ++d)
            ring.template issue<S>(d, rs, x, pstart, wave + 8u * d, lane);
        for (uint32_t i = lane; i < 2 * kBlock; i += 64)  // the block words start cleared
            sw[i] = 0;
        wave_lds_order();
        uint32_t *const swh = sw + half * kBlock;
        for (uint32_t q0 = wave; q0 < npair; q0 += 8u * D)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const uint32_t q = q0 + 8u * d;
            if (q >= npair)
                break;
            uint32_t dl[4];
            ring.template take<S>(d, lane, dl);
            ring.template issue<S>(d, rs, x, pstart, q + 8u * D, lane);
            const uint32_t t = 2u * q + half;  // the lane's block
            const bool live = t < nb;
            const uint4 rc = live ? L.rec[t] : make_uint4(0, 0, 0, 0);
            const uint32_t b = rc.x & 255u, k = rc.x >> 8;
            bool e[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                or_field(swh, 4 * ql + c, b, dl[c]);
                e[c] = live && nbits(dl[c]) > b;
            }
            // exceptions of the block before this lane's: those of the lanes
            // below it in its half, then its own earlier ones
            const uint64_t m0 = ballot(e[0]), m1 = ballot(e[1]), m2 = ballot(e[2]), m3 = ballot(e[3]);
            const uint32_t in_a = __builtin_popcount((uint32_t)m0) + __builtin_popcount((uint32_t)m1) +
                                  __builtin_popcount((uint32_t)m2) + __builtin_popcount((uint32_t)m3);
            uint32_t idx = lanes_below(m0) + lanes_below(m1) + lanes_below(m2) + lanes_below(m3) - (half ? in_a : 0u);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (e[c]) {
                    mbytes[3 * nb + rc.w + idx] = (uint8_t)(4 * ql + c);
                    const uint32_t hv = dl[c] >> b;
                    const uint32_t bit = rc.z + idx * k, sh = bit & 31u;
                    atomicOr(&tw[bit >> 5], hv << sh);
                    if (sh + k > 32u)
                        atomicOr(&tw[(bit >> 5) + 1], hv >> (32u - sh));
                    ++idx;
                }
            }
            wave_lds_order();
            if (live && ql < b) {  // the block's 4b words as b 16-byte stores
                uint4 *const sw4 = reinterpret_cast<uint4 *>(swh);
                reinterpret_cast<uint4 *>(page + hdr_w + rc.y)[ql] = sw4[ql];
                sw4[ql] = make_uint4(0, 0, 0, 0);  // cleared for the wavefront's next pass
            }
            wave_lds_order();
        }
        if constexpr (IN_LDS) {
            __syncthreads();
            uint4 *const dst = reinterpret_cast<uint4 *>(page + tail0);
            const uint4 *const src = reinterpret_cast<const uint4 *>(s_tail);
            for (uint32_t i = tid; i < tail_w / 4; i += T)
                dst[i] = src[i];
        }
    };
    __syncthreads();  // the page tables are read; the metadata area may overwrite them
    if (tail_w <= kPackTailWords)
        assemble(std::true_type{});
    else
        assemble(std::false_type{});
}

// ------------------------------------------------------------------------
// Tail (Variable Byte, Section 2.4), directory padding, header, length.

__global__ __launch_bounds__(128) void k_finish(const uint32_t *__restrict__ x, uint64_t n, uint32_t S,
                                                uint32_t codec, const uint32_t *__restrict__ units_words, uint64_t units,
                                                uint32_t dir_end, uint32_t *__restrict__ out,
                                                uint64_t *__restrict__ out_words)
{
    __shared__ uint32_t s_bytes[(kMaxTailBytes + 3) / 4 + 1];
    __shared__ uint32_t s_tot[2];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint64_t nfull = n / kBlock;
    const uint32_t tail = (uint32_t)(n % kBlock);
    const uint32_t E = 1 + S;
    const uint64_t ndir = units + (tail ? 1 : 0);
    const uint32_t tail_off = units ? dir_end + *units_words : dir_end;
    for (uint32_t i = tid; i < sizeof(s_bytes) / 4; i += 128)
        s_bytes[i] = 0;
    const uint32_t d = tid < tail ? delta_at(x, nfull * kBlock + tid, S) : 0u;
    const uint32_t nb7 = (nbits(d) + 6) / 7;
    const uint32_t len = tid < tail ? (nb7 ? nb7 : 1u) : 0u;
    const uint32_t inc = wave_scan_incl(len);
    if (lane == 63)
        s_tot[wave] = inc;
    __syncthreads();
    const uint32_t at = inc - len + (wave ? s_tot[0] : 0u);
    const uint32_t tail_bytes = s_tot[0] + s_tot[1];
    uint8_t *sb = reinterpret_cast<uint8_t *>(s_bytes);
    for (uint32_t k = 0; k < len; ++k)
        sb[at + k] = (uint8_t)(((d >> (7 * k)) & 127u) | (k + 1 == len ? 128u : 0u));
    __syncthreads();
    for (uint32_t i = tid; i < (tail_bytes + 3) / 4; i += 128)
        out[tail_off + i] = s_bytes[i];
    if (tail)
        write_dir_entry(out, units, ndir, S, tail_off, x, nfull * kBlock);
    for (uint64_t i = kHdrWords + ndir * E + tid; i < dir_end; i += 128)
        out[i] = 0;
    const uint32_t total = tail_off + (tail_bytes + 3) / 4;
    if (tid == 0) {
        out[0] = codec == WP_CODEC_BP     ? kMagicBP
                 : codec == WP_CODEC_BPV  ? kMagicBPV
                 : codec == WP_CODEC_BP32 ? kMagicBP32
                 : codec == WP_CODEC_FP32 ? kMagicFP32
                 : codec == WP_CODEC_SP   ? kMagicSP
                                          : kMagicFP;
        out[1] = (uint32_t)n;
        out[2] = (uint32_t)(n >> 32);
        out[3] = S;
        out[4] = (uint32_t)units;
        out[5] = tail_bytes;
        out[6] = tail_off;
        out[7] = total;
        *out_words = total;
    }
}

// the patched encoders for a stride known at compile time
#define WP_FP_ENC(kern, p32, args)                                                                         \
    do {                                                                                                   \
        if (stride == 0)                                                                                   \
            hipLaunchKernelGGL((kern<p32, 0u>), dim3((uint32_t)units), dim3(512), 0, st, WP_UNPAREN args); \
        else if (stride == 1)                                                                              \
            hipLaunchKernelGGL((kern<p32, 1u>), dim3((uint32_t)units), dim3(512), 0, st, WP_UNPAREN args); \
        else                                                                                               \
            hipLaunchKernelGGL((kern<p32, 4u>), dim3((uint32_t)units), dim3(512), 0, st, WP_UNPAREN args); \
    } while (0)
#define WP_UNPAREN(...) __VA_ARGS__

// Scratch bytes an encode call of `codec` over n integers uses: scan
// status, unit sizes, per-block metadata (and the SimplePFOR pages' word
// starts).
// Look-back status words of an encode call: the chained scan of the unit
// sizes, or the fused binary-packing encoder's tiles.
static uint64_t encode_status_words(int codec, uint64_t units)
{
    if (codec == WP_CODEC_BP || codec == WP_CODEC_BPV)
        return (uint64_t)kStatusWords * ((units + kEncTile - 1) / kEncTile + 1);
    return scan_status_words(units);
}

static uint64_t encode_scratch_bytes(int codec, uint64_t n)
{
    const bool paged = codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP;
    const uint64_t per = paged ? kFpBlocks : kBpBlocks;
    const uint64_t units = (n / kBlock + per - 1) / per;
    const uint64_t nblk = units * per;
    const uint64_t meta_off = encode_status_words(codec, units) * 8 + ((units * 4 + 255) & ~255ull);
    const uint64_t meta_len = (codec == WP_CODEC_BP || codec == WP_CODEC_BPV) ? nblk
                              : codec == WP_CODEC_BP32                      ? 4 * nblk
                                                                            : 3 * nblk;
    const uint64_t sp_len = codec == WP_CODEC_SP ? sp_scratch_bytes(units) + nblk * kSpWidthSlot : 0;
    return ((meta_off + meta_len + 255) & ~255ull) + sp_len + 256;
}

static int32_t encode_common(int codec, const uint32_t *in, uint64_t n, int32_t stride, uint32_t *out,
                             uint64_t cap, uint64_t *out_words, void *stream)
{
    if (stride != 0 && stride != 1 && stride != 4)
        return WP_ERR_INVALID_ARG;
    if (out == nullptr || out_words == nullptr || (n > 0 && in == nullptr))
        return WP_ERR_INVALID_ARG;
    if (!aligned16(out) || (reinterpret_cast<uintptr_t>(in) & 3u) || (reinterpret_cast<uintptr_t>(out_words) & 7u))
        return WP_ERR_INVALID_ARG;
    const uint64_t need = wp_max_compressed_words(codec, n);
    if (need == 0)
        return WP_ERR_INVALID_ARG;
    if (cap < need)
        return WP_ERR_CAPACITY;
    const bool paged = codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP;
    const uint64_t per = paged ? kFpBlocks : kBpBlocks;
    const uint64_t nfull = n / kBlock;
    const uint64_t units = (nfull + per - 1) / per;
    const uint64_t E = 1 + (uint64_t)stride;
    const uint64_t ndir = units + ((n % kBlock) ? 1 : 0);
    const uint32_t dir_end = (uint32_t)(kHdrWords + ((E * ndir + 3) & ~3ull));
    hipStream_t st = as_stream(stream);
    // scratch: scan status | unit sizes | per-block metadata
    const uint64_t status_words = encode_status_words(codec, units);
    const uint64_t sizes_off = status_words * 8;
    const uint64_t meta_off = sizes_off + ((units * 4 + 255) & ~255ull);
    const uint64_t nblk = units * per;
    char *scr = static_cast<char *>(stream_scratch(st, encode_scratch_bytes(codec, n)));
    if (scr == nullptr)
        return WP_ERR_HIP;
    uint64_t *status = reinterpret_cast<uint64_t *>(scr);
    uint32_t *sizes = reinterpret_cast<uint32_t *>(scr + sizes_off);
    uint8_t *meta = reinterpret_cast<uint8_t *>(scr + meta_off);
    const uint64_t meta_len = codec == WP_CODEC_BP32 ? 4 * nblk : 3 * nblk;
    uint8_t *spw = reinterpret_cast<uint8_t *>(scr + ((meta_off + meta_len + 255) & ~255ull));
    uint8_t *spx = spw + sp_scratch_bytes(units);  // SimplePFOR: exception widths per block
    (void)hipGetLastError();
    // the units' total length in words, for the tail's offset
    const uint32_t *units_words = sizes + (units ? units - 1 : 0);
    if (units && (codec == WP_CODEC_BP || codec == WP_CODEC_BPV)) {
        const uint64_t tiles = (units + kEncTile - 1) / kEncTile;
        if (tiles > 0x7FFFFFFFull)
            return WP_ERR_INVALID_ARG;
        launch_clear(status, status_words, st);
        if (codec == WP_CODEC_BP)
            hipLaunchKernelGGL(k_bp_encode<false>, dim3((uint32_t)tiles), dim3(kEncThreads), 0, st, in, n, (uint32_t)stride,
                               units, dir_end, out, status, sizes);
        else
            hipLaunchKernelGGL(k_bp_encode<true>, dim3((uint32_t)tiles), dim3(kEncThreads), 0, st, in, n, (uint32_t)stride,
                               units, dir_end, out, status, sizes);
        units_words = sizes;
    } else if (units) {
        if (codec == WP_CODEC_BP32)
            hipLaunchKernelGGL(k_bp32_analyze, dim3((uint32_t)units), dim3(256), 0, st, in, n, (uint32_t)stride,
                               meta, sizes);
        else if (codec == WP_CODEC_FP32)
            WP_FP_ENC(k_fp_analyze, true, (in, n, meta, nblk, sizes));
        else if (codec == WP_CODEC_FP)
            WP_FP_ENC(k_fp_analyze, false, (in, n, meta, nblk, sizes));
        else if (stride == 0)
            hipLaunchKernelGGL((k_sp_analyze8<0u>), dim3((uint32_t)units), dim3(512), 0, st, in, n, meta, nblk, sizes,
                               spx);
        else if (stride == 1)
            hipLaunchKernelGGL((k_sp_analyze8<1u>), dim3((uint32_t)units), dim3(512), 0, st, in, n, meta, nblk, sizes,
                               spx);
        else
            hipLaunchKernelGGL((k_sp_analyze<4u>), dim3((uint32_t)units), dim3(512), 0, st, in, n, meta, nblk, sizes,
                               spx);
        if (codec == WP_CODEC_SP) {
            // widths and counts as for patched pages; the page sizes depend
            // on the Simple-8b coding
            if (sp_encode_units(in, n, (uint32_t)stride, units, meta, nblk, sizes, status, spw, spx, dir_end, out, st) !=
                WP_OK)
                return WP_ERR_HIP;
        } else if (launch_inclusive_scan(sizes, units, status, st) != WP_OK)
            return WP_ERR_HIP;
        if (codec == WP_CODEC_BP32)
            hipLaunchKernelGGL(k_bp32_pack, dim3((uint32_t)units), dim3(256), 0, st, in, n, (uint32_t)stride, meta,
                               sizes, dir_end, out);
        else if (codec == WP_CODEC_FP32)
            WP_FP_ENC(k_fp_pack, true, (in, n, meta, nblk, sizes, dir_end, out));
        else if (codec == WP_CODEC_FP)
            WP_FP_ENC(k_fp_pack, false, (in, n, meta, nblk, sizes, dir_end, out));
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(128), 0, st, in, n, (uint32_t)stride, (uint32_t)codec, units_words, units,
                       dir_end, out, out_words);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

}  // namespace wp

using namespace wp;

extern "C" int32_t bp_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                             uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_BP, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t bp_vertical_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                                      uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_BPV, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t bp32_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                               uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_BP32, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t fastpfor32_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                                     uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_FP32, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t fastpfor_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                                   uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_FP, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t simplepfor_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                                     uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    return encode_common(WP_CODEC_SP, in, n, delta_stride, out, out_cap_words, out_words, stream);
}

extern "C" int32_t fastpfor_inline_encode(const uint32_t *in, uint64_t n, int32_t delta_stride, uint32_t *out,
                                          uint64_t out_cap_words, uint64_t *out_words, void *stream)
{
    if (delta_stride != 0 && delta_stride != 1 && delta_stride != 4)
        return WP_ERR_INVALID_ARG;
    if (out == nullptr || out_words == nullptr || (n > 0 && in == nullptr))
        return WP_ERR_INVALID_ARG;
    if (!aligned16(out) || (reinterpret_cast<uintptr_t>(in) & 3u) || (reinterpret_cast<uintptr_t>(out_words) & 7u))
        return WP_ERR_INVALID_ARG;
    const uint64_t need = wp_max_compressed_words(WP_CODEC_FPI, n);
    const uint64_t tmp_words = wp_max_compressed_words(WP_CODEC_FP32, n);
    if (need == 0 || tmp_words == 0)
        return WP_ERR_INVALID_ARG;
    if (out_cap_words < need)
        return WP_ERR_CAPACITY;
    const uint64_t units = (n / kBlock + kFpBlocks - 1) / kFpBlocks;
    const uint64_t E = 1 + (uint64_t)delta_stride;
    const uint64_t ndir = units + ((n % kBlock) ? 1 : 0);
    const uint32_t dir_end = (uint32_t)(kHdrWords + ((E * ndir + 3) & ~3ull));
    hipStream_t st = as_stream(stream);
    // scratch: the FastPFOR encoder's own | the FastPFOR stream | page sizes
    // | scan status | the FastPFOR stream's length
    const uint64_t common = (encode_scratch_bytes(WP_CODEC_FP32, n) + 255) & ~255ull;
    const uint64_t tmp_off = common;
    const uint64_t sizes_off = tmp_off + ((tmp_words * 4 + 255) & ~255ull);
    const uint64_t status_off = sizes_off + ((units * 4 + 255) & ~255ull);
    const uint64_t len_off = status_off + scan_status_words(units) * 8;
    char *scr = static_cast<char *>(stream_scratch(st, len_off + 256));
    if (scr == nullptr)
        return WP_ERR_HIP;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(scr + tmp_off);
    const int32_t rc = encode_common(WP_CODEC_FP32, in, n, delta_stride, tmp, tmp_words,
                                     reinterpret_cast<uint64_t *>(scr + len_off), stream);
    if (rc != WP_OK)
        return rc;
    return fpi_encode_pages(tmp, units, dir_end, reinterpret_cast<uint32_t *>(scr + sizes_off),
                            reinterpret_cast<uint64_t *>(scr + status_off), out, out_words, st);
}
