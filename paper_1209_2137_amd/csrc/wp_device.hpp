// Device building blocks of the wavepack decoders (gfx950, wave64).
//
// Every decoder here is a workgroup-wide routine: all threads of the
// workgroup call it together (it contains barriers). A workgroup has WAVES
// wavefronts; in each pass a lane owns VPL consecutive integers of one
// 128-integer block (VPL = 4 or 8, so a block spans 32 or 16 lanes and a
// wave covers 2 or 4 blocks).
//
// Per pass the steps are the ones of the paper's decoder, fused:
//   1. the packed words of the pass are staged from HBM into LDS with
//      16-byte loads (coalesced);
//   2. each lane extracts its VPL fields with a funnel shift of two LDS
//      words and a mask (Section 4: field i at bits [i*b, i*b+b));
//   3. patched pages OR each exception's high bits, shifted left by b, into
//      its position (Section 5);
//   4. the differential decoding of Section 3 is an inclusive prefix sum:
//      serial inside the lane, a DPP scan across the wavefront, an LDS
//      exchange across wavefronts, seeded by the unit's stored base;
//   5. lanes store their integers with 16-byte stores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wp {

constexpr uint32_t kBlock = 128;      // integers per block (Section 6.2)
constexpr uint32_t kBpBlocks = 16;    // blocks per binary-packing meta-block (Section 6.2)
constexpr uint32_t kFpBlocks = 512;   // blocks per patched page, 2^16 integers (Section 5)
constexpr uint32_t kBpUnitInts = kBlock * kBpBlocks;
constexpr uint32_t kFpUnitInts = kBlock * kFpBlocks;
constexpr uint32_t kMagicBP = 0x31425057u;  // "WPB1"
constexpr uint32_t kMagicFP = 0x31465057u;  // "WPF1"
constexpr uint32_t kMagicBP32 = 0x32335057u;  // "WP32"
constexpr uint32_t kB32 = 32;                 // BP32 block length (Section 6.2)
constexpr uint32_t kMagicFP32 = 0x33465057u;  // "WPF3"
constexpr uint32_t kMagicBPV = 0x31565057u;   // "WPV1"
constexpr uint32_t kMagicSP = 0x31535057u;    // "WPS1"
constexpr uint32_t kMagicFPI = 0x31495057u;   // "WPI1"

// Words of a page's exception array of `cnt` values at k bits, padded to a
// multiple of 128 values (SIMD-FastPFOR) or of 32 (FastPFOR, P32); either
// way the values form one stream of k-bit fields, least significant first.
// A FastPFOR page ends zero-padded to 4 words.
template <bool P32>
__device__ __forceinline__ uint32_t exc_array_words(uint32_t cnt, uint32_t k)
{
    return P32 ? ((cnt + 31u) / 32u) * k : ((cnt + kBlock - 1) / kBlock) * 4u * k;
}
constexpr uint32_t kHdrWords = 8;
constexpr uint32_t kMaxTailBytes = 127 * 5;
constexpr int kErrCorrupt = -3;

__host__ __device__ constexpr uint32_t pad4(uint32_t w) { return (w + 3u) & ~3u; }

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Number of set bits of `m` in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A pointer read from memory is generic to the compiler (flat loads and
// stores); rebuilding it as a global-memory pointer lets the compiler use
// global loads and stores.
template <typename T>
__device__ __forceinline__ T *as_global(T *p)
{
    typedef __attribute__((address_space(1))) T *GPtr;
    return (T *)(GPtr)reinterpret_cast<uintptr_t>(p);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Inclusive prefix sum inside each row of 16 lanes (row_shr 1, 2, 4, 8).
__device__ __forceinline__ uint32_t row_scan_incl(uint32_t v)
{
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);
    return v;
}

// Inclusive prefix sum over the 64 lanes: row scans, then row_bcast:15
// (rows 1 and 3 add the last lane of the row before) and row_bcast:31
// (rows 2 and 3 add lane 31).
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v)
{
    v = row_scan_incl(v);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);
    return v;
}

__device__ __forceinline__ uint32_t wave_read(uint32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Orders this wavefront's LDS accesses around a lane exchange (LDS
// instructions of one wavefront execute in issue order; this only stops the
// compiler from moving them).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t width_mask(uint32_t b) { return b >= 32u ? 0xffffffffu : ((1u << b) - 1u); }

// Raw buffer access (gfx9 buffer resource, dword3 = 0x00020000: 32-bit
// data, no swizzle). Loads at byte offsets beyond `bytes` return 0 without
// touching memory.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ BufRsrc make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t buf_load_u32(BufRsrc rs, uint32_t byte_off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)byte_off, 0, 0);
}

__device__ __forceinline__ uint4 buf_load_u4(BufRsrc rs, uint32_t byte_off)
{
    const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)byte_off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Decoded output goes out with the non-temporal hint (cache policy bit 1):
// it is written once and not read back by the decoder.
constexpr int kOutPolicy = 2;
//
// A 16-byte store reads its last data registers a little after issue; a
// vector instruction issued right behind it that overwrites them can
// change what is stored. Without the wait states below, decoding the 2^28
// patched list with two wavefronts per workgroup stored, in element 2 of
// lanes 12-15, 28-31, 44-47 and 60-63, the block width that the next
// instruction wrote into that register. The scheduling barriers keep the
// wait directly behind the store.
__device__ __forceinline__ void buf_store_u4(BufRsrc rs, uint32_t byte_off, uint32_t soff, uint4 v)
{
    const u32x4_t w = {v.x, v.y, v.z, v.w};
    __builtin_amdgcn_raw_buffer_store_b128(w, rs, (int)byte_off, (int)soff, kOutPolicy);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 1" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Stream header, read with uniform (scalar) loads.
struct Hdr {
    uint32_t magic, n_lo, n_hi, stride, n_units, tail_bytes, tail_off, total;
};

__device__ __forceinline__ Hdr load_hdr(const uint32_t *in)
{
    // uniform() keeps the fields in scalar registers also when `in` was
    // itself read from memory (a generic pointer, loaded per lane)
    Hdr h;
    h.magic = uniform(in[0]);
    h.n_lo = uniform(in[1]);
    h.n_hi = uniform(in[2]);
    h.stride = uniform(in[3]);
    h.n_units = uniform(in[4]);
    h.tail_bytes = uniform(in[5]);
    h.tail_off = uniform(in[6]);
    h.total = uniform(in[7]);
    return h;
}

// Validated header of one list stream, with derived sizes (uniform values).
struct ListHdr {
    uint32_t S, tail, tail_bytes, tail_off, total;
    uint64_t nfull, units, ndir, dir_end;
};

// Checks the 8-word header against the caller's n and the stream length
// and derives the directory geometry. `per` = blocks per unit.
__device__ __forceinline__ bool check_header(const uint32_t *__restrict__ in, uint64_t in_words, uint64_t n,
                                             uint32_t magic, uint32_t per, ListHdr &H)
{
    const Hdr h = load_hdr(in);
    const uint64_t hn = (uint64_t)h.n_lo | ((uint64_t)h.n_hi << 32);
    H.S = h.stride;
    H.nfull = n / kBlock;
    H.tail = (uint32_t)(n % kBlock);
    H.units = (H.nfull + per - 1) / per;
    H.ndir = H.units + (H.tail ? 1 : 0);
    H.dir_end = kHdrWords + (((1 + (uint64_t)H.S) * H.ndir + 3) & ~(uint64_t)3);
    H.tail_bytes = h.tail_bytes;
    H.tail_off = h.tail_off;
    H.total = h.total;
    return h.magic == magic && hn == n && (H.S == 0 || H.S == 1 || H.S == 4) && h.n_units == H.units &&
           h.total <= in_words && H.dir_end <= h.total && h.tail_off <= h.total && h.tail_off >= H.dir_end &&
           ((H.tail == 0) == (h.tail_bytes == 0));
}

// ------------------------------------------------------------------------
// Encoders: the directory entry of a unit (one workgroup per unit).

// directory entry: offset at word 8 + entry, bases after all ndir offsets;
// base_s = x[start - S + s], 0 before the array start
__device__ __forceinline__ void write_dir_entry(uint32_t *out, uint64_t entry, uint64_t ndir, uint32_t S,
                                                uint32_t off, const uint32_t *__restrict__ x, uint64_t start)
{
    const uint32_t tid = threadIdx.x;
    if (tid == 0)
        out[kHdrWords + entry] = off;
    else if (tid <= S)
        out[kHdrWords + ndir + entry * S + (tid - 1)] = (start + (tid - 1) >= S) ? x[start + (tid - 1) - S] : 0u;
}

__host__ __device__ __forceinline__ uint64_t dir_entries(uint64_t n, uint64_t per)
{
    const uint64_t nfull = n / kBlock;
    return (nfull + per - 1) / per + ((n % kBlock) ? 1 : 0);
}

// ------------------------------------------------------------------------
// LDS arena shared by all roles (a workgroup plays one role at a time).

template <int WAVES>
struct TailLds {
    uint32_t words[(kMaxTailBytes + 3) / 4 + 4];
    uint32_t vals[kBlock];
    uint32_t cnt[16 * 2];
    uint32_t bad;
};

// ------------------------------------------------------------------------
// Variable Byte tail (Section 2.4, remainder after the last block as in
// Section 6.2): up to 127 integers of 1..5 bytes, low 7-bit group first,
// top bit set on the last byte. Parallel parse: each byte is looked at by
// one lane; terminator bytes are counted with ballots to give each integer
// its index; the terminator's lane gathers the integer's bytes.
// WG: the whole workgroup of WAVES wavefronts takes part; otherwise one
// wavefront by itself (WAVES == 1, no workgroup barrier).
template <int WAVES, bool WG = true>
__device__ __forceinline__ bool tail_decode(const uint32_t *__restrict__ tw, uint32_t tail_bytes, uint32_t count,
                            uint32_t S, const uint32_t (&base)[4], uint32_t *__restrict__ out,
                            TailLds<WAVES> &L)
{
    static_assert(WG || WAVES == 1, "a single wavefront");
    constexpr int T = 64 * WAVES;
    constexpr int R = (kMaxTailBytes + T - 1) / T;
    static_assert(R * WAVES <= 32, "tail counters");
    const uint32_t lane = lane_id();
    const uint32_t tid = WG ? threadIdx.x : lane;
    const uint32_t wave = WG ? uniform(tid >> 6) : 0u;
    auto sync = [&]() __attribute__((always_inline)) {
        if constexpr (WG)
            __syncthreads();
        else
            wave_lds_order();
    };
    if (count == 0 || count >= kBlock || tail_bytes < count || tail_bytes > 5 * count)
        return false;
    const uint32_t nw = (tail_bytes + 3) / 4;
    for (uint32_t i = tid; i < nw; i += T)
        L.words[i] = tw[i];
    if (tid == 0)
        L.bad = 0;
    sync();
    const uint8_t *by = reinterpret_cast<const uint8_t *>(L.words);
    uint64_t m[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = r * T + tid;
        const bool f = i < tail_bytes && (by[i] & 0x80u);
        m[r] = ballot(f);
        if (lane == 0)
            L.cnt[r * WAVES + wave] = (uint32_t)__builtin_popcountll(m[r]);
    }
    sync();
    uint32_t total = 0;
    for (int c = 0; c < R * WAVES; ++c)
        total += L.cnt[c];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t i = r * T + tid;
        const bool f = i < tail_bytes && (by[i] & 0x80u);
        if (f) {
            uint32_t idx = lanes_below(m[r]);
            for (int c = 0; c < r * WAVES + (int)wave; ++c)
                idx += L.cnt[c];
            uint32_t s = i, len = 1;
            while (s > 0 && !(by[s - 1] & 0x80u) && len <= 5) {
                --s;
                ++len;
            }
            uint64_t v = 0;
            for (uint32_t k = 0; k < len && k < 5; ++k)
                v |= (uint64_t)(by[s + k] & 0x7fu) << (7 * k);
            if (len > 5 || v > 0xffffffffull || idx >= count)
                L.bad = 1;
            else
                L.vals[idx] = (uint32_t)v;
        }
    }
    sync();
    if (L.bad || total != count || !(by[tail_bytes - 1] & 0x80u))
        return false;
    if (wave == 0) {
        if (S == 4) {
            // class c = row, element m of the class is integer 4m + c
            const uint32_t c = lane >> 4, mm = 2 * (lane & 15);
            const uint32_t i0 = 4 * mm + c, i1 = 4 * (mm + 1) + c;
            uint32_t v0 = i0 < count ? L.vals[i0] : 0u;
            uint32_t v1 = i1 < count ? L.vals[i1] : 0u;
            v1 += v0;
            const uint32_t incl = row_scan_incl(v1);
            const uint32_t add = incl - v1 + base[c];
            if (i0 < count)
                out[i0] = v0 + add;
            if (i1 < count)
                out[i1] = v1 + add;
        } else {
            const uint32_t i0 = 2 * lane, i1 = 2 * lane + 1;
            uint32_t v0 = i0 < count ? L.vals[i0] : 0u;
            uint32_t v1 = i1 < count ? L.vals[i1] : 0u;
            if (S == 1) {
                v1 += v0;
                const uint32_t incl = wave_scan_incl(v1);
                const uint32_t add = incl - v1 + base[0];
                v0 += add;
                v1 += add;
            }
            if (i0 < count)
                out[i0] = v0;
            if (i1 < count)
                out[i1] = v1;
        }
    }
    return true;
}

// The list's tail entry (directory entry n_units): offset check, bases,
// then tail_decode. Called by a whole workgroup (WG) or one wavefront.
template <int WAVES, bool WG = true>
__device__ __forceinline__ bool decode_tail_entry(const uint32_t *__restrict__ in, const ListHdr &H, uint32_t *__restrict__ out,
                                  TailLds<WAVES> &L)
{
    const uint32_t off = uniform(in[kHdrWords + H.units]);
    const uint32_t *bp = in + kHdrWords + H.ndir + H.units * H.S;
    const uint32_t base[4] = {H.S > 0 ? uniform(bp[0]) : 0u, H.S > 1 ? uniform(bp[1]) : 0u,
                              H.S > 2 ? uniform(bp[2]) : 0u, H.S > 3 ? uniform(bp[3]) : 0u};
    if (!(off == H.tail_off && (uint64_t)off + (H.tail_bytes + 3) / 4 == H.total))
        return false;
    return tail_decode<WAVES, WG>(in + off, H.tail_bytes, H.tail, H.S, base, out + H.nfull * kBlock, L);
}

// Prefix sum of one pass held as four consecutive integers per lane, in
// place. stride 1: lane-serial sums, a wave scan of the lane totals, plus
// the carry; stride 4: one wave scan per residue class (each lane holds
// one integer of each class); stride 0: nothing. carry advances to the
// value(s) at the end of the pass.
template <uint32_t S>
__device__ __forceinline__ void scan_wave4(uint32_t (&x)[4], uint32_t (&carry)[4])
{
    if constexpr (S == 1) {
        x[1] += x[0];
        x[2] += x[1];
        x[3] += x[2];
        const uint32_t incl = wave_scan_incl(x[3]);
        const uint32_t add = incl - x[3] + carry[0];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            x[r] += add;
        carry[0] += wave_read(incl, 63);
    } else if constexpr (S == 4) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t incl = wave_scan_incl(x[c]);
            x[c] = incl + carry[c];
            carry[c] += wave_read(incl, 63);
        }
    }
}

// ------------------------------------------------------------------------
// Patched page (Section 5) decoded by segments of 64 blocks, one
// wavefront each, with no workgroup barrier: a segment is decoded in block
// order, four blocks (512 integers) per pass, the prefix sum carried from
// the segment's base (the unit's stored bases for the first segment, the
// page header's segment bases for the others). Everything else a segment
// needs follows from the page's metadata bytes: before its own blocks, the
// wavefront reads the widths and exception counts of the earlier segments'
// blocks (three byte loads per lane and segment, all in flight at once)
// for the packed-word and position offsets where its segment starts and,
// per array k, the exceptions before it (LDS atomics). A segment that is
// not the page's last checks its final running value against the next
// segment's stored base; the last one checks the page's totals.
//
// Block records {b | k << 8 | c << 16, word offset in the packed region,
// bit offset of the block's first exception's high part from the page
// start, index of its first exception in the page} are built a round of 64
// blocks ahead, lane = block: wave scans of 4b and c give the offsets, and
// the rank of the block's exceptions inside array k = maxb - b is the
// count of earlier rounds (per k, in LDS) plus one masked scan per distinct
// k of the round (exceptions are appended to array k in block order). The
// records of two rounds live in an LDS ring; a record past the last block
// holds b = c = 0 and the running offsets, so the passes need no special
// case at the page end.
//
// A pass: lanes 0..31 unpack blocks A and C, lanes 32..63 blocks B and D;
// lane q takes integers q, q+32, q+64, q+96 of its block (integer q + 32m
// starts at bit q*b + 32*m*b: word (q*b >> 5) + m*b at the same shift), one
// funnel shift of two LDS words each. The values go to the pass's area in
// block order, lane e ORs in exception e of the pass (its high part
// shifted left by b), then lane l reads integers 4l..4l+3 and 256+4l..
// 256+4l+3 for the prefix sum and two 16-byte stores. The packed words of
// a pass, and for each lane its exception's position byte and its high
// part (or the two words holding it), are fetched two passes ahead into
// named register slots.
//
// Three page kinds share this: SIMD-FastPFOR (exception arrays padded to
// 128 values), FastPFOR (padded to 32) and SimplePFOR, whose high parts
// are one Simple-8b array over the page in block order (Section 5, and
// the Simple-8b modes of Section 2). A SimplePFOR page holds the same
// segment bases and, per segment after the first, the Simple-8b word that
// holds the segment's first high part and that word's values before it,
// so its segments decode independently too. A SimplePFOR segment's high
// parts are decoded into an LDS ring as the passes need them: a wavefront
// takes up to 64 Simple-8b words at a time (lane i word i), a wave scan of
// the counts their selectors give places each word's integers, and the
// words are loaded one batch ahead.
enum : int { kPageFp = 0, kPageFp32 = 1, kPageSp = 2, kPageFpi = 3 };
// High parts held by a SimplePFOR segment's ring: the next pass's beyond
// its first 64 (those are fetched into registers), the fetched pass's, and
// one Simple-8b word: at most 4 * 102 - 64 + 4 * 102 + 59, since the cost
// rule never keeps more than 102 exceptions in a block (c (8 + maxb - b)
// < 128 (maxb - b)); a pass holding more is flagged. Not a power of two:
// 816 entries keep a segment at 11.5 KB of LDS, seven workgroups of two
// segments per compute unit (six with 1024).
constexpr uint32_t kSpRing = 816;
static_assert(kSpRing >= 4u * 102u - 64u + 4u * 102u + 59u, "a segment's high parts fit the ring");
constexpr uint32_t kSegBlocks = 64;  // blocks per segment of a patched page
constexpr uint32_t kSegInts = kSegBlocks * kBlock;
constexpr uint32_t kPageSegs = kFpBlocks / kSegBlocks;

// Wavefront items of a patched page of nb blocks: its segments (one for a
// page in the paper's layout).
template <int KIND>
__host__ __device__ constexpr uint32_t page_items(uint32_t nb)
{
    return KIND == kPageFpi ? 1u : (nb + kSegBlocks - 1) / kSegBlocks;
}

// A segment's packed words stream through a per-wavefront LDS ring in
// chunks of one 16-byte load per lane (256 words), kFpDepth chunks loaded
// ahead: each read from HBM is a contiguous kilobyte or more, not a pass's
// few hundred bytes between other wavefronts' stores.
constexpr uint32_t kFpCW = 256;
constexpr uint32_t kFpDepth = 2;
constexpr uint32_t kFpRing = 1024;        // >= kFpDepth * kFpCW + the largest pass (512 words)
constexpr uint32_t kFpMir = kBlock + 4;   // ring words mirrored after its end
static_assert(kFpRing >= kFpDepth * kFpCW + 4 * kBlock && (kFpRing & (kFpRing - 1)) == 0, "ring size");

// R: rounds of block records held (a segment is one round; a page in the
// paper's layout keeps two rounds in a ring).
template <int R>
struct alignas(16) FpLdsT {
    uint32_t ring[kFpRing + kFpMir];  // packed words of the segment
    uint32_t buf[4 * kBlock + 4];     // a pass's integers in block order
    uint4 rec[R][64];                 // block records of R rounds of 64 blocks
    uint32_t kcar[33];                // exceptions of the rounds built so far, per array k
    uint32_t excb[33];                // page word offset of array k
};
using FpWaveLds = FpLdsT<1>;

// A page in the paper's own layout (kPageFpi) is parsed into LDS first:
// per block its widths and count, and where its positions start in the
// byte array, which is held in LDS when it fits.
constexpr uint32_t kFpiBaWords = 3072;
struct alignas(16) FpiLds : FpLdsT<2> {
    uint32_t bm[kFpBlocks];      // block t: b | maxb << 8 | c << 16
    uint32_t posoff[kFpBlocks];  // block t: byte offset of its positions in the byte array
    uint32_t kc[33];             // array k's length (from its counter)
    uint32_t ba[kFpiBaWords];    // the byte array, when it fits
};

template <int KIND>
struct FpLdsSel {
    using T = FpLdsT<1>;
};
template <>
struct FpLdsSel<kPageFpi> {
    using T = FpiLds;
};
template <int KIND>
using FpLdsOf = typename FpLdsSel<KIND>::T;

struct alignas(16) SpWaveLds {
    FpLdsT<1> fp;
    uint32_t ring[kSpRing];  // decoded high parts, by their index in the page mod kSpRing
};

// What a pass needs, fetched ahead (per lane unless noted).
struct FpFetch {
    uint32_t pe;           // uniform: end of the pass's packed words, from the segment's first
    uint32_t u0, u1;       // blocks A|B (half 0), C|D (half 1): the lane's block width | its first
                           // word (from the segment's first) << 8
    uint32_t pos, lo, hi;  // exception `lane` of the pass: position byte, the words holding its high
                           // part (SimplePFOR: lo is the high part itself)
    uint32_t em;           // its bit shift | (b & 31) << 8 | its block in the pass << 16 | first of its block << 18
    uint32_t km;           // mask of its k high bits
    uint32_t ce, e0;       // uniform: exceptions of the pass, index of its first exception in the page
};

constexpr uint32_t kOutOfRange = 0xfffffff0u;  // a buffer offset beyond every page: reads nothing

__device__ __forceinline__ uint32_t buf_load_u8(BufRsrc rs, uint32_t byte_off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, (int)byte_off, 0, 0);
}

// Lane i gets v of lane i - 1 (DPP wave_shr:1); lane 0 gets `first`.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t first, uint32_t v)
{
    return __builtin_amdgcn_update_dpp(first, v, 0x138, 0xf, 0xf, false);
}

// Simple-8b modes (Section 2's table): selector s -> count | bits << 8.
__device__ __forceinline__ uint32_t s8_mode(uint32_t sel)
{
    // counts 240 120 60 30 20 15 12 10 8 7 6 5 4 3 2 1; bits 0 0 1 2 3 4 5 6 7 8 10 12 15 20 30 60
    constexpr uint64_t kCnt0 = 0x0a0c0f141e3c78f0ull;  // selectors 0..7, one byte each
    constexpr uint64_t kCnt1 = 0x0102030405060708ull;  // selectors 8..15
    constexpr uint64_t kBit0 = 0x0605040302010000ull;
    constexpr uint64_t kBit1 = 0x3c1e140f0c0a0807ull;
    const uint32_t sh = 8u * (sel & 7u);
    const uint32_t cnt = (uint32_t)(((sel & 8u) ? kCnt1 : kCnt0) >> sh) & 255u;
    const uint32_t bits = (uint32_t)(((sel & 8u) ? kBit1 : kBit0) >> sh) & 255u;
    return cnt | (bits << 8);
}

// Decodes segment `seg` of the patched page at `page` (16-byte aligned,
// `nwords` words, which must hold `nb` blocks; a page in the paper's
// layout is one segment) into its part of out[0, 128 nb) (the page's output) with
// differential coding of stride S, the page's first segment starting from
// `ubase` (the unit's stored bases). One wavefront; `ring` is the LDS ring
// of a SimplePFOR segment (KIND kPageSp), unused otherwise. Returns the
// segment's validity (uniform); every access stays inside the page, the
// segment's output range and the wavefront's LDS whatever the page holds.
template <uint32_t S, int KIND = kPageFp>
__device__ __forceinline__ bool fp_wave_page(const uint32_t *__restrict__ page, uint32_t nwords, uint32_t nb,
                                             uint32_t seg, const uint32_t (&ubase)[4], uint32_t *__restrict__ out,
                                             FpLdsOf<KIND> &L, uint32_t *ring = nullptr)
{
    constexpr bool SP = KIND == kPageSp;
    constexpr bool IN = KIND == kPageFpi;  // the paper's own page layout
    constexpr bool WHOLE = IN;             // one wavefront decodes the whole page
    constexpr uint32_t NR = WHOLE ? 2u : 1u;  // rounds of records held
    static_assert(sizeof(L.rec) / sizeof(L.rec[0]) >= NR, "the LDS record area holds every round in use");
    const uint32_t lane = lane_id();
    if (nwords < (IN ? 4u : 4u) || nb == 0 || nb > kFpBlocks || seg >= page_items<KIND>(nb))
        return false;
    const BufRsrc rpg = make_rsrc(page, nwords * 4u);
    const bool kl = lane < 32;
    // SIMD-FastPFOR / FastPFOR: [nblocks, packed_words, meta_bytes, bitset]
    // + a count per non-empty array; SimplePFOR: [nblocks, packed_words,
    // meta_bytes, Simple-8b words] + the segment entries; both + the
    // segment bases; the paper's layout: word 0 = the byte array's
    // counter, parsed below
    uint32_t packed_words, meta_bytes, w3, bitset, hdr_w;
    uint32_t cpos = 0, nba = 0, baw = 0;  // the paper's layout: counter word, byte array bytes and words
    bool ba_lds = false;                  // the byte array is held in LDS
    if constexpr (IN) {
        cpos = uniform(page[0]);
        if (cpos < 1 || cpos >= nwords || ((cpos - 1) & 3u))
            return false;
        nba = uniform(page[cpos]);
        baw = (nba + 3u) / 4u;
        if (nba > (3u + 127u) * nb || baw > nwords - cpos - 1u)
            return false;
        packed_words = cpos - 1u;
        hdr_w = 1;
        w3 = 0;
        meta_bytes = 0;  // 3 nb + the page's exceptions, once parsed
        ba_lds = baw <= kFpiBaWords;
    } else {
        const uint32_t h_nb = uniform(page[0]);
        packed_words = uniform(page[1]);
        meta_bytes = uniform(page[2]);
        w3 = uniform(page[3]);
        bitset = SP ? 0u : w3;
        const uint32_t nset0 = __builtin_popcount(bitset);
        // + the segment bases (SimplePFOR: and one Simple-8b entry per segment)
        hdr_w = pad4(4 + nset0 + (S + (SP ? 1u : 0u)) * (page_items<KIND>(nb) - 1));
        const uint32_t meta_w0 = ((meta_bytes + 15u) / 16u) * 4u;
        if (h_nb != nb || hdr_w > nwords || packed_words > nwords - hdr_w || meta_bytes < 3 * nb ||
            meta_bytes > 3 * nb + 127 * nb || meta_w0 > nwords - hdr_w - packed_words || (packed_words & 3u))
            return false;
    }
    const uint32_t nset = IN ? 0u : (uint32_t)__builtin_popcount(bitset);
    const uint32_t nseg = page_items<KIND>(nb);
    const uint32_t meta_w = ((meta_bytes + 15u) / 16u) * 4u;
    const uint32_t meta_at = (hdr_w + packed_words) * 4u;  // byte offset of the metadata
    const uint32_t pos_at = meta_at + 3u * nb;             // byte offset of the positions
    const uint32_t exc_at = hdr_w + packed_words + meta_w;
    const uint32_t ba_at = (cpos + 1u) * 4u;               // the paper's layout: byte offset of the byte array
    // the paper's layout: byte o of the byte array (o < nba), from LDS or the page
    auto ba_byte = [&](uint32_t o) __attribute__((always_inline)) -> uint32_t {
        if constexpr (IN) {
            if (ba_lds)
                return reinterpret_cast<const uint8_t *>(L.ba)[o];
            return buf_load_u8(rpg, ba_at + o);
        }
        return 0u;
    };
    if constexpr (IN) {
        // the byte array into LDS (eight 4-byte loads per lane in flight),
        // then walked record by record: b, maxb, and when maxb > b, c and
        // the c positions; then the exception arrays, each behind its
        // counter, one after the other behind the bitset
        if (ba_lds) {
            const BufRsrc rba = make_rsrc(page + cpos + 1, baw * 4u);
            for (uint32_t i0 = 0; i0 < baw; i0 += 512u) {
                uint32_t v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    v[r] = buf_load_u32(rba, (i0 + 64u * r + lane) * 4u);
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (i0 + 64u * r + lane < baw)
                        L.ba[i0 + 64u * r + lane] = v[r];
            }
            wave_lds_order();
        }
        uint32_t o = 0, ne = 0, pk = 0;
        bool pbad = false;
        for (uint32_t t = 0; t < nb; ++t) {
            const uint32_t b = uniform(o < nba ? ba_byte(o) : 255u);
            const uint32_t mb = uniform(o + 1u < nba ? ba_byte(o + 1u) : 255u);
            const uint32_t cc = uniform(o + 2u < nba ? ba_byte(o + 2u) : 0u);
            const uint32_t c = mb > b ? cc : 0u;
            pbad = pbad || b > 32u || mb > 32u || mb < b || (mb > b && (c == 0u || c >= kBlock)) ||
                   o + 2u + (mb > b ? 1u + c : 0u) > nba;
            if (pbad)
                break;
            if (lane == 0) {
                L.bm[t] = b | (mb << 8) | (c << 16);
                L.posoff[t] = o + 3u;
            }
            o += mb > b ? 3u + c : 2u;
            ne += c;
            pk += 4u * b;
        }
        if (pbad || o != nba || pk != packed_words)
            return false;
        meta_bytes = 3u * nb + ne;
        uint32_t xp = cpos + 1u + baw;
        if (xp >= nwords)
            return false;
        bitset = uniform(page[xp]);
        ++xp;
        for (uint32_t k = 1; k <= 32; ++k) {
            uint32_t cnt = 0, at = 0;
            if ((bitset >> (k - 1u)) & 1u) {
                if (xp >= nwords)
                    return false;
                cnt = uniform(page[xp]);
                const uint32_t words = ((cnt + 31u) / 32u) * k;
                if (cnt == 0u || cnt > nb * kBlock || words > nwords - xp - 1u)
                    return false;
                at = xp + 1u;
                xp += 1u + words;
            }
            if (lane == 0) {
                L.kc[k] = cnt;
                L.excb[k] = at;
            }
        }
        if (pad4(xp) != nwords)
            return false;
        if (lane == 32)
            L.excb[0] = 0, L.kc[0] = 0;
        if (lane < 33)
            L.kcar[lane] = 0;
        wave_lds_order();
    }
    // the segment: blocks [blk0, blk1)
    const uint32_t blk0 = WHOLE ? 0u : seg * kSegBlocks;
    const uint32_t blk1 = WHOLE ? nb : (nb - blk0 < kSegBlocks ? nb : blk0 + kSegBlocks);
    const bool last_seg = seg + 1 == nseg;
    uint32_t carry[4] = {ubase[0], ubase[1], ubase[2], ubase[3]};
    if constexpr (!WHOLE && S > 0) {
        if (seg > 0) {
            // segment bases follow the counts; inside the validated header
            const uint32_t *const sb = page + 4 + nset + S * (seg - 1);
#pragma unroll
            for (uint32_t t = 0; t < S; ++t)
                carry[t] = uniform(sb[t]);
        }
    }
    // relative round r of the segment: blocks blk0 + 64 r + lane
    auto load_meta = [&](uint32_t r, uint32_t &mb_, uint32_t &mm_, uint32_t &mc_) __attribute__((always_inline)) {
        const uint32_t jj = blk0 + 64u * r + lane;
        const bool own = jj < blk1;
        if constexpr (IN) {
            const uint32_t v = own ? L.bm[jj] : 0u;
            mb_ = v & 255u;
            mm_ = (v >> 8) & 255u;
            mc_ = v >> 16;
            return;
        }
        mb_ = buf_load_u8(rpg, own ? meta_at + jj : kOutOfRange);
        mm_ = buf_load_u8(rpg, own ? meta_at + nb + jj : kOutOfRange);
        mc_ = buf_load_u8(rpg, own ? meta_at + 2u * nb + jj : kOutOfRange);
    };
    // A segment's setup is a chain of dependent reads; every read that
    // needs only the header is issued here at once: the earlier segments'
    // metadata bytes, this segment's, and the L2 prefetch of its share of
    // the exception arrays (below).
    uint32_t m0 = 0, m1 = 0, m2 = 0;
    uint32_t eb[kPageSegs - 1], em[kPageSegs - 1], ec[kPageSegs - 1];
    uint4 pf[3];
    if constexpr (!WHOLE) {
        if (seg > 0) {
#pragma unroll
            for (uint32_t r = 0; r + 1 < kPageSegs; ++r) {
                const uint32_t jj = 64u * r + lane;
                const bool own = r < seg;
                eb[r] = buf_load_u8(rpg, own ? meta_at + jj : kOutOfRange);
                em[r] = buf_load_u8(rpg, own ? meta_at + nb + jj : kOutOfRange);
                ec[r] = buf_load_u8(rpg, own ? meta_at + 2u * nb + jj : kOutOfRange);
            }
        }
        load_meta(0, m0, m1, m2);
        // The exceptions' high parts and positions are read a few bytes per
        // pass from up to 32 arrays; fetched that way from HBM, between the
        // other wavefronts' stores, each read would be a small scattered
        // one. Instead each segment first reads its share of the page's
        // exception arrays (an equal part for each of the page's segments,
        // all of them decoded side by side) and its own positions with
        // contiguous 16-byte loads, so that the passes find those lines in
        // the L2 cache. The data is only folded into a register that an
        // empty asm statement consumes.
        const uint32_t ex_w = nwords - exc_at, share = (ex_w + nseg - 1) / nseg;
        const uint32_t pf_at = (exc_at + seg * share) * 4u;
        pf[0] = buf_load_u4(rpg, pf_at + lane * 16u);
        pf[1] = buf_load_u4(rpg, pf_at + 1024u + lane * 16u);
    }
    uint32_t kcnt = 0;
    if constexpr (IN) {
        kcnt = kl ? L.kc[lane + 1] : 0u;
    } else if constexpr (SP) {
        // the Simple-8b words run to the page end (zero-padded to 4 words)
        if ((w3 & 1u) || w3 > nwords - exc_at || pad4(exc_at + w3) != nwords)
            return false;
    } else {
        // exception array directory: lane k - 1 owns array k
        const bool set = kl && ((bitset >> (lane & 31u)) & 1u);
        const uint32_t ci = kl ? (uint32_t)__builtin_popcount(bitset & ((1u << (lane & 31u)) - 1u)) : 0u;
        kcnt = set ? page[4 + ci] : 0u;
        const bool badk = set && (kcnt == 0 || kcnt > nb * kBlock);
        const uint32_t wk = (set && !badk) ? exc_array_words<KIND == kPageFp32>(kcnt, lane + 1) : 0u;
        const uint32_t kincl = wave_scan_incl(wk);
        const uint32_t exc_end = exc_at + wave_read(kincl, 63);
        if (ballot(badk) != 0 || (KIND == kPageFp32 ? pad4(exc_end) : exc_end) != nwords)
            return false;
        if (kl)
            L.excb[lane + 1] = exc_at + kincl - wk;
        if (lane == 32)
            L.excb[0] = 0;
        if (lane < 33)
            L.kcar[lane] = 0;
        wave_lds_order();
    }

    bool bad = false;  // per lane, reduced at the end
    uint32_t pk_run = 0, pos_run = 0;
    if constexpr (!WHOLE) {
        // the earlier segments' blocks (all full rounds of 64): packed words,
        // positions and, per array k, exceptions before this segment
        if (seg > 0) {
            uint32_t pk_l = 0, pos_l = 0;
#pragma unroll
            for (uint32_t r = 0; r + 1 < kPageSegs; ++r) {
                const uint32_t k = (em[r] >= eb[r] && em[r] <= 32u) ? em[r] - eb[r] : 0u;
                pk_l += 4u * (eb[r] < 32u ? eb[r] : 32u);
                pos_l += ec[r];
                if (!SP && ec[r] != 0u && k != 0u)
                    atomicAdd(&L.kcar[k], ec[r]);
            }
            pk_run = wave_read(wave_scan_incl(pk_l), 63);
            pos_run = wave_read(wave_scan_incl(pos_l), 63);
            wave_lds_order();
        }
    }
    // the segment's packed words [yS, yX) of the packed region stream
    // through the ring (a SimplePFOR page's, all of them); words a corrupt
    // stream would place past the packed region are not read
    uint32_t yS = 0, wS = 0, yX = 0;  // the segment's first packed word and exception, its words' end
    BufRsrc rsp = make_rsrc(page, 0u);
    uint4 c0, c1;
    auto issue_ring = [&]() __attribute__((always_inline)) {
        const bool okx = yS <= yX && yX <= packed_words;
        rsp = make_rsrc(page + hdr_w + (okx ? yS : 0u), okx ? 4u * (yX - yS) : 0u);
        c0 = buf_load_u4(rsp, lane * 16u);
        __builtin_amdgcn_sched_barrier(0);
        c1 = buf_load_u4(rsp, (kFpCW + lane * 4u) * 4u);
        if constexpr (!WHOLE)
            pf[2] = buf_load_u4(rpg, ((pos_at + wS) & ~15u) + lane * 16u);
    };
    auto build_round = [&](uint32_t r, uint32_t bv, uint32_t mv, uint32_t cv) __attribute__((always_inline)) {
        // blocks past the segment read 0 for b, maxb and c
        bad = bad || bv > 32u || mv > 32u || mv < bv || cv >= kBlock || ((cv == 0u) != (mv == bv));
        const uint32_t k = (mv >= bv && mv <= 32u) ? mv - bv : 0u;
        const uint32_t bc = bv < 32u ? bv : 32u;  // a corrupt width stays within the pass's words
        const uint32_t bw = 4u * bc;
        const uint32_t iw = wave_scan_incl(bw), ip = wave_scan_incl(cv);
        const uint32_t y = pk_run + iw - bw, w = pos_run + ip - cv;
        pk_run += wave_read(iw, 63);
        pos_run += wave_read(ip, 63);
        if (!WHOLE && r == 0) {
            // a segment of a FastPFOR page is one round: its packed words
            // end here, and the ring's first loads go out before the ranks
            yX = pk_run;
            issue_ring();
        }
        uint32_t z = 0;
        if constexpr (!SP) {
            const uint32_t kc = L.kcar[k];
            uint32_t rk = 0;
            uint64_t todo = ballot(cv > 0u && k > 0u);
            while (todo) {
                const uint32_t lead = (uint32_t)__builtin_ctzll(todo);
                const uint32_t k0 = wave_read(k, (int)lead);
                const bool mine = cv > 0u && k == k0;
                const uint64_t mm = ballot(mine);
                const uint32_t xc = mine ? cv : 0u;
                const uint32_t incl = wave_scan_incl(xc);
                if (mine)
                    rk = incl - xc;
                if (lane == 0)
                    L.kcar[k0] = wave_read(kc, (int)lead) + wave_read(incl, 63);
                todo &= ~mm;
            }
            z = L.excb[k] * 32u + (kc + rk) * k;
        }
        L.rec[r % NR][lane] = make_uint4(bc | (k << 8) | (cv << 16), y, z, w);
        wave_lds_order();
    };
    const uint32_t npass = (blk1 - blk0 + 3) / 4;
    yS = pk_run;
    wS = pos_run;
    if constexpr (WHOLE)
        load_meta(0, m0, m1, m2);
    build_round(0, m0, m1, m2);
    if constexpr (WHOLE) {
        load_meta(1, m0, m1, m2);
        build_round(1, m0, m1, m2);
        load_meta(2, m0, m1, m2);
        yX = packed_words;
        issue_ring();
    }
    uint32_t written = 0;  // words of the segment already in the ring
    // chunk c goes to the ring (and its mirror), the slot reloads chunk c + 2;
    // slots are written and reloaded in a fixed order, so the wait for a
    // slot covers only older loads
    auto put = [&](uint4 &slot, uint32_t c) __attribute__((always_inline)) {
        const uint32_t pos = (c * kFpCW + lane * 4u) & (kFpRing - 1u);
        *reinterpret_cast<uint4 *>(&L.ring[pos]) = slot;
        if (pos < kFpMir)
            *reinterpret_cast<uint4 *>(&L.ring[kFpRing + pos]) = slot;
        slot = buf_load_u4(rsp, ((c + kFpDepth) * kFpCW + lane * 4u) * 4u);
    };
    // a pass reads at most 512 words from at or before `written`, so one
    // group of two chunks always brings the ring up to its end
    auto fill_to = [&](uint32_t need) __attribute__((always_inline)) {
        if (written < need) {
            const uint32_t c = written / kFpCW;
            put(c0, c);
            put(c1, c + 1);
            written += kFpDepth * kFpCW;
        }
    };

    // SimplePFOR: the ring holds the high parts [keep, dec) (indices in the
    // page); sw = next Simple-8b word, whose batch of 64 (lane i: word
    // sw + i) sits in plo/phi
    const uint32_t ns8 = SP ? w3 / 2u : 0u;
    uint32_t sw = 0, dec = 0, plo = 0, phi = 0;
    auto s8_load = [&]() __attribute__((always_inline)) {
        const uint32_t o = sw + lane < ns8 ? (exc_at + 2u * (sw + lane)) * 4u : kOutOfRange;
        plo = buf_load_u32(rpg, o);
        phi = buf_load_u32(rpg, o + 4u);
    };
    // decodes Simple-8b words until high part need - 1 is in the ring
    // (never overwriting [keep, dec)); with count_only, only counts them
    auto s8_fill = [&](uint32_t need, uint32_t keep, bool count_only) __attribute__((always_inline)) {
        while (dec < need && sw < ns8) {
            const bool live = sw + lane < ns8;
            const uint32_t md = s8_mode(phi >> 28);
            const uint32_t cnt = live ? (md & 255u) : 0u, bits = md >> 8;
            const uint32_t incl = wave_scan_incl(cnt);
            // accepted high parts stay inside one ring length from dec and
            // from keep, so no two of them, and none of [keep, dec), share
            // a slot (dec is below keep while a segment's first word is
            // read: its values before the segment are not needed)
            const uint32_t room = count_only ? 0xffffffffu : dec >= keep ? kSpRing - (dec - keep) : kSpRing;
            const uint64_t am = ballot(live && incl <= room);
            const uint32_t nacc = (uint32_t)__builtin_popcountll(am);
            if (nacc == 0) {  // a pass's high parts do not fit the ring: corrupt counts
                bad = true;
                break;
            }
            if (!count_only && ((am >> lane) & 1u)) {
                const uint64_t word = ((uint64_t)phi << 32) | plo;
                const uint64_t fm = bits >= 64u ? ~0ull : ((1ull << bits) - 1u);
                uint32_t at = dec + incl - cnt;
                for (uint32_t j = 0; j < cnt; ++j, ++at) {
                    const uint64_t v = bits ? (word >> (j * bits)) & fm : 0u;
                    bad = bad || (v >> 32) != 0u;
                    ring[at % kSpRing] = (uint32_t)v;
                }
            }
            dec += wave_read(incl, (int)nacc - 1);
            sw += nacc;
            s8_load();
        }
    };
    if constexpr (SP) {
        // a segment after the first starts on the Simple-8b word its entry
        // names, that word's first value being high part wS - skip
        if (seg > 0) {
            const uint32_t ent = uniform(page[4 + S * (nseg - 1) + seg - 1]);
            const uint32_t w0 = ent & 0xFFFFFFu, skip = ent >> 24;
            if (w0 > ns8 || skip > wS || skip >= 60u || (w0 == ns8 && skip != 0u))
                return false;
            sw = w0;
            dec = wS - skip;
        }
        s8_load();
    }

    const uint32_t jl = lane >> 5;
    // pass q's words and exceptions; `keep`: the first high part still to
    // be read from the ring (SimplePFOR)
    auto fetch = [&](uint32_t q, uint32_t keep) __attribute__((always_inline)) {
        FpFetch f;
        if (q >= npass) {  // past the segment: nothing to read
            f.pe = 0, f.u0 = f.u1 = f.pos = f.lo = f.hi = f.em = f.km = 0, f.ce = f.e0 = 0;
            return f;
        }
        const uint4 *const R = &L.rec[(q >> 4) % NR][(q & 15u) * 4u];
        const uint4 rA = R[jl], rC = R[2 + jl];
        const uint32_t yA = wave_read(rA.y, 0), wA = wave_read(rA.w, 0), wB = wave_read(rA.w, 32);
        const uint32_t wC = wave_read(rC.w, 0), xD = wave_read(rC.x, 32), yD = wave_read(rC.y, 32),
                       wD = wave_read(rC.w, 32);
        (void)yA;
        f.pe = yD + 4u * (xD & 255u) - yS;
        f.u0 = (rA.x & 255u) | ((rA.y - yS) << 8);
        f.u1 = (rC.x & 255u) | ((rC.y - yS) << 8);
        f.e0 = wA;
        f.ce = wD + ((xD >> 16) & 255u) - wA;
        // exception `lane`: its block j of the pass, then its place in array k
        const uint32_t j = (lane >= wB - wA ? 1u : 0u) + (lane >= wC - wA ? 1u : 0u) + (lane >= wD - wA ? 1u : 0u);
        const uint4 re = R[j];
        const uint32_t k = (re.x >> 8) & 255u;
        const uint32_t idx = wA + lane - re.w;
        const bool any = lane < f.ce;
        if constexpr (IN)
            f.pos = any ? ba_byte(L.posoff[blk0 + 4u * q + j] + idx) : 0u;
        else
            f.pos = buf_load_u8(rpg, any ? pos_at + wA + lane : kOutOfRange);
        uint32_t bit = 0;
        if constexpr (SP) {
            s8_fill(wA + f.ce, keep, false);
            f.lo = any ? ring[(wA + lane) % kSpRing] : 0u;
            f.hi = 0;
        } else {
            bit = re.z + idx * k;
            const uint32_t woff = any ? (bit >> 5) * 4u : kOutOfRange;
            f.lo = buf_load_u32(rpg, woff);
            f.hi = buf_load_u32(rpg, woff + 4u);
        }
        f.em = (bit & 31u) | ((re.x & 31u) << 8) | (j << 16) | (idx == 0u ? (1u << 18) : 0u);
        f.km = width_mask(k);
        return f;
    };

    const uint32_t qq = lane & 31u;
    uint32_t *const xw = &L.buf[jl * kBlock + qq];  // integer q of the lane's block of half 0
    // f: pass p, fetched; nx: pass p + 1, fetched (its exceptions beyond the
    // first 64 still read from the ring while f is refetched for p + 2)
    auto run_pass = [&](uint32_t p, FpFetch &f, const FpFetch &nx) __attribute__((always_inline)) {
        fill_to(f.pe);
        wave_lds_order();
        uint32_t v[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t u = h ? f.u1 : f.u0;
            const uint32_t b = u & 255u, qb = qq * b;
            // the block's words lie in [w0, w0 + 4b + 1) of the ring and its mirror
            const uint32_t w0 = ((u >> 8) + (qb >> 5)) & (kFpRing - 1u);
            const uint32_t mask = width_mask(b);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t wi = w0 + m * b;
                v[h][m] = __builtin_amdgcn_alignbit(L.ring[wi + 1], L.ring[wi], qb) & mask;
            }
        }
        wave_lds_order();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int m = 0; m < 4; ++m)
                xw[h * 2 * kBlock + 32 * m] = v[h][m];
        wave_lds_order();
        // exceptions: one per lane, the rest (more than 64 in the pass) in rounds
        const uint32_t prev = wave_shr1(0u, f.pos);
        if (lane < f.ce) {
            const uint32_t hv = SP ? f.lo : __builtin_amdgcn_alignbit(f.hi, f.lo, f.em) & f.km;
            atomicOr(&L.buf[((f.em >> 16) & 3u) * kBlock + (f.pos & (kBlock - 1u))], hv << ((f.em >> 8) & 31u));
            bad = bad || f.pos >= kBlock || (!((f.em >> 18) & 1u) && prev >= f.pos) || (SP && (hv & ~f.km) != 0u);
        }
        if (f.ce > 64u) {
            const uint4 *const R = &L.rec[(p >> 4) % NR][(p & 15u) * 4u];
            const uint32_t wA = f.e0, wB = wave_read(R[1].w, 0), wC = wave_read(R[2].w, 0),
                           wD = wave_read(R[3].w, 0);
            for (uint32_t e = 64u + lane; e - lane < f.ce; e += 64u) {
                if (e < f.ce) {
                    const uint32_t j = (e >= wB - wA ? 1u : 0u) + (e >= wC - wA ? 1u : 0u) + (e >= wD - wA ? 1u : 0u);
                    const uint4 re = R[j];
                    const uint32_t k = (re.x >> 8) & 255u, b = re.x & 31u;
                    const uint32_t idx = wA + e - re.w;
                    uint32_t pos, pprev;
                    if constexpr (IN) {
                        const uint32_t po = L.posoff[blk0 + 4u * p + j] + idx;
                        pos = ba_byte(po);
                        pprev = idx > 0u ? ba_byte(po - 1u) : 0u;
                    } else {
                        pos = buf_load_u8(rpg, pos_at + wA + e);
                        pprev = idx > 0u ? buf_load_u8(rpg, pos_at + wA + e - 1u) : 0u;
                    }
                    bad = bad || pos >= kBlock || (idx > 0u && pprev >= pos);
                    uint32_t hv;
                    if constexpr (SP) {
                        hv = ring[(wA + e) % kSpRing];
                        bad = bad || (hv & ~width_mask(k)) != 0u;
                    } else {
                        const uint32_t bit = re.z + idx * k;
                        const uint32_t lo = buf_load_u32(rpg, (bit >> 5) * 4u);
                        const uint32_t hw = buf_load_u32(rpg, (bit >> 5) * 4u + 4u);
                        hv = __builtin_amdgcn_alignbit(hw, lo, bit & 31u) & width_mask(k);
                    }
                    atomicOr(&L.buf[j * kBlock + (pos & (kBlock - 1u))], hv << b);
                }
            }
        }
        // beyond the page it reads nothing; the ring keeps the next pass's high parts
        f = fetch(p + 2, nx.e0 + (nx.ce < 64u ? nx.ce : 64u));
        wave_lds_order();
        const uint4 t0 = *reinterpret_cast<const uint4 *>(&L.buf[4 * lane]);
        const uint4 t1 = *reinterpret_cast<const uint4 *>(&L.buf[256 + 4 * lane]);
        uint32_t x[4] = {t0.x, t0.y, t0.z, t0.w}, y[4] = {t1.x, t1.y, t1.z, t1.w};
        if constexpr (S == 1) {
            x[1] += x[0];
            x[2] += x[1];
            x[3] += x[2];
            y[1] += y[0];
            y[2] += y[1];
            y[3] += y[2];
            const uint32_t ix = wave_scan_incl(x[3]), iy = wave_scan_incl(y[3]);
            const uint32_t tx = wave_read(ix, 63);
            const uint32_t ax = ix - x[3] + carry[0], ay = iy - y[3] + carry[0] + tx;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                x[r] += ax;
                y[r] += ay;
            }
            carry[0] += tx + wave_read(iy, 63);
        } else if constexpr (S == 4) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t ix = wave_scan_incl(x[c]), iy = wave_scan_incl(y[c]);
                const uint32_t tx = wave_read(ix, 63);
                x[c] = ix + carry[c];
                y[c] = iy + carry[c] + tx;
                carry[c] += tx + wave_read(iy, 63);
            }
        }
        // the pass's output; blocks past the segment fall outside the resource
        const BufRsrc rout = make_rsrc(out + (blk0 + 4u * p) * kBlock, (blk1 - blk0 - 4u * p) * (kBlock * 4u));
        buf_store_u4(rout, lane * 16u, 0u, make_uint4(x[0], x[1], x[2], x[3]));
        buf_store_u4(rout, 1024u + lane * 16u, 0u, make_uint4(y[0], y[1], y[2], y[3]));
    };
    // the ring keeps high parts from the segment's first exception on
    FpFetch f0 = fetch(0, wS);
    FpFetch f1 = fetch(1, wS + (f0.ce < 64u ? f0.ce : 64u));
    for (uint32_t p = 0; p < npass; p += 2) {
        if (p > 0 && (p & 15u) == 0) {
            // round p / 16 starts: build the next one, load the one after
            build_round((p >> 4) + 1, m0, m1, m2);
            load_meta((p >> 4) + 2, m0, m1, m2);
        }
        run_pass(p, f0, f1);
        if (p + 1 < npass)
            run_pass(p + 1, f1, f0);
        if constexpr (!WHOLE) {
            if (p == 2) {
                uint32_t t = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    t ^= pf[i].x ^ pf[i].y ^ pf[i].z ^ pf[i].w;
                asm volatile("" ::"v"(t));
            }
        }
    }
    // the page's last segment checks the totals: packed words, positions,
    // and each array's count (SimplePFOR: the Simple-8b words hold exactly
    // the page's exceptions); any other checks that its sums end on the
    // next segment's stored base
    if (last_seg) {
        bad = bad || pk_run != packed_words || 3u * nb + pos_run != meta_bytes;
        if constexpr (SP) {
            s8_fill(0xffffffffu, 0u, true);
            bad = bad || dec != pos_run;
        } else {
            bad = bad || (kl && L.kcar[lane + 1] != kcnt);
        }
    } else if constexpr (S > 0) {
        const uint32_t *const nsb = page + 4 + nset + S * seg;
#pragma unroll
        for (uint32_t t = 0; t < S; ++t)
            bad = bad || carry[t] != uniform(nsb[t]);
    }
    wave_lds_order();
    return ballot(bad) == 0;
}

// Full blocks of patched page u (512 except possibly the last).
__device__ __forceinline__ uint32_t page_blocks(const ListHdr &H, uint64_t u)
{
    const uint64_t left = H.nfull - u * kFpBlocks;
    return (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
}

// Segment `seg` of directory entry u (< H.units) of a patched-page stream
// decoded by one wavefront into out (the whole list's output): the entry's
// offset, length and bases, then fp_wave_page. Uniform result.
template <int KIND = kPageFp>
__device__ __forceinline__ bool fp_unit(const uint32_t *__restrict__ in, const ListHdr &H, uint64_t u, uint32_t seg,
                                        uint32_t *__restrict__ out, FpLdsOf<KIND> &L, uint32_t *ring = nullptr)
{
    const uint32_t off = uniform(in[kHdrWords + u]);
    const uint32_t end = (u + 1 < H.units) ? uniform(in[kHdrWords + u + 1]) : H.tail_off;
    const uint32_t *bp = in + kHdrWords + H.ndir + u * H.S;
    const uint32_t base[4] = {H.S > 0 ? uniform(bp[0]) : 0u, H.S > 1 ? uniform(bp[1]) : 0u,
                              H.S > 2 ? uniform(bp[2]) : 0u, H.S > 3 ? uniform(bp[3]) : 0u};
    const uint64_t left = H.nfull - u * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    if (!(off >= H.dir_end && end >= off && end <= H.total && (off & 3u) == 0))
        return false;
    const uint32_t *pg = in + off;
    uint32_t *po = out + u * kFpUnitInts;
    return H.S == 1   ? fp_wave_page<1, KIND>(pg, end - off, nb, seg, base, po, L, ring)
           : H.S == 4 ? fp_wave_page<4, KIND>(pg, end - off, nb, seg, base, po, L, ring)
                      : fp_wave_page<0, KIND>(pg, end - off, nb, seg, base, po, L, ring);
}

// ------------------------------------------------------------------------
// Full blocks held by meta-block u (16 except possibly the last).
__device__ __forceinline__ uint32_t unit_blocks(const ListHdr &H, uint64_t u)
{
    const uint64_t left = H.nfull - u * kBpBlocks;
    return (uint32_t)(left < kBpBlocks ? left : kBpBlocks);
}

constexpr uint32_t pow2ceil(uint32_t x)
{
    uint32_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

// Binary packing, one wavefront per run of meta-blocks (Section 6.2 format,
// Section 4 bit layout, Section 3 prefix sum).
//
// A wavefront decodes a run of consecutive meta-blocks by itself, so no
// workgroup barrier is involved. The run's compressed words (one contiguous
// range) stream through a private LDS ring in chunks of one 16-byte load
// per lane (256 words); DEPTH chunk loads stay in flight in named registers
// and are written to the ring a group at a time, whenever the next pass
// needs words that are not there yet.
//
// A pass decodes two blocks: lanes 0..31 the first, lanes 32..63 the
// second. Lane q of a block takes integers q, q+32, q+64 and q+96: integer
// q + 32m starts at bit q*b + 32*m*b, i.e. in word (q*b >> 5) + m*b at the
// same shift q*b & 31 for every m. Each integer costs an address add, a
// paired LDS read, a funnel shift and a mask, and the lanes of a block read
// consecutive words. The integers are then transposed through LDS so that
// lane l holds integers 4l..4l+3 of the pass for the prefix sum and the
// 16-byte stores.
//
// BP32 (B32): a pass is two meta-blocks of four 32-integer blocks, each
// meta-block behind its own descriptor word: eight blocks of eight lanes.
// Lane l takes integers 4l..4l+3 of the pass, four consecutive integers of
// one block, so its width, mask and block offset (the byte-wise prefix of
// the descriptor, one multiply) are computed once, the four fields follow
// each other at b bits, and the lane already holds what the prefix sum and
// the 16-byte store need: no transposition.
template <int DEPTH, bool B32 = false>
struct WaveGeo {
    static_assert(DEPTH >= 2 && DEPTH <= 4, "depth");
    static constexpr uint32_t CW = 256;               // words per chunk
    static constexpr uint32_t PASS = 2 * kBlock;      // integers of a pass
    // the most words a pass reads (BP32: two descriptors, and the next
    // pass's first descriptor, read ahead)
    static constexpr uint32_t PASSW = PASS + (B32 ? 3 : 0);
    // a group is written while the pass that needs it (at most PASSW words,
    // starting at or before the group) stays intact
    static constexpr uint32_t RB = pow2ceil(DEPTH * CW + PASSW);
    // ring words mirrored after the end: a block's reads run on past the
    // end (SIMD-BP128), or only one word does (BP32 wraps each address)
    static constexpr uint32_t MIR = B32 ? 4 : kBlock + 4;
    // words of the largest unit
    static constexpr uint32_t MAXU = (B32 ? kBpBlocks : 4) + kBpUnitInts;
};

template <int DEPTH, bool B32 = false>
struct alignas(16) WaveLds {
    uint32_t ring[WaveGeo<DEPTH, B32>::RB + WaveGeo<DEPTH, B32>::MIR];
    uint32_t xp[B32 ? 4 : WaveGeo<DEPTH, B32>::PASS];  // transposition of one pass (SIMD-BP128)
};

// Sum of the four byte lanes of each word, and whether any byte exceeds 32.
__device__ __forceinline__ uint32_t byte_sum(uint32_t d)
{
    const uint32_t s = (d & 0x00ff00ffu) + ((d >> 8) & 0x00ff00ffu);
    return (s & 0xffffu) + (s >> 16);
}
__device__ __forceinline__ bool byte_over32(uint32_t d)
{
    const uint32_t low5 = d & 0x1f1f1f1fu;
    const uint32_t nz = ((low5 + 0x7f7f7f7fu) & 0x80808080u) >> 7;  // low five bits non-zero
    const uint32_t b5 = (d >> 5) & 0x01010101u;                     // bit 5 set
    return (d & 0xc0c0c0c0u) != 0u || (nz & b5) != 0u;
}

// Decodes units [ua, ua + cnt) (cnt <= 63) of the list whose validated
// header is H, whose stride is S; one wavefront, its own LDS slice L.
// Returns the uniform validity of the run: on a bad run the wavefront
// stops, its output is unspecified but every store stays inside the run's
// output range.
//
// V (the four-lane vectorized block layout of Section 4, SIMD-BP128
// descriptors and sizes): lane q of a block takes integers 4q..4q+3, field
// q of each of the four 32-bit lanes, at the same bit offset q*b in each:
// two 16-byte LDS reads (the row holding the field start and the next
// row) and four funnel shifts, and again no transposition.
template <int DEPTH, uint32_t S, bool B32 = false, bool V = false>
__device__ __forceinline__ bool bp_wave_run(const uint32_t *__restrict__ in, const ListHdr &H, uint64_t ua, uint32_t cnt,
                            uint32_t *__restrict__ out, WaveLds<DEPTH, B32> &L)
{
    static_assert(!(B32 && V), "one block layout");
    using G = WaveGeo<DEPTH, B32>;
    constexpr uint32_t RB = G::RB, CW = G::CW;
    const uint32_t lane = lane_id();
    // the run's directory: lane i holds the offset of entry ua + i (i <= cnt)
    // and its bases
    uint32_t offv = 0;
    uint32_t bv[4] = {0u, 0u, 0u, 0u};
    if (lane <= cnt)
        offv = (ua + lane < H.units) ? in[kHdrWords + ua + lane] : H.tail_off;
    if (lane < cnt)
        for (uint32_t s = 0; s < S; ++s)
            bv[s] = in[kHdrWords + H.ndir + (ua + lane) * S + s];
    const uint32_t nxt = __shfl_down(offv, 1);
    const bool lane_bad = lane < cnt && (nxt < offv || nxt - offv > G::MAXU || (offv & 3u) != 0u);
    const uint32_t W0 = wave_read(offv, 0), Wend = wave_read(offv, cnt);
    if (ballot(lane_bad) != 0 || !(W0 >= H.dir_end && Wend <= H.total))
        return false;
    const uint32_t run_len = Wend - W0;  // <= 63 * MAXU words
    const BufRsrc rs = make_rsrc(in + W0, run_len * 4u);
    // output of the run: full blocks only (the tail belongs to another
    // workgroup); stores beyond the range are dropped by the hardware
    const uint64_t o0 = ua * kBpUnitInts;
    const uint64_t o1e = (ua + cnt) * kBpUnitInts, o2e = H.nfull * kBlock;
    const BufRsrc ro = make_rsrc(out + o0, (uint32_t)(((o1e < o2e ? o1e : o2e) - o0) * 4u));

    // slots are loaded, written and reloaded in the same order, so the
    // wait for a slot never covers a younger slot's load
    uint4 s0 = make_uint4(0, 0, 0, 0), s1 = s0, s2 = s0, s3 = s0;
    uint32_t written = 0;  // words of the run already in the ring
    if (run_len <= RB) {
        // the whole run fits the ring: every chunk loaded at once and
        // written before the first pass, so the passes' stores never share
        // a wait with a later load (a wait for a load also waits for every
        // older store)
        constexpr uint32_t NCH = RB / CW;
        uint4 ch[NCH];
#pragma unroll
        for (uint32_t k = 0; k < NCH; ++k)
            ch[k] = buf_load_u4(rs, (k * CW + lane * 4) * 4);  // beyond the run: zeros
#pragma unroll
        for (uint32_t k = 0; k < NCH; ++k) {
            const uint32_t pos = k * CW + lane * 4;
            *reinterpret_cast<uint4 *>(&L.ring[pos]) = ch[k];
            if (pos < G::MIR)
                *reinterpret_cast<uint4 *>(&L.ring[RB + pos]) = ch[k];
        }
        written = RB;
        wave_lds_order();
    } else {
        s0 = buf_load_u4(rs, (0 * CW + lane * 4) * 4);
        __builtin_amdgcn_sched_barrier(0);
        s1 = buf_load_u4(rs, (1 * CW + lane * 4) * 4);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DEPTH > 2)
            s2 = buf_load_u4(rs, (2 * CW + lane * 4) * 4);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (DEPTH > 3)
            s3 = buf_load_u4(rs, (3 * CW + lane * 4) * 4);
    }
    auto put = [&](uint4 &slot, uint32_t c) __attribute__((always_inline)) {
        const uint32_t pos = (c * CW + lane * 4) & (RB - 1);
        *reinterpret_cast<uint4 *>(&L.ring[pos]) = slot;
        if (pos < G::MIR)
            *reinterpret_cast<uint4 *>(&L.ring[RB + pos]) = slot;
        slot = buf_load_u4(rs, ((c + DEPTH) * CW + lane * 4) * 4);
    };
    // Brings the ring up to word `need` with at most one group: a pass
    // reads at most PASSW words starting at or before `written`, and a
    // descriptor starts where the previous meta-block ended, so one group
    // (DEPTH * CW >= PASSW words) always suffices for a consistent run (no
    // loop here: a loop would make every wait cover all younger stores).
    auto fill_to = [&](uint32_t need) __attribute__((always_inline)) {
        if (written < need) {
            const uint32_t c = written / CW;
            put(s0, c);
            put(s1, c + 1);
            if constexpr (DEPTH > 2)
                put(s2, c + 2);
            if constexpr (DEPTH > 3)
                put(s3, c + 3);
            written += DEPTH * CW;
        }
        return written >= need;
    };

    const uint32_t q = lane & 31u;
    const bool hi = lane >= 32u;
    const uint32_t sh32 = 8u * ((lane >> 3) & 3u), r4 = 4u * (lane & 7u);  // BP32 lane geometry
    uint32_t *const xw = &L.xp[lane + (hi ? 96u : 0u)];   // integer q of the lane's block
    const uint4 *const xr = reinterpret_cast<const uint4 *>(&L.xp[4 * lane]);
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t su = wave_read(offv, i) - W0, eu = wave_read(offv, i + 1) - W0;
        const uint32_t nb = unit_blocks(H, ua + i);
        if constexpr (B32) {
            uint32_t carry[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                carry[k] = wave_read(bv[k], i);
            const uint32_t sbase = i * (kBpUnitInts * 4u);
            uint32_t ps = su;     // the pass's first descriptor word
            uint32_t wmax = 0;    // widest block seen by the lane (checked at the unit's end)
            if (!fill_to(ps + G::PASSW))
                return false;
            uint32_t dnext = L.ring[ps & (RB - 1)];
            for (uint32_t p = 0; 2 * p < nb; ++p) {
                // one fill covers the largest pass and the next descriptor
                // (PASSW words from ps)
                if (!fill_to(ps + G::PASSW))
                    return false;
                const uint32_t dA = uniform(dnext);
                const bool hasB = 2 * p + 1 < nb;
                // (d * 0x01010101) >> 24: sum of the four widths (<= 128 when valid)
                const uint32_t pB = ps + 1u + ((dA * 0x01010101u) >> 24);
                const uint32_t dB = hasB ? uniform(L.ring[pB & (RB - 1)]) : 0u;
                const uint32_t pe = hasB ? pB + 1u + ((dB * 0x01010101u) >> 24) : pB;
                if (pe > eu)
                    return false;
                // the next pass's first descriptor, read now: its latency
                // overlaps this pass's unpacking
                dnext = L.ring[pe & (RB - 1)];
                // lane l: block jj = (l >> 3) & 3 of its meta-block,
                // integers 4r .. 4r+3 of the block, r = l & 7; byte jj of
                // d * 0x01010100 is the width of blocks 0..jj-1
                const uint32_t d = hi ? dB : dA;
                const uint32_t ex = hi ? dB * 0x01010100u : dA * 0x01010100u;
                const uint32_t b = (d >> sh32) & 255u;
                wmax = wmax > b ? wmax : b;
                const uint32_t o = (hi ? pB : ps) + 1u + ((ex >> sh32) & 255u);
                const uint32_t mask = width_mask(b);
                uint32_t pos = r4 * b;  // bit offset of the lane's first field
                uint32_t x[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t w = (o + (pos >> 5)) & (RB - 1);
                    x[k] = __builtin_amdgcn_alignbit(L.ring[w + 1], L.ring[w], pos) & mask;
                    pos += b;
                }
                scan_wave4<S>(x, carry);
                buf_store_u4(ro, lane * 16u, uniform(sbase + p * (G::PASS * 4u)), make_uint4(x[0], x[1], x[2], x[3]));
                ps = pe;
            }
            // widths <= 32, and the unit ends (zero-padded to 4 words)
            // where its last meta-block ends
            if (ballot(wmax > 32u) != 0 || ((ps - su + 3u) & ~3u) != eu - su)
                return false;
            continue;
        }
        if (!fill_to(su + 4))
            return false;
        const uint4 dsc = *reinterpret_cast<const uint4 *>(&L.ring[su & (RB - 1)]);
        const uint32_t d0 = uniform(dsc.x), d1 = uniform(dsc.y), d2 = uniform(dsc.z), d3 = uniform(dsc.w);
        // widths <= 32, none beyond the meta-block's blocks, sizes agree
        const uint32_t nbb = 8u * nb;  // descriptor bits in use
        const uint32_t k0 = nbb >= 32u ? 0u : (0xffffffffu << nbb);
        const uint32_t k1 = nbb >= 64u ? 0u : nbb <= 32u ? 0xffffffffu : (0xffffffffu << (nbb - 32u));
        const uint32_t k2 = nbb >= 96u ? 0u : nbb <= 64u ? 0xffffffffu : (0xffffffffu << (nbb - 64u));
        const uint32_t k3 = nbb >= 128u ? 0u : nbb <= 96u ? 0xffffffffu : (0xffffffffu << (nbb - 96u));
        const uint32_t sum = byte_sum(d0) + byte_sum(d1) + byte_sum(d2) + byte_sum(d3);
        if (byte_over32(d0) || byte_over32(d1) || byte_over32(d2) || byte_over32(d3) ||
            ((d0 & k0) | (d1 & k1) | (d2 & k2) | (d3 & k3)) != 0u || eu - su != 4u + 4u * sum)
            return false;
        uint32_t carry[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            carry[k] = wave_read(bv[k], i);
        uint32_t ps = su + 4;  // first word of the pass
        uint64_t dd = ((uint64_t)d1 << 32) | d0;
        const uint32_t sbase = i * (kBpUnitInts * 4u);
        for (uint32_t p = 0; 2 * p < nb; ++p) {
            if (p == 4)
                dd = ((uint64_t)d3 << 32) | d2;
            const uint32_t bA = (uint32_t)dd & 255u, bB = ((uint32_t)dd >> 8) & 255u;
            dd >>= 16;
            const uint32_t pe = ps + 4u * (bA + bB);
            if (!fill_to(pe))
                return false;
            const uint32_t b = hi ? bB : bA;
            const uint32_t st = hi ? ps + 4u * bA : ps;
            const uint32_t qb = q * b;
            const uint32_t mask = width_mask(b);
            uint32_t x[4];
            if constexpr (V) {
                // row (qb >> 5) of the block holds the start of field q of
                // every lane; rows are 16-byte aligned in the ring (blocks
                // are 4b words from a 16-byte aligned run), and the mirror
                // after the ring end covers the second row
                const uint32_t w0 = (st + 4u * (qb >> 5)) & (RB - 1);
                const uint4 r0 = *reinterpret_cast<const uint4 *>(&L.ring[w0]);
                const uint4 r1 = *reinterpret_cast<const uint4 *>(&L.ring[w0 + 4]);
                x[0] = __builtin_amdgcn_alignbit(r1.x, r0.x, qb) & mask;
                x[1] = __builtin_amdgcn_alignbit(r1.y, r0.y, qb) & mask;
                x[2] = __builtin_amdgcn_alignbit(r1.z, r0.z, qb) & mask;
                x[3] = __builtin_amdgcn_alignbit(r1.w, r0.w, qb) & mask;
            } else {
                const uint32_t w0 = (st + (qb >> 5)) & (RB - 1);
                uint32_t v[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint32_t w = w0 + m * b;
                    v[m] = __builtin_amdgcn_alignbit(L.ring[w + 1], L.ring[w], qb) & mask;
                }
                wave_lds_order();
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    xw[32 * m] = v[m];
                wave_lds_order();
                const uint4 t = *xr;
                x[0] = t.x;
                x[1] = t.y;
                x[2] = t.z;
                x[3] = t.w;
            }
            scan_wave4<S>(x, carry);
            buf_store_u4(ro, lane * 16u, sbase + p * (G::PASS * 4u), make_uint4(x[0], x[1], x[2], x[3]));
            ps = pe;
        }
    }
    return true;
}

}  // namespace wp
