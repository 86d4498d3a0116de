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
// LDS arena shared by all roles (a workgroup plays one role at a time).

// Page tables of a patched page (shared by the encoder and the decoder)
// plus, for the decoder, each wavefront's staging and transposition areas.
// The per-block tables are dead once the block records are built, so the
// passes' areas overlay them.
template <int WAVES>
struct FpLds {
    union {
        struct {
            uint32_t stage[WAVES][2 * kBlock + 4];  // a wavefront's two blocks of packed words (+1 word)
            uint32_t xp[WAVES][2 * kBlock];         // a wavefront's two blocks, transposed and patched
        };
        struct {
            uint8_t b[kFpBlocks];
            uint8_t mb[kFpBlocks];
            uint8_t c[kFpBlocks];
            uint32_t blkoff[kFpBlocks + 1];  // word offset of each block in the packed region
            uint32_t posoff[kFpBlocks + 1];  // offset of each block's positions
            uint32_t rank[kFpBlocks];        // index of the block's first exception in its array
        };
    };
    // per block: {b | k << 8 | c << 16, packed word offset, bit offset of its
    // first exception's high part, position offset}; zero past the last block
    // (the passes fetch up to four passes of 2 * WAVES blocks ahead)
    uint4 rec[kFpBlocks + 8 * WAVES];
    uint32_t ktot[WAVES][33];
    uint32_t kcar[33];
    uint32_t excbase[33];            // word offset of array k from the page start
    uint32_t kcnt[33];
    uint32_t stot[WAVES][2];
    uint32_t wtot[2][WAVES][4];
    uint32_t bad;
};

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
// Patched pages (Section 5): decoding a pair of blocks in one wavefront.
//
// Every block of a page is described by one 16-byte record {b | k << 8 |
// c << 16, packed word offset, bit offset of its first exception's high
// part, position offset}, k = maxb - b; the record arrays are zero-padded
// past the page's last block, so fetching beyond it reads nothing. A
// wavefront takes two blocks at a time and unpacks them as the
// binary-packing decoder does (lanes 0..31 the first, 32..63 the second,
// strided fields, LDS transpose); lane e patches exception e of the pair
// (position byte and k-bit high part, OR-ed in above bit b; a pair with
// more than 64 exceptions patches the rest in a slower loop). Each lane
// reads the record of its own block and the record of its exception's
// block; the pair's packed words, one exception per lane and everything
// needed to place it are fetched by `fetch` into registers ahead of use.
struct FpPairFetch {
    uint32_t bA, cA, ce;      // width and exceptions of block A, exceptions of the pair (uniform)
    uint4 pk;                 // the pair's packed words, 16 bytes per lane
    uint32_t pos, lo, hi;     // exception `lane`: position byte, words of its high part
    // exception `lane`: bit shift of its high part | its block's b << 8 |
    // 128 * (its block is B) << 16; bits 24..29: the width of the lane's own
    // block (lanes 0..31 block A, 32..63 block B)
    uint32_t em;
    uint32_t km;              // exception `lane`: mask of its k high bits
};

struct FpPair {
    const uint32_t *page;
    const uint4 *rec;  // the page's block records (LDS, zero-padded)
    uint32_t hdr_w, pos_at;
    BufRsrc rpg;
    uint32_t *stg, *xpw;  // this wavefront's staging and transposition areas (LDS)

    static constexpr uint32_t kOut = 0xfffffff0u;  // a buffer offset beyond every page: reads nothing

    // blocks jA, jA + 1 (records past the page are zero: no words, no exceptions)
    __device__ __forceinline__ FpPairFetch fetch(uint32_t jA) const
    {
        const uint32_t lane = lane_id();
        FpPairFetch f;
        const uint4 rm = rec[jA + (lane >> 5)];
        const uint32_t a0 = wave_read(rm.x, 0), b0 = wave_read(rm.x, 32), ay = wave_read(rm.y, 0);
        f.bA = a0 & 255u;
        f.cA = a0 >> 16;
        f.ce = f.cA + (b0 >> 16);
        const BufRsrc rp = make_rsrc(page + hdr_w + ay, 16u * (f.bA + (b0 & 255u)));
        f.pk = buf_load_u4(rp, lane * 16u);
        const bool inA = lane < f.cA;
        const uint4 re = rec[jA + (inA ? 0u : 1u)];
        const uint32_t idx = lane - (inA ? 0u : f.cA);
        const uint32_t k = (re.x >> 8) & 255u;
        const uint32_t bit = re.z + idx * k;
        const bool any = lane < f.ce;
        const uint32_t poff = any ? pos_at + re.w + idx : kOut;
        const uint32_t woff = any ? (bit >> 5) * 4u : kOut;
        f.pos = __builtin_amdgcn_raw_buffer_load_b8(rpg, (int)poff, 0, 0);
        f.lo = buf_load_u32(rpg, woff);
        f.hi = buf_load_u32(rpg, woff + 4u);
        f.em = (bit & 31u) | ((re.x & 255u) << 8) | (inA ? 0u : (kBlock << 16)) | ((rm.x & 255u) << 24);
        f.km = width_mask(k);
        return f;
    }

    // Unpacks and patches blocks jA, jA + 1 from f into the transposition
    // area; after it, lane l's integers 4l..4l+3 of the pair are read with
    // read_back(). f may be refilled once this returns. Exception positions
    // that are not below 128 or not ascending inside their block set `bad`
    // (a per-lane flag the caller reduces once per page).
    __device__ __forceinline__ void unpack_patch(const FpPairFetch &f, uint32_t jA, bool &bad) const
    {
        const uint32_t lane = lane_id();
        const uint32_t q = lane & 31u;
        const bool hi = lane >= 32u;
        *reinterpret_cast<uint4 *>(&stg[4 * lane]) = f.pk;
        wave_lds_order();
        const uint32_t b = f.em >> 24;
        const uint32_t qb = q * b;
        const uint32_t w0 = (hi ? 4u * f.bA : 0u) + (qb >> 5);
        const uint32_t mask = width_mask(b);
        uint32_t v[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const uint32_t wi = w0 + m * b;
            v[m] = __builtin_amdgcn_alignbit(stg[wi + 1], stg[wi], qb) & mask;
        }
        uint32_t *const xw = &xpw[lane + (hi ? 96u : 0u)];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            xw[32 * m] = v[m];
        wave_lds_order();
        // exceptions: one per lane, the rest (more than 64 in the pair) in rounds
        const uint32_t prev = (uint32_t)__shfl_up((int)f.pos, 1, 64);
        if (lane < f.ce) {
            const uint32_t hv = __builtin_amdgcn_alignbit(f.hi, f.lo, f.em) & f.km;
            atomicOr(&xpw[((f.em >> 16) & 255u) + (f.pos & (kBlock - 1u))], hv << ((f.em >> 8) & 255u));
            bad = bad || f.pos >= kBlock || (lane != 0 && lane != f.cA && prev >= f.pos);
        }
        for (uint32_t e0 = 64; e0 < f.ce; e0 += 64) {
            const uint32_t e = e0 + lane;
            if (e < f.ce) {
                const bool inA = e < f.cA;
                const uint4 re = rec[jA + (inA ? 0u : 1u)];
                const uint32_t idx = inA ? e : e - f.cA;
                const uint32_t k = (re.x >> 8) & 255u;
                const uint32_t bit = re.z + idx * k;
                const uint8_t *const pb = reinterpret_cast<const uint8_t *>(page) + pos_at + re.w + idx;
                const uint32_t pos = pb[0], pprev = idx > 0 ? pb[-1] : 0u;
                bad = bad || pos >= kBlock || (idx > 0 && pprev >= pos);
                const uint32_t lo = page[bit >> 5];
                const uint32_t hw = (bit & 31u) + k > 32u ? page[(bit >> 5) + 1u] : 0u;
                const uint32_t hv = __builtin_amdgcn_alignbit(hw, lo, bit) & width_mask(k);
                atomicOr(&xpw[(inA ? 0u : kBlock) + (pos & (kBlock - 1u))], hv << (re.x & 255u));
            }
        }
    }

    __device__ __forceinline__ void read_back(uint32_t (&x)[4]) const
    {
        wave_lds_order();
        const uint4 t = *reinterpret_cast<const uint4 *>(&xpw[4 * lane_id()]);
        x[0] = t.x;
        x[1] = t.y;
        x[2] = t.z;
        x[3] = t.w;
    }
};

// Patched page (Section 5) decoded by a whole workgroup. `page` points at
// the page header (16-byte aligned), `nwords` its length, `nb` the number
// of blocks it must hold. Setup (bounded by nb): the exception-array
// directory, the block metadata, block offsets in the packed region,
// offsets into the position bytes and, per block, the index of its first
// exception inside its array k = maxb - b (exceptions are appended to
// array k in block order, so this is the number of exceptions of earlier
// blocks with the same k); then the block records. Then passes of 2 * WAVES
// blocks: wavefront w decodes pair w of the pass (FpPair), the words and
// exceptions of the next SLOTS - 1 passes in flight; one barrier per pass
// hands the wavefront totals over for the prefix sum.
template <int WAVES, uint32_t S, int SLOTS = 3, bool P32 = false>
__device__ __forceinline__ bool fp_page(const uint32_t *__restrict__ page, uint32_t nwords, uint32_t nb,
                        const uint32_t (&base)[4], uint32_t *__restrict__ out, FpLds<WAVES> &L)
{
    constexpr int T = 64 * WAVES;
    static_assert(T <= (int)kFpBlocks, "setup maps at most one thread per block and round");
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    if (nwords < 4)
        return false;
    const uint32_t h_nb = uniform(page[0]), packed_words = uniform(page[1]), meta_bytes = uniform(page[2]),
                   bitset = uniform(page[3]);
    const uint32_t nset = __builtin_popcount(bitset);
    const uint32_t hdr_w = pad4(4 + nset);
    const uint32_t meta_w = ((meta_bytes + 15u) / 16u) * 4u;
    if (h_nb != nb || nb == 0 || hdr_w > nwords || packed_words > nwords - hdr_w ||
        meta_bytes < 3 * nb || meta_bytes > 3 * nb + 127 * nb || meta_w > nwords - hdr_w - packed_words ||
        (packed_words & 3u))
        return false;
    const uint32_t exc_at = hdr_w + packed_words + meta_w;
    const uint8_t *meta = reinterpret_cast<const uint8_t *>(page + hdr_w + packed_words);

    // exception array directory: lanes 0..31 of wave 0 own k = lane + 1
    if (wave == 0) {
        const bool kl = lane < 32;
        const uint32_t k = lane + 1;
        const bool set = kl && ((bitset >> (lane & 31u)) & 1u);
        const uint32_t ci = kl ? (uint32_t)__builtin_popcount(bitset & ((1u << (lane & 31u)) - 1u)) : 0u;
        const uint32_t cnt = set ? page[4 + ci] : 0u;
        const bool badk = set && (cnt == 0 || cnt > nb * kBlock);
        const uint32_t wk = (set && !badk) ? exc_array_words<P32>(cnt, k) : 0u;
        const uint32_t incl = wave_scan_incl(wk);
        const uint32_t tot = wave_read(incl, 63);
        const uint64_t anybad = ballot(badk);
        if (kl) {
            L.excbase[k] = exc_at + incl - wk;
            L.kcnt[k] = cnt;
        }
        if (lane < 33)
            L.kcar[lane] = 0;
        if (lane == 32) {
            L.excbase[0] = exc_at;
            L.kcnt[0] = 0;
        }
        if (lane == 0)
            L.bad = (anybad != 0 || (P32 ? pad4(exc_at + tot) : exc_at + tot) != nwords) ? 1u : 0u;
    }
    const uint32_t nbr = ((nb + T - 1) / T) * T;  // the rounds of the table pass (entries beyond nb are 0)
    for (uint32_t t = tid; t < nbr; t += T) {
        uint32_t b = 0, mb = 0, c = 0;
        if (t < nb) {
            b = meta[t];
            mb = meta[nb + t];
            c = meta[2 * nb + t];
        }
        L.b[t] = (uint8_t)b;
        L.mb[t] = (uint8_t)mb;
        L.c[t] = (uint8_t)c;
    }
    for (uint32_t i = tid; i < WAVES * 33; i += T)
        (&L.ktot[0][0])[i] = 0;
    __syncthreads();
    // validate block metadata
    for (uint32_t t = tid; t < nb; t += T) {
        const uint32_t b = L.b[t], mb = L.mb[t], c = L.c[t];
        if (b > 32 || mb > 32 || mb < b || c >= kBlock || ((c == 0) != (mb == b)))
            L.bad = 1;
    }
    uint32_t carry_w = 0, carry_p = 0;
    fp_tables<WAVES>(L, nb, carry_w, carry_p);
    if (tid == 0) {
        L.blkoff[kFpBlocks] = carry_w;
        if (carry_w != packed_words || 3 * nb + carry_p != meta_bytes)
            L.bad = 1;
    }
    if (tid >= 1 && tid <= 32 && L.kcar[tid] != L.kcnt[tid])
        L.bad = 1;
    __syncthreads();
    if (L.bad)
        return false;

    // block records (zero past the last block)
    const uint32_t pos_at = (hdr_w + packed_words) * 4u + 3u * nb;  // byte offset of the positions
    const BufRsrc rpg = make_rsrc(page, nwords * 4u);
    for (uint32_t t = tid; t < nb + 8 * WAVES; t += T) {
        if (t < nb) {
            const uint32_t b = L.b[t], k = (uint32_t)L.mb[t] - b, c = L.c[t];
            L.rec[t] = make_uint4(b | (k << 8) | (c << 16), L.blkoff[t],
                                  L.excbase[k <= 32 ? k : 0] * 32u + L.rank[t] * k, L.posoff[t]);
        } else {
            L.rec[t] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    __syncthreads();

    // passes of 2 * WAVES blocks
    constexpr uint32_t BPP = 2 * WAVES;
    const FpPair pair{page, L.rec, hdr_w, pos_at, rpg, L.stage[wave], L.xp[wave]};
    const BufRsrc rout = make_rsrc(out, nb * kBlock * 4u);
    uint32_t carry[4] = {base[0], base[1], base[2], base[3]};
    const uint32_t npass = (nb + BPP - 1) / BPP;
    bool bad_pos = false;
    // pass p from slot f; the slot is refilled with pass p + SLOTS as soon
    // as its words and exceptions have been used (named slots, so nothing
    // is copied between passes; with three, a wait for a slot's loads rarely
    // covers the stores of the two passes issued after them)
    static_assert(SLOTS == 2 || SLOTS == 3, "fetch slots");
    auto run_pass = [&](uint32_t p, FpPairFetch &f) __attribute__((always_inline)) {
        const uint32_t jA = p * BPP + 2u * wave;
        pair.unpack_patch(f, jA, bad_pos);
        f = pair.fetch((p + SLOTS) * BPP + 2u * wave);  // beyond the page it reads nothing
        uint32_t x[4];
        pair.read_back(x);
        // prefix sum: inside the wavefront, then across wavefronts
        if constexpr (S == 1) {
            x[1] += x[0];
            x[2] += x[1];
            x[3] += x[2];
            const uint32_t incl = wave_scan_incl(x[3]);
            if (lane == 63)
                L.wtot[p & 1][wave][0] = incl;
            __syncthreads();
            uint32_t before = carry[0], all = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint32_t tw = uniform(L.wtot[p & 1][w][0]);
                before += w < (int)wave ? tw : 0u;
                all += tw;
            }
            const uint32_t add = incl - x[3] + before;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                x[r] += add;
            carry[0] += all;
        } else if constexpr (S == 4) {
            uint32_t incl[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                incl[c] = wave_scan_incl(x[c]);
            if (lane == 63)
                *reinterpret_cast<uint4 *>(&L.wtot[p & 1][wave][0]) = make_uint4(incl[0], incl[1], incl[2], incl[3]);
            __syncthreads();
            uint32_t before[4] = {carry[0], carry[1], carry[2], carry[3]};
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint4 tw = *reinterpret_cast<const uint4 *>(&L.wtot[p & 1][w][0]);
                const uint32_t tv[4] = {uniform(tw.x), uniform(tw.y), uniform(tw.z), uniform(tw.w)};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    before[c] += w < (int)wave ? tv[c] : 0u;
                    carry[c] += tv[c];
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                x[c] = incl[c] + before[c];
        }
        buf_store_u4(rout, lane * 16u, uniform(jA * (kBlock * 4u)), make_uint4(x[0], x[1], x[2], x[3]));
    };
    uint32_t p = 0;
    if constexpr (SLOTS == 3) {
        FpPairFetch f0 = pair.fetch(2u * wave), f1 = pair.fetch(BPP + 2u * wave),
                    f2 = pair.fetch(2 * BPP + 2u * wave);
        for (; p + 3 <= npass; p += 3) {
            run_pass(p, f0);
            run_pass(p + 1, f1);
            run_pass(p + 2, f2);
        }
        if (p < npass)
            run_pass(p, f0);
        if (p + 1 < npass)
            run_pass(p + 1, f1);
    } else {
        FpPairFetch f0 = pair.fetch(2u * wave), f1 = pair.fetch(BPP + 2u * wave);
        for (; p + 2 <= npass; p += 2) {
            run_pass(p, f0);
            run_pass(p + 1, f1);
        }
        if (p < npass)
            run_pass(p, f0);
    }
    const bool any_bad_pos = ballot(bad_pos) != 0;
    if (lane == 0 && any_bad_pos)
        L.bad = 1;
    __syncthreads();
    return L.bad == 0;
}

// A small patched page (nb <= 64 blocks) decoded by one wavefront, with no
// workgroup barrier: the same setup with one lane per block (tables by wave
// scans, ranks by one masked scan per distinct k), then the pairs in order
// with the prefix sum carried inside the wavefront. Used by the batched
// decoder for the short lists' pages.
struct alignas(16) FpWaveLds {
    uint32_t stage[2 * kBlock + 4];
    uint32_t xp[2 * kBlock];
    uint4 rec[64 + 8];  // zero past the last block (fetches run two pairs ahead)
};

template <uint32_t S, bool P32 = false>
__device__ __forceinline__ bool fp_small_page(const uint32_t *__restrict__ page, uint32_t nwords, uint32_t nb,
                              const uint32_t (&base)[4], uint32_t *__restrict__ out, FpWaveLds &L)
{
    const uint32_t lane = lane_id();
    if (nwords < 4 || nb == 0 || nb > 64)
        return false;
    const uint32_t h_nb = uniform(page[0]), packed_words = uniform(page[1]), meta_bytes = uniform(page[2]),
                   bitset = uniform(page[3]);
    const uint32_t nset = __builtin_popcount(bitset);
    const uint32_t hdr_w = pad4(4 + nset);
    const uint32_t meta_w = ((meta_bytes + 15u) / 16u) * 4u;
    if (h_nb != nb || hdr_w > nwords || packed_words > nwords - hdr_w || meta_bytes < 3 * nb ||
        meta_bytes > 3 * nb + 127 * nb || meta_w > nwords - hdr_w - packed_words || (packed_words & 3u))
        return false;
    const uint32_t exc_at = hdr_w + packed_words + meta_w;
    const uint8_t *meta = reinterpret_cast<const uint8_t *>(page + hdr_w + packed_words);
    // exception array directory: lane k - 1 owns array k
    const bool kl = lane < 32;
    const uint32_t kown = lane + 1;
    const bool set = kl && ((bitset >> (lane & 31u)) & 1u);
    const uint32_t ci = kl ? (uint32_t)__builtin_popcount(bitset & ((1u << (lane & 31u)) - 1u)) : 0u;
    const uint32_t cnt = set ? page[4 + ci] : 0u;
    const bool badk = set && (cnt == 0 || cnt > nb * kBlock);
    const uint32_t wk = (set && !badk) ? exc_array_words<P32>(cnt, kown) : 0u;
    const uint32_t kincl = wave_scan_incl(wk);
    const uint32_t excb = exc_at + kincl - wk;  // lane k - 1: first word of array k
    const uint32_t exc_end = exc_at + wave_read(kincl, 63);
    bool bad = ballot(badk) != 0 || (P32 ? pad4(exc_end) : exc_end) != nwords;
    // blocks: lane j owns block j
    const bool own = lane < nb;
    const uint32_t b = own ? meta[lane] : 0u, mb = own ? meta[nb + lane] : 0u, c = own ? meta[2 * nb + lane] : 0u;
    bad = bad || ballot(own && (b > 32 || mb > 32 || mb < b || c >= kBlock || ((c == 0) != (mb == b)))) != 0;
    const uint32_t k = own && mb >= b ? mb - b : 0u;
    const uint32_t bincl = wave_scan_incl(4u * b), cincl = wave_scan_incl(c);
    const uint32_t cnt_all = wave_read(wave_scan_incl(cnt), 63);
    bad = bad || wave_read(bincl, 63) != packed_words || 3 * nb + wave_read(cincl, 63) != meta_bytes ||
          wave_read(cincl, 63) != cnt_all;
    // rank of each block's first exception in its array: one masked scan per distinct k
    uint32_t rank = 0;
    uint64_t todo = ballot(c > 0 && k >= 1 && k <= 32);
    while (todo) {
        const uint32_t lead = (uint32_t)__builtin_ctzll(todo);
        const uint32_t k0 = wave_read(k, lead);
        const bool mine = c > 0 && k == k0;
        const uint64_t mm = ballot(mine);
        const uint32_t xc = mine ? c : 0u;
        const uint32_t incl = wave_scan_incl(xc);
        if (mine)
            rank = incl - xc;
        bad = bad || wave_read(incl, 63) != wave_read(cnt, (int)k0 - 1);
        todo &= ~mm;
    }
    const uint32_t eb = __shfl(excb, (int)(k >= 1 ? k - 1 : 0));
    const uint32_t pos_at = (hdr_w + packed_words) * 4u + 3u * nb;
    const BufRsrc rpg = make_rsrc(page, nwords * 4u);
    if (own)
        L.rec[lane] = make_uint4(b | (k << 8) | (c << 16), bincl - 4u * b, (c > 0 ? eb * 32u + rank * k : 0u),
                                 cincl - c);
    if (lane < 8)
        L.rec[nb + lane] = make_uint4(0u, 0u, 0u, 0u);
    if (bad)
        return false;
    wave_lds_order();

    const FpPair pair{page, L.rec, hdr_w, pos_at, rpg, L.stage, L.xp};
    const BufRsrc rout = make_rsrc(out, nb * kBlock * 4u);
    uint32_t carry[4] = {base[0], base[1], base[2], base[3]};
    const uint32_t npass = (nb + 1) / 2;
    bool bad_pos = false;
    auto run_pass = [&](uint32_t p, FpPairFetch &f) __attribute__((always_inline)) {
        pair.unpack_patch(f, 2u * p, bad_pos);
        f = pair.fetch(2u * (p + 2));
        uint32_t x[4];
        pair.read_back(x);
        scan_wave4<S>(x, carry);
        buf_store_u4(rout, lane * 16u, p * (2u * kBlock * 4u), make_uint4(x[0], x[1], x[2], x[3]));
    };
    FpPairFetch f0 = pair.fetch(0), f1 = pair.fetch(2);
    uint32_t p = 0;
    for (; p + 2 <= npass; p += 2) {
        run_pass(p, f0);
        run_pass(p + 1, f1);
    }
    if (p < npass)
        run_pass(p, f0);
    wave_lds_order();
    return ballot(bad_pos) == 0;
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
    uint4 s0, s1, s2, s3;
    s0 = buf_load_u4(rs, (0 * CW + lane * 4) * 4);
    __builtin_amdgcn_sched_barrier(0);
    s1 = buf_load_u4(rs, (1 * CW + lane * 4) * 4);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DEPTH > 2)
        s2 = buf_load_u4(rs, (2 * CW + lane * 4) * 4);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DEPTH > 3)
        s3 = buf_load_u4(rs, (3 * CW + lane * 4) * 4);
    uint32_t written = 0;  // words of the run already in the ring
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
