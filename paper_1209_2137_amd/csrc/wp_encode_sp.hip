// SimplePFOR pages (Section 5, SimplePFOR; Simple-8b of Section 2): the
// encoder's per-page kernels. Widths, exception counts and positions are
// those of the patched pages (the same cost rule, computed by the patched
// encoder's analysis kernel); the exceptions' high parts of a page, in
// block order, are coded once with Simple-8b.
//
// One workgroup of four wavefronts per page, in chunks of blocks whose
// exceptions fit a 4096-entry LDS ring (a page's 7000 or so exceptions in
// two chunks; at most 102 per block under the cost rule, so a chunk holds at
// least nine groups of four blocks). Two kernels, as for every unit: the
// size kernel finds the page's Simple-8b words and its length, the chained
// scan turns lengths into offsets, and the packer writes the page.
//
// Size kernel, per chunk:
//  1. gather: the patched analysis (in its SimplePFOR form) has written
//     each block's exceptions' high-part widths, one byte each in position
//     order, to a 128-byte slot per block; 16 lanes per block copy them into
//     the ring at their index in the page (the input is not read again);
//  2. counts: Simple-8b's greedy choice at a position depends only on the
//     high parts from there on, so every position gets, in parallel, the
//     number of values the greedy word starting there would hold: the largest
//     count whose width holds the widest of that many values (a count that
//     fits makes every smaller count fit, so the scan stops at the first
//     that does not: three or four values of width near 17 are read);
//  3. walk: the word starts are the chain 0, 0 + count(0), ... . By windows
//     of 64 positions: every position's exit from its window (the chain's
//     first position past the window) by pointer jumping within the window;
//     the windows' entries one after another (one lookup per window); then
//     one lane per window walks its window from its entry. The word starts
//     go to scratch (16-bit indices, per page), with the words after each
//     chunk.
// The chunk's counts are computed for positions whose 60 following high
// parts are in the ring (the last 59 of a chunk wait for the next one, which
// the ring keeps them for), and the walk stops at the first word start
// beyond them.
//
// Packer, per chunk: the wavefronts load four blocks at a time (64 lanes,
// eight values each), find each block's exceptions (16 lanes per block),
// keep their high parts in the ring at their index in the page and write
// the blocks' low bits (staged in LDS, stored as words) and the metadata
// bytes (widths, maximum widths, counts, positions); then one thread per
// word of the chunk assembles it from the ring (its count: the distance to
// the next word's start) with the segment entries it holds.
#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

namespace {

constexpr uint32_t kSpThreads = 256;
constexpr uint32_t kSpWaves = kSpThreads / 64;
constexpr uint32_t kSpR = 4096;                 // ring of a page's high parts, by index mod kSpR
constexpr uint32_t kSpChunkExc = kSpR - 64;     // a chunk's exceptions: the ring keeps the 59 before them too
constexpr uint32_t kSpQuadInts = 4u * kBlock;   // a wavefront's step: four blocks, eight values a lane
constexpr uint32_t kSpDepth = 4;                // the packer's steps in flight per wavefront
static_assert(kSpChunkExc >= 4u * 102u, "a chunk holds at least one step's exceptions");

__device__ __forceinline__ uint32_t sp_nbits(uint32_t x) { return 32u - (uint32_t)__clz((int)x); }

// Words of a SimplePFOR page's header: 4, then for each 64-block segment
// after the first S bases and one Simple-8b entry, padded to 4.
__device__ __forceinline__ uint32_t sp_hdr_words(uint32_t nb, uint32_t S)
{
    return pad4(4u + (S + 1u) * (page_items<kPageFp>(nb) - 1u));
}

// Simple-8b's non-zero modes by increasing count (selectors 15 down to 2):
// values per word and their width.
constexpr uint32_t kS8Modes = 14;
__device__ constexpr uint8_t kS8Cnt[kS8Modes] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 15, 20, 30, 60};
__device__ constexpr uint8_t kS8Bits[kS8Modes] = {60, 30, 20, 15, 12, 10, 8, 7, 6, 5, 4, 3, 2, 1};

// Values in the greedy word starting at position p (avail high parts from
// p on, widths in the ring): the largest count whose width holds the widest
// of its first `count` values. Count 1 always fits (a high part has at most
// 32 bits).
__device__ __forceinline__ uint32_t sp_greedy_count(const uint8_t *__restrict__ wd, uint32_t p, uint32_t avail)
{
    uint32_t w = 0, best = 1;
#pragma unroll
    for (uint32_t j = 0; j < kS8Modes; ++j) {
        const uint32_t c = kS8Cnt[j];
        if (c > avail)
            break;
#pragma unroll
        for (uint32_t m = j ? kS8Cnt[j - 1] : 0u; m < c; ++m) {
            const uint32_t v = wd[(p + m) & (kSpR - 1u)];
            w = v > w ? v : w;
        }
        if (w > kS8Bits[j])
            break;
        best = c;
    }
    return best;
}

// Selector of the word holding `count` values.
__device__ __forceinline__ uint32_t sp_selector(uint32_t count)
{
    uint32_t j = 0;
#pragma unroll
    for (uint32_t i = 0; i < kS8Modes - 1; ++i)
        j += count > kS8Cnt[i] ? 1u : 0u;
    return 15u - j;
}

// Per-page scratch of the two kernels: the words after each chunk (at most
// 16 chunks: each but the last holds nine or more steps), the page's word
// count, then the word starts (indices of their first high part; a word
// holds at least one, so at most as many words as exceptions).
constexpr uint32_t kSpMaxExc = kFpBlocks * 102u;  // the cost rule's bound on a page's exceptions
constexpr uint32_t kSpTab = 32;                   // chunk table words; the last: the page's words
static_assert(kSpChunkExc / (4u * 102u) >= 9u && (kFpBlocks / 4u + 8u) / 9u < kSpTab, "chunks fit the table");
constexpr uint64_t kSpSlotBytes = 4u * kSpTab + 2u * kSpMaxExc;
static_assert(kSpMaxExc < 65536u && kSpSlotBytes % 16u == 0, "16-bit word starts; aligned slots");

template <bool WRITE>
struct SpLds {
    uint32_t exc[kFpBlocks + 1];             // exceptions before block t in the page (exc[nb]: all)
    uint32_t blk[WRITE ? kFpBlocks + 1 : 1];  // (packer) block t's first packed word, from the packed region
    uint32_t hv[WRITE ? kSpR : 1];            // (packer) high parts (ring)
    uint32_t st[WRITE ? kSpWaves * 512u : 1];  // (packer) a wavefront's step of low bits: four blocks of at most 128 words
    uint32_t pos0;                           // (size) the chain's first word start in the chunk
    uint32_t pw;                             // packed words of the page
    uint8_t b[kFpBlocks], mb[WRITE ? kFpBlocks : 1], c[kFpBlocks];
    uint8_t wd[WRITE ? 1 : kSpR];             // (size) widths of the high parts (ring)
    uint8_t cnt[WRITE ? 1 : kSpR];            // (size) values of the greedy word starting there (ring)
    uint8_t xo[WRITE ? 1 : kSpR];             // (size) where the chain from there leaves its window, past its end
};

// Deltas of the eight values of lane `lane` in step q of the page (values
// 512 q + 8 lane ...), from the step's two loads and, for lane 0, the four
// values before the step.
template <uint32_t S>
__device__ __forceinline__ void sp_deltas(const uint4 &a, const uint4 &bq, const uint4 &pv, uint32_t lane,
                                          uint32_t (&d)[8])
{
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, bq.x, bq.y, bq.z, bq.w};
    if constexpr (S == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            d[k] = v[k];
    } else if constexpr (S == 1) {
        uint32_t prev = (uint32_t)__shfl_up((int)v[7], 1, 64);
        if (lane == 0)
            prev = pv.w;
        d[0] = v[0] - prev;
#pragma unroll
        for (int k = 1; k < 8; ++k)
            d[k] = v[k] - v[k - 1];
    } else {
        uint32_t p[4] = {(uint32_t)__shfl_up((int)v[4], 1, 64), (uint32_t)__shfl_up((int)v[5], 1, 64),
                         (uint32_t)__shfl_up((int)v[6], 1, 64), (uint32_t)__shfl_up((int)v[7], 1, 64)};
        if (lane == 0)
            p[0] = pv.x, p[1] = pv.y, p[2] = pv.z, p[3] = pv.w;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            d[k] = v[k] - p[k];
#pragma unroll
        for (int k = 4; k < 8; ++k)
            d[k] = v[k] - v[k - 4];
    }
}

}  // namespace

// One workgroup per page. WRITE = false: the page's length in words into
// sizes[p], its word starts and chunk table into its scratch slot `spw`.
// WRITE = true (sizes: inclusive sums of the page lengths): the page at its
// offset, its directory entry, header, low bits, metadata and Simple-8b
// words, from its slot.
template <uint32_t S, bool WRITE>
__global__ __launch_bounds__(kSpThreads) void k_sp_page(const uint32_t *__restrict__ x, uint64_t n,
                                                        const uint8_t *__restrict__ meta, uint64_t nblk,
                                                        uint32_t *__restrict__ sizes, uint8_t *__restrict__ spw,
                                                        const uint8_t *__restrict__ spx, uint32_t dir_end,
                                                        uint32_t *__restrict__ out)
{
    __shared__ SpLds<WRITE> L;
    const uint64_t p = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - p * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    const uint64_t pstart = p * kFpUnitInts;
    uint32_t *const tab = reinterpret_cast<uint32_t *>(spw + p * kSpSlotBytes);
    uint16_t *const starts = reinterpret_cast<uint16_t *>(spw + p * kSpSlotBytes + 4u * kSpTab);
    // the page's metadata, then exclusive sums of 4b and c in block order
    for (uint32_t t = tid; t < nb; t += kSpThreads) {
        L.b[t] = meta[p * kFpBlocks + t];
        if constexpr (WRITE)
            L.mb[t] = meta[nblk + p * kFpBlocks + t];
        L.c[t] = meta[2 * nblk + p * kFpBlocks + t];
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t cw = 0, cc = 0;
        for (uint32_t t0 = 0; t0 < nb; t0 += 64) {
            const uint32_t t = t0 + lane;
            const uint32_t bw = t < nb ? 4u * L.b[t] : 0u, c = t < nb ? (uint32_t)L.c[t] : 0u;
            const uint32_t iw = wave_scan_incl(bw), ic = wave_scan_incl(c);
            if (t < nb) {
                if constexpr (WRITE)
                    L.blk[t] = cw + iw - bw;
                L.exc[t] = cc + ic - c;
            }
            cw += wave_read(iw, 63);
            cc += wave_read(ic, 63);
        }
        if (lane == 0) {
            L.exc[nb] = cc;
            L.pw = cw;
            if constexpr (WRITE)
                L.blk[nb] = cw;
        }
    }
    __syncthreads();
    const uint32_t nexc = L.exc[nb];
    const uint32_t nseg = page_items<kPageFp>(nb), hw = sp_hdr_words(nb, S);
    const uint32_t meta_bytes = 3u * nb + nexc;
    const uint32_t meta_w = ((meta_bytes + 15u) / 16u) * 4u;
    const uint32_t packed = L.pw;
    // exceptions before each segment (uniform)
    uint32_t sege[kPageSegs];
#pragma unroll
    for (uint32_t g = 0; g < kPageSegs; ++g)
        sege[g] = uniform(L.exc[kSegBlocks * g < nb ? kSegBlocks * g : nb]);
    uint32_t off = 0, s8_at = 0, s8w = 0, total = 0;
    uint32_t *page = nullptr, *s8 = nullptr, *entries = nullptr;
    uint8_t *md = nullptr;
    if constexpr (WRITE) {
        const uint32_t size = sizes[p] - (p ? sizes[p - 1] : 0u);
        off = dir_end + sizes[p] - size;
        s8_at = hw + packed + meta_w;
        s8w = size - s8_at;  // Simple-8b words and the page's end padding
        write_dir_entry(out, p, dir_entries(n, kFpBlocks), S, off, x, pstart);
        page = out + off;
        md = reinterpret_cast<uint8_t *>(page + hw + packed);
        s8 = page + s8_at;
        entries = page + 4u + S * (nseg - 1u);
        total = uniform(tab[kSpTab - 1u]);
    }
    const BufRsrc rs = make_rsrc(x + pstart, nb * kBlock * 4u);
    const uint32_t nq = (nb + 3u) / 4u;
    auto exc_q = [&](uint32_t q) __attribute__((always_inline)) { return L.exc[4u * q < nb ? 4u * q : nb]; };
    uint32_t qa = 0, lo = 0, ci = 0, k0 = 0;
    uint32_t pos = 0, words = 0;  // (size, wavefront 0) the chain's next word start, words so far
    while (qa < nq) {
        // the chunk: steps [qa, qb) with at most kSpChunkExc exceptions
        const uint32_t ea = exc_q(qa);
        uint32_t qb = qa + 1u, hiq = nq;
        while (qb < hiq) {  // largest qb with exc_q(qb) - ea <= kSpChunkExc
            const uint32_t mid = (qb + hiq + 1u) / 2u;
            if (exc_q(mid) - ea <= kSpChunkExc)
                qb = mid;
            else
                hiq = mid - 1u;
        }
        const uint32_t eb = exc_q(qb);
        const uint32_t hi = qb == nq ? nexc : (eb >= lo + 59u ? eb - 59u : lo);
        if constexpr (!WRITE)
            if (tid == 0)
                L.pos0 = pos;
        if constexpr (!WRITE) {
            // 1. gather: the chunk's widths from the analysis's per-block
            // slots, 16 lanes a block and eight bytes a lane, eight blocks
            // a thread in flight
            constexpr uint32_t J = 8, BPS = kSpThreads / 16u;  // blocks per step
            const uint32_t t0 = 4u * qa, t1 = 4u * qb < nb ? 4u * qb : nb;
            const uint32_t r = tid & 15u;
            for (uint32_t tb = t0 + (tid >> 4); tb < t1; tb += J * BPS) {
                uint2 v[J];
#pragma unroll
                for (uint32_t j = 0; j < J; ++j) {
                    const uint32_t t = tb + j * BPS;
                    const uint32_t c = t < t1 ? (uint32_t)L.c[t] : 0u;
                    v[j] = 8u * r < c ? *reinterpret_cast<const uint2 *>(spx + (p * kFpBlocks + t) * kSpWidthSlot + 8u * r)
                                      : make_uint2(0, 0);
                }
#pragma unroll
                for (uint32_t j = 0; j < J; ++j) {
                    const uint32_t t = tb + j * BPS;
                    const uint32_t c = t < t1 ? (uint32_t)L.c[t] : 0u;
                    if (8u * r < c) {
                        const uint32_t at = L.exc[t] + 8u * r;
                        const uint64_t w = v[j].x | ((uint64_t)v[j].y << 32);
#pragma unroll
                        for (uint32_t k = 0; k < 8; ++k)
                            if (8u * r + k < c)
                                L.wd[(at + k) & (kSpR - 1u)] = (uint8_t)(w >> (8u * k));
                    }
                }
            }
        } else {
            // 1. gather: the wavefront takes steps wave, wave + 4, ... of the
            // chunk, kSpDepth of them in flight (a step's slot is refilled as
            // soon as its values are taken)
            uint4 va[kSpDepth], vb[kSpDepth], pv[kSpDepth];
            auto issue = [&](uint32_t d, uint32_t q) __attribute__((always_inline)) {
                pv[d] = make_uint4(0, 0, 0, 0);
                if (q < qb) {
                    va[d] = buf_load_u4(rs, (q * kSpQuadInts + 8u * lane) * 4u);
                    vb[d] = buf_load_u4(rs, (q * kSpQuadInts + 8u * lane + 4u) * 4u);
                    if (S != 0 && lane == 0) {
                        if (q != 0)
                            pv[d] = buf_load_u4(rs, (q * kSpQuadInts - 4u) * 4u);
                        else if (pstart >= 4)
                            pv[d] = make_uint4(x[pstart - 4], x[pstart - 3], x[pstart - 2], x[pstart - 1]);
                    }
                }
            };
#pragma unroll
            for (uint32_t d = 0; d < kSpDepth; ++d)
                issue(d, qa + wave + kSpWaves * d);
            for (uint32_t q0 = qa + wave; q0 < qb; q0 += kSpWaves * kSpDepth) {
#pragma unroll
                for (uint32_t d = 0; d < kSpDepth; ++d) {
                    const uint32_t q = q0 + kSpWaves * d;
                    if (q >= qb)
                        break;
                    uint32_t dv[8];
                    sp_deltas<S>(va[d], vb[d], pv[d], lane, dv);
                    issue(d, q + kSpWaves * kSpDepth);
                    const uint32_t t = 4u * q + (lane >> 4), r = lane & 15u;
                    const bool in = t < nb;
                    const uint32_t b = in ? (uint32_t)L.b[t] : 32u;
                    uint32_t emask = 0;
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        emask |= (sp_nbits(dv[k]) > b ? 1u : 0u) << k;
                    const uint32_t ce = (uint32_t)__builtin_popcount(emask);
                    const uint32_t incl16 = row_scan_incl(ce);  // rows of 16 lanes are the blocks
                    uint32_t at = in ? L.exc[t] + incl16 - ce : 0u;
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if ((emask >> k) & 1u) {
                            L.hv[at & (kSpR - 1u)] = dv[k] >> b;
                            md[3u * nb + at] = (uint8_t)(8u * r + k);
                            ++at;
                        }
                    // low b bits of the eight values: b bytes from byte b * r
                    // of the block, staged with the step's other blocks (whose
                    // packed words follow one another), then stored as words
                    const uint32_t w0 = L.blk[4u * q];
                    uint8_t *const stb = reinterpret_cast<uint8_t *>(L.st + 512u * wave);
                    if (in) {
                        const uint32_t m = width_mask(b);
                        uint64_t acc = 0;
                        uint32_t nbit = 0, o = 4u * (L.blk[t] - w0) + b * r;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            acc |= (uint64_t)(dv[k] & m) << nbit;
                            nbit += b;
                            while (nbit >= 8u) {
                                stb[o++] = (uint8_t)acc;
                                acc >>= 8;
                                nbit -= 8u;
                            }
                        }
                        if (r == 0) {
                            md[t] = (uint8_t)b;
                            md[nb + t] = L.mb[t];
                            md[2u * nb + t] = L.c[t];
                        }
                    }
                    wave_lds_order();
                    const uint32_t nw4 = L.blk[4u * q + 4u < nb ? 4u * q + 4u : nb] - w0;
                    uint32_t *const pkw = page + hw + w0;
                    for (uint32_t i = lane; i < nw4; i += 64u)
                        pkw[i] = L.st[512u * wave + i];
                    wave_lds_order();
                }
            }
        }
        __syncthreads();
        if constexpr (WRITE) {
            // the chunk's words [k0, k1): one thread per word, from the ring;
            // the word starts of four words a thread are loaded at once
            const uint32_t k1 = uniform(tab[ci]);
            const uint32_t kend = k1 < total ? k1 : total;
            constexpr uint32_t U = 4;
            for (uint32_t kb = k0 + tid; kb < kend; kb += U * kSpThreads) {
                uint32_t qs[U], qe[U];
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t k = kb + u * kSpThreads;
                    qs[u] = k < kend ? (uint32_t)starts[k] : 0u;
                    qe[u] = k < kend ? (k + 1u < total ? (uint32_t)starts[k + 1u] : nexc) : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < U; ++u) {
                    const uint32_t k = kb + u * kSpThreads;
                    if (k >= kend)
                        break;
                    const uint32_t q = qs[u];
                    const uint32_t c = qe[u] - q;
                    const uint32_t sel = sp_selector(c);
                    const uint32_t bits = s8_mode(sel) >> 8;
                    uint64_t wv = 0;
                    for (uint32_t m = 0; m < c && m < 60u; ++m)
                        wv |= (uint64_t)L.hv[(q + m) & (kSpR - 1u)] << (m * bits);
                    s8[2u * k] = (uint32_t)wv;
                    s8[2u * k + 1u] = (uint32_t)(wv >> 32) | (sel << 28);
#pragma unroll
                    for (uint32_t g = 1; g < kPageSegs; ++g)
                        if (g < nseg && sege[g] >= q && sege[g] - q < c)
                            entries[g - 1u] = k | ((sege[g] - q) << 24);
                }
            }
            k0 = k1;
        } else {
            // 2. greedy counts of positions [lo, hi)
            for (uint32_t q = lo + tid; q < hi; q += kSpThreads)
                L.cnt[q & (kSpR - 1u)] = (uint8_t)sp_greedy_count(L.wd, q, nexc - q);
            __syncthreads();
            // 3. the chain from pos0 through [pos0, hi), by windows of 64
            // positions from pos0. (a) every position's exit from its
            // window: the chain's first position at or past the window's
            // end, by pointer jumping within the window (six rounds cover 64
            // steps), four windows a wavefront at a time
            const uint32_t pos0 = L.pos0;
            const uint32_t span = hi > pos0 ? hi - pos0 : 0u;
            const uint32_t nw = (span + 63u) / 64u;  // at most kSpR / 64
            for (uint32_t w0 = wave; w0 < nw; w0 += 4u * kSpWaves) {
                uint32_t X[4], lim[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t w = w0 + kSpWaves * u, base = pos0 + 64u * w;
                    lim[u] = w < nw ? (hi - base < 64u ? hi - base : 64u) : 0u;
                    const uint32_t c = lane < lim[u] ? (uint32_t)L.cnt[(base + lane) & (kSpR - 1u)] : 0u;
                    X[u] = lane + (c ? c : (lane < lim[u] ? 1u : 0u));
                }
#pragma unroll
                for (int k = 0; k < 6; ++k)
#pragma unroll
                    for (uint32_t u = 0; u < 4; ++u) {
                        const bool inside = X[u] < lim[u];
                        const uint32_t t = (uint32_t)__builtin_amdgcn_ds_bpermute(
                            (int)(4u * (inside ? X[u] : lane)), (int)X[u]);
                        X[u] = inside ? t : X[u];
                    }
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u)
                    if (lane < lim[u])
                        L.xo[(pos0 + 64u * (w0 + kSpWaves * u) + lane) & (kSpR - 1u)] = (uint8_t)(X[u] - lim[u]);
            }
            __syncthreads();
            if (wave == 0) {
                // (b) the windows' entries, one after the other: lane w
                // keeps window w's
                uint32_t e = pos0, mine = 0;
                for (uint32_t w = 0; w < nw; ++w) {
                    mine = lane == w ? e : mine;
                    const uint32_t base = pos0 + 64u * w;
                    const uint32_t end = base + (hi - base < 64u ? hi - base : 64u);
                    e = e < end ? end + uniform((uint32_t)L.xo[e & (kSpR - 1u)]) : e;
                }
                pos = e;
                // (c) lane w walks window w from its entry: its word starts,
                // after those of the windows before
                uint64_t mask = 0;
                if (lane < nw) {
                    const uint32_t base = pos0 + 64u * lane;
                    const uint32_t end = base + (hi - base < 64u ? hi - base : 64u);
                    for (uint32_t q = mine; q < end;) {
                        mask |= 1ull << (q - base);
                        const uint32_t c = L.cnt[q & (kSpR - 1u)];
                        q += c ? c : 1u;
                    }
                }
                const uint32_t cw = (uint32_t)__builtin_popcountll(mask);
                const uint32_t incl = wave_scan_incl(cw);
                uint32_t k = words + incl - cw;
                for (uint64_t m = mask; m != 0; m &= m - 1u, ++k)
                    if (k < kSpMaxExc)
                        starts[k] = (uint16_t)(pos0 + 64u * lane + (uint32_t)__builtin_ctzll(m));
                words += wave_read(incl, 63);
                if (lane == 0)
                    tab[ci] = words;
            }
        }
        __syncthreads();
        qa = qb;
        lo = hi;
        ++ci;
    }
    if constexpr (!WRITE) {
        if (tid == 0) {
            tab[kSpTab - 1u] = words;
            sizes[p] = pad4(hw + packed + meta_w + 2u * words);
        }
        return;
    } else {
        if (wave != 0)
            return;
        // zero padding after the words, up to the page's end
        for (uint32_t w = 2u * total + lane; w < s8w; w += 64)
            s8[w] = 0u;
        // entries of segments with no exception at or after their start
#pragma unroll
        for (uint32_t g = 1; g < kPageSegs; ++g)
            if (lane == 0 && g < nseg && sege[g] >= nexc)
                entries[g - 1u] = total;
        // segment bases: the S values before each segment after the first;
        // then the header's padding
        if (lane < S * (nseg - 1u)) {
            const uint32_t g = 1u + lane / (S ? S : 1u), t = lane % (S ? S : 1u);
            page[4u + lane] = x[pstart + (uint64_t)g * kSegInts - S + t];
        }
        if (4u + (S + 1u) * (nseg - 1u) + lane < hw)
            page[4u + (S + 1u) * (nseg - 1u) + lane] = 0u;
        if (lane == 0) {
            page[0] = nb;
            page[1] = packed;
            page[2] = meta_bytes;
            page[3] = 2u * total;
        }
        // the metadata's padding to 16 bytes
        for (uint32_t i = meta_bytes + lane; i < 4u * meta_w; i += 64u)
            md[i] = 0;
    }
}

}  // namespace wp

using namespace wp;

namespace wp {

// Scratch bytes of the SimplePFOR kernels for `units` pages.
uint64_t sp_scratch_bytes(uint64_t units) { return units * kSpSlotBytes; }

// SimplePFOR pages of one encode call: size, offsets, pages. `meta` holds
// the patched analysis's widths, maximum widths and counts; `spw` has
// sp_scratch_bytes(units) bytes.
int32_t sp_encode_units(const uint32_t *in, uint64_t n, uint32_t stride, uint64_t units, const uint8_t *meta,
                        uint64_t nblk, uint32_t *sizes, uint64_t *status, uint8_t *spw, const uint8_t *spx,
                        uint32_t dir_end, uint32_t *out, hipStream_t st)
{
#define WP_SP_LAUNCH(W, ...)                                                                                    \
    do {                                                                                                        \
        if (stride == 0)                                                                                        \
            hipLaunchKernelGGL((k_sp_page<0u, W>), dim3((uint32_t)units), dim3(kSpThreads), 0, st, __VA_ARGS__); \
        else if (stride == 1)                                                                                   \
            hipLaunchKernelGGL((k_sp_page<1u, W>), dim3((uint32_t)units), dim3(kSpThreads), 0, st, __VA_ARGS__); \
        else                                                                                                    \
            hipLaunchKernelGGL((k_sp_page<4u, W>), dim3((uint32_t)units), dim3(kSpThreads), 0, st, __VA_ARGS__); \
    } while (0)
    WP_SP_LAUNCH(false, in, n, meta, nblk, sizes, spw, spx, 0u, out);
    if (launch_inclusive_scan(sizes, units, status, st) != WP_OK)
        return WP_ERR_HIP;
    WP_SP_LAUNCH(true, in, n, meta, nblk, sizes, spw, spx, dir_end, out);
#undef WP_SP_LAUNCH
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

}  // namespace wp
