// Intersection of two posting lists held decoded on the device: the values
// present in both of two strictly increasing arrays a and b, ascending (the
// conjunctive-query step that consumes decoded lists).
//
// Each element of a is looked up in b by binary search. A workgroup takes a
// tile of 1024 consecutive elements of a; two wavefronts bound the tile's
// range of b (64 probes per round trip), and every thread then searches its four
// consecutive elements inside that range, each search starting where the
// previous one ended (a is increasing). Pass 1 writes one flag byte per
// element of a and the tile's match count; an in-place inclusive scan of the
// counts (the chained scan of delta_decode_inplace) gives every tile its
// output offset; pass 2 writes the flagged elements in order.
//
// With the second list still compressed, the directory serves as a skip
// list: every unit's stored base is the value just before the unit, so a
// strictly increasing list's unit e holds values in (base_e, base_{e+1}].
// The decode pass takes one unit per wavefront (or workgroup, for pages):
// it searches the first list for a value in its unit's range and decodes
// the unit only then (the decoders' wavefront and page routines, into the
// caller's work buffer at the unit's own positions); the lookups then
// search the directory for the unit, then the unit's values. Random access
// by key uses the same decode pass with the key range in place of the
// first list, then two wavefront searches for the range's ends.
#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

constexpr uint32_t kIsThreads = 256, kIsPer = 4, kIsTile = kIsThreads * kIsPer;

// First index in [lo, hi) whose value is >= v (hi if none).
__device__ __forceinline__ uint64_t lower_bound(const uint32_t *__restrict__ b, uint64_t lo, uint64_t hi, uint32_t v)
{
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (b[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// lower_bound by a whole wavefront (uniform arguments and result) over
// b[i * stride], i in [lo, hi): 64 probes per round trip, the range
// shrinking 64-fold each time.
__device__ __forceinline__ uint64_t wave_lower_bound(const uint32_t *__restrict__ b, uint64_t lo, uint64_t hi,
                                                     uint32_t v, uint64_t stride = 1)
{
    const uint32_t lane = lane_id();
    for (;;) {
        const uint64_t len = hi - lo;
        const uint64_t step = len > 64 ? (len + 63) / 64 : 1;
        const uint64_t p = lo + lane * step;
        const bool lt = p < hi && b[p * stride] < v;
        const uint32_t c = (uint32_t)__builtin_popcountll(ballot(lt));
        if (len <= 64 || c == 0)
            return lo + (len <= 64 ? c : 0u);
        const uint64_t nhi = lo + c * step;
        lo = lo + (c - 1) * step + 1;
        hi = nhi < hi ? nhi : hi;
    }
}

// Block-wide inclusive sum of one value per thread (256 threads); `part`
// holds kIsThreads / 64 words of LDS.
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t v, uint32_t *part, uint32_t &total)
{
    const uint32_t lane = lane_id(), wave = uniform(threadIdx.x >> 6);
    const uint32_t incl = wave_scan_incl(v);
    if (lane == 63)
        part[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (uint32_t w = 0; w < kIsThreads / 64; ++w) {
        const uint32_t t = part[w];
        before += w < wave ? t : 0u;
        all += t;
    }
    total = all;
    return before + incl;
}

__global__ __launch_bounds__(kIsThreads) void k_isect_flag(const uint32_t *__restrict__ a, uint64_t na,
                                                           const uint32_t *__restrict__ b, uint64_t nb,
                                                           uint8_t *__restrict__ flags,
                                                           uint32_t *__restrict__ counts)
{
    __shared__ uint64_t s_range[2];
    __shared__ uint32_t s_part[kIsThreads / 64];
    const uint64_t t0 = (uint64_t)blockIdx.x * kIsTile;
    const uint64_t tend = t0 + kIsTile < na ? t0 + kIsTile : na;
    // the tile's range of b: wavefront 0 bounds its first element, 1 its last
    const uint32_t wave = uniform(threadIdx.x >> 6);
    if (wave < 2) {
        const uint64_t r = wave_lower_bound(b, 0, nb, a[wave == 0 ? t0 : tend - 1]);
        if (lane_id() == 0)
            s_range[wave] = wave == 0 ? r : (r < nb ? r + 1 : nb);
    }
    __syncthreads();
    uint64_t lo = s_range[0];
    const uint64_t hi = s_range[1];
    const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kIsPer;
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t r = 0; r < kIsPer; ++r) {
        const uint64_t i = i0 + r;
        if (i < tend) {
            const uint32_t v = a[i];
            lo = lower_bound(b, lo, hi, v);
            const bool hit = lo < hi && b[lo] == v;
            flags[i] = hit ? 1u : 0u;
            cnt += hit ? 1u : 0u;
        }
    }
    uint32_t total;
    block_scan_incl(cnt, s_part, total);
    if (threadIdx.x == 0)
        counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kIsThreads) void k_isect_write(const uint32_t *__restrict__ a, uint64_t na,
                                                            const uint8_t *__restrict__ flags,
                                                            const uint32_t *__restrict__ incl,
                                                            uint32_t *__restrict__ out,
                                                            uint64_t *__restrict__ out_count)
{
    __shared__ uint32_t s_part[kIsThreads / 64];
    const uint64_t t0 = (uint64_t)blockIdx.x * kIsTile;
    const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kIsPer;
    uint32_t f[kIsPer];
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t r = 0; r < kIsPer; ++r) {
        f[r] = i0 + r < na ? flags[i0 + r] : 0u;
        cnt += f[r];
    }
    uint32_t total;
    uint32_t o = block_scan_incl(cnt, s_part, total) - cnt;
    o += blockIdx.x > 0 ? incl[blockIdx.x - 1] : 0u;
#pragma unroll
    for (uint32_t r = 0; r < kIsPer; ++r) {
        if (f[r])
            out[o++] = a[i0 + r];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *out_count = incl[blockIdx.x];
}

// ---------------------------------------------------------------------
// Second list compressed. Directory entry e (units, then the tail entry)
// covers the list's integers [e * per * 128, ...) and, for a strictly
// increasing list, values in (base_e, base_{e+1}] where base_e is the last
// of the entry's stored bases (the value just before the entry); entry 0 has
// no lower bound and the last entry no upper bound. A stream without
// differential coding (stride 0) has no such bounds: every entry is
// decoded and lookups search the whole decoded list.

struct DirView {
    const uint32_t *in;
    ListHdr H;
    uint32_t per;  // blocks per unit
    __device__ __forceinline__ uint32_t base(uint64_t e) const
    {
        return in[kHdrWords + H.ndir + e * H.S + (H.S - 1)];
    }
    // first integer of entry e (the tail entry starts after the last full block)
    __device__ __forceinline__ uint64_t first_int(uint64_t e) const
    {
        const uint64_t f = e * per * (uint64_t)kBlock, t = H.nfull * kBlock;
        return f < t ? f : t;
    }
};

__device__ __forceinline__ bool dir_view(const uint32_t *in, uint64_t in_words, uint64_t n, int32_t codec,
                                         DirView &D)
{
    D.in = in;
    D.per = (codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP) ? kFpBlocks : kBpBlocks;
    const uint32_t magic = codec == WP_CODEC_BP     ? kMagicBP
                           : codec == WP_CODEC_BPV  ? kMagicBPV
                           : codec == WP_CODEC_BP32 ? kMagicBP32
                           : codec == WP_CODEC_FP32 ? kMagicFP32
                           : codec == WP_CODEC_SP   ? kMagicSP
                                                    : kMagicFP;
    return check_header(in, in_words, n, magic, D.per, D.H);
}

// Decodes the wanted entries of a binary-packing (SIMD-BP128 or BP32)
// stream into out (one wavefront per unit; the tail entry by a wavefront of
// its own).
template <uint32_t S, bool B32, bool V>
__device__ __forceinline__ bool bp_unit(const uint32_t *in, const ListHdr &H, uint64_t u, uint32_t *out,
                                        WaveLds<2, B32> &L)
{
    return bp_wave_run<2, S, B32, V>(in, H, u, 1, out, L);
}

template <bool B32>
union IsectWaveLds {
    WaveLds<2, B32> r;
    TailLds<1> tail;
};

// Whether entry e is to be decoded (uniform over the wavefront). With a
// short list a (strictly increasing, na values): whether some element of a
// lies in the entry's values, (base_e, base_{e+1}] for a strictly
// increasing list, found by a wavefront search of a. Without it: whether
// the entry's values can lie in [klo, khi], [base_e, base_{e+1}] for a
// non-decreasing list. base_e is the last of the entry's stored bases (the
// value just before it); entry 0 has no lower bound and the last entry no
// upper bound; without differential coding every entry counts.
__device__ __forceinline__ bool entry_wanted(const uint32_t *__restrict__ in, const ListHdr &H, uint64_t e,
                                             const uint32_t *__restrict__ a, uint64_t na, uint32_t klo,
                                             uint32_t khi)
{
    if (H.S == 0)
        return true;
    const uint32_t *const bases = in + kHdrWords + H.ndir + (H.S - 1);
    const bool last = e + 1 == H.ndir;
    if (a != nullptr) {
        if (e > 0 && bases[e * H.S] == 0xFFFFFFFFu)
            return false;  // nothing can lie above the largest value
        const uint64_t i = e == 0 ? 0 : wave_lower_bound(a, 0, na, bases[e * H.S] + 1u);
        return i < na && (last || a[i] <= bases[(e + 1) * H.S]);
    }
    const bool above_lo = last || bases[(e + 1) * H.S] >= klo;  // some value can be >= klo
    const bool below_hi = e == 0 || bases[e * H.S] <= khi;      // some value can be <= khi
    return above_lo && below_hi;
}

template <bool B32, bool V>
__global__ __launch_bounds__(256) void k_isect_decode_bp(const uint32_t *__restrict__ in, uint64_t in_words,
                                                         uint64_t n, const uint32_t *__restrict__ a, uint64_t na,
                                                         uint32_t klo, uint32_t khi, uint32_t *__restrict__ out,
                                                         int *__restrict__ err)
{
    __shared__ IsectWaveLds<B32> L[4];
    ListHdr H;
    if (!check_header(in, in_words, n, B32 ? kMagicBP32 : V ? kMagicBPV : kMagicBP, kBpBlocks, H))
        return;  // reported by k_isect_flag_dir or k_range_bounds
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint64_t e = (uint64_t)blockIdx.x * 4 + wave;
    if (e >= H.ndir || !entry_wanted(in, H, e, a, na, klo, khi))
        return;
    bool ok;
    if (e < H.units)
        ok = H.S == 1   ? bp_unit<1, B32, V>(in, H, e, out, L[wave].r)
             : H.S == 4 ? bp_unit<4, B32, V>(in, H, e, out, L[wave].r)
                        : bp_unit<0, B32, V>(in, H, e, out, L[wave].r);
    else
        ok = decode_tail_entry<1, false>(in, H, out, L[wave].tail);
    if (!ok && lane_id() == 0)
        *err = kErrCorrupt;
}

union IsectPageLds {
    FpWaveLds page;
    SpWaveLds sp;
    TailLds<1> tail;
};

// Decodes the wanted entries of a patched-page stream (one wavefront per
// 64-block segment of a page, four per workgroup;
// P32: exception arrays padded to 32 values).
template <int KIND>
__global__ __launch_bounds__(256) void k_isect_decode_fp(const uint32_t *__restrict__ in, uint64_t in_words,
                                                         uint64_t n, const uint32_t *__restrict__ a, uint64_t na,
                                                         uint32_t klo, uint32_t khi, uint32_t *__restrict__ out,
                                                         int *__restrict__ err)
{
    __shared__ IsectPageLds L[4];
    ListHdr H;
    const uint32_t magic = KIND == kPageSp ? kMagicSP : KIND == kPageFp32 ? kMagicFP32 : kMagicFP;
    if (!check_header(in, in_words, n, magic, kFpBlocks, H))
        return;  // reported by k_isect_flag_dir or k_range_bounds
    const uint32_t wave = uniform(threadIdx.x >> 6);
    constexpr uint32_t per = kPageSegs;
    const uint64_t item = (uint64_t)blockIdx.x * 4 + wave;
    const uint64_t u = item / per;
    const uint32_t seg = (uint32_t)(item % per);
    if (u >= H.ndir || seg >= (u == H.units ? 1u : page_items<KIND>(page_blocks(H, u))) ||
        !entry_wanted(in, H, u, a, na, klo, khi))
        return;
    bool ok;
    if (u == H.units)
        ok = decode_tail_entry<1, false>(in, H, out, L[wave].tail);
    else if constexpr (KIND == kPageSp)
        ok = fp_unit<KIND>(in, H, u, seg, out, L[wave].sp.fp, L[wave].sp.ring);
    else
        ok = fp_unit<KIND>(in, H, u, seg, out, L[wave].page);
    if (!ok && lane_id() == 0)
        *err = kErrCorrupt;
}

// Pass 1 against the decoded entries: each element of a finds its entry by
// a search of the directory's bases, then itself inside the entry's values.
__global__ __launch_bounds__(kIsThreads) void k_isect_flag_dir(const uint32_t *__restrict__ a, uint64_t na,
                                                               const uint32_t *__restrict__ in, uint64_t in_words,
                                                               uint64_t n, int32_t codec,
                                                               const uint32_t *__restrict__ b,
                                                               uint8_t *__restrict__ flags,
                                                               uint32_t *__restrict__ counts, int *__restrict__ err)
{
    __shared__ uint32_t s_part[kIsThreads / 64];
    DirView D;
    const bool valid = dir_view(in, in_words, n, codec, D);
    if (!valid && blockIdx.x == 0 && threadIdx.x == 0)
        *err = kErrCorrupt;
    const uint64_t t0 = (uint64_t)blockIdx.x * kIsTile;
    const uint64_t i0 = t0 + (uint64_t)threadIdx.x * kIsPer;
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t r = 0; r < kIsPer; ++r) {
        const uint64_t i = i0 + r;
        if (i >= na)
            break;
        const uint32_t v = a[i];
        bool hit = false;
        if (valid) {
            uint64_t lo = 0, hi = n;
            if (D.H.S != 0) {
                // entry: number of entries e >= 1 whose base is below v
                uint64_t l = 1, h = D.H.ndir;
                while (l < h) {
                    const uint64_t m = l + ((h - l) >> 1);
                    if (D.base(m) < v)
                        l = m + 1;
                    else
                        h = m;
                }
                const uint64_t e = l - 1;
                lo = D.first_int(e);
                hi = e + 1 < D.H.ndir ? D.first_int(e + 1) : n;
                hi = hi < n ? hi : n;
            }
            const uint64_t pos = lower_bound(b, lo, hi, v);
            hit = pos < hi && b[pos] == v;
        }
        flags[i] = hit ? 1u : 0u;
        cnt += hit ? 1u : 0u;
    }
    uint32_t total;
    block_scan_incl(cnt, s_part, total);
    if (threadIdx.x == 0)
        counts[blockIdx.x] = total;
}

// ---------------------------------------------------------------------
// Random access by key. The decode kernels above take the entries whose
// values can lie in [klo, khi] (entry_wanted); every entry in which one of
// the two searches below ends is among them: the search for v ends in the
// entry with base_e < v <= base_{e+1}.

// The index range [i0, i1) of the values in [klo, khi]: wavefront 0 finds
// the first value >= klo, wavefront 1 the first value > khi, each by the
// directory's bases (the entry), then inside the entry's decoded values.
__global__ __launch_bounds__(128) void k_range_bounds(const uint32_t *__restrict__ in, uint64_t in_words, uint64_t n,
                                                      int32_t codec, uint32_t klo, uint32_t khi,
                                                      const uint32_t *__restrict__ vals,
                                                      uint64_t *__restrict__ range, int *__restrict__ err)
{
    DirView D;
    const bool valid = dir_view(in, in_words, n, codec, D);
    if (!valid && threadIdx.x == 0)
        *err = kErrCorrupt;
    const uint32_t wave = uniform(threadIdx.x >> 6);
    uint64_t r = 0;
    if (valid) {
        // first value >= v, v = klo or khi + 1 (none above 0xffffffff)
        const bool past_top = wave == 1 && khi == 0xffffffffu;
        const uint32_t v = wave == 0 ? klo : khi + 1u;
        if (past_top) {
            r = n;
        } else if (D.H.S == 0) {
            r = wave_lower_bound(vals, 0, n, v);
        } else {
            // entry: the last e whose base is below v (entry 0 has no base)
            const uint32_t *bases = in + kHdrWords + D.H.ndir + (D.H.S - 1);
            const uint64_t e = D.H.ndir > 1 ? wave_lower_bound(bases, 1, D.H.ndir, v, D.H.S) - 1 : 0;
            const uint64_t lo = D.first_int(e);
            uint64_t hi = e + 1 < D.H.ndir ? D.first_int(e + 1) : n;
            hi = hi < n ? hi : n;
            r = wave_lower_bound(vals, lo, hi, v);
        }
    }
    if (lane_id() == 0)
        range[wave] = r;
}

__global__ void k_isect_none(uint64_t *__restrict__ out_count)
{
    if (threadIdx.x == 0)
        *out_count = 0;
}

}  // namespace wp

using namespace wp;

// scratch: scan status | tile counts | one flag byte per element of a
struct IsectScratch {
    uint64_t *status;
    uint32_t *counts;
    uint8_t *flags;
};

static bool isect_scratch(hipStream_t st, uint64_t tiles, uint64_t na, IsectScratch &S)
{
    const uint64_t status_bytes = scan_status_words(tiles) * sizeof(uint64_t);
    const uint64_t counts_off = (status_bytes + 255) & ~255ull;
    const uint64_t flags_off = (counts_off + tiles * sizeof(uint32_t) + 255) & ~255ull;
    char *scr = static_cast<char *>(stream_scratch(st, flags_off + na + 1));
    if (scr == nullptr)
        return false;
    S.status = reinterpret_cast<uint64_t *>(scr);
    S.counts = reinterpret_cast<uint32_t *>(scr + counts_off);
    S.flags = reinterpret_cast<uint8_t *>(scr + flags_off);
    return true;
}

extern "C" int32_t wp_intersect(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out,
                                uint64_t *out_count, void *stream)
{
    if (out_count == nullptr || (na > 0 && (a == nullptr || out == nullptr)) || (nb > 0 && b == nullptr) ||
        (reinterpret_cast<uintptr_t>(out_count) & 7u) || na > 0xFFFFFFFFull)
        return WP_ERR_INVALID_ARG;
    hipStream_t st = as_stream(stream);
    (void)hipGetLastError();
    if (na == 0 || nb == 0) {
        hipLaunchKernelGGL(k_isect_none, dim3(1), dim3(64), 0, st, out_count);
        return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
    }
    const uint64_t tiles = (na + kIsTile - 1) / kIsTile;
    IsectScratch S;
    if (!isect_scratch(st, tiles, na, S))
        return WP_ERR_HIP;
    hipLaunchKernelGGL(k_isect_flag, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, b, nb, S.flags,
                       S.counts);
    if (launch_inclusive_scan(S.counts, tiles, S.status, st) != WP_OK)
        return WP_ERR_HIP;
    hipLaunchKernelGGL(k_isect_write, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, S.flags, S.counts, out,
                       out_count);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

extern "C" int32_t wp_intersect_compressed(const uint32_t *a, uint64_t na, const uint32_t *b_comp, uint64_t b_words,
                                           uint64_t nb, int32_t codec, uint32_t *b_work, uint32_t *out,
                                           uint64_t *out_count, void *stream)
{
    if (out_count == nullptr || (na > 0 && (a == nullptr || out == nullptr)) || b_comp == nullptr ||
        b_words < kHdrWords || (nb > 0 && b_work == nullptr) || (reinterpret_cast<uintptr_t>(out_count) & 7u) ||
        na > 0xFFFFFFFFull ||
        (codec != WP_CODEC_BP && codec != WP_CODEC_FP && codec != WP_CODEC_BP32 && codec != WP_CODEC_FP32 &&
         codec != WP_CODEC_SP &&
         codec != WP_CODEC_BPV) ||
        !aligned16(b_comp) ||
        !aligned16(b_work) || nb > 0xFFFFFFFFull * 32ull)
        return WP_ERR_INVALID_ARG;
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    hipStream_t st = as_stream(stream);
    (void)hipGetLastError();
    if (na == 0 || nb == 0) {
        hipLaunchKernelGGL(k_isect_none, dim3(1), dim3(64), 0, st, out_count);
        return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
    }
    const uint64_t per =
        (codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP) ? kFpBlocks : kBpBlocks;
    const uint64_t nfull = nb / kBlock;
    const uint64_t nent = (nfull + per - 1) / per + ((nb % kBlock) ? 1 : 0);
    const uint64_t tiles = (na + kIsTile - 1) / kIsTile;
    IsectScratch S;
    if (nent > 0x0FFFFFFFull || !isect_scratch(st, tiles, na, S))
        return WP_ERR_HIP;
    if (codec == WP_CODEC_BP)
        hipLaunchKernelGGL((k_isect_decode_bp<false, false>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                           b_comp, b_words, nb, a, na, 0u, 0u, b_work, ds->err);
    else if (codec == WP_CODEC_BPV)
        hipLaunchKernelGGL((k_isect_decode_bp<false, true>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                           b_comp, b_words, nb, a, na, 0u, 0u, b_work, ds->err);
    else if (codec == WP_CODEC_BP32)
        hipLaunchKernelGGL((k_isect_decode_bp<true, false>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                           b_comp, b_words, nb, a, na, 0u, 0u, b_work, ds->err);
    else if (codec == WP_CODEC_SP)
        hipLaunchKernelGGL(k_isect_decode_fp<kPageSp>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, b_comp,
                           b_words, nb, a, na, 0u, 0u, b_work, ds->err);
    else if (codec == WP_CODEC_FP32)
        hipLaunchKernelGGL(k_isect_decode_fp<kPageFp32>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, b_comp, b_words, nb,
                           a, na, 0u, 0u, b_work, ds->err);
    else
        hipLaunchKernelGGL(k_isect_decode_fp<kPageFp>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, b_comp, b_words, nb,
                           a, na, 0u, 0u, b_work, ds->err);
    hipLaunchKernelGGL(k_isect_flag_dir, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, b_comp, b_words, nb,
                       codec, b_work, S.flags, S.counts, ds->err);
    if (launch_inclusive_scan(S.counts, tiles, S.status, st) != WP_OK)
        return WP_ERR_HIP;
    hipLaunchKernelGGL(k_isect_write, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, S.flags, S.counts, out,
                       out_count);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

extern "C" int32_t wp_decode_range(const uint32_t *in, uint64_t in_words, uint64_t n, int32_t codec,
                                   uint32_t key_lo, uint32_t key_hi, uint32_t *out, uint64_t *range, void *stream)
{
    if (in == nullptr || in_words < kHdrWords || range == nullptr || (n > 0 && out == nullptr) ||
        (reinterpret_cast<uintptr_t>(range) & 7u) || key_lo > key_hi ||
        (codec != WP_CODEC_BP && codec != WP_CODEC_FP && codec != WP_CODEC_BP32 && codec != WP_CODEC_FP32 &&
         codec != WP_CODEC_SP &&
         codec != WP_CODEC_BPV) ||
        !aligned16(in) || !aligned16(out) || n > 0xFFFFFFFFull * 32ull)
        return WP_ERR_INVALID_ARG;
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    hipStream_t st = as_stream(stream);
    (void)hipGetLastError();
    const uint64_t per =
        (codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP) ? kFpBlocks : kBpBlocks;
    const uint64_t nfull = n / kBlock;
    const uint64_t nent = (nfull + per - 1) / per + ((n % kBlock) ? 1 : 0);
    if (nent > 0x0FFFFFFFull)
        return WP_ERR_INVALID_ARG;
    if (nent > 0) {
        // no short list: each entry's own bases against the key range decide (entry_wanted)
        const uint32_t *const nf = nullptr;
        if (codec == WP_CODEC_BP)
            hipLaunchKernelGGL((k_isect_decode_bp<false, false>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                               in, in_words, n, nf, 0, key_lo, key_hi, out, ds->err);
        else if (codec == WP_CODEC_BPV)
            hipLaunchKernelGGL((k_isect_decode_bp<false, true>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                               in, in_words, n, nf, 0, key_lo, key_hi, out, ds->err);
        else if (codec == WP_CODEC_BP32)
            hipLaunchKernelGGL((k_isect_decode_bp<true, false>), dim3((uint32_t)((nent + 3) / 4)), dim3(256), 0, st,
                               in, in_words, n, nf, 0, key_lo, key_hi, out, ds->err);
        else if (codec == WP_CODEC_SP)
            hipLaunchKernelGGL(k_isect_decode_fp<kPageSp>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, in,
                               in_words, n, nf, 0, key_lo, key_hi, out, ds->err);
        else if (codec == WP_CODEC_FP32)
            hipLaunchKernelGGL(k_isect_decode_fp<kPageFp32>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, in, in_words, n, nf,
                               0, key_lo, key_hi, out, ds->err);
        else
            hipLaunchKernelGGL(k_isect_decode_fp<kPageFp>, dim3((uint32_t)((nent * kPageSegs + 3) / 4)), dim3(256), 0, st, in, in_words, n, nf,
                               0, key_lo, key_hi, out, ds->err);
    }
    hipLaunchKernelGGL(k_range_bounds, dim3(1), dim3(128), 0, st, in, in_words, n, codec, key_lo, key_hi, out,
                       range, ds->err);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}
