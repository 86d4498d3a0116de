// Intersection of two posting lists held decoded on the device: the values
// present in both of two strictly increasing arrays a and b, ascending (the
// conjunctive-query step that consumes decoded lists).
//
// Each element of a is looked up in b by binary search. A workgroup takes a
// tile of 1024 consecutive elements of a; one thread bounds the tile's range
// of b with two searches, and every thread then searches its four
// consecutive elements inside that range, each search starting where the
// previous one ended (a is increasing). Pass 1 writes one flag byte per
// element of a and the tile's match count; an in-place inclusive scan of the
// counts (the chained scan of delta_decode_inplace) gives every tile its
// output offset; pass 2 writes the flagged elements in order.
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
    if (threadIdx.x == 0) {
        const uint64_t lo = lower_bound(b, 0, nb, a[t0]);
        const uint64_t hi = lower_bound(b, lo, nb, a[tend - 1]);
        s_range[0] = lo;
        s_range[1] = hi < nb ? hi + 1 : nb;
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

__global__ void k_isect_none(uint64_t *__restrict__ out_count)
{
    if (threadIdx.x == 0)
        *out_count = 0;
}

}  // namespace wp

using namespace wp;

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
    // scratch: scan status | tile counts | one flag byte per element of a
    const uint64_t status_bytes = scan_status_words(tiles) * sizeof(uint64_t);
    const uint64_t counts_off = (status_bytes + 255) & ~255ull;
    const uint64_t flags_off = (counts_off + tiles * sizeof(uint32_t) + 255) & ~255ull;
    char *scr = static_cast<char *>(stream_scratch(st, flags_off + na));
    if (scr == nullptr)
        return WP_ERR_HIP;
    uint64_t *status = reinterpret_cast<uint64_t *>(scr);
    uint32_t *counts = reinterpret_cast<uint32_t *>(scr + counts_off);
    uint8_t *flags = reinterpret_cast<uint8_t *>(scr + flags_off);
    hipLaunchKernelGGL(k_isect_flag, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, b, nb, flags, counts);
    if (launch_inclusive_scan(counts, tiles, status, st) != WP_OK)
        return WP_ERR_HIP;
    hipLaunchKernelGGL(k_isect_write, dim3((uint32_t)tiles), dim3(kIsThreads), 0, st, a, na, flags, counts, out,
                       out_count);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}
