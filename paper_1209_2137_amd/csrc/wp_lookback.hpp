// Decoupled look-back (Merrill & Garland) across the tiles of one launch,
// shared by the in-place prefix sum and the fused binary-packing encoder.
//
// status[0] is the launch's tile counter (tiles take their index from it, so
// a tile's predecessors always started first); tile t owns the eight words
// status[8 (t + 1) ...]: its aggregates (words 0..3) and its inclusive
// prefixes (words 4..7), one per residue class in use. Each status word is
// {flag << 32 | value}, written and read with device-scope relaxed atomics
// so that flag and value always travel together and no cache-wide release
// is needed.
#pragma once

#include "wp_device.hpp"

namespace wp {

constexpr uint64_t kFlagAgg = 1ull << 32;
constexpr uint64_t kFlagInc = 2ull << 32;
constexpr int kStatusWords = 8;  // per tile: aggregate[4], inclusive[4]

__device__ __forceinline__ void st_status(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t ld_status(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run by one whole wavefront of tile `tile`: publishes the tile's NC
// aggregates agg[c], reads its predecessors' status 64 at a time (lane i:
// tile pos - 1 - i) until one has published its inclusive prefix, and
// returns in pre[c] the sum of every earlier tile's values plus `init`
// (the value before tile 0); then publishes the tile's inclusive prefix
// pre[c] + agg[c]. Waits only on tiles that started earlier.
template <int NC>
__device__ __forceinline__ void wave_lookback(uint64_t *__restrict__ status, uint32_t tile, const uint32_t (&agg)[4],
                                              uint32_t init, uint32_t (&pre)[4])
{
    const uint32_t lane = lane_id();
    uint64_t *const my = status + kStatusWords + (uint64_t)tile * kStatusWords;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        pre[c] = init;
    if (tile == 0) {
        if (lane < (uint32_t)NC)
            st_status(my + 4 + lane, kFlagInc | (uint32_t)(init + agg[lane & 3]));
        return;
    }
    if (lane < (uint32_t)NC)
        st_status(my + lane, kFlagAgg | agg[lane & 3]);
    uint32_t acc[4] = {0, 0, 0, 0};
    int64_t pos = (int64_t)tile;
    for (;;) {
        const int64_t t = pos - 1 - (int64_t)lane;
        // per lane: state of predecessor t (2 = inclusive, 1 = aggregate, 0 = not ready)
        uint32_t state = 0;
        uint32_t val[4] = {0, 0, 0, 0};
        if (t < 0) {
            state = 2;
            val[0] = val[1] = val[2] = val[3] = init;
        } else {
            const uint64_t *st = status + kStatusWords + (uint64_t)t * kStatusWords;
            bool inc = true, ag = true;
            uint64_t w[4];
            for (int c = 0; c < NC; ++c) {
                w[c] = ld_status(st + 4 + c);
                inc = inc && (w[c] >> 32) == 2;
            }
            if (inc) {
                state = 2;
                for (int c = 0; c < NC; ++c)
                    val[c] = (uint32_t)w[c];
            } else {
                for (int c = 0; c < NC; ++c) {
                    w[c] = ld_status(st + c);
                    ag = ag && (w[c] >> 32) == 1;
                }
                if (ag) {
                    state = 1;
                    for (int c = 0; c < NC; ++c)
                        val[c] = (uint32_t)w[c];
                }
            }
        }
        const uint64_t incm = ballot(state == 2);
        const uint64_t notready = ballot(state == 0);
        const uint32_t first = incm ? (uint32_t)__builtin_ctzll(incm) : 64u;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
        if (notready & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        for (int c = 0; c < NC; ++c) {
            const uint32_t x = lane <= first ? val[c] : 0u;
            acc[c] += wave_read(wave_scan_incl(x), 63);
        }
        if (first < 64)
            break;
        pos -= 64;
    }
    for (int c = 0; c < NC; ++c)
        pre[c] = acc[c];
    if (lane < (uint32_t)NC) {
        uint32_t mine = 0;
        for (int c = 0; c < NC; ++c)
            if ((uint32_t)c == lane)
                mine = pre[c] + agg[c];
        st_status(my + 4 + lane, kFlagInc | mine);
    }
}

}  // namespace wp
