// delta_decode_inplace: the in-place prefix sum of Section 3 over a whole
// device array, in one pass (read 4 B + write 4 B per integer).
//
// Tiles of 32768 integers (1024 threads x 8 rows x 4 integers, 128 KB)
// take their index from an atomic counter, so a tile's predecessors always
// started first. Large tiles matter: the inclusive prefix advances by at
// most one look-back window (64 tiles) per device-scope round trip. Each
// tile scans locally, publishes its aggregate, then looks back
// over its predecessors (a whole wavefront reads 64 of them at once) until
// it meets one that has published its inclusive prefix (decoupled look-back,
// Merrill & Garland). Each status is one 64-bit word {flag, value} written
// and read with device-scope relaxed atomics, so flag and value always
// travel together and no cache-wide release is needed. Stride 4 keeps four
// independent sums (residue classes mod 4): four status words per kind.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "wp_device.hpp"
#include "wp_host.hpp"
#include "wp_lookback.hpp"

namespace wp {

constexpr int kScanWaves = 16;
constexpr int kScanT = 64 * kScanWaves;
// Rows per tile for stride 1 and stride 4: tiles of 32768 integers. The
// chained scan completes at most about 64 tiles per device-scope round
// trip; with tiles of 16384 integers that capped the 2^28 stride-1 scan at
// about 475 us, with 32768 it runs at the device copy's rate.
#ifndef WP_SCAN_ROWS1
#define WP_SCAN_ROWS1 8
#endif
#ifndef WP_SCAN_ROWS4
#define WP_SCAN_ROWS4 8
#endif
constexpr int kRows1 = WP_SCAN_ROWS1, kRows4 = WP_SCAN_ROWS4;
constexpr uint32_t tile_ints(uint32_t S) { return kScanT * 4u * (S == 1 ? kRows1 : kRows4); }
// the smaller of the two strides' tiles: status arrays sized for it fit both
constexpr uint32_t kMinTileInts = tile_ints(1) < tile_ints(4) ? tile_ints(1) : tile_ints(4);
__global__ void k_fill_zero(uint64_t *__restrict__ p, uint64_t count)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0;
}

// counter lives in status[0]; tile t's words at status[8 + 8t ...]
template <uint32_t S>
__global__ __launch_bounds__(kScanT) void k_delta_scan(uint32_t *__restrict__ data, uint64_t n, uint32_t init,
                                                       uint64_t *__restrict__ status)
{
    constexpr int kScanRows = S == 1 ? kRows1 : kRows4;
    constexpr uint32_t kTileInts = tile_ints(S);
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_tot[kScanRows][kScanWaves][4];
    __shared__ uint32_t s_excl[4];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    if (tid == 0)
        s_tile = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long *>(status), 1ull);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t t0 = (uint64_t)tile * kTileInts;
    uint32_t *const tb = data + t0;  // uniform tile base; rows at 32-bit offsets
    const bool full = t0 + kTileInts <= n;
    uint32_t v[kScanRows][4];
    if (full) {
#pragma unroll
        for (int m = 0; m < kScanRows; ++m) {
            const uint4 x = *reinterpret_cast<const uint4 *>(tb + m * (kScanT * 4) + 4 * tid);
            v[m][0] = x.x, v[m][1] = x.y, v[m][2] = x.z, v[m][3] = x.w;
        }
    } else {
        const uint32_t left = (uint32_t)(n - t0);
#pragma unroll
        for (int m = 0; m < kScanRows; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t i = m * (kScanT * 4) + 4 * tid + r;
                v[m][r] = i < left ? tb[i] : 0u;
            }
    }
    // local inclusive scans: per row, lane-serial then across the wavefront;
    // the wavefront's exclusive prefix is folded in at once
#pragma unroll
    for (int m = 0; m < kScanRows; ++m) {
        if constexpr (S == 1) {
            v[m][1] += v[m][0];
            v[m][2] += v[m][1];
            v[m][3] += v[m][2];
            const uint32_t incl = wave_scan_incl(v[m][3]);
            const uint32_t ex = incl - v[m][3];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[m][r] += ex;
            if (lane == 63)
                s_tot[m][wave][0] = incl;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t incl = wave_scan_incl(v[m][c]);
                v[m][c] = incl;
                if (lane == 63)
                    s_tot[m][wave][c] = incl;
            }
        }
    }
    __syncthreads();
    // add the earlier (row, wave) segments inside the tile: the rows x waves
    // segment totals, in tile order, are K wavefronts' worth (K per lane,
    // consecutive), so one wave scan per residue class gives every
    // segment's offset
    constexpr int K = kScanRows * kScanWaves / 64;
    static_assert(kScanRows * kScanWaves == 64 * K && (K == 1 || K == 2), "one or two segments per lane");
    constexpr int NC = S == 1 ? 1 : 4;
    uint32_t agg[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        uint32_t sv[K], lsum = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sv[k] = (&s_tot[0][0][0])[(lane * K + k) * 4 + c];  // segment (q / W, q % W), q = K lane + k
            lsum += sv[k];
        }
        const uint32_t incl = wave_scan_incl(lsum);
        const uint32_t ex0 = incl - lsum, ex1 = ex0 + sv[0];
        agg[c] = wave_read(incl, 63);
#pragma unroll
        for (int m = 0; m < kScanRows; ++m) {
            const int q = m * kScanWaves + (int)wave;
            const uint32_t o0 = __builtin_amdgcn_readlane(ex0, q / K);
            const uint32_t off = (K == 2 && (q & 1)) ? __builtin_amdgcn_readlane(ex1, q / K) : o0;
            if constexpr (S == 1) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    v[m][r] += off;
            } else {
                v[m][c] += off;
            }
        }
    }
    // publish and look back (wave 0)
    if (wave == 0) {
        uint32_t pre[4];
        wave_lookback<NC>(status, tile, agg, init, pre);
        if (lane == 0)
            for (int c = 0; c < 4; ++c)
                s_excl[c] = pre[c];
    }
    __syncthreads();
    const uint32_t e0 = s_excl[0], e1 = s_excl[1], e2 = s_excl[2], e3 = s_excl[3];
#pragma unroll
    for (int m = 0; m < kScanRows; ++m) {
        if constexpr (S == 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[m][r] += e0;
        } else {
            v[m][0] += e0;
            v[m][1] += e1;
            v[m][2] += e2;
            v[m][3] += e3;
        }
    }
    if (full) {
#pragma unroll
        for (int m = 0; m < kScanRows; ++m)
            *reinterpret_cast<uint4 *>(tb + m * (kScanT * 4) + 4 * tid) =
                make_uint4(v[m][0], v[m][1], v[m][2], v[m][3]);
    } else {
        const uint32_t left = (uint32_t)(n - t0);
#pragma unroll
        for (int m = 0; m < kScanRows; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t i = m * (kScanT * 4) + 4 * tid + r;
                if (i < left)
                    tb[i] = v[m][r];
            }
    }
}

// ------------------------------------------------------------------------

struct ScratchKey {
    int dev;
    hipStream_t st;
    bool operator==(const ScratchKey &o) const { return dev == o.dev && st == o.st; }
};
struct ScratchHash {
    size_t operator()(const ScratchKey &k) const
    {
        return std::hash<void *>()(reinterpret_cast<void *>(k.st)) ^ (size_t)k.dev;
    }
};
struct ScratchBuf {
    void *p = nullptr;
    size_t bytes = 0;
};
static std::mutex g_smu;
static std::unordered_map<ScratchKey, ScratchBuf, ScratchHash> g_scratch;

void *stream_scratch(hipStream_t stream, size_t bytes)
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_smu);
    ScratchBuf &b = g_scratch[ScratchKey{d, stream}];
    if (b.bytes >= bytes && b.p)
        return b.p;
    if (b.p) {
        if (hipStreamSynchronize(stream) != hipSuccess)
            return nullptr;
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess)
        return nullptr;
    b.p = p;
    b.bytes = want;
    return p;
}

}  // namespace wp

using namespace wp;

namespace wp {

// status words for n integers (sized for the smaller of the two strides'
// tiles, so one size fits both)
uint64_t scan_status_words(uint64_t n)
{
    const uint64_t tiles = (n + kMinTileInts - 1) / kMinTileInts;
    return (uint64_t)kStatusWords * (tiles + 1);
}

static int32_t launch_scan(uint32_t *data, uint64_t n, uint32_t init, uint32_t stride, uint64_t *status,
                           hipStream_t st, bool timed)
{
    const uint32_t ti = tile_ints(stride);
    const uint64_t tiles = (n + ti - 1) / ti;
    const uint64_t words = (uint64_t)kStatusWords * (tiles + 1);
    hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, status, words);
    const LaunchEvents e = timed ? take_launch_events() : LaunchEvents{};
    if (stride == 1)
        hipExtLaunchKernelGGL(k_delta_scan<1>, dim3((uint32_t)tiles), dim3(kScanT), 0, st, e.start, e.stop, 0, data, n,
                              init, status);
    else
        hipExtLaunchKernelGGL(k_delta_scan<4>, dim3((uint32_t)tiles), dim3(kScanT), 0, st, e.start, e.stop, 0, data, n,
                              init, status);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

void launch_clear(uint64_t *p, uint64_t count, hipStream_t st)
{
    if (count)
        hipLaunchKernelGGL(k_fill_zero, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, st, p, count);
}

int32_t launch_inclusive_scan(uint32_t *data, uint64_t n, uint64_t *status, hipStream_t st)
{
    if (n == 0)
        return WP_OK;
    return launch_scan(data, n, 0u, 1u, status, st, false);
}

}  // namespace wp

extern "C" int32_t delta_decode_inplace(uint32_t *data, uint64_t n, uint32_t init, int32_t stride, void *stream)
{
    if (stride != 1 && stride != 4)
        return WP_ERR_INVALID_ARG;
    if (n == 0)
        return WP_OK;
    if (data == nullptr || !aligned16(data))
        return WP_ERR_INVALID_ARG;
    const uint64_t tiles = (n + kMinTileInts - 1) / kMinTileInts;
    if (tiles > 0x7FFFFFFFull)
        return WP_ERR_INVALID_ARG;
    hipStream_t st = as_stream(stream);
    uint64_t *status = static_cast<uint64_t *>(stream_scratch(st, scan_status_words(n) * sizeof(uint64_t)));
    if (status == nullptr)
        return WP_ERR_HIP;
    (void)hipGetLastError();
    return launch_scan(data, n, init, (uint32_t)stride, status, st, true);
}

// ------------------------------------------------------------------------
// The same scan with its status words in a fixed array of the library's
// code object, for callers that cannot allocate. Every device holds its own
// copy of the array at its own address, looked up once per device with
// hipGetSymbolAddress; host code passes only that address to kernels and
// never uses the array's name.

namespace wp {

constexpr uint64_t kNoAllocMaxN = 1ull << 28;
constexpr uint64_t kNoAllocWords = (uint64_t)kStatusWords * ((kNoAllocMaxN + kMinTileInts - 1) / kMinTileInts + 1);

static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

static std::mutex g_nmu;
static std::vector<uint64_t *> g_noalloc_ptr;  // per device, nullptr until looked up

static uint64_t *noalloc_scratch()
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_nmu);
    if ((int)g_noalloc_ptr.size() <= d)
        g_noalloc_ptr.resize(d + 1, nullptr);
    if (g_noalloc_ptr[d] == nullptr) {
        uint64_t *ptr = nullptr;
        if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return nullptr;
        g_noalloc_ptr[d] = ptr;
    }
    return g_noalloc_ptr[d];
}

}  // namespace wp

extern "C" int32_t delta_decode_inplace_noalloc(uint32_t *data, uint64_t n, uint32_t init, int32_t stride,
                                                void *stream)
{
    if (stride != 1 && stride != 4)
        return WP_ERR_INVALID_ARG;
    if (n > kNoAllocMaxN)
        return WP_ERR_CAPACITY;
    if (n == 0)
        return WP_OK;
    if (data == nullptr || !aligned16(data))
        return WP_ERR_INVALID_ARG;
    uint64_t *status = noalloc_scratch();
    if (status == nullptr)
        return WP_ERR_HIP;
    (void)hipGetLastError();
    // launch_scan clears the status words it uses with a fill kernel first
    return launch_scan(data, n, init, (uint32_t)stride, status, as_stream(stream), true);
}
