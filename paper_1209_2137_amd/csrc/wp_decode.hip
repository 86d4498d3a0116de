// Single-list decoders: bp_decode, bp32_decode and fastpfor_decode.
//
// Units are independent because the directory stores each unit's offset
// and base value(s): no cross-workgroup dependency, no second pass.
//
// Binary packing: every wavefront decodes its own contiguous run of
// meta-blocks (bp_wave_run); a workgroup is just WAVES such runs side by
// side. The workgroup after the last run decodes the Variable Byte tail.
// BP32 streams (32-integer blocks) take the same kernel in its B32 mode,
// SIMD-BP128 streams with the four-lane block layout in its V mode.
//
// Patched pages: one wavefront per 64-block segment of a page
// (fp_wave_page), a workgroup being WAVES such segments side by side;
// FastPFOR streams (exception arrays padded to 32 values) take the same
// kernel in its P32 mode; a SimplePFOR page is one wavefront.
#include <mutex>
#include <vector>

#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

template <int WAVES, int DEPTH, bool B32>
union BpKernelLds {
    WaveLds<DEPTH, B32> w[WAVES];
    TailLds<WAVES> tail;
};

// Wavefront w of workgroup g decodes run g * WAVES + w: units
// [run * upw, run * upw + upw) of one list.
template <int WAVES, int DEPTH, bool B32 = false, bool V = false>
__global__ __launch_bounds__(64 * WAVES) void k_bp_decode(const uint32_t *__restrict__ in, uint64_t in_words,
                                                          uint32_t *__restrict__ out, uint64_t n,
                                                          int *__restrict__ err, uint32_t upw)
{
    __shared__ BpKernelLds<WAVES, DEPTH, B32> L;
    ListHdr H;
    if (!check_header(in, in_words, n, B32 ? kMagicBP32 : V ? kMagicBPV : kMagicBP, kBpBlocks, H)) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            *err = kErrCorrupt;
        return;
    }
    const uint64_t nruns = (H.units + upw - 1) / upw;
    const uint64_t nwg = (nruns + WAVES - 1) / WAVES;
    if (blockIdx.x >= nwg) {
        if (blockIdx.x == nwg && H.tail)
            if (!decode_tail_entry<WAVES>(in, H, out, L.tail) && threadIdx.x == 0)
                *err = kErrCorrupt;
        return;
    }
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint64_t r = (uint64_t)blockIdx.x * WAVES + wave;
    if (r >= nruns)
        return;
    const uint64_t ua = r * upw;
    const uint32_t cnt = (uint32_t)((H.units - ua) < upw ? (H.units - ua) : upw);
    const bool ok = H.S == 1   ? bp_wave_run<DEPTH, 1, B32, V>(in, H, ua, cnt, out, L.w[wave])
                    : H.S == 4 ? bp_wave_run<DEPTH, 4, B32, V>(in, H, ua, cnt, out, L.w[wave])
                               : bp_wave_run<DEPTH, 0, B32, V>(in, H, ua, cnt, out, L.w[wave]);
    if (!ok && lane_id() == 0)
        *err = kErrCorrupt;
}

template <int KIND>
union FpWaveItemLds {
    FpWaveLds page;
    SpWaveLds sp;  // SimplePFOR pages also hold a ring of decoded high parts
    TailLds<1> tail;
};
template <>
union FpWaveItemLds<kPageFp> {
    FpWaveLds page;
    TailLds<1> tail;
};
template <>
union FpWaveItemLds<kPageFp32> {
    FpWaveLds page;
    TailLds<1> tail;
};
template <>
union FpWaveItemLds<kPageFpi> {
    FpiLds page;
    TailLds<1> tail;
};

// Wavefronts resident per SIMD that the patched-page kernel is compiled
// for (register budget).
#ifndef WP_FP_MIN_WAVES
#define WP_FP_MIN_WAVES 8
#endif

// Wavefront w of workgroup g takes item i = g * WAVES + w: segment i % 8 of
// page i / 8 (SimplePFOR: page i); the item after the last page's decodes
// the tail. KIND: SIMD-FastPFOR, FastPFOR or SimplePFOR pages.
template <int WAVES, int KIND = kPageFp>
__global__ __launch_bounds__(64 * WAVES, WP_FP_MIN_WAVES) void k_fp_decode(const uint32_t *__restrict__ in, uint64_t in_words,
                                                          uint32_t *__restrict__ out, uint64_t n,
                                                          int *__restrict__ err)
{
    __shared__ FpWaveItemLds<KIND> L[WAVES];
    ListHdr H;
    const uint32_t magic = KIND == kPageSp     ? kMagicSP
                           : KIND == kPageFp32 ? kMagicFP32
                           : KIND == kPageFpi  ? kMagicFPI
                                               : kMagicFP;
    if (!check_header(in, in_words, n, magic, kFpBlocks, H)) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            *err = kErrCorrupt;
        return;
    }
    const uint32_t wave = uniform(threadIdx.x >> 6);
    constexpr uint32_t per = page_items<KIND>(kFpBlocks);
    const uint64_t item = (uint64_t)blockIdx.x * WAVES + wave;
    const uint64_t u = item / per;
    const uint32_t seg = (uint32_t)(item % per);
    bool ok = true;
    if (u == H.units) {
        if (H.tail && seg == 0)
            ok = decode_tail_entry<1, false>(in, H, out, L[wave].tail);
    } else if (u < H.units && seg < page_items<KIND>(page_blocks(H, u))) {
        if constexpr (KIND == kPageSp)
            ok = fp_unit<KIND>(in, H, u, seg, out, L[wave].sp.fp, L[wave].sp.ring);
        else
            ok = fp_unit<KIND>(in, H, u, seg, out, L[wave].page);
    }
    if (!ok && lane_id() == 0)
        *err = kErrCorrupt;
}

// ------------------------------------------------------------------------
// Host side

static std::mutex g_mu;
static std::vector<DevState> g_dev;
static thread_local LaunchEvents t_events;

// The error word kernels report corrupt streams into: one per device, in
// the library's own code object (zero when the code object loads), so no
// decoder call allocates. Host code reaches it through the address that
// hipGetSymbolAddress returns for the current device, never through this
// name.
static __device__ __align__(16) int g_err_word[4];

LaunchEvents take_launch_events()
{
    const LaunchEvents e = t_events;
    t_events = LaunchEvents{};
    return e;
}
// per tuning slot: SIMD-BP128 (both block layouts), patched pages (both
// paddings), BP32
static Tune g_tune[3] = {{4, 4, kBpRunsPerCu, 2}, {4, 4, 0, 0}, {4, 4, kBpRunsPerCu, 2}};

static int tune_slot(int codec)
{
    return (codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP || codec == WP_CODEC_FPI) ? 1
           : codec == WP_CODEC_BP32                                                ? 2
                                                                                   : 0;
}

DevState *dev_state()
{
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= d)
        g_dev.resize(d + 1);
    DevState &s = g_dev[d];
    if (s.err == nullptr) {
        void *e = nullptr;
        if (hipGetSymbolAddress(&e, HIP_SYMBOL(g_err_word)) != hipSuccess || e == nullptr)
            return nullptr;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess)
            cus = 256;
        s.err = static_cast<int *>(e);
        s.cus = cus;
        s.device = d;
    }
    return &s;
}

Tune decode_tune(int codec)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_tune[tune_slot(codec)];
}

static bool valid_tune(int codec, int waves, int vpl)
{
    (void)codec;
    return (waves == 1 || waves == 2 || waves == 4 || waves == 8) && vpl == 4;
}

template <int WAVES, int DEPTH, bool B32 = false, bool V = false>
static void launch_bp(uint64_t grid, hipStream_t st, const uint32_t *in, uint64_t in_words, uint32_t *out,
                      uint64_t n, int *err, uint32_t upw)
{
    launch_timed(k_bp_decode<WAVES, DEPTH, B32, V>, dim3((uint32_t)grid), dim3(64 * WAVES), st, in, in_words, out,
                 n, err, upw);
}

template <int WAVES>
static void launch_fp(int kind, uint64_t grid, hipStream_t st, const uint32_t *in, uint64_t in_words, uint32_t *out,
                      uint64_t n, int *err)
{
    if (kind == kPageFp32)
        launch_timed(k_fp_decode<WAVES, kPageFp32>, dim3((uint32_t)grid), dim3(64 * WAVES), st, in, in_words, out,
                     n, err);
    else if (kind == kPageSp)
        launch_timed(k_fp_decode<WAVES, kPageSp>, dim3((uint32_t)grid), dim3(64 * WAVES), st, in, in_words, out, n,
                     err);
    else if (kind == kPageFpi)
        launch_timed(k_fp_decode<1, kPageFpi>, dim3((uint32_t)grid), dim3(64), st, in, in_words, out, n, err);
    else
        launch_timed(k_fp_decode<WAVES, kPageFp>, dim3((uint32_t)grid), dim3(64 * WAVES), st, in, in_words, out, n,
                     err);
}

static int32_t decode_common(int codec, const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                             void *stream)
{
    if (in == nullptr || in_words < kHdrWords || (n > 0 && out == nullptr))
        return WP_ERR_INVALID_ARG;
    if (!aligned16(in) || !aligned16(out))
        return WP_ERR_INVALID_ARG;
    if (n > 0xFFFFFFFFull * 32ull)
        return WP_ERR_INVALID_ARG;
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    const bool paged = codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP || codec == WP_CODEC_FPI;
    const uint64_t per = paged ? kFpBlocks : kBpBlocks;
    const uint64_t nfull = n / kBlock;
    const uint64_t units = (nfull + per - 1) / per;
    const uint64_t has_tail = (n % kBlock) ? 1 : 0;
    hipStream_t st = as_stream(stream);
    const Tune t = decode_tune(codec);
    (void)hipGetLastError();
    if (!paged) {
        // runs of upw meta-blocks, one per wavefront: about wg_per_cu runs
        // per compute unit
        const uint64_t target = (uint64_t)ds->cus * (uint64_t)(t.wg_per_cu > 0 ? t.wg_per_cu : kBpRunsPerCu);
        uint64_t upw = (units + target - 1) / (target ? target : 1);
        upw = upw < 1 ? 1 : (upw > 63 ? 63 : upw);
        const uint64_t nruns = (units + upw - 1) / upw;
        uint64_t grid = (nruns + t.waves - 1) / t.waves + has_tail;
        grid = grid ? grid : 1;
        if (grid > 0x7FFFFFFFull)
            return WP_ERR_INVALID_ARG;
        const uint32_t u32 = (uint32_t)upw;
        const bool b32 = codec == WP_CODEC_BP32, vert = codec == WP_CODEC_BPV;
#define WP_BP_D(W, D)                                                                                           \
    (b32    ? launch_bp<W, D, true>(grid, st, in, in_words, out, n, ds->err, u32)                               \
     : vert ? launch_bp<W, D, false, true>(grid, st, in, in_words, out, n, ds->err, u32)                        \
            : launch_bp<W, D>(grid, st, in, in_words, out, n, ds->err, u32))
#define WP_BP(W) (t.depth >= 4 ? WP_BP_D(W, 4) : t.depth == 3 ? WP_BP_D(W, 3) : WP_BP_D(W, 2))
        if (t.waves == 1)
            WP_BP(1);
        else if (t.waves == 2)
            WP_BP(2);
        else if (t.waves == 4)
            WP_BP(4);
        else
            WP_BP(8);
#undef WP_BP
#undef WP_BP_D
    } else {
        // one wavefront per segment (the paper's layout: per page, one
        // wavefront per workgroup, for its LDS), then one for the tail;
        // SimplePFOR segments at most two per workgroup (each holds 16 KB
        // of LDS: the ring of decoded high parts besides the packed words)
        const uint64_t per_page = codec == WP_CODEC_FPI ? 1 : kPageSegs;
        const int waves = codec == WP_CODEC_FPI ? 1 : codec == WP_CODEC_SP ? (t.waves < 2 ? t.waves : 2) : t.waves;
        const uint64_t wpg = (uint64_t)waves;
        uint64_t grid = (units * per_page + has_tail + wpg - 1) / wpg;
        grid = grid ? grid : 1;
        if (grid > 0x7FFFFFFFull)
            return WP_ERR_INVALID_ARG;
        const int kind = codec == WP_CODEC_FP32 ? kPageFp32
                         : codec == WP_CODEC_SP ? kPageSp
                         : codec == WP_CODEC_FPI ? kPageFpi
                                                 : kPageFp;
        if (waves == 1)
            launch_fp<1>(kind, grid, st, in, in_words, out, n, ds->err);
        else if (waves == 2)
            launch_fp<2>(kind, grid, st, in, in_words, out, n, ds->err);
        else if (waves == 4)
            launch_fp<4>(kind, grid, st, in, in_words, out, n, ds->err);
        else
            launch_fp<8>(kind, grid, st, in, in_words, out, n, ds->err);
    }
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

}  // namespace wp

using namespace wp;

extern "C" int32_t bp_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n, void *stream)
{
    return decode_common(WP_CODEC_BP, in, in_words, out, n, stream);
}

extern "C" int32_t fastpfor_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                                   void *stream)
{
    return decode_common(WP_CODEC_FP, in, in_words, out, n, stream);
}

extern "C" int32_t bp32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n, void *stream)
{
    return decode_common(WP_CODEC_BP32, in, in_words, out, n, stream);
}

extern "C" int32_t fastpfor32_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                                     void *stream)
{
    return decode_common(WP_CODEC_FP32, in, in_words, out, n, stream);
}

extern "C" int32_t simplepfor_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                                     void *stream)
{
    return decode_common(WP_CODEC_SP, in, in_words, out, n, stream);
}

extern "C" int32_t fastpfor_inline_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                                          void *stream)
{
    return decode_common(WP_CODEC_FPI, in, in_words, out, n, stream);
}

extern "C" int32_t bp_vertical_decode(const uint32_t *in, uint64_t in_words, uint32_t *out, uint64_t n,
                                      void *stream)
{
    return decode_common(WP_CODEC_BPV, in, in_words, out, n, stream);
}

extern "C" int32_t wp_set_decode_tune(int32_t codec, int32_t waves, int32_t vpl, int32_t depth, int32_t wg_per_cu)
{
    if ((codec != WP_CODEC_BP && codec != WP_CODEC_FP && codec != WP_CODEC_BP32 && codec != WP_CODEC_FP32 &&
         codec != WP_CODEC_BPV && codec != WP_CODEC_SP && codec != WP_CODEC_FPI) ||
        !valid_tune(codec, waves, vpl) || wg_per_cu < 0 ||
        wg_per_cu > 1024 || depth < 0 || depth == 1 || depth > 4)
        return WP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune[tune_slot(codec)] = Tune{waves, vpl, wg_per_cu, depth ? depth : 2};
    return WP_OK;
}

extern "C" int32_t wp_time_next_launch(void *start_event, void *stop_event)
{
    t_events.start = reinterpret_cast<hipEvent_t>(start_event);
    t_events.stop = reinterpret_cast<hipEvent_t>(stop_event);
    return WP_OK;
}

extern "C" int32_t wp_check(void *stream)
{
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess)
        return WP_ERR_HIP;
    int v = 0;
    if (hipMemcpy(&v, ds->err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return WP_ERR_HIP;
    if (v != 0 && hipMemset(ds->err, 0, sizeof(int)) != hipSuccess)
        return WP_ERR_HIP;
    return v;
}

extern "C" const char *wp_strerror(int32_t code)
{
    switch (code) {
    case WP_OK:
        return "ok";
    case WP_ERR_INVALID_ARG:
        return "invalid argument";
    case WP_ERR_CAPACITY:
        return "output capacity too small";
    case WP_ERR_CORRUPT:
        return "corrupt compressed stream";
    case WP_ERR_HIP:
        return "HIP runtime error";
    default:
        return "unknown error";
    }
}

extern "C" uint64_t wp_max_compressed_words(int32_t codec, uint64_t n)
{
    if (codec != WP_CODEC_BP && codec != WP_CODEC_FP && codec != WP_CODEC_BP32 && codec != WP_CODEC_FP32 &&
        codec != WP_CODEC_BPV && codec != WP_CODEC_SP && codec != WP_CODEC_FPI)
        return 0;
    const uint64_t nfull = n / kBlock, tail = n % kBlock;
    const uint64_t per = (codec == WP_CODEC_FP || codec == WP_CODEC_FP32 || codec == WP_CODEC_SP ||
                          codec == WP_CODEC_FPI) ? kFpBlocks
                                                                                                 : kBpBlocks;
    const uint64_t units = (nfull + per - 1) / per;
    uint64_t w = kHdrWords + ((5 * (units + 1) + 3) & ~3ull);
    if (codec == WP_CODEC_BP || codec == WP_CODEC_BPV) {
        w += units * 4 + nfull * 128;  // descriptor + every block at 32 bits
    } else if (codec == WP_CODEC_BP32) {
        // a descriptor word per meta-block, every block at 32 bits, at most
        // three words of padding per unit
        w += units * 3 + nfull * (1 + 128);
    } else if (codec == WP_CODEC_FPI) {
        // page: offset word, byte counter, bitset, 32 array counters and 3
        // words of padding; packed <= 128 words per block; byte array <=
        // 130 bytes per block + 3 bytes of padding; exception bits of a
        // block <= 127 * 32; at most 31 values of padding per array
        w += units * (1 + 1 + 1 + 32 + 3 + 1 + 32 * 31) + nfull * (128 + 33 + 127);
    } else if (codec == WP_CODEC_SP) {
        // page header <= 39 words (4, seven segment bases of up to four
        // words, seven segment entries) and 3 words of padding; packed <= 128
        // words per block; metadata <= 131 bytes per block + 16 bytes
        // padding; at most one 64-bit Simple-8b word (two words) per exception
        w += units * (39 + 3 + 4) + nfull * (128 + 33 + 1 + 2 * 128);
    } else {
        // page header <= 64 words (4, a count per array, seven segment
        // bases of up to four words); metadata <= 130 bytes per block + 16
        // bytes padding; packed <= 128 words per block; exception bits of a
        // block <= 127 * 32; one group of padding for each of the 32 arrays
        w += units * (64 + 4 + 32 * 4 * 32) + nfull * (128 + 33 + 127);
    }
    w += (tail * 5 + 3) / 4;
    return w > 0xFFFFFFFFull ? 0 : w;
}
