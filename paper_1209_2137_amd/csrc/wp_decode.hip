// Single-list decoders: bp_decode and fastpfor_decode.
//
// One workgroup per unit (a 2048-integer meta-block or a 2^16-integer page)
// plus one for the Variable Byte tail. Units are independent because the
// directory stores each unit's base value(s), so there is no cross-workgroup
// dependency and no second pass over the output.
#include <mutex>
#include <vector>

#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

// Decodes directory entry u of one list stream (unit u, or the tail when
// u == n_units). Called by every thread of the workgroup.
template <int CODEC, int WAVES, int VPL, typename Lds>
__device__ void decode_entry(const uint32_t *__restrict__ in, uint64_t in_words, uint32_t *__restrict__ out,
                             uint64_t n, uint64_t u, int *__restrict__ err, Lds &L)
{
    const Hdr h = load_hdr(in);
    const uint32_t per = CODEC == 0 ? kBpBlocks : kFpBlocks;
    const uint64_t hn = (uint64_t)h.n_lo | ((uint64_t)h.n_hi << 32);
    const uint32_t S = h.stride;
    const uint64_t nfull = n / kBlock;
    const uint32_t tail = (uint32_t)(n % kBlock);
    const uint64_t units = (nfull + per - 1) / per;
    const uint64_t E = 1 + (uint64_t)S;
    const uint64_t ndir = units + (tail ? 1 : 0);
    const uint64_t dir_end = kHdrWords + ((E * ndir + 3) & ~(uint64_t)3);
    bool ok = h.magic == (CODEC == 0 ? kMagicBP : kMagicFP) && hn == n && (S == 0 || S == 1 || S == 4) &&
              h.n_units == units && h.total <= in_words && dir_end <= h.total && h.tail_off <= h.total &&
              ((tail == 0) == (h.tail_bytes == 0));
    if (!ok) {
        if (u == 0 && threadIdx.x == 0)
            *err = kErrCorrupt;
        return;
    }
    if (u >= ndir)
        return;
    const uint32_t *ent = in + kHdrWords + u * E;
    uint32_t base[4] = {0u, 0u, 0u, 0u};
    for (uint32_t s = 0; s < S; ++s)
        base[s] = ent[1 + s];
    const uint32_t off = ent[0];
    if (u == units) {
        ok = off == h.tail_off && off >= dir_end && (uint64_t)off + (h.tail_bytes + 3) / 4 == h.total;
        if (ok)
            ok = tail_decode<WAVES>(in + off, h.tail_bytes, tail, S, base, out + nfull * kBlock, L.tail);
    } else {
        const uint32_t end = (u + 1 < units) ? in[kHdrWords + (u + 1) * E] : h.tail_off;
        ok = off >= dir_end && end >= off && end <= h.total && (off & 3u) == 0;
        const uint64_t left = nfull - u * per;
        const uint32_t nb = (uint32_t)(left < per ? left : per);
        if (ok) {
            if constexpr (CODEC == 0)
                ok = bp_unit<WAVES, VPL>(in + off, end - off, nb, S, base, out + u * per * kBlock, L.bp);
            else
                ok = fp_page<WAVES, VPL>(in + off, end - off, nb, S, base, out + u * per * kBlock, L.fp);
        }
    }
    if (!ok && threadIdx.x == 0)
        *err = kErrCorrupt;
}

template <int WAVES, int VPL>
union BpUnion {
    BpLds<WAVES, VPL> bp;
    TailLds<WAVES> tail;
};

template <int WAVES, int VPL>
union FpUnion {
    FpLds<WAVES, VPL> fp;
    TailLds<WAVES> tail;
};

template <int WAVES, int VPL>
__global__ __launch_bounds__(64 * WAVES) void k_bp_decode(const uint32_t *__restrict__ in, uint64_t in_words,
                                                          uint32_t *__restrict__ out, uint64_t n,
                                                          int *__restrict__ err)
{
    __shared__ BpUnion<WAVES, VPL> L;
    struct {
        BpLds<WAVES, VPL> &bp;
        TailLds<WAVES> &tail;
    } view{L.bp, L.tail};
    decode_entry<0, WAVES, VPL>(in, in_words, out, n, blockIdx.x, err, view);
}

template <int WAVES, int VPL>
__global__ __launch_bounds__(64 * WAVES) void k_fp_decode(const uint32_t *__restrict__ in, uint64_t in_words,
                                                          uint32_t *__restrict__ out, uint64_t n,
                                                          int *__restrict__ err)
{
    __shared__ FpUnion<WAVES, VPL> L;
    struct {
        FpLds<WAVES, VPL> &fp;
        TailLds<WAVES> &tail;
    } view{L.fp, L.tail};
    decode_entry<1, WAVES, VPL>(in, in_words, out, n, blockIdx.x, err, view);
}

// ------------------------------------------------------------------------
// Host side

static std::mutex g_mu;
static std::vector<DevState> g_dev;
static Tune g_tune[2] = {{8, 4}, {8, 4}};

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
        int *e = nullptr;
        if (hipMalloc(&e, 16) != hipSuccess)
            return nullptr;
        if (hipMemset(e, 0, 16) != hipSuccess) {
            (void)hipFree(e);
            return nullptr;
        }
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess)
            cus = 256;
        s.err = e;
        s.cus = cus;
        s.device = d;
    }
    return &s;
}

Tune decode_tune(int codec) { return g_tune[codec == WP_CODEC_FP ? 1 : 0]; }

static bool valid_tune(int codec, int waves, int vpl)
{
    if (codec == WP_CODEC_BP)
        return (waves == 2 && vpl == 8) || (waves == 4 && (vpl == 4 || vpl == 8)) || (waves == 8 && vpl == 4);
    return (waves == 4 || waves == 8) && (vpl == 4 || vpl == 8);
}

template <int WAVES, int VPL>
static void launch_bp(uint64_t grid, hipStream_t st, const uint32_t *in, uint64_t in_words, uint32_t *out,
                      uint64_t n, int *err)
{
    hipLaunchKernelGGL((k_bp_decode<WAVES, VPL>), dim3((uint32_t)grid), dim3(64 * WAVES), 0, st, in, in_words,
                       out, n, err);
}

template <int WAVES, int VPL>
static void launch_fp(uint64_t grid, hipStream_t st, const uint32_t *in, uint64_t in_words, uint32_t *out,
                      uint64_t n, int *err)
{
    hipLaunchKernelGGL((k_fp_decode<WAVES, VPL>), dim3((uint32_t)grid), dim3(64 * WAVES), 0, st, in, in_words,
                       out, n, err);
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
    const uint64_t per = codec == WP_CODEC_BP ? kBpBlocks : kFpBlocks;
    const uint64_t nfull = n / kBlock;
    const uint64_t ndir = (nfull + per - 1) / per + ((n % kBlock) ? 1 : 0);
    const uint64_t grid = ndir ? ndir : 1;
    if (grid > 0x7FFFFFFFull)
        return WP_ERR_INVALID_ARG;
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    hipStream_t st = as_stream(stream);
    const Tune t = decode_tune(codec);
    (void)hipGetLastError();
    if (codec == WP_CODEC_BP) {
        if (t.waves == 2 && t.vpl == 8)
            launch_bp<2, 8>(grid, st, in, in_words, out, n, ds->err);
        else if (t.waves == 4 && t.vpl == 4)
            launch_bp<4, 4>(grid, st, in, in_words, out, n, ds->err);
        else if (t.waves == 4 && t.vpl == 8)
            launch_bp<4, 8>(grid, st, in, in_words, out, n, ds->err);
        else
            launch_bp<8, 4>(grid, st, in, in_words, out, n, ds->err);
    } else {
        if (t.waves == 4 && t.vpl == 4)
            launch_fp<4, 4>(grid, st, in, in_words, out, n, ds->err);
        else if (t.waves == 4 && t.vpl == 8)
            launch_fp<4, 8>(grid, st, in, in_words, out, n, ds->err);
        else if (t.waves == 8 && t.vpl == 8)
            launch_fp<8, 8>(grid, st, in, in_words, out, n, ds->err);
        else
            launch_fp<8, 4>(grid, st, in, in_words, out, n, ds->err);
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

extern "C" int32_t wp_set_decode_tune(int32_t codec, int32_t waves, int32_t vpl)
{
    if ((codec != WP_CODEC_BP && codec != WP_CODEC_FP) || !valid_tune(codec, waves, vpl))
        return WP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune[codec] = Tune{waves, vpl};
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
    if (codec != WP_CODEC_BP && codec != WP_CODEC_FP)
        return 0;
    const uint64_t nfull = n / kBlock, tail = n % kBlock;
    const uint64_t per = codec == WP_CODEC_BP ? kBpBlocks : kFpBlocks;
    const uint64_t units = (nfull + per - 1) / per;
    uint64_t w = kHdrWords + ((5 * (units + 1) + 3) & ~3ull);
    if (codec == WP_CODEC_BP) {
        w += units * 4 + nfull * 128;  // descriptor + every block at 32 bits
    } else {
        // page header <= 36 words; metadata <= 130 bytes per block + 16 bytes
        // padding; packed <= 128 words per block; exception bits of a block
        // <= 127 * 32; one group of padding for each of the 32 arrays
        w += units * (36 + 4 + 32 * 4 * 32) + nfull * (128 + 33 + 127);
    }
    w += (tail * 5 + 3) / 4;
    return w > 0xFFFFFFFFull ? 0 : w;
}
