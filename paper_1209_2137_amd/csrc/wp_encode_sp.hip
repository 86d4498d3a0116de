// SimplePFOR pages (Section 5, SimplePFOR; Simple-8b of Section 2): the
// encoder's per-page kernels. Widths, exception counts and positions are
// those of the patched pages (the same cost rule, computed by the patched
// encoder's analysis kernel); the exceptions' high parts of a page, in
// block order, are coded once with Simple-8b.
//
// Simple-8b's greedy choice is sequential: the next word starts where the
// previous one ended. One wavefront per page walks it. The page's high
// parts stream, block by block, into a 512-entry LDS window (each block's
// exceptions found with ballots); for the next word the 64 lanes take the
// next 64 high parts' widths, a prefix maximum over the lanes gives the
// widest of the first c for every c, and lane s tests selector s (count
// available, widest of its first `count` within its width) at once. The
// first selector that passes is the greedy one. High parts are never zero
// (an exception is wider than its block's width), so selectors 0 and 1
// (runs of zeros) never pass and only selectors 2..15 are tested.
//
// Two passes, as for every unit: k_sp_size runs the coding to size each
// page (packed words, metadata, Simple-8b words), the chained scan turns
// sizes into offsets, and k_sp_pack writes the page: its header, the
// blocks' low bits, the metadata bytes (widths, maximum widths, counts,
// positions) and, from one wavefront, the same coding again, now writing
// its words.
#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

namespace {

constexpr uint32_t kSpWin = 512;  // high parts held by a page's coding window

__device__ __forceinline__ uint32_t sp_nbits(uint32_t x) { return 32u - (uint32_t)__clz((int)x); }

__device__ __forceinline__ uint32_t sp_delta(const uint32_t *__restrict__ x, uint64_t i, uint32_t S)
{
    const uint32_t v = x[i];
    if (S == 0)
        return v;
    return i >= S ? v - x[i - S] : v;
}

// Inclusive maximum over the 64 lanes (values >= 0): row steps, then the
// two row broadcasts, as in wave_scan_incl.
__device__ __forceinline__ uint32_t wave_max_incl(uint32_t v)
{
    auto step = [&](uint32_t o) __attribute__((always_inline)) { v = o > v ? o : v; };
    step(__builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false));
    step(__builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false));
    step(__builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false));
    step(__builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false));
    step(__builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false));
    step(__builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_read(wave_scan_incl(v), 63); }

// Words of a SimplePFOR page's header: 4, then for each 64-block segment
// after the first S bases and one Simple-8b entry, padded to 4.
__device__ __forceinline__ uint32_t sp_hdr_words(uint32_t nb, uint32_t S)
{
    return pad4(4u + (S + 1u) * (page_items<kPageFp>(nb) - 1u));
}

// The greedy Simple-8b coding of page `p`'s high parts (nexc of them), by
// one wavefront; with WRITE the words go to s8 (two 32-bit words each, low
// half first), and the entry of each segment g = 1 .. nseg - 1 (seg_e[g]:
// the exceptions before it) to entries[g - 1]: the index of the word
// holding high part seg_e[g] | the word's values before it << 24, or the
// word count when seg_e[g] = nexc. Returns the number of 64-bit words
// (uniform).
template <uint32_t S, bool WRITE>
__device__ uint32_t sp_code(const uint32_t *__restrict__ x, uint64_t pstart, uint32_t nb,
                            const uint8_t *__restrict__ mb, const uint8_t *__restrict__ mc, uint32_t nexc,
                            uint32_t *__restrict__ s8, uint32_t *win, const uint32_t *seg_e = nullptr,
                            uint32_t nseg = 1, uint32_t *__restrict__ entries = nullptr)
{
    const uint32_t lane = lane_id();
    // selector tested by this lane (2..15): its count and width
    const uint32_t my_sel = lane >= 2 && lane <= 15 ? lane : 15u;
    const uint32_t my_md = s8_mode(my_sel);
    const uint32_t my_cnt = my_md & 255u, my_bits = my_md >> 8;
    uint32_t t = 0, produced = 0, i = 0, words = 0;
    while (i < nexc) {
        // the window holds at least the next 64 high parts (or all that are left)
        while (t < nb && produced - i < 64u) {
            const uint32_t b = uniform(mb[t]), c = uniform(mc[t]);
            if (c != 0u) {
                const uint64_t j0 = pstart + (uint64_t)t * kBlock + lane;
                const uint32_t d0 = sp_delta(x, j0, S), d1 = sp_delta(x, j0 + 64, S);
                const bool e0 = sp_nbits(d0) > b, e1 = sp_nbits(d1) > b;
                const uint64_t m0 = ballot(e0), m1 = ballot(e1);
                const uint32_t n0 = (uint32_t)__builtin_popcountll(m0);
                if (e0)
                    win[(produced + lanes_below(m0)) & (kSpWin - 1u)] = d0 >> b;
                if (e1)
                    win[(produced + n0 + lanes_below(m1)) & (kSpWin - 1u)] = d1 >> b;
                produced += n0 + (uint32_t)__builtin_popcountll(m1);
                wave_lds_order();
            }
            ++t;
        }
        const uint32_t avail = nexc - i;
        const bool live = lane < avail;
        const uint32_t hv = live ? win[(i + lane) & (kSpWin - 1u)] : 0u;
        const uint32_t widest = wave_max_incl(live ? sp_nbits(hv) : 64u);
        // widest of the first my_cnt high parts
        const uint32_t wc = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((my_cnt - 1u) * 4u), (int)widest);
        const bool pass = lane >= 2 && lane <= 15 && my_cnt <= avail && wc <= my_bits;
        const uint32_t sel = (uint32_t)__builtin_ctzll(ballot(pass));  // selector 15 always passes
        const uint32_t md = s8_mode(sel);
        const uint32_t cnt = md & 255u, bits = md >> 8;
        if constexpr (WRITE) {
            // the fields do not overlap: their sum is the word
            const uint64_t f = lane < cnt ? (uint64_t)hv << (lane * bits) : 0ull;
            const uint32_t lo = wave_sum((uint32_t)f), hi = wave_sum((uint32_t)(f >> 32)) | (sel << 28);
            if (lane == 0) {
                s8[2 * words] = lo;
                s8[2 * words + 1] = hi;
            }
            // lane g: segment g's first high part in this word?
            if (lane >= 1 && lane < nseg) {
                const uint32_t e = seg_e[lane];
                if (e >= i && e < i + cnt)
                    entries[lane - 1] = words | ((e - i) << 24);
            }
        }
        ++words;
        i += cnt;
        wave_lds_order();
    }
    if constexpr (WRITE) {
        if (lane >= 1 && lane < nseg && seg_e[lane] >= nexc)
            entries[lane - 1] = words;
    }
    return words;
}

// Packed words and exceptions of page p from its blocks' metadata: sums
// over the blocks (uniform).
__device__ __forceinline__ void sp_page_sums(const uint8_t *__restrict__ mb, const uint8_t *__restrict__ mc,
                                             uint32_t nb, uint32_t &packed, uint32_t &nexc)
{
    const uint32_t lane = lane_id();
    uint32_t pw = 0, ne = 0;
    for (uint32_t t = lane; t < nb; t += 64) {
        pw += 4u * mb[t];
        ne += mc[t];
    }
    packed = wave_sum(pw);
    nexc = wave_sum(ne);
}

}  // namespace

// One wavefront per page: the page's length in words.
template <uint32_t S>
__global__ __launch_bounds__(64) void k_sp_size(const uint32_t *__restrict__ x, uint64_t n,
                                                const uint8_t *__restrict__ meta, uint64_t nblk,
                                                uint32_t *__restrict__ sizes)
{
    __shared__ uint32_t win[kSpWin];
    const uint64_t p = blockIdx.x;
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - p * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    const uint8_t *mb = meta + p * kFpBlocks, *mm = meta + nblk + p * kFpBlocks, *mc = meta + 2 * nblk + p * kFpBlocks;
    (void)mm;
    uint32_t packed, nexc;
    sp_page_sums(mb, mc, nb, packed, nexc);
    const uint32_t words = sp_code<S, false>(x, p * kFpUnitInts, nb, mb, mc, nexc, nullptr, win);
    const uint32_t meta_w = ((3u * nb + nexc + 15u) / 16u) * 4u;
    if (lane_id() == 0)
        sizes[p] = pad4(sp_hdr_words(nb, S) + packed + meta_w + 2u * words);
}

// One workgroup of four wavefronts per page: wavefront 0 writes the page
// header (with the segment bases and entries) and codes the high parts
// into their place; the others write the packed low bits (16 lanes per
// block, each eight values = b whole bytes) and the metadata bytes, and
// clear the metadata's padding.
template <uint32_t S>
__global__ __launch_bounds__(256) void k_sp_pack(const uint32_t *__restrict__ x, uint64_t n,
                                                 const uint8_t *__restrict__ meta, uint64_t nblk,
                                                 const uint32_t *__restrict__ incl, uint32_t dir_end,
                                                 uint32_t *__restrict__ out)
{
    __shared__ uint32_t win[kSpWin];
    __shared__ uint32_t s_blk[kFpBlocks];  // block t's first packed word (from the packed region)
    __shared__ uint32_t s_exc[kFpBlocks];  // block t's first exception in the page
    __shared__ uint32_t s_tot[2];
    __shared__ uint32_t s_sege[kPageSegs];  // exceptions before each segment
    const uint64_t p = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint64_t nfull = n / kBlock;
    const uint64_t left = nfull - p * kFpBlocks;
    const uint32_t nb = (uint32_t)(left < kFpBlocks ? left : kFpBlocks);
    const uint8_t *mb = meta + p * kFpBlocks, *mm = meta + nblk + p * kFpBlocks, *mc = meta + 2 * nblk + p * kFpBlocks;
    const uint64_t pstart = p * kFpUnitInts;
    // block offsets: exclusive sums of 4b and c in block order (wavefront 0)
    if (wave == 0) {
        uint32_t cw = 0, cc = 0;
        for (uint32_t t0 = 0; t0 < nb; t0 += 64) {
            const uint32_t t = t0 + lane;
            const uint32_t bw = t < nb ? 4u * mb[t] : 0u, c = t < nb ? (uint32_t)mc[t] : 0u;
            const uint32_t iw = wave_scan_incl(bw), ic = wave_scan_incl(c);
            if (t < nb) {
                s_blk[t] = cw + iw - bw;
                s_exc[t] = cc + ic - c;
            }
            cw += wave_read(iw, 63);
            cc += wave_read(ic, 63);
        }
        if (lane == 0)
            s_tot[0] = cw, s_tot[1] = cc;
    }
    __syncthreads();
    const uint32_t packed = s_tot[0], nexc = s_tot[1];
    const uint32_t nseg = page_items<kPageFp>(nb), hw = sp_hdr_words(nb, S);
    if (wave == 0 && lane < kPageSegs)
        s_sege[lane] = lane < nseg ? s_exc[kSegBlocks * lane] : 0u;
    const uint32_t meta_bytes = 3u * nb + nexc;
    const uint32_t meta_w = ((meta_bytes + 15u) / 16u) * 4u;
    const uint32_t size = incl[p] - (p ? incl[p - 1] : 0u);
    const uint32_t off = dir_end + incl[p] - size;
    const uint32_t s8_at = hw + packed + meta_w;
    const uint32_t s8w = size - s8_at;  // Simple-8b words and the page's end padding
    write_dir_entry(out, p, dir_entries(n, kFpBlocks), S, off, x, pstart);
    uint32_t *page = out + off;
    if (wave == 0) {
        wave_lds_order();
        const uint32_t words = sp_code<S, true>(x, pstart, nb, mb, mc, nexc, page + s8_at, win, s_sege, nseg,
                                                page + 4 + S * (nseg - 1u));
        // zero padding after the words, up to the page's end
        for (uint32_t w = 2u * words + lane; w < s8w; w += 64)
            page[s8_at + w] = 0u;
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
            page[3] = 2u * words;
        }
        return;
    }
    // waves 1..3: blocks in groups of four, 16 lanes per block
    uint8_t *const pk = reinterpret_cast<uint8_t *>(page + hw);
    uint8_t *const md = reinterpret_cast<uint8_t *>(page + hw + packed);
    const uint32_t g = lane >> 4, r = lane & 15u;
    for (uint32_t t0 = 4u * (wave - 1u); t0 < nb; t0 += 12u) {
        const uint32_t t = t0 + g;
        const bool in = t < nb;
        const uint32_t b = in ? (uint32_t)mb[t] : 0u;
        uint32_t d[8];
        uint32_t emask = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            d[k] = in ? sp_delta(x, pstart + (uint64_t)t * kBlock + 8u * r + k, S) : 0u;
            emask |= (sp_nbits(d[k]) > b ? 1u : 0u) << k;
        }
        if (in) {
            // low b bits of the eight values: b bytes from byte b * r of the block
            const uint32_t m = width_mask(b);
            uint64_t acc = 0;
            uint32_t nbit = 0, o = 4u * s_blk[t] + b * r;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc |= (uint64_t)(d[k] & m) << nbit;
                nbit += b;
                while (nbit >= 8u) {
                    pk[o++] = (uint8_t)acc;
                    acc >>= 8;
                    nbit -= 8u;
                }
            }
        }
        // positions of the block's exceptions, in order: rank = exceptions of
        // the lanes before this one in the block's 16, then within the lane
        const uint32_t cnt = (uint32_t)__builtin_popcount(emask);
        const uint32_t incl16 = row_scan_incl(cnt);  // rows of 16 lanes are the blocks
        uint32_t at = in ? 3u * nb + s_exc[t] + incl16 - cnt : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (in && ((emask >> k) & 1u))
                md[at++] = (uint8_t)(8u * r + k);
        if (in && r == 0) {
            md[t] = (uint8_t)b;
            md[nb + t] = mm[t];
            md[2u * nb + t] = mc[t];
        }
    }
    // the metadata's padding to 16 bytes
    for (uint32_t i = meta_bytes + (tid - 64u); i < 4u * meta_w; i += 192u)
        md[i] = 0;
}

}  // namespace wp

using namespace wp;

namespace wp {

// SimplePFOR pages of one encode call: size, offsets, pages. `meta` holds
// the patched analysis's widths, maximum widths and counts.
int32_t sp_encode_units(const uint32_t *in, uint64_t n, uint32_t stride, uint64_t units, const uint8_t *meta,
                        uint64_t nblk, uint32_t *sizes, uint64_t *status, uint32_t dir_end, uint32_t *out,
                        hipStream_t st)
{
#define WP_SP_LAUNCH(kern, threads, ...)                                                                   \
    do {                                                                                                   \
        if (stride == 0)                                                                                   \
            hipLaunchKernelGGL(kern<0u>, dim3((uint32_t)units), dim3(threads), 0, st, __VA_ARGS__);         \
        else if (stride == 1)                                                                              \
            hipLaunchKernelGGL(kern<1u>, dim3((uint32_t)units), dim3(threads), 0, st, __VA_ARGS__);         \
        else                                                                                               \
            hipLaunchKernelGGL(kern<4u>, dim3((uint32_t)units), dim3(threads), 0, st, __VA_ARGS__);         \
    } while (0)
    WP_SP_LAUNCH(k_sp_size, 64, in, n, meta, nblk, sizes);
    if (launch_inclusive_scan(sizes, units, status, st) != WP_OK)
        return WP_ERR_HIP;
    WP_SP_LAUNCH(k_sp_pack, 256, in, n, meta, nblk, sizes, dir_end, out);
#undef WP_SP_LAUNCH
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

}  // namespace wp
