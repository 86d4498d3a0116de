// fastpfor_inline_encode: FastPFOR pages in the paper's own layout
// (Section 5 and its page-layout figure). The widths, exceptions and
// packed arrays are exactly those of the FastPFOR pages with arrays padded
// to 32 values, so the stream is encoded in that form first (into the
// library's scratch) and each page is then rearranged:
//   k_fpi_size   one wavefront per page: its length in the paper's layout
//   (the chained scan of the lengths gives every page its offset)
//   k_fpi_pack   one workgroup per page: the offset word, the packed words,
//                the byte array (record offsets by a workgroup scan over
//                the blocks: 2 bytes, or 3 + c when the block has
//                exceptions), the bitset and each array behind its counter
//   k_fpi_finish header, directory (new offsets, the same bases) and the
//                Variable Byte tail.
#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

namespace {

// The FastPFOR page at `pg` (stride S): its header fields and where its
// parts start (words from the page start).
struct Fp32Page {
    uint32_t nb, packed, meta_bytes, bitset, nset, hdr_w, meta_w, exc_at;
};

__device__ __forceinline__ Fp32Page fp32_page(const uint32_t *pg, uint32_t S)
{
    Fp32Page f;
    f.nb = uniform(pg[0]);
    f.packed = uniform(pg[1]);
    f.meta_bytes = uniform(pg[2]);
    f.bitset = uniform(pg[3]);
    f.nset = (uint32_t)__builtin_popcount(f.bitset);
    f.hdr_w = pad4(4u + f.nset + S * (page_items<kPageFp32>(f.nb) - 1u));
    f.meta_w = ((f.meta_bytes + 15u) / 16u) * 4u;
    f.exc_at = f.hdr_w + f.packed + f.meta_w;
    return f;
}

__device__ __forceinline__ uint32_t fpi_wave_sum(uint32_t v) { return wave_read(wave_scan_incl(v), 63); }

}  // namespace

// One wavefront per page: the page's length in the paper's layout.
__global__ __launch_bounds__(64) void k_fpi_size(const uint32_t *__restrict__ tmp, uint32_t *__restrict__ sizes)
{
    const uint32_t p = blockIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t S = uniform(tmp[3]);
    const uint32_t *pg = tmp + uniform(tmp[kHdrWords + p]);
    const Fp32Page f = fp32_page(pg, S);
    const uint8_t *c = reinterpret_cast<const uint8_t *>(pg + f.hdr_w + f.packed) + 2u * f.nb;
    uint32_t nz = 0;
    for (uint32_t t = lane; t < f.nb; t += 64)
        nz += c[t] != 0 ? 1u : 0u;
    nz = fpi_wave_sum(nz);
    // arrays: a counter and ceil(count / 32) * k words each
    uint32_t aw = 0;
    if (lane < 32 && ((f.bitset >> lane) & 1u)) {
        const uint32_t k = lane + 1u;
        const uint32_t cnt = pg[4u + (uint32_t)__builtin_popcount(f.bitset & ((1u << lane) - 1u))];
        aw = 1u + ((cnt + 31u) / 32u) * k;
    }
    aw = fpi_wave_sum(aw);
    const uint32_t nba = 2u * f.nb + nz + (f.meta_bytes - 3u * f.nb);
    if (lane == 0)
        sizes[p] = pad4(1u + f.packed + 1u + (nba + 3u) / 4u + 1u + aw);
}

// One workgroup of 512 threads (thread t = block t) per page.
__global__ __launch_bounds__(512) void k_fpi_pack(const uint32_t *__restrict__ tmp, const uint32_t *__restrict__ incl,
                                                  uint32_t dir_end, uint32_t *__restrict__ out)
{
    __shared__ uint32_t s_part[8][2];
    __shared__ uint32_t s_arr[32][3];  // array k - 1: words, offset in the new page, offset in the old
    const uint32_t p = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(tid >> 6);
    const uint32_t S = uniform(tmp[3]);
    const uint32_t *pg = tmp + uniform(tmp[kHdrWords + p]);
    const Fp32Page f = fp32_page(pg, S);
    const uint32_t size = incl[p] - (p ? incl[p - 1] : 0u);
    uint32_t *const q = out + dir_end + incl[p] - size;  // the page in the paper's layout
    const uint8_t *const meta = reinterpret_cast<const uint8_t *>(pg + f.hdr_w + f.packed);
    // block t: its record's length in the byte array and its positions
    const bool in = tid < f.nb;
    const uint32_t b = in ? meta[tid] : 0u, mb = in ? meta[f.nb + tid] : 0u, c = in ? meta[2u * f.nb + tid] : 0u;
    const uint32_t rl = in ? (c ? 3u + c : 2u) : 0u;
    const uint32_t ri = wave_scan_incl(rl), ci = wave_scan_incl(c);
    if (lane == 63)
        s_part[wave][0] = ri, s_part[wave][1] = ci;
    __syncthreads();
    uint32_t ro = ri - rl, co = ci - c, nba = 0, ntot = 0;
    for (uint32_t w = 0; w < 8; ++w) {
        if (w < wave)
            ro += s_part[w][0], co += s_part[w][1];
        nba += s_part[w][0];
        ntot += s_part[w][1];
    }
    const uint32_t cpos = 1u + f.packed, baw = (nba + 3u) / 4u;
    // the offset word, the packed words, the byte counter
    if (tid == 0) {
        q[0] = cpos;
        q[cpos] = nba;
    }
    for (uint32_t i = tid; i < f.packed; i += 512)
        q[1u + i] = pg[f.hdr_w + i];
    // the byte array: the last word first cleared of padding, then records
    uint8_t *const ba = reinterpret_cast<uint8_t *>(q + cpos + 1u);
    if (tid < 4u * baw - nba)
        ba[nba + tid] = 0;
    if (in) {
        ba[ro] = (uint8_t)b;
        ba[ro + 1u] = (uint8_t)mb;
        if (c) {
            ba[ro + 2u] = (uint8_t)c;
            const uint8_t *pos = meta + 3u * f.nb + co;
            for (uint32_t e = 0; e < c; ++e)
                ba[ro + 3u + e] = pos[e];
        }
    }
    // the bitset, then each array behind its counter: offsets by lane
    // k - 1 of wavefront 0, then every array copied by the whole workgroup
    uint32_t xq = cpos + 1u + baw;
    if (tid == 0)
        q[xq] = f.bitset;
    ++xq;
    if (wave == 0) {
        const bool set = lane < 32 && ((f.bitset >> lane) & 1u);
        const uint32_t k = lane + 1u;
        const uint32_t cnt = set ? pg[4u + (uint32_t)__builtin_popcount(f.bitset & ((1u << lane) - 1u))] : 0u;
        const uint32_t words = set ? ((cnt + 31u) / 32u) * k : 0u;
        const uint32_t wi = wave_scan_incl(set ? 1u + words : 0u), wf = wave_scan_incl(words);
        const uint32_t at_q = xq + wi - (set ? 1u + words : 0u), at_f = f.exc_at + wf - words;
        if (set)
            q[at_q] = cnt;
        if (lane < 32) {
            s_arr[lane][0] = words;
            s_arr[lane][1] = at_q + 1u;
            s_arr[lane][2] = at_f;
        }
        const uint32_t end = xq + wave_read(wi, 63);
        for (uint32_t i = end + lane; i < size; i += 64)
            q[i] = 0;
    }
    __syncthreads();
    for (uint32_t k = 0; k < 32; ++k) {
        const uint32_t words = s_arr[k][0], at_q = s_arr[k][1], at_f = s_arr[k][2];
        for (uint32_t i = tid; i < words; i += 512)
            q[at_q + i] = pg[at_f + i];
    }
    (void)ntot;
}

// Header, directory and tail of the rearranged stream.
__global__ __launch_bounds__(256) void k_fpi_finish(const uint32_t *__restrict__ tmp, const uint32_t *__restrict__ incl,
                                                    uint64_t units, uint32_t dir_end, uint32_t *__restrict__ out,
                                                    uint64_t *__restrict__ out_words)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t S = tmp[3], tail_bytes = tmp[5], tail_off_f = tmp[6], total_f = tmp[7];
    const uint64_t ndir = units + (tail_bytes ? 1u : 0u);
    const uint32_t tail_off = units ? dir_end + incl[units - 1] : dir_end;
    for (uint64_t u = tid; u < units; u += 256)
        out[kHdrWords + u] = dir_end + (u ? incl[u - 1] : 0u);
    if (tail_bytes && tid == 0)
        out[kHdrWords + units] = tail_off;
    for (uint64_t i = tid; i < ndir * S; i += 256)
        out[kHdrWords + ndir + i] = tmp[kHdrWords + ndir + i];
    for (uint64_t i = kHdrWords + ndir * (1u + S) + tid; i < dir_end; i += 256)
        out[i] = 0;
    for (uint32_t i = tid; i < total_f - tail_off_f; i += 256)
        out[tail_off + i] = tmp[tail_off_f + i];
    const uint32_t total = tail_off + (total_f - tail_off_f);
    if (tid == 0) {
        out[0] = kMagicFPI;
        for (int i = 1; i < 6; ++i)
            out[i] = tmp[i];
        out[6] = tail_off;
        out[7] = total;
        *out_words = total;
    }
}

}  // namespace wp

namespace wp {

int32_t fpi_encode_pages(const uint32_t *tmp, uint64_t units, uint32_t dir_end, uint32_t *sizes, uint64_t *status,
                         uint32_t *out, uint64_t *out_words, hipStream_t st)
{
    if (units) {
        hipLaunchKernelGGL(k_fpi_size, dim3((uint32_t)units), dim3(64), 0, st, tmp, sizes);
        if (launch_inclusive_scan(sizes, units, status, st) != WP_OK)
            return WP_ERR_HIP;
        hipLaunchKernelGGL(k_fpi_pack, dim3((uint32_t)units), dim3(512), 0, st, tmp, sizes, dir_end, out);
    }
    hipLaunchKernelGGL(k_fpi_finish, dim3(1), dim3(256), 0, st, tmp, sizes, units, dir_end, out, out_words);
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

}  // namespace wp
