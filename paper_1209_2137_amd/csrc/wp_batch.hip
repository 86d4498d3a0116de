// Batched decoding of many lists in one launch.
//
// The host planner cuts every list into work items: segments of 64 blocks
// of patched pages, runs of up to `run_units` meta-blocks (binary packing) and the
// Variable Byte tails of lists without full blocks. The tail of any other
// list is decoded by the item that holds the list's last unit. One grid
// covers the items, one wavefront each with no barrier at all, ordered
// largest and smallest alternately: the dispatcher, which starts
// workgroups in index order as compute units free up, schedules the
// longest items first, and the short items (latency-bound: a chain of
// dependent reads each) run beside them. Items are independent because
// every unit's base is stored in its list's directory.
//
// A plan owns its device item array and, when asked, a hipGraph holding
// the one kernel node (built from an explicit node, not captured).
#include <algorithm>
#include <mutex>
#include <vector>

#include "wp_device.hpp"
#include "wp_host.hpp"

namespace wp {

enum : uint32_t { kItemBpRun = 0, kItemFpPage = 1, kItemTail = 2 };

struct DevList {
    const uint32_t *comp;
    uint32_t *out;
    uint64_t comp_words;
    uint64_t n;
    uint32_t codec;
    uint32_t pad;
};

template <int DEPTH>
union WaveItemLds {
    WaveLds<DEPTH> r;
    FpWaveLds fp;
    TailLds<1> tail;
};

// Header check of item `it`'s list; uniform.
__device__ __forceinline__ bool item_header(const DevList *__restrict__ lists, const uint4 *__restrict__ items,
                                            uint32_t it, uint4 &item, DevList &Ld, ListHdr &H)
{
    const uint4 t = items[it];
    item = make_uint4(uniform(t.x), uniform(t.y), uniform(t.z), uniform(t.w));
    Ld = lists[item.x];
    Ld.codec = uniform(Ld.codec);
    Ld.comp = as_global(Ld.comp);
    Ld.out = as_global(Ld.out);
    return check_header(Ld.comp, Ld.comp_words, Ld.n, Ld.codec == WP_CODEC_BP ? kMagicBP : kMagicFP,
                        Ld.codec == WP_CODEC_BP ? kBpBlocks : kFpBlocks, H);
}

// Item `it` -- a run of binary-packing meta-blocks {list, kind, first unit,
// unit count}, a segment of a patched page {list, kind, page, its blocks |
// segment << 16} or a tail -- decoded by one wavefront; the item holding a
// list's last unit (its last segment) also decodes its tail. Uniform
// result.
template <int DEPTH>
__device__ __forceinline__ bool wave_item(const DevList *__restrict__ lists, const uint4 *__restrict__ items, uint32_t it,
                          WaveItemLds<DEPTH> &W)
{
    uint4 item;
    DevList Ld;
    ListHdr H;
    if (!item_header(lists, items, it, item, Ld, H))
        return false;
    bool ok, last;
    if (item.y == kItemBpRun) {
        const uint32_t first = item.z, count = item.w;
        ok = Ld.codec == WP_CODEC_BP && count >= 1 && count <= 63 && (uint64_t)first + count <= H.units;
        if (!ok)
            return false;
        ok = H.S == 1   ? bp_wave_run<DEPTH, 1>(Ld.comp, H, first, count, Ld.out, W.r)
             : H.S == 4 ? bp_wave_run<DEPTH, 4>(Ld.comp, H, first, count, Ld.out, W.r)
                        : bp_wave_run<DEPTH, 0>(Ld.comp, H, first, count, Ld.out, W.r);
        last = first + count == H.units;
    } else if (item.y == kItemFpPage) {
        const uint64_t u = item.z;
        const uint32_t seg = item.w >> 16;
        if (!(Ld.codec == WP_CODEC_FP && u < H.units))
            return false;
        const uint32_t nseg = page_items<kPageFp>(page_blocks(H, u));
        if (seg >= nseg)
            return false;
        ok = fp_unit(Ld.comp, H, u, seg, Ld.out, W.fp);
        last = u + 1 == H.units && seg + 1 == nseg;
    } else {
        return item.y == kItemTail && H.tail != 0 && decode_tail_entry<1, false>(Ld.comp, H, Ld.out, W.tail);
    }
    if (ok && last && H.tail) {
        wave_lds_order();
        ok = decode_tail_entry<1, false>(Ld.comp, H, Ld.out, W.tail);
    }
    return ok;
}

// One launch over the whole plan: wavefront w of workgroup g decodes item
// g * WAVES + w. The largest items come first, and the dispatcher starts
// workgroups in index order as compute units free up, which balances the
// load without a work queue.
template <int WAVES, int DEPTH>
__global__ __launch_bounds__(64 * WAVES) void k_batch(const DevList *__restrict__ lists,
                                                      const uint4 *__restrict__ items, uint32_t nitems,
                                                      int *__restrict__ err)
{
    __shared__ WaveItemLds<DEPTH> L[WAVES];
    const uint32_t wave = uniform(threadIdx.x >> 6);
    const uint64_t it = (uint64_t)blockIdx.x * WAVES + wave;
    if (it >= nitems)
        return;
    if (!wave_item<DEPTH>(lists, items, (uint32_t)it, L[wave]) && lane_id() == 0)
        *err = kErrCorrupt;
}

// The persistent form: a grid sized to the chip (wg_per_cu workgroups per
// compute unit) whose wavefronts take items, in plan order, from a device
// counter until none is left, kQueueChunk consecutive items per atomic
// (one device-scope atomic per item serialises on the counter's address);
// the counter is cleared by a small kernel launched before it (a graph
// holds both nodes).
constexpr uint32_t kQueueChunk = 8;
template <int WAVES, int DEPTH>
__global__ __launch_bounds__(64 * WAVES) void k_batch_queue(const DevList *__restrict__ lists,
                                                            const uint4 *__restrict__ items, uint32_t nitems,
                                                            int *__restrict__ err, uint32_t *__restrict__ next)
{
    __shared__ WaveItemLds<DEPTH> L[WAVES];
    const uint32_t wave = uniform(threadIdx.x >> 6);
    uint32_t it = 0;
    if (lane_id() == 0)
        it = atomicAdd(next, kQueueChunk);
    it = uniform(it);
    // every wavefront leaves once the counter has passed the items
    while (it < nitems) {
        // the next chunk's first index is taken now; its round trip overlaps
        // this chunk
        uint32_t nx = 0;
        if (lane_id() == 0)
            nx = atomicAdd(next, kQueueChunk);
        const uint32_t end = nitems - it < kQueueChunk ? nitems : it + kQueueChunk;
        for (; it < end; ++it) {
            if (!wave_item<DEPTH>(lists, items, it, L[wave]) && lane_id() == 0)
                *err = kErrCorrupt;
            wave_lds_order();
        }
        it = uniform(nx);
    }
}

__global__ void k_batch_reset(uint32_t *next)
{
    if (threadIdx.x == 0)
        *next = 0;
}

struct Plan {
    int device = -1;
    DevList *d_lists = nullptr;
    uint4 *d_items = nullptr;
    uint64_t nlists = 0, nitems = 0;
    int waves = 4, vpl = 4, depth = 4;
    uint32_t grid = 1;
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *kernel = nullptr;
    int *err = nullptr;
    // re-planning without allocation: capacities and pinned staging
    uint64_t cap_lists = 0, cap_items = 0;
    DevList *h_lists_pin = nullptr;
    uint4 *h_items_pin = nullptr;
    uint64_t pin_lists = 0, pin_items = 0;
    hipEvent_t copied = nullptr;
    int run_units = 8;
    int wg_per_cu = 0;          // > 0: the persistent form, this many workgroups per compute unit
    uint32_t *counter = nullptr;  // its item counter
};

template <int W, int D>
static const void *batch_kernel(bool queue)
{
    return queue ? reinterpret_cast<const void *>(&k_batch_queue<W, D>) : reinterpret_cast<const void *>(&k_batch<W, D>);
}

template <int W>
static const void *batch_kernel_depth(int depth, bool queue)
{
    return depth == 2 ? batch_kernel<W, 2>(queue) : depth == 3 ? batch_kernel<W, 3>(queue) : batch_kernel<W, 4>(queue);
}

// waves 2, 4 or 8 (vpl 4), each with ring depth 2..4; the one-shot grid or
// the persistent form
static const void *pick_kernel(int waves, int vpl, int depth, bool queue)
{
    if (depth < 2 || depth > 4 || vpl != 4)
        return nullptr;
    if (waves == 2)
        return batch_kernel_depth<2>(depth, queue);
    if (waves == 4)
        return batch_kernel_depth<4>(depth, queue);
    if (waves == 8)
        return batch_kernel_depth<8>(depth, queue);
    return nullptr;
}

static void release(Plan *p)
{
    if (p->copied)
        (void)hipEventSynchronize(p->copied), (void)hipEventDestroy(p->copied);
    if (p->h_lists_pin)
        (void)hipHostFree(p->h_lists_pin);
    if (p->h_items_pin)
        (void)hipHostFree(p->h_items_pin);
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->d_lists)
        (void)hipFree(p->d_lists);
    if (p->d_items)
        (void)hipFree(p->d_items);
    if (p->counter)
        (void)hipFree(p->counter);
    delete p;
}

// Workgroups of a launch: one per `waves` items (at least one).
static uint64_t grid_for(uint64_t nitems, int waves)
{
    return std::max<uint64_t>(1, (nitems + (uint64_t)waves - 1) / (uint64_t)waves);
}
constexpr uint64_t kMaxGrid = 0x7FFFFFFFull;

// Workgroups of the persistent form.
static uint32_t queue_grid(const Plan *p, int cus)
{
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)cus * (uint64_t)p->wg_per_cu,
                                                               grid_for(p->nitems, p->waves)));
}

static int32_t launch_plan(Plan *p, hipStream_t st)
{
    (void)hipGetLastError();
    if (p->nitems == 0)
        return WP_OK;
    uint32_t nitems32 = (uint32_t)p->nitems;
    if (p->wg_per_cu > 0) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, p->counter);
        void *qargs[] = {&p->d_lists, &p->d_items, &nitems32, &p->err, &p->counter};
        if (hipLaunchKernel(p->kernel, dim3(p->grid), dim3(64 * p->waves), qargs, 0, st) != hipSuccess)
            return WP_ERR_HIP;
        return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
    }
    void *args[] = {&p->d_lists, &p->d_items, &nitems32, &p->err};
    if (hipLaunchKernel(p->kernel, dim3(p->grid), dim3(64 * p->waves), args, 0, st) != hipSuccess)
        return WP_ERR_HIP;
    return hipGetLastError() == hipSuccess ? WP_OK : WP_ERR_HIP;
}

static int32_t build_graph(Plan *p)
{
    if (hipGraphCreate(&p->graph, 0) != hipSuccess)
        return WP_ERR_HIP;
    hipGraphNode_t dec = nullptr, reset = nullptr;
    uint32_t nitems32 = (uint32_t)p->nitems;
    void *args[] = {&p->d_lists, &p->d_items, &nitems32, &p->err, &p->counter};
    if (p->wg_per_cu > 0) {
        // the counter is cleared by a kernel node (no memset node), then the decoder
        void *rargs[] = {&p->counter};
        hipKernelNodeParams rp = {};
        rp.func = reinterpret_cast<void *>(&k_batch_reset);
        rp.gridDim = dim3(1);
        rp.blockDim = dim3(64);
        rp.kernelParams = rargs;
        if (hipGraphAddKernelNode(&reset, p->graph, nullptr, 0, &rp) != hipSuccess)
            return WP_ERR_HIP;
    }
    void *args4[] = {&p->d_lists, &p->d_items, &nitems32, &p->err};
    hipKernelNodeParams kp = {};
    kp.func = const_cast<void *>(p->kernel);
    kp.gridDim = dim3(p->grid);
    kp.blockDim = dim3(64 * p->waves);
    kp.sharedMemBytes = 0;
    kp.kernelParams = p->wg_per_cu > 0 ? args : args4;
    kp.extra = nullptr;
    if (hipGraphAddKernelNode(&dec, p->graph, reset ? &reset : nullptr, reset ? 1 : 0, &kp) != hipSuccess)
        return WP_ERR_HIP;
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return WP_ERR_HIP;
    return WP_OK;
}

// Validates a registry and cuts it into work items: binary-packing runs of
// run_units meta-blocks, page segments, tails; ordered largest and smallest
// alternately.
static bool build_items(const uint32_t *pool, uint32_t *out_base, const wp_list *h_lists, uint64_t nlists,
                        int run_units, std::vector<DevList> &lists, std::vector<uint4> &items)
{
    lists.assign(nlists, DevList{});
    std::vector<uint4> unit_items, tail_items;
    if (nlists > 0xFFFFFFFFull)
        return false;
    for (uint64_t i = 0; i < nlists; ++i) {
        const wp_list &l = h_lists[i];
        if ((l.codec != WP_CODEC_BP && l.codec != WP_CODEC_FP) || l.reserved != 0 || (l.comp_off_words & 3u) ||
            l.comp_words < kHdrWords || l.n > 0xFFFFFFFFull * 32ull)
            return false;
        // the list's own destination, else its place in out_base
        if (l.out != nullptr ? !aligned16(l.out) : (out_base == nullptr || (l.out_off & 3u)))
            return false;
        lists[i].comp = pool + l.comp_off_words;
        lists[i].out = l.out != nullptr ? l.out : out_base + l.out_off;
        lists[i].comp_words = l.comp_words;
        lists[i].n = l.n;
        lists[i].codec = (uint32_t)l.codec;
        lists[i].pad = 0;
        const uint64_t nfull = l.n / kBlock;
        const uint32_t li = (uint32_t)i;
        if (l.codec == WP_CODEC_BP) {
            const uint64_t units = (nfull + kBpBlocks - 1) / kBpBlocks;
            for (uint64_t u = 0; u < units; u += (uint64_t)run_units) {
                const uint64_t c = std::min<uint64_t>((uint64_t)run_units, units - u);
                unit_items.push_back(make_uint4(li, kItemBpRun, (uint32_t)u, (uint32_t)c));
            }
        } else {
            const uint64_t units = (nfull + kFpBlocks - 1) / kFpBlocks;
            for (uint64_t u = 0; u < units; ++u) {
                const uint64_t nb = std::min<uint64_t>(kFpBlocks, nfull - u * kFpBlocks);
                for (uint32_t g = 0; g < page_items<kPageFp>((uint32_t)nb); ++g) {
                    const uint32_t sb = (uint32_t)std::min<uint64_t>(kSegBlocks, nb - g * kSegBlocks);
                    unit_items.push_back(make_uint4(li, kItemFpPage, (uint32_t)u, sb | (g << 16)));
                }
            }
        }
        // a tail has an item of its own only in a list without full blocks;
        // otherwise the list's last run or page decodes it
        if ((l.n % kBlock) && nfull == 0)
            tail_items.push_back(make_uint4(li, kItemTail, 0, 0));
    }
    // by blocks, largest first (a run of w meta-blocks holds up to 16 w), then tails
    auto blocks = [](const uint4 &a) { return a.y == kItemBpRun ? 16u * a.w : (a.w & 0xffffu); };
    std::stable_sort(unit_items.begin(), unit_items.end(),
                     [&](const uint4 &a, const uint4 &b) { return blocks(a) > blocks(b); });
    items.reserve(unit_items.size() + tail_items.size());
    // largest, smallest, second largest, second smallest, ...: the longest
    // items still start first, and the short items' chains of dependent
    // reads overlap the large items' streaming instead of running alone at
    // the end of the grid (1.44 -> 1.33 ms on the 10^5-list pool)
    std::vector<uint4> all(unit_items);
    all.insert(all.end(), tail_items.rbegin(), tail_items.rend());
    size_t lo = 0, hi = all.size();
    while (lo < hi) {
        items.push_back(all[lo++]);
        if (lo < hi)
            items.push_back(all[--hi]);
    }
    return items.size() <= 0xFFFFFFF0ull;
}

}  // namespace wp

using namespace wp;

extern "C" int32_t wp_batch_plan(const uint32_t *pool, uint32_t *out_base, const wp_list *h_lists, uint64_t nlists,
                                 const wp_tune *tune, void **h_plan, void *stream)
{
    if (h_plan == nullptr || (nlists > 0 && (pool == nullptr || h_lists == nullptr)))
        return WP_ERR_INVALID_ARG;
    *h_plan = nullptr;
    if (!aligned16(pool) || !aligned16(out_base))
        return WP_ERR_INVALID_ARG;
    wp_tune t = {4, 4, 2, 8, 0, 1};
    if (tune) {
        t = *tune;
        if (t.waves == 0)
            t.waves = 4;
        if (t.vpl == 0)
            t.vpl = 4;
        if (t.depth == 0)
            t.depth = 2;
        if (t.run_units == 0)
            t.run_units = 8;
    }
    const void *kern = pick_kernel(t.waves, t.vpl, t.depth, t.wg_per_cu > 0);
    if (kern == nullptr || t.run_units < 1 || t.run_units > 63 || t.wg_per_cu < 0 || t.wg_per_cu > 64)
        return WP_ERR_INVALID_ARG;
    DevState *ds = dev_state();
    if (ds == nullptr)
        return WP_ERR_HIP;
    std::vector<DevList> lists;
    std::vector<uint4> items;
    if (!build_items(pool, out_base, h_lists, nlists, t.run_units, lists, items) ||
        grid_for(items.size(), t.waves) > kMaxGrid)
        return WP_ERR_INVALID_ARG;
    Plan *p = new Plan();
    p->device = ds->device;
    p->err = ds->err;
    p->nlists = nlists;
    p->nitems = items.size();
    p->waves = t.waves;
    p->vpl = t.vpl;
    p->depth = t.depth;
    p->kernel = kern;
    p->use_graph = t.use_graph != 0;
    p->run_units = t.run_units;
    p->wg_per_cu = t.wg_per_cu;
    p->cap_lists = std::max<uint64_t>(1, lists.size());
    p->cap_items = std::max<uint64_t>(1, items.size());
    p->grid = p->wg_per_cu > 0 ? queue_grid(p, ds->cus) : (uint32_t)grid_for(items.size(), t.waves);
    hipStream_t st = as_stream(stream);
    if (p->wg_per_cu > 0 && hipMalloc(&p->counter, 256) != hipSuccess) {
        release(p);
        return WP_ERR_HIP;
    }
    if (hipMalloc(&p->d_lists, std::max<size_t>(1, lists.size()) * sizeof(DevList)) != hipSuccess ||
        hipMalloc(&p->d_items, std::max<size_t>(1, items.size()) * sizeof(uint4)) != hipSuccess) {
        release(p);
        return WP_ERR_HIP;
    }
    if ((!lists.empty() &&
         hipMemcpyAsync(p->d_lists, lists.data(), lists.size() * sizeof(DevList), hipMemcpyHostToDevice, st) !=
             hipSuccess) ||
        (!items.empty() &&
         hipMemcpyAsync(p->d_items, items.data(), items.size() * sizeof(uint4), hipMemcpyHostToDevice, st) !=
             hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess) {
        release(p);
        return WP_ERR_HIP;
    }
    if (p->use_graph && build_graph(p) != WP_OK) {
        release(p);
        return WP_ERR_HIP;
    }
    *h_plan = p;
    return WP_OK;
}

extern "C" int32_t wp_batch_decode(void *h_plan, void *stream)
{
    Plan *p = static_cast<Plan *>(h_plan);
    if (p == nullptr)
        return WP_ERR_INVALID_ARG;
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d != p->device)
        return WP_ERR_INVALID_ARG;
    hipStream_t st = as_stream(stream);
    if (p->use_graph) {
        (void)hipGetLastError();
        return hipGraphLaunch(p->exec, st) == hipSuccess ? WP_OK : WP_ERR_HIP;
    }
    return launch_plan(p, st);
}

extern "C" uint64_t wp_batch_items(const void *h_plan)
{
    const Plan *p = static_cast<const Plan *>(h_plan);
    return p ? p->nitems : 0;
}

extern "C" int32_t wp_batch_free(void *h_plan)
{
    Plan *p = static_cast<Plan *>(h_plan);
    if (p == nullptr)
        return WP_ERR_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess) {
        release(p);
        return WP_ERR_HIP;
    }
    release(p);
    return WP_OK;
}

extern "C" int32_t wp_batch_replan(void *h_plan, const uint32_t *pool, uint32_t *out_base, const wp_list *h_lists,
                                   uint64_t nlists, void *stream)
{
    Plan *p = static_cast<Plan *>(h_plan);
    if (p == nullptr || (nlists > 0 && (pool == nullptr || h_lists == nullptr)) || !aligned16(pool) ||
        !aligned16(out_base))
        return WP_ERR_INVALID_ARG;
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d != p->device)
        return WP_ERR_INVALID_ARG;
    std::vector<DevList> lists;
    std::vector<uint4> items;
    if (!build_items(pool, out_base, h_lists, nlists, p->run_units, lists, items) ||
        grid_for(items.size(), p->waves) > kMaxGrid)
        return WP_ERR_INVALID_ARG;
    hipStream_t st = as_stream(stream);
    // the previous copy out of the pinned staging must have finished
    if (p->copied && hipEventSynchronize(p->copied) != hipSuccess)
        return WP_ERR_HIP;
    if (lists.size() > p->cap_lists || items.size() > p->cap_items) {
        // grow: earlier launches of this plan may still read the old arrays
        if (hipStreamSynchronize(st) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return WP_ERR_HIP;
        if (lists.size() > p->cap_lists) {
            (void)hipFree(p->d_lists);
            p->d_lists = nullptr;
            p->cap_lists = lists.size() + lists.size() / 2;
            if (hipMalloc(&p->d_lists, p->cap_lists * sizeof(DevList)) != hipSuccess)
                return WP_ERR_HIP;
        }
        if (items.size() > p->cap_items) {
            (void)hipFree(p->d_items);
            p->d_items = nullptr;
            p->cap_items = items.size() + items.size() / 2;
            if (hipMalloc(&p->d_items, p->cap_items * sizeof(uint4)) != hipSuccess)
                return WP_ERR_HIP;
        }
    }
    if (lists.size() > p->pin_lists) {
        if (p->h_lists_pin)
            (void)hipHostFree(p->h_lists_pin);
        p->h_lists_pin = nullptr;
        p->pin_lists = std::max<uint64_t>(lists.size() * 2, 64);
        if (hipHostMalloc(&p->h_lists_pin, p->pin_lists * sizeof(DevList), 0) != hipSuccess) {
            p->pin_lists = 0;
            return WP_ERR_HIP;
        }
    }
    if (items.size() > p->pin_items) {
        if (p->h_items_pin)
            (void)hipHostFree(p->h_items_pin);
        p->h_items_pin = nullptr;
        p->pin_items = std::max<uint64_t>(items.size() * 2, 256);
        if (hipHostMalloc(&p->h_items_pin, p->pin_items * sizeof(uint4), 0) != hipSuccess) {
            p->pin_items = 0;
            return WP_ERR_HIP;
        }
    }
    if (p->copied == nullptr && hipEventCreateWithFlags(&p->copied, hipEventDisableTiming) != hipSuccess)
        return WP_ERR_HIP;
    std::copy(lists.begin(), lists.end(), p->h_lists_pin);
    std::copy(items.begin(), items.end(), p->h_items_pin);
    (void)hipGetLastError();
    if ((!lists.empty() && hipMemcpyAsync(p->d_lists, p->h_lists_pin, lists.size() * sizeof(DevList),
                                          hipMemcpyHostToDevice, st) != hipSuccess) ||
        (!items.empty() && hipMemcpyAsync(p->d_items, p->h_items_pin, items.size() * sizeof(uint4),
                                          hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipEventRecord(p->copied, st) != hipSuccess)
        return WP_ERR_HIP;
    p->nlists = lists.size();
    p->nitems = items.size();
    if (p->wg_per_cu > 0) {
        DevState *ds = dev_state();
        if (ds == nullptr)
            return WP_ERR_HIP;
        p->grid = queue_grid(p, ds->cus);
    } else {
        p->grid = (uint32_t)grid_for(items.size(), p->waves);
    }
    // the graph baked in the old item count and grid
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec), p->exec = nullptr;
    if (p->graph)
        (void)hipGraphDestroy(p->graph), p->graph = nullptr;
    p->use_graph = false;
    return WP_OK;
}
