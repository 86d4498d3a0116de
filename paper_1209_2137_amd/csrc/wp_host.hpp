// Host-side state shared by the wavepack translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wavepack.h"

namespace wp {

// Per-device state: the address of the device's error word (a static
// device variable of the library; kernels report corrupt streams into it)
// and the device's compute-unit count.
struct DevState {
    int *err = nullptr;
    int cus = 0;
    int device = -1;
};

// Returns the current device's state, filling it on first use (a symbol
// lookup, no allocation). nullptr if HIP fails.
DevState *dev_state();

// Scratch memory owned by the library for one (device, stream) pair: calls
// on one stream run in order, so they can share it. Grows on demand (the
// old buffer is released after synchronising the stream). nullptr on failure.
void *stream_scratch(hipStream_t stream, size_t bytes);

// Decoder configuration for the single-list entry points.
struct Tune {
    int waves;
    int vpl;
    int wg_per_cu;  // binary packing: runs (one per wavefront) per compute unit (0 = default)
    int depth;      // binary packing: 16-byte chunk loads in flight per wavefront (2..4)
};

// Default binary-packing runs per compute unit. Many short runs (down to
// one meta-block per wavefront) let the hardware dispatcher balance the
// load: wavefronts that finish early take the next runs.
constexpr int kBpRunsPerCu = 128;
Tune decode_tune(int codec);

// In-place inclusive prefix sum of data[0..n) on `st` (the chained scan of
// delta_decode_inplace, stride 1, init 0). `status` must hold
// scan_status_words(n) zero-or-garbage words; it is cleared on the stream.
uint64_t scan_status_words(uint64_t n);
int32_t launch_inclusive_scan(uint32_t *data, uint64_t n, uint64_t *status, hipStream_t st);

// Clears `count` 64-bit words on `st` with a kernel (look-back status words
// before a chained scan).
void launch_clear(uint64_t *p, uint64_t count, hipStream_t st);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// The SimplePFOR pages of an encode call (after the patched analysis has
// written every block's width, maximum width and exception count to
// `meta`): page sizes into `sizes` and each page's Simple-8b word starts
// into `spw` (sp_scratch_bytes(units) bytes), the sizes' chained scan
// (`status` as for launch_inclusive_scan), then the pages themselves.
// `spx`: each block's exceptions' high-part widths, one byte each in
// position order, from byte k * kSpWidthSlot for block k (written by the
// patched analysis in its SimplePFOR form).
constexpr uint32_t kSpWidthSlot = 128;  // at least the cost rule's 102 exceptions per block
uint64_t sp_scratch_bytes(uint64_t units);
int32_t sp_encode_units(const uint32_t *in, uint64_t n, uint32_t stride, uint64_t units, const uint8_t *meta,
                        uint64_t nblk, uint32_t *sizes, uint64_t *status, uint8_t *spw, const uint8_t *spx,
                        uint32_t dir_end, uint32_t *out, hipStream_t st);

// Rearranges the FastPFOR stream `tmp` (arrays padded to 32) into pages of
// the paper's own layout in `out`: page sizes, their chained scan, the
// pages, then header, directory and tail; the length goes to out_words.
int32_t fpi_encode_pages(const uint32_t *tmp, uint64_t units, uint32_t dir_end, uint32_t *sizes, uint64_t *status,
                         uint32_t *out, uint64_t *out_words, hipStream_t st);

// Events the calling thread's next decoder launch records when its main
// kernel starts and ends (set by wp_time_next_launch); taking them clears
// them.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
LaunchEvents take_launch_events();

// Launches kernel(args...) on st, recording the thread's launch events
// around it if any are set.
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    const LaunchEvents e = take_launch_events();
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e.start, e.stop, 0, args...);
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace wp
