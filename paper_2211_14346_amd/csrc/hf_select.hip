// Cut chain launchers (the device code is in hf_cuts.hpp), the counter
// reduction, and the device-side cut reordering.  Compiled with
// -ffp-contract=off.
#include <math.h>

#include "hf_cuts.hpp"
#include "hf_device.hpp"
#include "hf_internal.hpp"
#include "hf_rtc.hpp"

namespace hf {

static_assert(kChainBlock == kSelBlock, "the compiled-chain launch uses the chain kernel's block size");

namespace {

constexpr int kSelMaxGrid = 2048;

// One block per counter word: sums the per-block partial rows and adds the
// total to the caller's counters.
__global__ __launch_bounds__(256) void k_select_reduce(const uint64_t *__restrict__ partial, int nblocks, int width,
                                                       uint64_t *__restrict__ counters) {
    __shared__ uint64_t s_w[256 / kWave];
    const int t = blockIdx.x;
    uint64_t s = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[(size_t)b * width + t];
    for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (int w = 0; w < 256 / kWave; ++w) tot += s_w[w];
        counters[t] += tot;
    }
}

}  // namespace

int select_grid(int64_t n) {
    int64_t g = (n + kSelBlock - 1) / kSelBlock;
    if (g < 1) g = 1;
    if (g > kSelMaxGrid) g = kSelMaxGrid;
    return (int)g;
}

size_t select_ws_bytes(int64_t n, int n_cuts) {
    return (size_t)select_grid(n) * (size_t)n_cuts * 3 * sizeof(uint64_t);
}

hipError_t launch_select(const EvView &ev, const CutTable &ct, const int32_t *order, uint8_t *survive,
                         hf_counters_t *counters, void *ws, hipStream_t s) {
    const int grid = select_grid(ev.n);
    uint64_t *partial = static_cast<uint64_t *>(ws);
    hipLaunchKernelGGL(k_select_t<NoUserCuts>, dim3(grid), dim3(kSelBlock), 0, s, ev, ct, order, survive, partial,
                       (const int32_t *)nullptr, (const int64_t *)nullptr, (int64_t)0, 0, ct.n);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return launch_select_reduce(partial, grid, ct.n, counters, s);
}

hipError_t launch_select_segment(const EvView &ev, const CutTable &ct, const int32_t *order, int pos_begin,
                                 int pos_end, const int32_t *idx, const int64_t *count, int64_t capacity,
                                 uint8_t *survive, hf_counters_t *counters, void *ws, hipStream_t s) {
    const int grid = select_grid(idx ? capacity : ev.n);
    uint64_t *partial = static_cast<uint64_t *>(ws);
    hipLaunchKernelGGL(k_select_t<NoUserCuts>, dim3(grid), dim3(kSelBlock), 0, s, ev, ct, order, survive, partial,
                       idx, count, capacity, pos_begin, pos_end);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    return launch_select_reduce(partial, grid, ct.n, counters, s);
}

hipError_t launch_select_reduce(const uint64_t *partial, int grid, int n_cuts, hf_counters_t *counters,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_select_reduce, dim3(n_cuts * 3), dim3(256), 0, s, partial, grid, n_cuts * 3,
                       reinterpret_cast<uint64_t *>(counters));
    return hipGetLastError();
}

// ---------------------------------------------------------------- reordering
// The greedy placement of hf_reorder_stats (section 5.2) on the device, so
// that a recorded step can reorder its cuts without a host round trip.  One
// thread: at most HF_MAX_CUTS cuts.  The rank arithmetic is the host's
// (correctly rounded FP64 division, no contraction in this unit), so both
// produce the same order.
__global__ void k_reorder(const hf_counters_t *__restrict__ counters, CutTable ct, int32_t *__restrict__ order) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    __shared__ double rank[HF_MAX_CUTS];
    for (int c = 0; c < ct.n; ++c) {
        const hf_counters_t k = counters[c];
        const double p = k.reached ? (double)k.passed / (double)k.reached : 1.0;
        const double cost = k.reached ? (double)k.cost / (double)k.reached : 0.0;
        const double rej = 1.0 - p;
        rank[c] = cost / (rej > 1e-9 ? rej : 1e-9);
    }
    uint64_t placed = 0;
    for (int pos = 0; pos < ct.n; ++pos) {
        int best = -1;
        for (int c = 0; c < ct.n; ++c) {
            if ((placed >> c) & 1ull) continue;
            if (ct.c[c].dep_mask & ~placed) continue;
            if (best < 0 || rank[c] < rank[best]) best = c;
        }
        if (best < 0) return;  // cyclic: rejected on the host before the launch
        order[pos] = best;
        placed |= 1ull << best;
    }
}

hipError_t launch_reorder(const hf_counters_t *counters, const CutTable &ct, int32_t *order, hipStream_t s) {
    hipLaunchKernelGGL(k_reorder, dim3(1), dim3(64), 0, s, counters, ct, order);
    return hipGetLastError();
}

}  // namespace hf
