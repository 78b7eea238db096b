// Ingest from a packed transfer format: a chunk crosses the host link with
// its per-event object counts as bytes (instead of 32-bit offsets) and its
// charges and b-tags as bytes (instead of float32), and the device rebuilds
// the structure-of-arrays layout of hf_events_t from them: the offsets by an
// exclusive prefix sum of the counts (per tile of kTile events a sum, the
// tile sums scanned by one block, then each tile scanned from its offset),
// the charge and b-tag columns by widening the bytes.  Integer and byte work
// only: the rebuilt columns equal the unpacked ones bit for bit.
#include "hf_device.hpp"
#include "hf_internal.hpp"
#include "hf_unpack.hpp"

namespace hf {
namespace {

constexpr int kBlock = 256;
constexpr int kPer = 16;                 // counts per thread (one 16-byte load)
constexpr int kTile = kBlock * kPer;     // counts per tile

// Exclusive scan of v over the block; total receives the block's sum.
__device__ __forceinline__ uint64_t block_scan(uint64_t v, uint64_t *s_w, uint64_t &total) {
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    uint64_t inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) base += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

// the kPer counts of this thread in tile t (zeros past n)
__device__ __forceinline__ void load_counts(const uint8_t *cnt, int64_t n, int64_t t, uint32_t c[kPer]) {
    const int64_t k0 = t * kTile + (int64_t)threadIdx.x * kPer;
    if (k0 + kPer <= n) {
        const uint4 w = *reinterpret_cast<const uint4 *>(cnt + k0);  // 16-byte aligned: k0 is a multiple of 16
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int u = 0; u < kPer; ++u) c[u] = (words[u / 4] >> (8 * (u % 4))) & 0xffu;
    } else {
#pragma unroll
        for (int u = 0; u < kPer; ++u) c[u] = k0 + u < n ? cnt[k0 + u] : 0u;
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack_tiles(const uint8_t *__restrict__ lc, const uint8_t *__restrict__ jc,
                                                         int64_t n, uint64_t *__restrict__ tsum) {
    __shared__ uint64_t s_w[kBlock / kWave];
    const int64_t nt = (n + kTile - 1) / kTile;
    uint32_t c[kPer];
    uint64_t total;
    load_counts(lc, n, blockIdx.x, c);
    uint64_t v = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) v += c[u];
    block_scan(v, s_w, total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
    load_counts(jc, n, blockIdx.x, c);
    v = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) v += c[u];
    block_scan(v, s_w, total);
    if (threadIdx.x == 0) tsum[nt + 1 + blockIdx.x] = total;
}

// tile sums -> tile offsets (exclusive), grand totals at [nt] of each half
__global__ __launch_bounds__(kBlock) void k_unpack_top(int64_t n, uint64_t *__restrict__ tsum) {
    __shared__ uint64_t s_w[kBlock / kWave];
    const int64_t nt = (n + kTile - 1) / kTile;
    for (int half = 0; half < 2; ++half) {
        uint64_t *ts = tsum + half * (nt + 1);
        uint64_t carry = 0;
        for (int64_t c0 = 0; c0 < nt; c0 += kBlock) {
            const int64_t t = c0 + threadIdx.x;
            const uint64_t v = t < nt ? ts[t] : 0;
            uint64_t total;
            const uint64_t ex = block_scan(v, s_w, total);
            if (t < nt) ts[t] = carry + ex;
            carry += total;
        }
        if (threadIdx.x == 0) ts[nt] = carry;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_unpack_apply(const uint8_t *__restrict__ lc,
                                                         const uint8_t *__restrict__ jc, int64_t n,
                                                         const uint64_t *__restrict__ tsum,
                                                         uint32_t *__restrict__ loff, uint32_t *__restrict__ joff) {
    __shared__ uint64_t s_w[kBlock / kWave];
    const int64_t nt = (n + kTile - 1) / kTile;
    const int64_t k0 = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kPer;
    for (int half = 0; half < 2; ++half) {
        const uint8_t *cnt = half ? jc : lc;
        uint32_t *off = half ? joff : loff;
        const uint64_t *ts = tsum + half * (nt + 1);
        uint32_t c[kPer];
        load_counts(cnt, n, blockIdx.x, c);
        uint64_t v = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) v += c[u];
        uint64_t total;
        uint64_t run = ts[blockIdx.x] + block_scan(v, s_w, total);
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (k0 + u < n) off[k0 + u] = (uint32_t)run;
            run += c[u];
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = (uint32_t)ts[nt];
    }
}

// charges and b-tags: bytes -> float32
__global__ __launch_bounds__(kBlock) void k_unpack_cast(const int8_t *__restrict__ q8, int64_t n_lep,
                                                        const uint8_t *__restrict__ b8, int64_t n_jet,
                                                        float *__restrict__ q, float *__restrict__ b) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_jet || i < n_lep; i += stride) {
        if (i < n_lep) q[i] = (float)q8[i];
        if (i < n_jet) b[i] = (float)b8[i];
    }
}

}  // namespace

size_t unpack_ws_bytes(int64_t n) {
    const int64_t nt = n > 0 ? (n + kTile - 1) / kTile : 0;
    return (size_t)(2 * (nt + 1)) * sizeof(uint64_t);
}

hipError_t launch_unpack(int64_t n, const uint8_t *lc, const uint8_t *jc, int64_t n_lep, int64_t n_jet,
                         const int8_t *q8, const uint8_t *b8, uint32_t *loff, uint32_t *joff, float *q, float *b,
                         void *ws, hipStream_t s) {
    uint64_t *tsum = static_cast<uint64_t *>(ws);
    // an empty chunk still gets its offsets[0] = 0 (one block, no counts)
    const unsigned nt = n > 0 ? (unsigned)((n + kTile - 1) / kTile) : 1u;
    hipLaunchKernelGGL(k_unpack_tiles, dim3(nt), dim3(kBlock), 0, s, lc, jc, n, tsum);
    hipLaunchKernelGGL(k_unpack_top, dim3(1), dim3(kBlock), 0, s, n, tsum);
    hipLaunchKernelGGL(k_unpack_apply, dim3(nt), dim3(kBlock), 0, s, lc, jc, n, tsum, loff, joff);
    const int64_t m = n_lep > n_jet ? n_lep : n_jet;
    if (m > 0) {
        int64_t g = (m + kBlock - 1) / kBlock;
        if (g > 4096) g = 4096;
        hipLaunchKernelGGL(k_unpack_cast, dim3((unsigned)g), dim3(kBlock), 0, s, q8, n_lep, b8, n_jet, q, b);
    }
    return hipGetLastError();
}

}  // namespace hf
