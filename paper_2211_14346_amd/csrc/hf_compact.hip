// Stream compaction of a byte mask into ascending indices (paper section 3:
// the events that pass every cut form the filtered output).
//
// Single pass with decoupled look-back.  A tile is 512 threads x 16 bytes;
// tiles are numbered by an atomic ticket in the order blocks start, so a
// tile only ever waits on tiles whose blocks are already running.  Each
// thread loads its 16 mask bytes with one 128-bit load when aligned, counts
// them, the block scans the counts (wave64 shuffles + LDS), publishes its
// aggregate, and its first wavefront looks back over a window of 64
// predecessors per round trip (one device-scope load per lane, a ballot for
// the nearest inclusive prefix, a wave reduction of the aggregates before
// it), then publishes its inclusive prefix and the block scatters.  HBM
// traffic: 1 byte per entry read, 4 bytes per kept entry written.
//
// Status words (64 bit): bits 62-63 = 0 (not ready), 1 (aggregate), 2
// (inclusive prefix); bits 0-61 the value.  A tiny first kernel clears the
// status words and the ticket, so the pair can be recorded in a graph.
#include <atomic>
#include <mutex>

#include "hf_device.hpp"
#include "hf_internal.hpp"

namespace hf {
namespace {

constexpr int kCB = 512;
constexpr int kCPT = 16;
constexpr int kTile = kCB * kCPT;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr size_t kHeader = 256;  // ticket lives in the first 256 bytes

__global__ void k_compact_init(uint64_t *status, int64_t n_tiles, uint32_t *ticket) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *ticket = 0;
    for (int64_t t = i; t < n_tiles; t += (int64_t)gridDim.x * blockDim.x) status[t] = 0;
}

__device__ __forceinline__ uint64_t load_status(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_status(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kCB) void k_compact(const uint8_t *__restrict__ mask, int64_t capacity,
                                                 const int64_t *__restrict__ d_n, int64_t index_base,
                                                 const int32_t *__restrict__ map, int32_t *__restrict__ idx,
                                                 int64_t *__restrict__ count, uint64_t *status, uint32_t *ticket,
                                                 int64_t n_tiles, int aligned) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wsum[kCB / kWave];
    __shared__ uint64_t s_prefix;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    int64_t n = capacity;
    if (d_n) {
        const int64_t dn = *d_n;
        n = dn < 0 ? 0 : (dn < capacity ? dn : capacity);
    }
    const int64_t first = tile * kTile + (int64_t)tid * kCPT;

    // ---- load 16 flags
    uint32_t bits = 0;
    if (aligned && first + kCPT <= n) {
        const uint4 v = *reinterpret_cast<const uint4 *>(mask + first);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b) bits |= (((w[q] >> (8 * b)) & 0xffu) ? 1u : 0u) << (4 * q + b);
    } else {
#pragma unroll
        for (int j = 0; j < kCPT; ++j)
            if (first + j < n && mask[first + j]) bits |= 1u << j;
    }
    const uint32_t cnt = (uint32_t)__popc(bits);

    // ---- block exclusive scan of the per-thread counts
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) s_wsum[wave] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kCB / kWave; ++w) {
        if (w < wave) wbase += s_wsum[w];
        total += s_wsum[w];
    }
    const uint32_t excl_thread = wbase + incl - cnt;

    // ---- publish aggregate, look back (first wavefront), publish inclusive prefix
    if (wave == 0) {
        uint64_t prefix = 0;
        if (tile == 0) {
            if (lane == 0) store_status(&status[0], kFlagInc | (uint64_t)total);
        } else {
            if (lane == 0) store_status(&status[tile], kFlagAgg | (uint64_t)total);
            int64_t top = tile - 1;  // newest predecessor of the current window
            while (true) {
                const int64_t j = top - lane;
                const uint64_t st = j >= 0 ? load_status(&status[j]) : kFlagInc;  // before tile 0: prefix 0
                const uint64_t flag = st & ~kValMask;
                const uint64_t inc = ballot(flag == kFlagInc);
                const uint64_t ready = ballot(flag != 0);
                // lanes up to and including the nearest inclusive prefix must all be ready
                const int first = inc ? __ffsll((unsigned long long)inc) - 1 : kWave - 1;
                const uint64_t need = first == kWave - 1 ? ~0ull : ((2ull << first) - 1);
                if ((ready & need) != need) continue;  // a predecessor is still counting
                uint64_t v = (lane <= first && j >= 0) ? (st & kValMask) : 0;
                for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
                prefix += v;
                if (inc) break;
                top -= kWave;
            }
            if (lane == 0) store_status(&status[tile], kFlagInc | (prefix + total));
        }
        if (lane == 0) {
            s_prefix = prefix;
            if (tile == n_tiles - 1) *count = (int64_t)(prefix + total);
        }
    }
    __syncthreads();

    // ---- scatter
    int64_t out = (int64_t)s_prefix + excl_thread;
    while (bits) {
        const int j = __ffs(bits) - 1;
        bits &= bits - 1;
        const int64_t e = first + j;
        idx[out++] = map ? map[e] : (int32_t)(index_base + e);
    }
}

}  // namespace

static int64_t n_tiles_for(int64_t capacity) {
    const int64_t t = (capacity + kTile - 1) / kTile;
    return t < 1 ? 1 : t;
}

size_t compact_ws_bytes(int64_t capacity) { return kHeader + (size_t)n_tiles_for(capacity) * sizeof(uint64_t); }

hipError_t launch_compact(const uint8_t *mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                          const int32_t *map, int32_t *idx, int64_t *count, void *ws, hipStream_t s) {
    const int64_t nt = n_tiles_for(capacity);
    uint32_t *ticket = static_cast<uint32_t *>(ws);
    uint64_t *status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kHeader);
    int init_grid = (int)((nt + 255) / 256);
    if (init_grid > 1024) init_grid = 1024;
    hipLaunchKernelGGL(k_compact_init, dim3(init_grid), dim3(256), 0, s, status, nt, ticket);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int aligned = (reinterpret_cast<uintptr_t>(mask) % 16) == 0;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nt), dim3(kCB), 0, s, mask, capacity, d_n, index_base, map, idx,
                       count, status, ticket, nt, aligned);
    return hipGetLastError();
}

// ---- workspace held by the library (hf_compact_noalloc)
//
// Ticket and status words of up to HF_COMPACT_NOALLOC_MAX_ENTRIES mask
// entries, one copy per device for the life of the process.  On the host the
// name `scratch` is only a stand-in for the symbol: its device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes =
    kHeader + (size_t)((HF_COMPACT_NOALLOC_MAX_ENTRIES + kTile - 1) / kTile) * sizeof(uint64_t);

}  // namespace hf

static __device__ __align__(256) uint8_t scratch[hf::kStaticScratchBytes];

namespace hf {
namespace {
constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

hipError_t compact_static_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            if (!p) return hipErrorInvalidSymbol;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

hipError_t launch_compact_noalloc(const uint8_t *mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                                  const int32_t *map, int32_t *idx, int64_t *count, hipStream_t s) {
    if (compact_ws_bytes(capacity) > kStaticScratchBytes) return hipErrorInvalidValue;
    void *ws = nullptr;
    hipError_t e = compact_static_scratch(&ws);
    if (e != hipSuccess) return e;
    // the first kernel of launch_compact clears the ticket and the status words
    return launch_compact(mask, capacity, d_n, index_base, map, idx, count, ws, s);
}

}  // namespace hf
