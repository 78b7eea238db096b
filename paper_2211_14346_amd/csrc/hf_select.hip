// Cut chain over structure-of-arrays events (paper section 3: each cut is a
// boolean predicate of one event; section 5.2: per-cut filter ratios and
// costs drive the ordering).
//
// One lane per event, 64 events per wavefront, grid-stride over the chunk.
// Cuts run in the order held in device memory; a lane stops at its first
// failure and a wavefront skips the remaining cuts (and their column loads)
// once all 64 lanes have failed, which is how a good order saves HBM
// traffic.  Per-cut reached/passed counts come from wavefront ballots and the
// cost from the shader clock; each block reduces its waves in LDS and writes
// one partial row, and a second small kernel folds the partial rows into the
// caller's counters (no atomics, deterministic).
//
// Derived quantities (MET^2, M_ll^2, Delta R^2) are formed in FP64 from the
// float32 columns and compared without square roots; thresholds are float32
// values widened to FP64.  This file is compiled with -ffp-contract=off.
#include <math.h>

#include "hf_device.hpp"
#include "hf_internal.hpp"

namespace hf {
namespace {

constexpr int kSelBlock = 256;
constexpr int kSelWaves = kSelBlock / kWave;
constexpr int kSelMaxGrid = 2048;

__device__ __forceinline__ bool lep_ok(const EvView &ev, uint32_t k, float ptmin, float etamax) {
    return ev.lep_pt[k] > ptmin && fabsf(ev.lep_eta[k]) < etamax;
}

__device__ __forceinline__ bool jet_ok(const EvView &ev, uint32_t k, float ptmin, float etamax) {
    return ev.jet_pt[k] > ptmin && fabsf(ev.jet_eta[k]) < etamax;
}

__device__ __forceinline__ double fold_dphi(double d) {
    while (d > M_PI) d -= 2.0 * M_PI;
    while (d < -M_PI) d += 2.0 * M_PI;
    return d;
}

// Objects are visited in chunks of kChunk whose columns are loaded together
// (predicated loads, issued back to back), so that a chunk costs one memory
// round trip rather than one per object; the predicates and sums are then
// evaluated in object order exactly as a plain loop would.
constexpr int kChunk = 4;

__device__ bool eval_cut(const EvView &ev, int64_t e, const hf_cut_t &c) {
    switch (c.kind) {
    case HF_CUT_LEP_N_OS: {
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        int n = 0;
        float qprod = 1.0f;
        for (uint32_t c0 = l0; c0 < l1; c0 += kChunk) {
            float pt[kChunk], eta[kChunk], q[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const bool in = c0 + u < l1;
                pt[u] = in ? ev.lep_pt[c0 + u] : 0.0f;
                eta[u] = in ? ev.lep_eta[c0 + u] : 0.0f;
                q[u] = in ? ev.lep_q[c0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (c0 + u < l1 && pt[u] > c.f[0] && fabsf(eta[u]) < c.f[1]) {
                    ++n;
                    qprod *= q[u];
                }
        }
        if (n != c.i[0]) return false;
        if (c.i[1] && n == 2 && !(qprod < 0.0f)) return false;
        return true;
    }
    case HF_CUT_JET_N_MIN:
    case HF_CUT_BTAG_N_MIN:
    case HF_CUT_BTAG_N_EQ: {
        const bool tag = c.kind != HF_CUT_JET_N_MIN;
        const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
        int n = 0;
        for (uint32_t c0 = j0; c0 < j1; c0 += kChunk) {
            float pt[kChunk], eta[kChunk], bt[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const bool in = c0 + u < j1;
                pt[u] = in ? ev.jet_pt[c0 + u] : 0.0f;
                eta[u] = in ? ev.jet_eta[c0 + u] : 0.0f;
                bt[u] = (in && tag) ? ev.jet_btag[c0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                n += (c0 + u < j1 && pt[u] > c.f[0] && fabsf(eta[u]) < c.f[1] && (!tag || bt[u] > c.f[2])) ? 1 : 0;
        }
        return c.kind == HF_CUT_BTAG_N_EQ ? n == c.i[0] : n >= c.i[0];
    }
    case HF_CUT_MET_MIN: {
        const double mx = ev.met_x[e], my = ev.met_y[e], t = c.f[0];
        return mx * mx + my * my > t * t;
    }
    case HF_CUT_MLL_MIN: {
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        double E = 0, px = 0, py = 0, pz = 0;
        int n = 0;
        for (uint32_t c0 = l0; c0 < l1 && n < 2; c0 += kChunk) {
            float pt[kChunk], eta[kChunk], phi[kChunk], en[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const bool in = c0 + u < l1;
                pt[u] = in ? ev.lep_pt[c0 + u] : 0.0f;
                eta[u] = in ? ev.lep_eta[c0 + u] : 0.0f;
                phi[u] = in ? ev.lep_phi[c0 + u] : 0.0f;
                en[u] = in ? ev.lep_e[c0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (n < 2 && c0 + u < l1 && pt[u] > c.f[0] && fabsf(eta[u]) < c.f[1]) {
                    const double dpt = pt[u];
                    E += en[u];
                    px += dpt * cos((double)phi[u]);
                    py += dpt * sin((double)phi[u]);
                    pz += dpt * sinh((double)eta[u]);
                    ++n;
                }
        }
        if (n < 2) return false;
        const double m2 = E * E - px * px - py * py - pz * pz;
        const double t = c.f[2];
        return m2 > 0.0 && m2 > t * t;
    }
    case HF_CUT_FWD_JET_VETO: {
        const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
        for (uint32_t c0 = j0; c0 < j1; c0 += kChunk) {
            float pt[kChunk], ae[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const bool in = c0 + u < j1;
                pt[u] = in ? ev.jet_pt[c0 + u] : 0.0f;
                ae[u] = in ? fabsf(ev.jet_eta[c0 + u]) : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (c0 + u < j1 && pt[u] > c.f[0] && ae[u] >= c.f[1] && ae[u] < c.f[2]) return false;
        }
        return true;
    }
    case HF_CUT_LEP_ISO: {
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
        const double dr = c.f[4];
        const double dr2 = dr * dr;
        for (uint32_t a = l0; a < l1; ++a) {
            if (!lep_ok(ev, a, c.f[0], c.f[1])) continue;
            const double leta = ev.lep_eta[a], lphi = ev.lep_phi[a];
            for (uint32_t c0 = j0; c0 < j1; c0 += kChunk) {
                float pt[kChunk], eta[kChunk], phi[kChunk];
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const bool in = c0 + u < j1;
                    pt[u] = in ? ev.jet_pt[c0 + u] : 0.0f;
                    eta[u] = in ? ev.jet_eta[c0 + u] : 0.0f;
                    phi[u] = in ? ev.jet_phi[c0 + u] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    if (!(c0 + u < j1 && pt[u] > c.f[2] && fabsf(eta[u]) < c.f[3])) continue;
                    const double deta = leta - (double)eta[u];
                    const double dphi = fold_dphi(lphi - (double)phi[u]);
                    if (deta * deta + dphi * dphi < dr2) return false;
                }
            }
        }
        return true;
    }
    case HF_CUT_MTW_MIN: {
        // leading selected lepton; M_T^2 = 2 (pT_l MET - pT_l . MET)
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        for (uint32_t c0 = l0; c0 < l1; c0 += kChunk) {
            float pt[kChunk], eta[kChunk], phi[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const bool in = c0 + u < l1;
                pt[u] = in ? ev.lep_pt[c0 + u] : 0.0f;
                eta[u] = in ? ev.lep_eta[c0 + u] : 0.0f;
                phi[u] = in ? ev.lep_phi[c0 + u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (c0 + u < l1 && pt[u] > c.f[0] && fabsf(eta[u]) < c.f[1]) {
                    const double dpt = pt[u];
                    const double px = dpt * cos((double)phi[u]), py = dpt * sin((double)phi[u]);
                    const double mx = ev.met_x[e], my = ev.met_y[e];
                    const double met = sqrt(mx * mx + my * my);
                    const double mt2 = 2.0 * (dpt * met - (px * mx + py * my));
                    const double t = c.f[2];
                    return mt2 > t * t;
                }
        }
        return false;
    }
    default:
        return true;
    }
}

__global__ __launch_bounds__(kSelBlock) void k_select(EvView ev, CutTable ct, const int32_t *__restrict__ order,
                                                      uint8_t *__restrict__ survive,
                                                      uint64_t *__restrict__ partial) {
    __shared__ hf_cut_t s_cut[HF_MAX_CUTS];
    __shared__ int s_order[HF_MAX_CUTS];
    __shared__ uint64_t s_cnt[kSelWaves][HF_MAX_CUTS * 3];
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int nc = ct.n;
    if (tid < nc) {
        const int o = order[tid];
        s_order[tid] = (o >= 0 && o < nc) ? o : -1;
        s_cut[tid] = ct.c[tid];
    }
    for (int t = tid; t < kSelWaves * HF_MAX_CUTS * 3; t += kSelBlock) (&s_cnt[0][0])[t] = 0;
    __syncthreads();

    const int64_t stride = (int64_t)gridDim.x * kSelBlock;
    for (int64_t base = (int64_t)blockIdx.x * kSelBlock + wave * kWave; base < ev.n; base += stride) {
        const int64_t e = base + lane;
        bool alive = e < ev.n;
        for (int k = 0; k < nc; ++k) {
            const int c = s_order[k];
            if (c < 0 || s_cut[c].kind == HF_CUT_RECO) continue;
            const uint64_t am = ballot(alive);
            if (am == 0) break;
            const uint64_t t0 = __builtin_amdgcn_s_memtime();
            bool pass = false;
            if (alive) pass = eval_cut(ev, e, s_cut[c]);
            const uint64_t pm = ballot(pass);
            const uint64_t t1 = __builtin_amdgcn_s_memtime();
            if (lane == 0) {
                s_cnt[wave][3 * c + 0] += (uint64_t)popc64(am);
                s_cnt[wave][3 * c + 1] += (uint64_t)popc64(pm);
                s_cnt[wave][3 * c + 2] += t1 - t0;
            }
            alive = pass;
        }
        if (e < ev.n) survive[e] = alive ? 1 : 0;
    }
    __syncthreads();
    for (int t = tid; t < nc * 3; t += kSelBlock) {
        uint64_t s = 0;
#pragma unroll
        for (int w = 0; w < kSelWaves; ++w) s += s_cnt[w][t];
        partial[(size_t)blockIdx.x * nc * 3 + t] = s;
    }
}

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
    hipLaunchKernelGGL(k_select, dim3(grid), dim3(kSelBlock), 0, s, ev, ct, order, survive, partial);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_select_reduce, dim3(ct.n * 3), dim3(256), 0, s, partial, grid, ct.n * 3,
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
