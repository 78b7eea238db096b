// Device code of the cut chain (paper section 3: each cut is a boolean
// predicate of one event; section 5.2: per-cut filter ratios and costs drive
// the ordering), shared by the library's own chain kernel and by chains with
// user predicates compiled at run time.
//
// One lane per event, 64 events per wavefront, grid-stride over the chunk.
// Cuts run in the order held in device memory; a lane stops at its first
// failure and a wavefront skips the remaining cuts (and their column loads)
// once all 64 lanes have failed, which is how a good order saves HBM
// traffic.  Per-cut reached/passed counts come from wavefront ballots and the
// cost from the shader clock; each block reduces its waves in LDS and writes
// one partial row, which a second small kernel folds into the caller's
// counters (no atomics, deterministic).
//
// Derived quantities (MET^2, M_ll^2, Delta R^2, M_T^2) are formed in FP64
// from the float32 columns and compared without square roots where
// possible; thresholds are float32 values widened to FP64.  Every unit that
// includes this file compiles it with -ffp-contract=off.
#pragma once

#include "hf_device.hpp"
#include "hf_internal.hpp"

namespace hf {

constexpr int kSelBlock = 256;
constexpr int kSelWaves = kSelBlock / kWave;

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

__device__ inline bool eval_cut(const EvView &ev, int64_t e, const hf_cut_t &c) {
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
    case HF_CUT_JET_N_RANGE: {
        const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
        int n = 0;
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
                n += (c0 + u < j1 && pt[u] > c.f[0] && ae[u] >= c.f[1] && ae[u] < c.f[2]) ? 1 : 0;
        }
        return n >= c.i[0] && n <= c.i[1];
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

// The chain kernel.  User::eval(u, ev, e) evaluates user predicate u (cuts of
// kind HF_CUT_USER, u = the cut's i[0]); the library's own instantiation has
// none, a chain compiled at run time supplies them.
//
// A launch evaluates the cuts at positions [pos_begin, pos_end) of the order
// (a segment of the chain) over all events of the chunk (idx == nullptr;
// survive indexed by event) or over the compacted ids idx[0, min(*count,
// capacity)) (survive indexed by position; an id outside the chunk fails
// without being counted), so that the later cuts of a chain can run on the
// compacted survivors of the earlier ones.
template <class User>
__global__ __launch_bounds__(kSelBlock) void k_select_t(EvView ev, CutTable ct, const int32_t *__restrict__ order,
                                                        uint8_t *__restrict__ survive,
                                                        uint64_t *__restrict__ partial,
                                                        const int32_t *__restrict__ idx,
                                                        const int64_t *__restrict__ count, int64_t capacity,
                                                        int pos_begin, int pos_end) {
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

    int64_t n_items = ev.n;
    if (idx) {
        const int64_t S = *count;
        n_items = S < 0 ? 0 : (S > capacity ? capacity : S);
    }
    const int64_t stride = (int64_t)gridDim.x * kSelBlock;
    for (int64_t base = (int64_t)blockIdx.x * kSelBlock + wave * kWave; base < n_items; base += stride) {
        const int64_t item = base + lane;
        int64_t e = item;
        bool alive = item < n_items;
        if (idx && alive) {
            e = (int64_t)idx[item] - ev.index_base;
            alive = e >= 0 && e < ev.n;
        }
        for (int k = pos_begin; k < pos_end; ++k) {
            const int c = s_order[k];
            if (c < 0 || s_cut[c].kind == HF_CUT_RECO) continue;
            const uint64_t am = ballot(alive);
            if (am == 0) break;
            const uint64_t t0 = __builtin_amdgcn_s_memtime();
            bool pass = false;
            if (alive)
                pass = s_cut[c].kind == HF_CUT_USER ? User::eval(s_cut[c].i[0], ev, e, s_cut[c].i[1])
                                                    : eval_cut(ev, e, s_cut[c]);
            const uint64_t pm = ballot(pass);
            const uint64_t t1 = __builtin_amdgcn_s_memtime();
            if (lane == 0) {
                s_cnt[wave][3 * c + 0] += (uint64_t)popc64(am);
                s_cnt[wave][3 * c + 1] += (uint64_t)popc64(pm);
                s_cnt[wave][3 * c + 2] += t1 - t0;
            }
            alive = pass;
        }
        if (item < n_items) survive[item] = alive ? 1 : 0;
    }
    __syncthreads();
    for (int t = tid; t < nc * 3; t += kSelBlock) {
        uint64_t s = 0;
#pragma unroll
        for (int w = 0; w < kSelWaves; ++w) s += s_cnt[w][t];
        partial[(size_t)blockIdx.x * nc * 3 + t] = s;
    }
}

// Column accessor of user predicates: object i of the event's list, or 0
// when i is outside it (a predicate cannot read past its event).
__device__ __forceinline__ float user_col(const float *col, uint32_t base, uint32_t n, int i) {
    return (unsigned)i < n ? col[base + (unsigned)i] : 0.0f;
}

// No user predicates (the library's own chain kernel).
struct NoUserCuts {
    __device__ static bool eval(int, const EvView &, int64_t, int32_t) { return true; }
};

}  // namespace hf
