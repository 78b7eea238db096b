// Single-neutrino chi^2 reconstruction of one-lepton events (paper section
// 6.2, Eq. (chi2)).  The missing transverse momentum is the neutrino's
// transverse momentum; its p_z follows from the W mass (two roots of a
// quadratic, or the real part of a complex pair); the assignment of the
// selected jets to the expected top quarks and W bosons that minimises
//   chi^2 = sum_k (m_top_k - m_t)^2 / sigma_t^2 + sum_m (m_W_m - m_W)^2 / sigma_W^2
// is kept.  Topologies: t-channel (top = j l nu, W = l nu), Wt (adds the
// two-jet W p q) and semileptonic ttbar (adds the hadronic top h p q).
//
// One thread per compacted event, everything in FP64 (the inputs are FP32
// columns; converting them and the few masses per assignment costs little
// next to reading them).
//
// t-channel streams through the event's jets: each selected jet is
// converted and scored against both neutrino roots as it is read, so
// nothing is kept per jet.
//
// Wt and semileptonic ttbar keep the candidates' FP64 4-vectors in LDS
// (structure of arrays over the block's threads) and split chi^2 into the
// leptonic part A(j, r) = chi_t(j l nu_r) + chi_W(l nu_r), minimised over the
// roots per jet first, and the hadronic part that depends on (h, p, q) only.
// Each two-jet W and three-jet top is then built once, not once per
// leptonic jet and root; the sums are formed in the same order as the
// plain definition (leptonic top, leptonic W, hadronic W, hadronic top).
// Ties go to the first assignment in the order (root, j, h, p, q).
#include <math.h>

#include "hf_device.hpp"
#include "hf_internal.hpp"

namespace hf {
namespace {

constexpr int kMaxC = HF_MAX_CANDS;
constexpr int kTchanBlock = 256;
constexpr int kComboBlock = 64;  // threads per block of the combinatorial kernels (LDS per thread)

__device__ __forceinline__ int64_t clamp_count(const int64_t *count, int64_t capacity) {
    const int64_t S = *count;
    return S < 0 ? 0 : (S > capacity ? capacity : S);
}

// Azimuths are in [-pi, pi]: sincospi of phi / pi needs no wide argument
// reduction (sincos's large-argument path would cost a scratch buffer).
__device__ __forceinline__ void to_cart(float pt, float eta, float phi, float e, double v[4]) {
    double s, c;
    sincospi((double)phi * 0.31830988618379067, &s, &c);
    v[0] = (double)e;
    v[1] = (double)pt * c;
    v[2] = (double)pt * s;
    v[3] = (double)pt * sinh((double)eta);
}

__device__ __forceinline__ double mass4(double e, double x, double y, double z) {
    const double m2 = e * e - x * x - y * y - z * z;
    return m2 > 0.0 ? sqrt(m2) : 0.0;
}

__device__ __forceinline__ double sq(double x) { return x * x; }

// Lexicographic (chi^2, key): the smaller wins.
__device__ __forceinline__ bool better(double c, uint32_t key, double bc, uint32_t bkey) {
    return c < bc || (c == bc && key < bkey);
}

// Leading selected lepton of event e (pT > min, |eta| < max); -1 if none.
__device__ __forceinline__ int64_t leading_lepton(const EvView &ev, int64_t e, const SemilepArgs &a) {
    const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
    for (uint32_t c0 = l0; c0 < l1; c0 += 4) {
        float pt[4], eta[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = c0 + u < l1;
            pt[u] = in ? ev.lep_pt[c0 + u] : 0.0f;
            eta[u] = in ? ev.lep_eta[c0 + u] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u < l1 && pt[u] > a.lep_pt_min && fabsf(eta[u]) < a.lep_eta_max) return c0 + u;
    }
    return -1;
}

// Candidate jets of event e: the selected ones in input order, at most
// max_cands; their absolute positions go to the calling thread's LDS list
// jl[c * stride] (an LDS list rather than a register array, which dynamic
// indexing would send to scratch).  pT and eta are read four jets at a time.
__device__ __forceinline__ int select_jets(const EvView &ev, int64_t e, const SemilepArgs &a, uint32_t *jl,
                                           int stride) {
    const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
    int nc = 0;
    for (uint32_t c0 = j0; c0 < j1 && nc < a.max_cands; c0 += 4) {
        float pt[4], eta[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = c0 + u < j1;
            pt[u] = in ? ev.jet_pt[c0 + u] : 0.0f;
            eta[u] = in ? ev.jet_eta[c0 + u] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u < j1 && nc < a.max_cands && pt[u] > a.jet_pt_min && fabsf(eta[u]) < a.jet_eta_max)
                jl[(nc++) * stride] = c0 + u;
    }
    return nc;
}

// The event's lepton, neutrino p_z candidates (W mass, section 6.2) and the
// leptonic W per candidate.  Returns the candidate count (0: no lepton).
struct Leptonic {
    double w[2][4];  // l + nu_r
    double pz[2];
    double cw[2];    // (m(l nu_r) - m_W)^2 / sigma_W^2
    double mw[2];
    int kind[2];     // 0/1 minus/plus root, 2 real part
    int nr;
};

// Entry r of a two-entry array by selection, keeping the array in registers.
template <typename T>
__device__ __forceinline__ T at2(const T (&x)[2], int r) {
    return r ? x[1] : x[0];
}

__device__ __forceinline__ Leptonic leptonic(const EvView &ev, int64_t e, int64_t kl, const SemilepArgs &a) {
    Leptonic L;
    L.nr = 0;
    double l[4];
    to_cart(ev.lep_pt[kl], ev.lep_eta[kl], ev.lep_phi[kl], ev.lep_e[kl], l);
    const double mx = (double)ev.met_x[e], my = (double)ev.met_y[e];
    // E_l sqrt(pT^2 + pz^2) = mu + pz_l pz  ->  a pz^2 - 2 mu pz_l pz + (E_l^2 pT^2 - mu^2) = 0
    const double ml2 = l[0] * l[0] - l[1] * l[1] - l[2] * l[2] - l[3] * l[3];
    const double qa = l[0] * l[0] - l[3] * l[3];
    if (!(qa > 0.0)) return L;
    const double pt2 = mx * mx + my * my;
    const double mu = 0.5 * (a.m_w * a.m_w - ml2) + l[1] * mx + l[2] * my;
    const double d = mu * mu - qa * pt2;
    if (d < 0.0) {
        L.pz[0] = mu * l[3] / qa;
        L.kind[0] = 2;
        L.nr = 1;
    } else {
        const double s = l[0] * sqrt(d);
        L.pz[0] = (mu * l[3] - s) / qa;
        L.pz[1] = (mu * l[3] + s) / qa;
        L.kind[0] = 0;
        L.kind[1] = 1;
        L.nr = 2;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (r >= L.nr) break;
        const double pz = L.pz[r];
        const double en = sqrt(pt2 + pz * pz);
        L.w[r][0] = l[0] + en;
        L.w[r][1] = l[1] + mx;
        L.w[r][2] = l[2] + my;
        L.w[r][3] = l[3] + pz;
        L.mw[r] = mass4(L.w[r][0], L.w[r][1], L.w[r][2], L.w[r][3]);
        L.cw[r] = sq(L.mw[r] - a.m_w) * a.inv_sw2;
    }
    return L;
}

__device__ __forceinline__ void write_none(const SemilepOutView &o, int64_t k) {
    o.has_sol[k] = 0;
    o.root[k] = -1;
    o.best_j[k] = o.best_h[k] = o.best_p[k] = o.best_q[k] = -1;
    for (int q = 0; q < 3; ++q) o.nu[3 * k + q] = HF_NO_SOLUTION;
    o.m_tl[k] = o.m_wl[k] = o.m_th[k] = o.m_wh[k] = o.chi2[k] = HF_NO_SOLUTION;
}

// RECO counters: passed += events with a solution (one atomic per block),
// reached += S (block 0).
template <int kBlock>
__device__ __forceinline__ void fold_counters(bool have, int64_t S, hf_counters_t *counter) {
    __shared__ uint32_t s_pass[kBlock / kWave];
    const uint64_t m = ballot(have);
    if (lane_id() == 0) s_pass[threadIdx.x / kWave] = (uint32_t)popc64(m);
    __syncthreads();
    if (threadIdx.x == 0 && counter) {
        uint64_t tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) tot += s_pass[w];
        if (tot) atomicAdd((unsigned long long *)&counter->passed, (unsigned long long)tot);
        if (blockIdx.x == 0) atomicAdd((unsigned long long *)&counter->reached, (unsigned long long)S);
    }
}

// ---------------------------------------------------------------- t-channel
__global__ __launch_bounds__(kTchanBlock) void k_semilep_tchan(EvView ev, const int32_t *__restrict__ idx,
                                                               const int64_t *__restrict__ count, int64_t capacity,
                                                               SemilepArgs a, SemilepOutView o,
                                                               hf_counters_t *__restrict__ counter) {
    __shared__ uint32_t s_jl[kMaxC * kTchanBlock];
    const int64_t S = clamp_count(count, capacity);
    const int64_t k = (int64_t)blockIdx.x * kTchanBlock + threadIdx.x;
    bool have = false;
    if (k < S) {
        const int64_t e = (int64_t)idx[k] - ev.index_base;
        const int64_t kl = (e >= 0 && e < ev.n) ? leading_lepton(ev, e, a) : -1;
        if (kl >= 0) {
            const Leptonic L = leptonic(ev, e, kl, a);
            uint32_t *jl = s_jl + threadIdx.x;
            const int nc = L.nr > 0 ? select_jets(ev, e, a, jl, kTchanBlock) : 0;
            const uint32_t j0 = ev.jet_off[e];
            double best = 0.0, bmt = 0.0;
            uint32_t bkey = 0xffffffffu;
            int bj = -1, br = 0;
            // one jet per iteration; the next jet's columns are loaded before
            // this one is converted and scored
            uint32_t q = nc > 0 ? jl[0] : j0;
            float pt = nc > 0 ? ev.jet_pt[q] : 0.0f, eta = nc > 0 ? ev.jet_eta[q] : 0.0f;
            float phi = nc > 0 ? ev.jet_phi[q] : 0.0f, en = nc > 0 ? ev.jet_e[q] : 0.0f;
            for (int c = 0; c < nc; ++c) {
                const bool more = c + 1 < nc;
                const uint32_t qn = more ? jl[(c + 1) * kTchanBlock] : q;
                const float npt = more ? ev.jet_pt[qn] : 0.0f, neta = more ? ev.jet_eta[qn] : 0.0f;
                const float nphi = more ? ev.jet_phi[qn] : 0.0f, nen = more ? ev.jet_e[qn] : 0.0f;
                double v[4];
                to_cart(pt, eta, phi, en, v);
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (r >= L.nr) break;
                    const double mt = mass4(L.w[r][0] + v[0], L.w[r][1] + v[1], L.w[r][2] + v[2], L.w[r][3] + v[3]);
                    const double chi = sq(mt - a.m_t) * a.inv_st2 + L.cw[r];
                    const uint32_t key = (uint32_t)(r * 64 + c);
                    if (bj < 0 || better(chi, key, best, bkey)) {
                        best = chi;
                        bkey = key;
                        bj = (int)(q - j0);
                        br = r;
                        bmt = mt;
                    }
                }
                q = qn;
                pt = npt;
                eta = neta;
                phi = nphi;
                en = nen;
            }
            if (bj >= 0) {
                have = true;
                o.has_sol[k] = 1;
                o.root[k] = (int8_t)at2(L.kind, br);
                o.best_j[k] = (int16_t)bj;
                o.best_h[k] = o.best_p[k] = o.best_q[k] = -1;
                o.nu[3 * k + 0] = (double)ev.met_x[e];
                o.nu[3 * k + 1] = (double)ev.met_y[e];
                o.nu[3 * k + 2] = at2(L.pz, br);
                o.m_tl[k] = bmt;
                o.m_wl[k] = at2(L.mw, br);
                o.m_th[k] = o.m_wh[k] = HF_NO_SOLUTION;
                o.chi2[k] = best;
            }
        }
        if (!have) write_none(o, k);
    }
    fold_counters<kTchanBlock>(have, S, counter);
}

// ------------------------------------------------ Wt and semileptonic ttbar
// Candidate 4-vectors in LDS, s_v[(c * 4 + q) * kComboBlock + thread].
template <bool kTT>
__global__ __launch_bounds__(kComboBlock) void k_semilep_combo(EvView ev, const int32_t *__restrict__ idx,
                                                               const int64_t *__restrict__ count, int64_t capacity,
                                                               SemilepArgs a, SemilepOutView o,
                                                               hf_counters_t *__restrict__ counter) {
    __shared__ double s_v[kMaxC * 4 * kComboBlock];
    __shared__ uint16_t s_loc[kMaxC * kComboBlock];
    __shared__ uint32_t s_jl[kMaxC * kComboBlock];
    const int t = threadIdx.x;
    auto V = [&](int c, int q) -> double & { return s_v[(c * 4 + q) * kComboBlock + t]; };
    const int64_t S = clamp_count(count, capacity);
    const int64_t k = (int64_t)blockIdx.x * kComboBlock + t;
    const int need = kTT ? 4 : 3;
    bool have = false;
    if (k < S) {
        const int64_t e = (int64_t)idx[k] - ev.index_base;
        const int64_t kl = (e >= 0 && e < ev.n) ? leading_lepton(ev, e, a) : -1;
        int nc = 0;
        if (kl >= 0) {
            uint32_t *jl = s_jl + t;
            nc = select_jets(ev, e, a, jl, kComboBlock);
            if (nc >= need) {
                const uint32_t j0 = ev.jet_off[e];
                for (int c = 0; c < nc; ++c) {
                    const uint32_t q = jl[c * kComboBlock];
                    double v[4];
                    to_cart(ev.jet_pt[q], ev.jet_eta[q], ev.jet_phi[q], ev.jet_e[q], v);
                    for (int u = 0; u < 4; ++u) V(c, u) = v[u];
                    s_loc[c * kComboBlock + t] = (uint16_t)(q - j0);
                }
            }
        }
        Leptonic L;
        L.nr = 0;
        if (kl >= 0 && nc >= need) L = leptonic(ev, e, kl, a);
        if (L.nr > 0) {
            // leptonic part per jet, minimised over the roots (ties: the first root)
            double A[kMaxC], MT[kMaxC];
            int R[kMaxC];
#pragma unroll
            for (int j = 0; j < kMaxC; ++j) {
                A[j] = INFINITY;
                MT[j] = 0.0;
                R[j] = 0;
                if (j < nc) {
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        if (r >= L.nr) break;
                        const double mt = mass4(L.w[r][0] + V(j, 0), L.w[r][1] + V(j, 1), L.w[r][2] + V(j, 2),
                                                L.w[r][3] + V(j, 3));
                        const double c = sq(mt - a.m_t) * a.inv_st2 + L.cw[r];
                        if (c < A[j]) {
                            A[j] = c;
                            MT[j] = mt;
                            R[j] = r;
                        }
                    }
                }
            }
            double best = INFINITY, bmth = HF_NO_SOLUTION, bmwh = 0.0;
            uint32_t bkey = 0xffffffffu;
            int bj = -1, bh = -1, bp = -1, bq = -1;
            for (int p = 0; p < nc; ++p)
                for (int q = p + 1; q < nc; ++q) {
                    double w[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) w[u] = V(p, u) + V(q, u);
                    const double mwh = mass4(w[0], w[1], w[2], w[3]);
                    const double cwh = sq(mwh - a.m_w) * a.inv_sw2;
                    const int nh = kTT ? nc : 1;
                    for (int hi = 0; hi < nh; ++hi) {
                        const int h = kTT ? hi : -1;
                        if (kTT && (h == p || h == q)) continue;
                        double cth = 0.0, mth = HF_NO_SOLUTION;
                        if (kTT) {
                            mth = mass4(w[0] + V(h, 0), w[1] + V(h, 1), w[2] + V(h, 2), w[3] + V(h, 3));
                            cth = sq(mth - a.m_t) * a.inv_st2;
                        }
                        const uint32_t hk = kTT ? (uint32_t)h : 0u;
#pragma unroll
                        for (int j = 0; j < kMaxC; ++j) {
                            if (j >= nc || j == p || j == q || j == h) continue;
                            double c = A[j] + cwh;
                            if (kTT) c += cth;
                            const uint32_t key = ((((uint32_t)R[j] * 16u + j) * 16u + hk) * 16u + p) * 16u + q;
                            if (better(c, key, best, bkey)) {
                                best = c;
                                bkey = key;
                                bj = j;
                                bh = h;
                                bp = p;
                                bq = q;
                                bmth = mth;
                                bmwh = mwh;
                            }
                        }
                    }
                }
            if (bj >= 0) {
                have = true;
                int r = 0;
                double mt = 0.0;
#pragma unroll
                for (int j = 0; j < kMaxC; ++j)
                    if (j == bj) {
                        r = R[j];
                        mt = MT[j];
                    }
                o.has_sol[k] = 1;
                o.root[k] = (int8_t)at2(L.kind, r);
                o.best_j[k] = (int16_t)s_loc[bj * kComboBlock + t];
                o.best_h[k] = (int16_t)(bh >= 0 ? s_loc[bh * kComboBlock + t] : -1);
                o.best_p[k] = (int16_t)s_loc[bp * kComboBlock + t];
                o.best_q[k] = (int16_t)s_loc[bq * kComboBlock + t];
                o.nu[3 * k + 0] = (double)ev.met_x[e];
                o.nu[3 * k + 1] = (double)ev.met_y[e];
                o.nu[3 * k + 2] = at2(L.pz, r);
                o.m_tl[k] = mt;
                o.m_wl[k] = at2(L.mw, r);
                o.m_th[k] = bmth;
                o.m_wh[k] = bmwh;
                o.chi2[k] = best;
            }
        }
        if (!have) write_none(o, k);
    }
    fold_counters<kComboBlock>(have, S, counter);
}

}  // namespace

hipError_t launch_semilep(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity,
                          const SemilepArgs &a, const SemilepOutView &out, hf_counters_t *counter, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    if (a.topology == HF_TOPO_TCHAN) {
        const int64_t nb = (capacity + kTchanBlock - 1) / kTchanBlock;
        hipLaunchKernelGGL(k_semilep_tchan, dim3((unsigned)nb), dim3(kTchanBlock), 0, s, ev, idx, count, capacity, a,
                           out, counter);
    } else {
        const int64_t nb = (capacity + kComboBlock - 1) / kComboBlock;
        if (a.topology == HF_TOPO_WT)
            hipLaunchKernelGGL(k_semilep_combo<false>, dim3((unsigned)nb), dim3(kComboBlock), 0, s, ev, idx, count,
                               capacity, a, out, counter);
        else
            hipLaunchKernelGGL(k_semilep_combo<true>, dim3((unsigned)nb), dim3(kComboBlock), 0, s, ev, idx, count,
                               capacity, a, out, counter);
    }
    return hipGetLastError();
}

}  // namespace hf
