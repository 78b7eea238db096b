// Dileptonic chi^2 fit with a split of the missing transverse momentum
// (paper section 6.2): the two neutrinos share E_T^miss, each neutrino's p_z
// follows from its W mass, and Eq. (chi2) with two tops (b l+ nu, bbar l-
// nubar) and two W is minimised over the split, the ordered b-candidate
// pairings and the p_z roots.  For Wt events (one top, two W) each
// candidate forms the top with either lepton and the other W stands alone.
//
// The split is an offset (u, v) from the even split, nu_T = MET/2 + (u, v),
// nubar_T = MET/2 - (u, v), searched on an n_grid x n_grid grid over
// [-half_range, half_range]^2 and refined n_refine times on a 5 x 5 grid
// around the best point at a quarter of the previous step.
//
// A block of four wavefronts takes four compacted events, one per
// wavefront, lanes over grid points.  A lead wavefront stages all four
// (sixteen lanes per event: the objects' columns loaded at once, ballots for
// the selection and the candidate order, each object the fit uses converted
// on the lane holding it) and forms the split-independent lepton terms,
// keeping FP64 4-vectors in LDS; after a barrier every wavefront scans its
// own event's grid; after another the lead wavefront writes the four events'
// outputs, two lanes per event.  Staging and outputs touch a few lanes per
// event, so sharing one wavefront between four events cuts their issued
// instructions fourfold.  At a grid point chi^2 separates: the l+ side
// depends on (i, r1) only and the l- side on (j, r2) only, so a lane forms
// A+(i) = min over r1 of chi_t + chi_W for every candidate i, A-(j) likewise,
// and the best ordered pairing i != j from the smallest two A- values, at
// O(candidates) rather than O(candidates^2) per point.  A butterfly argmin
// (value, then point index) gives the level's best; a refined point replaces
// the best only when strictly smaller, as in a sequential scan.  FP64
// throughout.
#include <math.h>

#include "hf_chi2.hpp"
#include "hf_device.hpp"
#include "hf_internal.hpp"
#include "hf_reco_math.hpp"

namespace hf {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxC = HF_MAX_CANDS;
constexpr int kRefPts = 25;  // points of a refinement level (5 x 5)
constexpr int kSeg = kWave / kWaves;  // staging lanes per event

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int64_t clamp_count(const int64_t *count, int64_t capacity) {
    const int64_t S = *count;
    return S < 0 ? 0 : (S > capacity ? capacity : S);
}

__device__ __forceinline__ void to_cart(float pt, float eta, float phi, float e, double v[4]) {
    double s, c;
    sincospi((double)phi * 0.31830988618379067, &s, &c);  // |phi| <= pi: no wide reduction
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

// sqrt(v) for v >= kTiny to about 2^-46 relative: the hardware reciprocal
// square root (good to about 2^-23) and one Goldschmidt step, without the
// final correction to the last ulp.  Used for the p_z roots and the chi^2
// terms of every grid point, where the fit is issue-bound; the winner's
// outputs are recomputed with the library square root.  Callers clamp the
// argument to kTiny instead of testing for zero (one max instead of a compare
// and two selects): sqrt(kTiny) = 1e-150 stands for 0, a difference far
// below FP64 rounding of any chi^2 term at GeV scales.
constexpr double kTiny = 1e-300;
__device__ __forceinline__ double sqrt_fit(double v) {
    const double y = __builtin_amdgcn_rsq(v);
    const double s = v * y, h = 0.5 * y;
    return fma(s, fma(-s, h, 0.5), s);
}

// A lepton's split-independent terms: its 4-vector, (m_W^2 - m_l^2) / 2 and
// a = E^2 - p_z^2 with its reciprocal (the p_z quadratic's leading term).
struct Lep {
    double l[4];
    double c0, qa, inv_qa, inv_e;
};

__device__ __forceinline__ Lep make_lep(const double *l, const Chi2Args &a) {
    Lep L;
    for (int c = 0; c < 4; ++c) L.l[c] = l[c];
    const double ml2 = l[0] * l[0] - l[1] * l[1] - l[2] * l[2] - l[3] * l[3];
    L.c0 = 0.5 * (a.m_w * a.m_w - ml2);
    L.qa = l[0] * l[0] - l[3] * l[3];
    L.inv_qa = L.qa > 0.0 ? 1.0 / L.qa : 0.0;
    L.inv_e = l[0] > 0.0 ? 1.0 / l[0] : 0.0;
    return L;
}

// One lepton side at one split point: the neutrino p_z candidates from the
// W mass (both roots of the squared condition, or the real part), l + nu
// and the W term of chi^2 per candidate.  With h = mu + p_zl p_z the W
// condition reads E_l E_nu = h: a real root with h >= 0 solves it unsquared,
// so E_nu = h / E_l and l + nu lies on the W mass shell (W term zero); the
// squaring's extra root and the real part of a complex pair take E_nu from
// the mass shell and get their W term computed.  Both real roots have the
// sign of mu (|p_zl| sqrt(d) < E_l |mu|), so neighbouring split points --
// the lanes of a wave -- mostly agree, and the square roots of the other
// case are skipped for a wave where no lane needs them.  Square roots use
// the hardware estimate with one refinement (sqrt_fit); the quadratic's
// division is exact.
struct Side {
    double w[2][4];
    double pz[2];
    double cw[2];
    int kind[2];
    int n;
};

__device__ __forceinline__ Side side(const Lep &L, double nx, double ny, const Chi2Args &a) {
    Side S;
    S.n = 0;
    if (!(L.qa > 0.0)) return S;
    const double *l = L.l;
    const double pt2 = nx * nx + ny * ny;
    const double mu = L.c0 + l[1] * nx + l[2] * ny;
    const double d = mu * mu - L.qa * pt2;
    const double ml3 = mu * l[3];
    bool shell[2] = {false, false};
    if (d < 0.0) {
        S.pz[0] = ml3 * L.inv_qa;
        S.kind[0] = 2;
        S.n = 1;
    } else {
        const double s = l[0] * sqrt_fit(fmax(d, kTiny));
        S.pz[0] = (ml3 - s) * L.inv_qa;
        S.pz[1] = (ml3 + s) * L.inv_qa;
        S.kind[0] = 0;
        S.kind[1] = 1;
        S.n = 2;
        shell[0] = mu + l[3] * S.pz[0] >= 0.0;
        shell[1] = mu + l[3] * S.pz[1] >= 0.0;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (r >= S.n) break;
        double en = fma(l[3], S.pz[r], mu) * L.inv_e;
        S.cw[r] = 0.0;
        if (ballot(!shell[r])) {
            if (!shell[r]) en = sqrt_fit(fmax(pt2 + S.pz[r] * S.pz[r], kTiny));
        }
        S.w[r][0] = l[0] + en;
        S.w[r][1] = l[1] + nx;
        S.w[r][2] = l[2] + ny;
        S.w[r][3] = l[3] + S.pz[r];
        if (ballot(!shell[r])) {
            if (!shell[r])
                S.cw[r] = sq(sqrt_fit(fmax(S.w[r][0] * S.w[r][0] - S.w[r][1] * S.w[r][1] -
                                           S.w[r][2] * S.w[r][2] - S.w[r][3] * S.w[r][3], kTiny)) -
                             a.m_w) * a.inv_sw2;
        }
    }
    return S;
}

// top term of chi^2 for candidate b with l + nu = w
__device__ __forceinline__ double top_term(double b0, double b1, double b2, double b3, const double *w,
                                           const Chi2Args &a) {
    const double e = b0 + w[0], x = b1 + w[1], y = b2 + w[2], z = b3 + w[3];
    return sq(sqrt_fit(fmax(e * e - x * x - y * y - z * z, kTiny)) - a.m_t) * a.inv_st2;
}

template <typename T>
__device__ __forceinline__ T at2(const T (&x)[2], int r) {
    return r ? x[1] : x[0];
}

// The best (chi^2, packed i | j << 4 | r1 << 8 | r2 << 9) at one split point.
// The l- side goes first and keeps only its two smallest terms (first index
// on ties); the l+ side then pairs each candidate i with the smallest l-
// term of a j != i.  Nothing per candidate is kept.
__device__ __forceinline__ double side_min(const double *b, const Side &S, const Chi2Args &a, int &root) {
    double t = INFINITY;
    root = 0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (r < S.n) {
            const double v = top_term(b[0], b[1], b[2], b[3], S.w[r], a) + S.cw[r];
            if (v < t) {
                t = v;
                root = r;
            }
        }
    return t;
}

__device__ __forceinline__ double point_best(const Lep &LP, const Lep &LM, const double *cv, int nc, double mx,
                                             double my, double u, double v, const Chi2Args &a, int &packed) {
    const Side P = side(LP, 0.5 * mx + u, 0.5 * my + v, a);
    const Side M = side(LM, 0.5 * mx - u, 0.5 * my - v, a);
    double va = INFINITY, vb = INFINITY;
    int ja = -1, jb = -1, ra = 0, rb = 0;
    for (int c = 0; c < nc; ++c) {
        int r;
        const double t = side_min(cv + 4 * c, M, a, r);
        if (t < va) {
            vb = va;
            jb = ja;
            rb = ra;
            va = t;
            ja = c;
            ra = r;
        } else if (t < vb) {
            vb = t;
            jb = c;
            rb = r;
        }
    }
    double best = INFINITY;
    packed = 0;
    for (int i = 0; i < nc; ++i) {
        int r1;
        const double t1 = side_min(cv + 4 * i, P, a, r1);
        const bool other = i != ja;
        const int j = other ? ja : jb;
        const double t = t1 + (other ? va : vb);
        if (j >= 0 && t < best) {
            best = t;
            packed = i | (j << 4) | (r1 << 8) | ((other ? ra : rb) << 9);
        }
    }
    return best;
}

// The smallest W term of a side and its root (first on ties); INFINITY
// when the side has no p_z candidate.
__device__ __forceinline__ double w_min(const Side &S, int &root) {
    double t = INFINITY;
    root = 0;
#pragma unroll
    for (int r = 0; r < 2; ++r)
        if (r < S.n && S.cw[r] < t) {
            t = S.cw[r];
            root = r;
        }
    return t;
}

// One top (Wt, section 6.2): candidate i forms the top with l+ (the l- W
// standing alone), then with l- (the l+ W alone); the first minimum in the
// order (candidate, side).  Packed as for two tops with 15 in the index of
// the side without a top.
__device__ __forceinline__ double point_best1(const Lep &LP, const Lep &LM, const double *cv, int nc, double mx,
                                              double my, double u, double v, const Chi2Args &a, int &packed) {
    const Side P = side(LP, 0.5 * mx + u, 0.5 * my + v, a);
    const Side M = side(LM, 0.5 * mx - u, 0.5 * my - v, a);
    int rwp, rwm;
    const double wp = w_min(P, rwp), wm = w_min(M, rwm);
    double best = INFINITY;
    packed = 0;
    for (int i = 0; i < nc; ++i) {
        int r;
        const double tp = side_min(cv + 4 * i, P, a, r) + wm;
        if (tp < best) {
            best = tp;
            packed = i | (15 << 4) | (r << 8) | (rwm << 9);
        }
        const double tm = wp + side_min(cv + 4 * i, M, a, r);
        if (tm < best) {
            best = tm;
            packed = 15 | (i << 4) | (rwp << 8) | (r << 9);
        }
    }
    return best;
}

// Wave argmin of (value, point index); every lane gets the winner.  The
// minimum value first (four in-row DPP steps, then across rows by
// shuffles); a ballot finds the lanes holding it, and among several the
// smallest point index wins (a second reduction, on the index).
__device__ __forceinline__ void wave_argmin(double &val, int &pidx, int &packed) {
    double m = val;
    m = fmin(m, dpp_f64<0xB1>(m));
    m = fmin(m, dpp_f64<0x4E>(m));
    m = fmin(m, dpp_f64<0x141>(m));
    m = fmin(m, dpp_f64<0x140>(m));
    m = fmin(m, __shfl_xor(m, 16));
    m = fmin(m, __shfl_xor(m, 32));
    const uint64_t at = ballot(val == m);
    int wl = (int)__builtin_ctzll(at);
    if ((at & (at - 1)) != 0) {
        int q = ((at >> lane_id()) & 1ull) ? pidx : 0x7fffffff;
        q = min(q, dpp_i32<0xB1>(q));
        q = min(q, dpp_i32<0x4E>(q));
        q = min(q, dpp_i32<0x141>(q));
        q = min(q, dpp_i32<0x140>(q));
        q = min(q, __shfl_xor(q, 16));
        q = min(q, __shfl_xor(q, 32));
        wl = (int)__builtin_ctzll(ballot(((at >> lane_id()) & 1ull) && pidx == q));
    }
    val = __shfl(val, wl);
    pidx = __shfl(pidx, wl);
    packed = __shfl(packed, wl);
}

// Lep fields in LDS: the 4-vector, then c0, qa, inv_qa, inv_e
__device__ __forceinline__ void put_lep(double *d, const Lep &L) {
    for (int c = 0; c < 4; ++c) d[c] = L.l[c];
    d[4] = L.c0;
    d[5] = L.qa;
    d[6] = L.inv_qa;
    d[7] = L.inv_e;
}

__device__ __forceinline__ Lep get_lep(const double *d) {
    Lep L;
    for (int c = 0; c < 4; ++c) L.l[c] = d[c];
    L.c0 = d[4];
    L.qa = d[5];
    L.inv_qa = d[6];
    L.inv_e = d[7];
    return L;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__global__ __launch_bounds__(kBlock) void k_chi2(EvView ev, const int32_t *__restrict__ idx,
                                                 const int64_t *__restrict__ count, int64_t capacity, Chi2Args a,
                                                 Chi2OutView o, hf_counters_t *__restrict__ counter) {
    // one event per wavefront: event kb + w for wavefront w of the block
    __shared__ double s_lep[kWaves][8];       // the first two selected leptons
    __shared__ double s_cv[kWaves][kMaxC * 4];  // the b candidates
    __shared__ double s_fv[kWaves][8];        // the first two untagged selected jets
    __shared__ double s_L[kWaves][2][8];      // Lep of l+ and l-
    __shared__ double s_met[kWaves][2];
    __shared__ double s_res[kWaves][3];       // best split (u, v) and chi^2
    __shared__ int s_loc[kWaves][kMaxC];
    __shared__ int s_floc[kWaves][2];
    __shared__ int s_evi[kWaves][2];          // fit (0/1), candidate count
    __shared__ int s_pk[kWaves];              // best packed pairing and roots
    __shared__ float s_q[kWaves][2];          // charges of the first two selected leptons
    __shared__ double s_t[kWaves][kRefPts][kMaxC];  // refinement: l+ term per point and candidate
    __shared__ int s_r[kWaves][kRefPts][kMaxC];     // and its p_z root
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int64_t S = clamp_count(count, capacity);
    const int64_t kb = (int64_t)blockIdx.x * kWaves;  // the block's first event
    if (kb >= S) {
        if (threadIdx.x == 0 && counter && blockIdx.x == 0)
            atomicAdd((unsigned long long *)&counter->reached, (unsigned long long)S);
        return;
    }
    const int need = a.n_top == 1 ? 1 : 2;
    // the block's lead wavefront stages all four events and writes their outputs;
    // which one it is rotates with the block, so that no SIMD takes every block's share
    const int lead = (int)(blockIdx.x & (kWaves - 1));
    if (wave == lead) {
        // ---- staging, by the lead wavefront for all of the block's events: lanes
        // [kSeg s, kSeg (s + 1)) over the objects of event kb + s, leptons then jets,
        // every column loaded at once.  The first two selected leptons go to slots 0
        // and 1 by selection rank; the tagged selected jets (or all selected jets) to
        // candidate slots in input order, capped; the first two untagged selected jets
        // to filler slots.  Each object the fit uses is converted on the lane that
        // holds it.
        const int seg = lane / kSeg, sl = lane % kSeg, shift = seg * kSeg;
        const int64_t ks = kb + seg;
        uint32_t l0 = 0, j0 = 0, nlep = 0, nobj = 0;
        float fmx = 0.0f, fmy = 0.0f;
        if (ks < S) {
            const int64_t e = (int64_t)idx[ks] - ev.index_base;
            if (e >= 0 && e < ev.n) {
                l0 = ev.lep_off[e];
                j0 = ev.jet_off[e];
                const uint32_t l1 = ev.lep_off[e + 1], j1 = ev.jet_off[e + 1];
                fmx = ev.met_x[e];
                fmy = ev.met_y[e];
                nlep = l1 > l0 ? l1 - l0 : 0u;
                nobj = nlep + (j1 > j0 ? j1 - j0 : 0u);
            }
        }
        const bool all = a.pair_mode == HF_PAIR_ALL_JETS;
        const uint32_t segmask = (uint32_t)((1ull << kSeg) - 1ull), below = (1u << sl) - 1u;
        int nl = 0, ncand = 0, nfill = 0;
        for (uint32_t c0 = 0; ballot(c0 < nobj); c0 += kSeg) {
            const uint32_t o = c0 + (uint32_t)sl;
            const bool in = o < nobj, isl = o < nlep;
            const uint32_t q = isl ? l0 + o : j0 + (o - nlep);
            float pt = 0.0f, eta = 0.0f, phi = 0.0f, en = 0.0f, aux = 0.0f;
            if (in) {
                pt = (isl ? ev.lep_pt : ev.jet_pt)[q];
                eta = (isl ? ev.lep_eta : ev.jet_eta)[q];
                phi = (isl ? ev.lep_phi : ev.jet_phi)[q];
                en = (isl ? ev.lep_e : ev.jet_e)[q];
                aux = (isl ? ev.lep_q : ev.jet_btag)[q];
            }
            const bool lsel = in && isl && pt > a.lep_pt_min && fabsf(eta) < a.lep_eta_max;
            const bool jsel = in && !isl && pt > a.jet_pt_min && fabsf(eta) < a.jet_eta_max;
            const bool tag = all || aux > a.btag_min;
            const uint32_t ml = (uint32_t)(ballot(lsel) >> shift) & segmask;
            const uint32_t mt = (uint32_t)(ballot(jsel && tag) >> shift) & segmask;
            const uint32_t mu = (uint32_t)(ballot(jsel && !tag) >> shift) & segmask;
            const int lrank = nl + __popc(ml & below);
            const int pos = ncand + __popc(mt & below);
            const int frank = nfill + __popc(mu & below);
            double *dst = nullptr;
            if (lsel && lrank < 2) {
                dst = &s_lep[seg][4 * lrank];
                s_q[seg][lrank] = aux;
            } else if (jsel && tag && pos < a.max_cands) {
                dst = &s_cv[seg][4 * pos];
                s_loc[seg][pos] = (int)(q - j0);
            } else if (jsel && !tag && frank < 2) {
                dst = &s_fv[seg][4 * frank];
                s_floc[seg][frank] = (int)(q - j0);
            }
            if (dst) {
                double v[4];
                to_cart(pt, eta, phi, en, v);
                for (int c = 0; c < 4; ++c) dst[c] = v[c];
            }
            nl += __popc(ml);
            ncand = min(a.max_cands, ncand + __popc(mt));
            nfill += __popc(mu);
        }
        wave_sync();
        // exactly two selected leptons of opposite charges, l+ the positive one; fewer
        // than two candidates: the leading untagged selected jets fill
        int ok = 0, prank = 0;
        if (nl == 2 && s_q[seg][0] * s_q[seg][1] < 0.0f) {
            prank = s_q[seg][0] > 0.0f ? 0 : 1;
            const int nf = (all || ncand >= 2) ? 0 : min(nfill, 2 - ncand);
            if (sl < 4 * nf) s_cv[seg][4 * ncand + sl] = s_fv[seg][sl];
            if (sl < nf) s_loc[seg][ncand + sl] = s_floc[seg][sl];
            ncand += nf;
            ok = ncand >= need ? 1 : 0;
        }
        if (sl == 0) {
            s_evi[seg][0] = ok;
            s_evi[seg][1] = ncand;
            s_met[seg][0] = (double)fmx;
            s_met[seg][1] = (double)fmy;
        }
        // the split-independent lepton terms, lanes 2 s (l+) and 2 s + 1 (l-)
        const int src = ((lane >> 1) & (kWaves - 1)) * kSeg;
        const int prank_of = __shfl(prank, src), ok_of = __shfl(ok, src);
        if (lane < 2 * kWaves && ok_of) {
            const int s = lane >> 1, r = (lane & 1) ? 1 - prank_of : prank_of;
            put_lep(&s_L[s][lane & 1][0], make_lep(&s_lep[s][4 * r], a));
        }
    }
    __syncthreads();

    // ---- the grid scan of the wavefront's event, over all lanes
    if (kb + wave < S && uniform(s_evi[wave][0])) {
        const int nc = uniform(s_evi[wave][1]);
        const Lep LP = get_lep(&s_L[wave][0][0]), LM = get_lep(&s_L[wave][1][0]);
        const double mx = s_met[wave][0], my = s_met[wave][1];
        const double *cv = &s_cv[wave][0];
        // ---- coarse grid
        const int N = a.n_grid;
        double step = 2.0 * a.half_range / (double)(N - 1);
        double bval = INFINITY, bu = 0.0, bv = 0.0;
        int bpk = 0;
        {
            double val = INFINITY;
            int pidx = 0x7fffffff, pk = 0;
            // row and column of point p = p0 + lane, advanced by 64 points per pass
            // (no integer division in the loop)
            int row = lane / N, col = lane % N;
            const int drow = kWave / N, dcol = kWave % N;
            for (int p0 = 0; p0 < N * N; p0 += kWave) {
                const int p = p0 + lane;
                if (p < N * N) {
                    int q;
                    const double pu = -a.half_range + step * row, pv = -a.half_range + step * col;
                    const double t = a.n_top == 1 ? point_best1(LP, LM, cv, nc, mx, my, pu, pv, a, q)
                                                  : point_best(LP, LM, cv, nc, mx, my, pu, pv, a, q);
                    if (t < val) {
                        val = t;
                        pidx = p;
                        pk = q;
                    }
                }
                row += drow;
                col += dcol;
                if (col >= N) {
                    col -= N;
                    ++row;
                }
            }
            wave_argmin(val, pidx, pk);
            bval = val;
            bpk = pk;
            bu = -a.half_range + step * (pidx / N);
            bv = -a.half_range + step * (pidx % N);
        }
        // ---- refinements: 5 x 5 around the best point, a quarter of the step.
        // 25 points would leave most lanes idle, so the two lepton sides go to
        // different lanes: lanes [0, 25) take the l+ side of point q = lane and
        // keep each candidate's term in LDS, lanes [32, 57) the l- side of point
        // q = lane - 32 and keep its two smallest terms, which then go to the l+
        // lane of the same point (the same operations as point_best).
        for (int level = 0; level < a.n_refine && a.n_top == 1; ++level) {
            // one top: lanes [0, 25) take the whole point
            step *= 0.25;
            double val = INFINITY;
            int pidx = 0x7fffffff, pk = 0;
            if (lane < kRefPts) {
                const double u = bu + step * (lane / 5 - 2), v = bv + step * (lane % 5 - 2);
                val = point_best1(LP, LM, cv, nc, mx, my, u, v, a, pk);
                pidx = lane;
            }
            wave_argmin(val, pidx, pk);
            if (val < bval) {
                bval = val;
                bpk = pk;
                bu = bu + step * (pidx / 5 - 2);
                bv = bv + step * (pidx % 5 - 2);
            }
        }
        for (int level = 0; level < a.n_refine && a.n_top != 1; ++level) {
            step *= 0.25;
            const bool plus = lane < 32;
            const int q = plus ? lane : lane - 32;
            double va = INFINITY, vb = INFINITY;
            int ja = -1, jb = -1, ra = 0, rb = 0;
            if (q < kRefPts) {
                const double u = bu + step * (q / 5 - 2), v = bv + step * (q % 5 - 2);
                // one side() on selected inputs: the halves of the wavefront take
                // different leptons, and two calls would both run under masks
                Lep L;
                for (int c = 0; c < 4; ++c) L.l[c] = plus ? LP.l[c] : LM.l[c];
                L.c0 = plus ? LP.c0 : LM.c0;
                L.qa = plus ? LP.qa : LM.qa;
                L.inv_qa = plus ? LP.inv_qa : LM.inv_qa;
                L.inv_e = plus ? LP.inv_e : LM.inv_e;
                const double nx = plus ? 0.5 * mx + u : 0.5 * mx - u;
                const double ny = plus ? 0.5 * my + v : 0.5 * my - v;
                const Side Sd = side(L, nx, ny, a);
                for (int c = 0; c < nc; ++c) {
                    int r;
                    const double t = side_min(cv + 4 * c, Sd, a, r);
                    if (plus) {
                        s_t[wave][q][c] = t;
                        s_r[wave][q][c] = r;
                    } else if (t < va) {
                        vb = va;
                        jb = ja;
                        rb = ra;
                        va = t;
                        ja = c;
                        ra = r;
                    } else if (t < vb) {
                        vb = t;
                        jb = c;
                        rb = r;
                    }
                }
            }
            wave_sync();
            const int src = (lane + 32) & (kWave - 1);
            const double mva = __shfl(va, src), mvb = __shfl(vb, src);
            const int mja = __shfl(ja, src), mjb = __shfl(jb, src);
            const int mra = __shfl(ra, src), mrb = __shfl(rb, src);
            double val = INFINITY;
            int pidx = 0x7fffffff, pk = 0;
            if (plus && q < kRefPts) {
                double best = INFINITY;
                int packed = 0;
                for (int i = 0; i < nc; ++i) {
                    const double t1 = s_t[wave][q][i];
                    const int r1 = s_r[wave][q][i];
                    const bool other = i != mja;
                    const int j = other ? mja : mjb;
                    const double t = t1 + (other ? mva : mvb);
                    if (j >= 0 && t < best) {
                        best = t;
                        packed = i | (j << 4) | (r1 << 8) | ((other ? mra : mrb) << 9);
                    }
                }
                val = best;
                pidx = q;
                pk = packed;
            }
            wave_argmin(val, pidx, pk);
            wave_sync();  // the next level overwrites the l+ terms
            if (val < bval) {
                bval = val;
                bpk = pk;
                bu = bu + step * (pidx / 5 - 2);
                bv = bv + step * (pidx % 5 - 2);
            }
        }
        if (lane == 0) {
            s_res[wave][0] = bu;
            s_res[wave][1] = bv;
            s_res[wave][2] = bval;
            s_pk[wave] = bpk;
        }
    }
    __syncthreads();
    if (wave != lead) return;

    // ---- outputs, by the lead wavefront: lanes 2 s (l+ side) and 2 s + 1 (l- side)
    // of event kb + s, the winner's kinematics in the definition's order of operations
    const int s = (lane >> 1) & (kWaves - 1);
    const int64_t k = kb + s;
    const bool minus = lane & 1;
    const bool mine = lane < 2 * kWaves && k < S;
    bool have = false;
    double ct = 0.0, cwt = 0.0;
    if (mine && s_evi[s][0]) {
        const double bu = s_res[s][0], bv = s_res[s][1];
        have = s_res[s][2] < INFINITY;  // no p_z candidate at all leaves none
        if (have) {
            const int bpk = s_pk[s];
            const double mx = s_met[s][0], my = s_met[s][1];
            const Lep L = get_lep(&s_L[s][minus ? 1 : 0][0]);
            const int i = bpk & 15, j = (bpk >> 4) & 15, r1 = (bpk >> 8) & 1, r2 = (bpk >> 9) & 1;
            const int c = minus ? j : i, r = minus ? r2 : r1;
            const double nx = minus ? 0.5 * mx - bu : 0.5 * mx + bu;
            const double ny = minus ? 0.5 * my - bv : 0.5 * my + bv;
            const Side Sd = side(L, nx, ny, a);
            const double z = at2(Sd.pz, r);
            const double nu[4] = {sqrt(nx * nx + ny * ny + z * z), nx, ny, z};
            // one top: index 15 marks the side without it
            const bool has_top = c != 15;
            double w[4], t[4];
            for (int q = 0; q < 4; ++q) {
                w[q] = L.l[q] + nu[q];
                t[q] = (has_top ? s_cv[s][4 * c + q] : 0.0) + w[q];
            }
            const double mw = mass4(w[0], w[1], w[2], w[3]), mt = mass4(t[0], t[1], t[2], t[3]);
            const double st2 = a.sigma_t * a.sigma_t, sw2 = a.sigma_w * a.sigma_w;
            ct = has_top ? sq(mt - a.m_t) / st2 : 0.0;
            cwt = sq(mw - a.m_w) / sw2;
            (minus ? o.root_nubar : o.root_nu)[k] = (int8_t)at2(Sd.kind, r);
            (minus ? o.best_j : o.best_i)[k] = (int16_t)(has_top ? s_loc[s][c] : -1);
            double *onu = minus ? o.nubar : o.nu;
            for (int q = 0; q < 3; ++q) onu[3 * k + q] = nu[q + 1];
            (minus ? o.m_tbar : o.m_t)[k] = has_top ? mt : HF_NO_SOLUTION;
            (minus ? o.m_wm : o.m_wp)[k] = mw;
        }
    }
    // the l- terms to the l+ lane, summed in the definition's order
    const double ct_m = __shfl(ct, lane | 1), cw_m = __shfl(cwt, lane | 1);
    if (mine && !minus) {
        if (have) {
            o.has_sol[k] = 1;
            o.chi2[k] = ct + cwt + ct_m + cw_m;
            o.split[2 * k] = s_res[s][0];
            o.split[2 * k + 1] = s_res[s][1];
        } else {
            o.has_sol[k] = 0;
            o.root_nu[k] = o.root_nubar[k] = -1;
            o.best_i[k] = o.best_j[k] = -1;
            for (int c = 0; c < 3; ++c) o.nu[3 * k + c] = o.nubar[3 * k + c] = HF_NO_SOLUTION;
            o.m_t[k] = o.m_tbar[k] = o.m_wp[k] = o.m_wm[k] = o.chi2[k] = HF_NO_SOLUTION;
            o.split[2 * k] = o.split[2 * k + 1] = HF_NO_SOLUTION;
        }
    }
    // RECO counters: one atomic per block
    const uint32_t tot = (uint32_t)popc64(ballot(mine && !minus && have));
    if (lane == 0 && counter) {
        if (tot) atomicAdd((unsigned long long *)&counter->passed, (unsigned long long)tot);
        if (blockIdx.x == 0) atomicAdd((unsigned long long *)&counter->reached, (unsigned long long)S);
    }
}

}  // namespace

hipError_t launch_chi2(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity, const Chi2Args &a,
                       const Chi2OutView &out, hf_counters_t *counter, hipStream_t s) {
    if (capacity <= 0) return hipSuccess;
    const int64_t nb = (capacity + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(k_chi2, dim3((unsigned)nb), dim3(kBlock), 0, s, ev, idx, count, capacity, a, out, counter);
    return hipGetLastError();
}

}  // namespace hf
