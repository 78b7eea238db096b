// Dileptonic ttbar kinematic reconstruction over the compacted events
// (paper section 4: W and top mass constraints for every lepton / b-jet
// pairing, over resolution-smeared pseudo-experiments, the most probable
// solution kept; the event fails the last cut when no solution exists).
//
// Kernels, in launch order.
//
// k_stage: eight lanes per compacted event; selects the leptons and b
// candidates, writes their FP64 Cartesian 4-vectors to a record, the
// event's count of lane granules (16 variations each; none when no
// pairing is valid) and an empty best record.
//
// k_scan_*: exclusive prefix sum of the granule counts (the worklist: the
// variations of all events laid end to end, each event padded to whole
// granules).
//
// k_search: persistent grid; each wavefront takes a contiguous range of
// 64-lane blocks of the worklist.  A block holds up to four events (small
// variation counts are packed) or one slice of a large one (large counts
// are split over blocks and wavefronts).  The wavefront copies the block's
// records into LDS and adds, per candidate and lepton side, the constants of
// the linear maps and of the conic's quadratic part.  Each lane draws its
// variation (Philox4x32-10 + Box-Muller in precision T) and, for every
// pairing of its event, assembles the eliminant quartic in FP64 and brackets
// its real roots (critical points from the closed-form cubic in T, one FP64
// Newton step each); the wavefront then deals the root intervals out 64 at
// a time: Halley iteration in FP64, recovery and polish of (x, y), the acceptance
// test, the energies' signs and the score, each result handed back to the
// lane that owns the variation.  A segmented argmax with a total-order
// tie-break (score, then smallest variation, pairing, x) gives each event's
// winner; an event that crosses a range boundary leaves partial records.
//
// k_fixup: merges the partial records of events that crossed a range.
//
// k_epilogue: one thread per event; recomputes the winner's kinematics in
// FP64 (draws recomputed bit-identically in T), writes the outputs, the
// H -> bb candidate mass, and folds the RECO counters.
//
// T = float (HF_PREC_MIXED): draws and root seeds in FP32.
// T = double (HF_PREC_FP64): everything in FP64.
#include <math.h>

#include "hf_device.hpp"
#include "hf_internal.hpp"
#include "hf_reco_math.hpp"

namespace hf {
namespace {

constexpr int kRecoBlock = 256;
constexpr int kRecoWaves = kRecoBlock / kWave;
constexpr int kMaxC = HF_MAX_CANDS;
constexpr int kNoBest = 0x7fffffff;
constexpr size_t kWsHeader = 2048;
// Event counters of the one-wavefront-per-event search: kTicketClasses of
// them at words kTicketWord + 16 c of the workspace header, each on its own
// 128-byte line.
constexpr int kTicketWord = 16;
constexpr int kTicketClasses = 8;
constexpr int kGran = 16;              // lanes per granule of the worklist
constexpr int kGpb = kWave / kGran;    // granules per 64-lane block: at most 4 events per block
constexpr int kSideCap = 24;           // side-constant slots shared by a block's events
constexpr int kMaxSearchWaves = 8192;  // bound on the search grid (partial-record space)
constexpr int kScanTile = 1024;        // elements per block of the prefix sum

// Per-event result of the search, read by the epilogue.
struct BestRec {
    double score, x, y;
    int32_t v, p, nsol, nc;
};

// One compacted event as the reconstruction sees it, built by k_stage: the
// two selected leptons and the b candidates as nominal FP64 (E, px, py, pz),
// in the order of the candidate rule; nc = 0 when the lepton selection
// fails (or the id lies outside the chunk).  640 bytes = 80 words, copied
// into LDS by a wavefront with two loads per lane.
struct StageRec {
    double lp[4], lm[4];    // l+ and l-
    double met[2];          // nominal MET x, y
    double ml2p, ml2m;      // squared masses of l+ and l-
    double sigma[kMaxC];    // jet energy resolution at the nominal energy
    uint64_t g;             // global event id (the generator's counter)
    int32_t jidx[kMaxC];    // candidate -> jet index within the event
    int32_t nc, V;          // number of candidates, of variations
    double cand[kMaxC][4];  // b candidates
};
constexpr int kRecWords = (int)(sizeof(StageRec) / 8);
static_assert(sizeof(StageRec) == 640 && kRecWords > kWave && kRecWords <= 2 * kWave, "record layout");

// Best solution of an event seen by one wavefront at a boundary of its range
// of blocks, merged by k_fixup.  k = -1: none; k = -2: the range is empty.
struct PartRec {
    int64_t k;
    int32_t cont;  // the event continues past the end of the range
    int32_t nsol, v, p, nc, pad;
    double score, x, y;
};

template <typename T>
struct WaveStageEv {
    StageRec rec;
    double sp[kMaxC][kSide];  // side constants with l+
    double sm[kMaxC][kSide];  // side constants with l-
    T z[kMaxC][kWave];  // per-lane draw of each candidate
    T zl[4][kWave];     // per-lane draws of l+, l-, MET x, MET y
};

template <typename T>
struct WaveStage {
    StageRec rec[kGpb];             // the block's events
    double sp[kSideCap][kSide];     // side constants with l+ (slot base + candidate)
    double sm[kSideCap][kSide];     // side constants with l-
    int okp[kSideCap], okm[kSideCap];
    double res_w[kWave], res_x[kWave], res_y[kWave];  // stage-2 results, by queue position
    int res_ok[kWave];
    double gb_s[kGpb], gb_x[kGpb], gb_y[kGpb];       // per-granule best
    int gb_v[kGpb], gb_p[kGpb], gb_n[kGpb];
    T z[kMaxC][kWave];  // per-lane draw of each candidate of the lane's event
    T zl[4][kWave];     // per-lane draws of l+, l-, MET x, MET y
    PartRec headp, tailp;  // partial records of the range's first and last event
    int queue[4 * kWave];  // stage-2 queue: source lane | interval << 6
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Nominal Cartesian 4-vector (E, px, py, pz) from the float32 columns, FP64.
__device__ __forceinline__ void polar_to_cart(float pt, float eta, float phi, float e, double out[4]) {
    double s, c;
    sincos((double)phi, &s, &c);
    out[0] = (double)e;
    out[1] = (double)pt * c;
    out[2] = (double)pt * s;
    out[3] = (double)pt * sinh((double)eta);
}

// "a is better than b": higher score, then smaller variation, pairing, x.
__device__ __forceinline__ bool better(double sa, int va, int pa, double xa, double sb, int vb, int pb, double xb) {
    if (sa != sb) return sa > sb;
    if (va != vb) return va < vb;
    if (pa != pb) return pa < pb;
    return xa < xb;
}

// Scale factor max(1 + sigma z, 0.01), formed in FP64 from a draw in T.
template <typename T>
__device__ __forceinline__ double smear(double sigma, T z) {
    const double s = 1.0 + sigma * (double)z;
    return s > 0.01 ? s : 0.01;
}

__device__ __forceinline__ bool lep_sel(const EvView &ev, uint32_t k, const RecoArgs &a) {
    return ev.lep_pt[k] > a.lep_pt_min && fabsf(ev.lep_eta[k]) < a.lep_eta_max;
}

__device__ __forceinline__ bool jet_sel(const EvView &ev, uint32_t k, const RecoArgs &a) {
    return ev.jet_pt[k] > a.jet_pt_min && fabsf(ev.jet_eta[k]) < a.jet_eta_max;
}

template <typename X>
__device__ __forceinline__ X from_lane(X v, int src) {
    return __shfl(v, src);
}

// In-row lane exchanges by DPP (no LDS round trip): kCtrl is the DPP control
// word (quad_perm 0xB1 = lane ^ 1, 0x4E = lane ^ 2; 0x141 = row_half_mirror,
// lane i <-> 7 - i within eight lanes; 0x140 = row_mirror, i <-> 15 - i
// within sixteen).  Every pattern used is a permutation inside each row, so
// no lane reads outside the wavefront.
template <int kCtrl>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, kCtrl, 0xF, 0xF, false);
}

template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(dpp_i32<kCtrl>(hi), dpp_i32<kCtrl>(lo));
}

__device__ __forceinline__ int64_t clamp_count(const int64_t *count, int64_t capacity) {
    const int64_t S = *count;
    return S < 0 ? 0 : (S > capacity ? capacity : S);
}

// Eight lanes per compacted event (eight events per wavefront): selection of
// the two leptons (exactly two selected, opposite charges; l+ first) and of
// the b candidates (b-tagged selected jets in input order up to max_cands,
// filled up to two with the leading untagged selected jets; or every
// selected jet), converted to FP64 Cartesian 4-vectors.  The lanes of an
// event read its objects eight at a time; ballots restricted to the event's
// eight bits give the selection, the candidates' order and the first
// untagged jets; each lane then converts and writes at most two candidates,
// and the record's fields are written by the lanes that own them.  Spreading
// an event over lanes keeps many more wavefronts in flight than one thread
// per event, which is what hides the chain of dependent loads.
constexpr int kStageLanes = 8;
constexpr int kStageEvents = 256 / kStageLanes;  // events per block

__global__ __launch_bounds__(256) void k_stage(EvView ev, const int32_t *__restrict__ idx,
                                               const int64_t *__restrict__ count, int64_t capacity, RecoArgs a,
                                               StageRec *__restrict__ stage, int32_t *__restrict__ gcnt,
                                               BestRec *__restrict__ best) {
    __shared__ uint32_t s_jl[kStageEvents][kMaxC];  // candidates' jet positions
    __shared__ double s_lep[kStageEvents][8];       // l+ then l-
    const int lane = lane_id(), sub = lane & (kStageLanes - 1);
    const int slot = threadIdx.x / kStageLanes;
    const int shift = lane & ~(kStageLanes - 1);     // the event's first lane in the wave
    const uint64_t lt = lanemask_lt() >> shift;      // lanes of this event below this one (low bits)
    const int64_t S = clamp_count(count, capacity);
    const int64_t k = (int64_t)blockIdx.x * kStageEvents + slot;
    if (k >= S) return;  // whole events only: the eight lanes of an event leave together
    StageRec &r = stage[k];
    const uint64_t g = (uint64_t)idx[k];
    const int64_t e = (int64_t)g - ev.index_base;
    const bool in_chunk = e >= 0 && e < ev.n;  // ids outside the chunk get no solution
    auto bits = [&](bool p) { return (uint32_t)((ballot(p) >> shift) & 0xffu); };
    int nc = 0, V = 0;
    uint32_t kp = 0, km = 0;
    bool lep_ok = false;
    if (in_chunk) {
        V = ev.n_var ? (int)ev.n_var[e] : a.n_var_uniform;
        // ---- leptons: the first two selected, and how many are selected
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        int nl = 0;
        uint32_t ka = 0, kb = 0;
        for (uint32_t c0 = l0; c0 < l1; c0 += kStageLanes) {
            const uint32_t q = c0 + sub;
            const bool in = q < l1;
            const float pt = in ? ev.lep_pt[q] : 0.0f, eta = in ? ev.lep_eta[q] : 0.0f;
            uint32_t m = bits(in && pt > a.lep_pt_min && fabsf(eta) < a.lep_eta_max);
            while (m && nl < 2) {
                const uint32_t b = c0 + (uint32_t)(__ffs(m) - 1);
                if (nl == 0) ka = b;
                else kb = b;
                ++nl;
                m &= m - 1;
            }
            nl += __popc(m);
        }
        if (nl == 2) {
            const float qa = ev.lep_q[ka], qb = ev.lep_q[kb];
            lep_ok = qa * qb < 0.0f;
            kp = qa > 0.0f ? ka : kb;
            km = qa > 0.0f ? kb : ka;
        }
        if (lep_ok) {
            // ---- b candidates
            const int cap = a.max_cands < kMaxC ? a.max_cands : kMaxC;
            const bool all = a.pair_mode == HF_PAIR_ALL_JETS;
            const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
            int nfill = 0;
            uint32_t f0 = 0, f1 = 0;
            for (uint32_t c0 = j0; c0 < j1; c0 += kStageLanes) {
                const uint32_t q = c0 + sub;
                const bool in = q < j1;
                const float pt = in ? ev.jet_pt[q] : 0.0f, eta = in ? ev.jet_eta[q] : 0.0f;
                const float bt = in ? ev.jet_btag[q] : 0.0f;
                const bool sel = in && pt > a.jet_pt_min && fabsf(eta) < a.jet_eta_max;
                const bool tag = all || bt > a.btag_min;
                const uint32_t mt = bits(sel && tag);
                uint32_t mu = bits(sel && !tag);
                const int pos = nc + __popc(mt & (uint32_t)lt);
                if (sel && tag && pos < cap) s_jl[slot][pos] = q;
                nc = min(cap, nc + __popc(mt));
                while (mu && nfill < 2) {
                    const uint32_t b = c0 + (uint32_t)(__ffs(mu) - 1);
                    if (nfill == 0) f0 = b;
                    else f1 = b;
                    ++nfill;
                    mu &= mu - 1;
                }
                nfill += __popc(mu);
            }
            if (!all) {
                // leading untagged selected jets fill the list up to two
                if (nc < 2 && nfill > 0) {
                    if (sub == 0) s_jl[slot][nc] = f0;
                    ++nc;
                }
                if (nc < 2 && nfill > 1) {
                    if (sub == 0) s_jl[slot][nc] = f1;
                    ++nc;
                }
            }
        }
    }
    if (!lep_ok) nc = 0;
    // ---- the record: leptons by lanes 0 and 1, candidates two per lane
    uint32_t okp = 0, okm = 0;
    if (nc > 0) {
        const uint32_t j0 = ev.jet_off[e];
        if (sub < 2) {
            const uint32_t q = sub == 0 ? kp : km;
            double v[4];
            polar_to_cart(ev.lep_pt[q], ev.lep_eta[q], ev.lep_phi[q], ev.lep_e[q], v);
            double *dst = sub == 0 ? r.lp : r.lm;
            for (int c = 0; c < 4; ++c) {
                dst[c] = v[c];
                s_lep[slot][4 * sub + c] = v[c];
            }
            const double m2 = v[0] * v[0] - v[1] * v[1] - v[2] * v[2] - v[3] * v[3];
            if (sub == 0) r.ml2p = m2;
            else r.ml2m = m2;
        }
        wave_sync();
        double lp[4], lm[4];
        for (int c = 0; c < 4; ++c) {
            lp[c] = s_lep[slot][c];
            lm[c] = s_lep[slot][4 + c];
        }
        for (int c = sub; c < nc; c += kStageLanes) {
            const uint32_t q = s_jl[slot][c];
            double v[4];
            const float en = ev.jet_e[q];
            polar_to_cart(ev.jet_pt[q], ev.jet_eta[q], ev.jet_phi[q], en, v);
            for (int u = 0; u < 4; ++u) r.cand[c][u] = v[u];
            r.sigma[c] = sqrt(a.jet_a * a.jet_a / (double)en + a.jet_c * a.jet_c);
            r.jidx[c] = (int32_t)(q - j0);
            // valid sides (the same test as make_side)
            double sd[kSide];
            if (make_side(lp, v, sd)) okp |= 1u << c;
            if (make_side(lm, v, sd)) okm |= 1u << c;
        }
    }
    // the event's masks: OR over its eight lanes
#pragma unroll
    for (int off = 1; off < kStageLanes; off <<= 1) {
        okp |= __shfl_xor(okp, off);
        okm |= __shfl_xor(okm, off);
    }
    if (sub == 2) {
        r.g = g;
        if (in_chunk) {
            r.met[0] = (double)ev.met_x[e];
            r.met[1] = (double)ev.met_y[e];
        }
        r.nc = nc;
        r.V = V;
    }
    if (sub == 3) {
        int npair = 0;
        for (int c = 0; c < nc; ++c)
            if ((okp >> c) & 1u) npair += __popc(okm & ~(1u << c));
        gcnt[k] = (npair > 0 && V > 0) ? (V + kGran - 1) / kGran : 0;
        BestRec b;
        b.score = -INFINITY;
        b.x = b.y = 0.0;
        b.v = b.p = kNoBest;
        b.nsol = 0;
        b.nc = nc;
        best[k] = b;
    }
}

// ------------------------------------------------------------ prefix sum
// Exclusive prefix sum of the granule counts: per tile of kScanTile counts a
// total (k_scan_tiles), the tile totals scanned by one block (k_scan_top),
// then each tile's counts scanned from its tile offset (k_scan_apply).
// gofs[S] receives the grand total.

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *s_w, int64_t &total) {
    // 256 threads: wave inclusive scans, then the four wave totals
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    int64_t inc = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(inc, off);
        if (lane >= off) inc += o;
    }
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
        if (w < wave) base += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t *__restrict__ gcnt,
                                                    const int64_t *__restrict__ count, int64_t capacity,
                                                    int64_t *__restrict__ tsum) {
    __shared__ int64_t s_w[256 / kWave];
    const int64_t S = clamp_count(count, capacity);
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    if (t0 >= S && blockIdx.x > 0) return;
    int64_t v = 0;
#pragma unroll
    for (int u = 0; u < kScanTile / 256; ++u) {
        const int64_t k = t0 + (int64_t)threadIdx.x * (kScanTile / 256) + u;
        if (k < S) v += gcnt[k];
    }
    int64_t total;
    block_exclusive_scan(v, s_w, total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_top(const int64_t *__restrict__ count, int64_t capacity,
                                                  int64_t *__restrict__ tsum) {
    __shared__ int64_t s_w[256 / kWave];
    const int64_t S = clamp_count(count, capacity);
    const int64_t nt = S > 0 ? (S + kScanTile - 1) / kScanTile : 1;
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nt; c0 += 256) {
        const int64_t t = c0 + threadIdx.x;
        const int64_t v = t < nt ? tsum[t] : 0;
        int64_t total;
        const int64_t ex = block_exclusive_scan(v, s_w, total);
        if (t < nt) tsum[t] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t *__restrict__ gcnt,
                                                    const int64_t *__restrict__ count, int64_t capacity,
                                                    const int64_t *__restrict__ tsum, int64_t *__restrict__ gofs) {
    __shared__ int64_t s_w[256 / kWave];
    const int64_t S = clamp_count(count, capacity);
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    if (t0 >= S) {
        if (blockIdx.x == 0 && threadIdx.x == 0) gofs[0] = 0;  // S == 0
        return;
    }
    constexpr int kPer = kScanTile / 256;
    int64_t c[kPer];
    int64_t v = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t k = t0 + (int64_t)threadIdx.x * kPer + u;
        c[u] = k < S ? gcnt[k] : 0;
        v += c[u];
    }
    int64_t total;
    int64_t run = tsum[blockIdx.x] + block_exclusive_scan(v, s_w, total);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t k = t0 + (int64_t)threadIdx.x * kPer + u;
        if (k < S) gofs[k] = run;
        run += c[u];
        if (k == S - 1) gofs[S] = run;
    }
}

// ------------------------------------------------------------ search

// Largest k in [lo, hi) with gofs[k] <= G, given gofs[lo] <= G (gofs is
// non-decreasing): a 64-ary search, one load per lane per round.
__device__ int64_t find_event(const int64_t *__restrict__ gofs, int64_t lo, int64_t hi, int64_t G) {
    const int lane = lane_id();
    while (hi - lo > kWave) {
        const int64_t step = (hi - lo + kWave - 1) / kWave;
        const int64_t pos = lo + (int64_t)lane * step;
        const bool le = pos < hi && gofs[pos] <= G;
        const int c = popc64(ballot(le));  // >= 1: gofs[lo] <= G
        lo += (int64_t)(c - 1) * step;
        const int64_t nh = lo + step;
        hi = nh < hi ? nh : hi;
    }
    const int64_t pos = lo + lane;
    const bool le = pos < hi && gofs[pos] <= G;
    return lo + popc64(ballot(le)) - 1;
}

// Merge b into a by the total order of better(); solution counts add up.
struct Acc {
    double s, x, y;
    int v, p, n;
};

__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    if (better(b.s, b.v, b.p, b.x, a.s, a.v, a.p, a.x)) {
        a.s = b.s;
        a.v = b.v;
        a.p = b.p;
        a.x = b.x;
        a.y = b.y;
    }
    a.n += b.n;
}

template <typename T>
__global__ __launch_bounds__(kRecoBlock, 2) void k_search(const int64_t *__restrict__ count, int64_t capacity,
                                                          RecoArgs a, const StageRec *__restrict__ stage,
                                                          const int64_t *__restrict__ gofs,
                                                          BestRec *__restrict__ best_out, PartRec *__restrict__ part,
                                                          uint64_t *__restrict__ wstats) {
    __shared__ WaveStage<T> stage_all[kRecoWaves];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    WaveStage<T> &st = stage_all[wave];
    const int64_t S = clamp_count(count, capacity);
    const int64_t wid = (int64_t)blockIdx.x * kRecoWaves + wave;
    const int64_t nw = (int64_t)gridDim.x * kRecoWaves;
    const double mt2_mw2 = a.m_t * a.m_t - a.m_w * a.m_w;
    const double mw2 = a.m_w * a.m_w;
    uint64_t acc_var = 0, acc_pair = 0, acc_int = 0, acc_sol = 0;
    const uint64_t lt = lanemask_lt();

    // this wavefront's contiguous range of 64-lane blocks
    const int64_t NG = S > 0 ? gofs[S] : 0;
    const int64_t NB = (NG + kGpb - 1) / kGpb;
    const int64_t b0 = wid * NB / nw, b1 = (wid + 1) * NB / nw;
    const uint64_t *recw = reinterpret_cast<const uint64_t *>(stage);

    // open event (lane 0 keeps the accumulator; the others follow uniformly)
    int64_t open_k = -1;
    int open_nc = 0;
    bool open_head = false;
    Acc acc{-INFINITY, 0.0, 0.0, kNoBest, kNoBest, 0};
    // the partial records live in LDS (lane 0 writes them) rather than in
    // registers for the whole kernel
    if (lane == 0) {
        st.headp.k = b0 < b1 ? -1 : -2;
        st.tailp.k = -1;
        st.headp.cont = st.tailp.cont = 0;
    }

    auto flush = [&](bool cont) {
        if (open_k < 0) return;
        if (lane == 0) {
            if (open_head || cont) {
                PartRec &pr = open_head ? st.headp : st.tailp;
                pr.k = open_k;
                pr.cont = cont ? 1 : 0;
                pr.nsol = acc.n;
                pr.v = acc.v;
                pr.p = acc.p;
                pr.nc = open_nc;
                pr.score = acc.s;
                pr.x = acc.x;
                pr.y = acc.y;
            } else {
                BestRec r;
                r.score = acc.s;
                r.x = acc.x;
                r.y = acc.y;
                r.v = acc.v;
                r.p = acc.p;
                r.nsol = acc.n;
                r.nc = open_nc;
                best_out[open_k] = r;
            }
        }
        open_k = -1;
        open_head = false;
    };

    int64_t kc = b0 < b1 ? find_event(gofs, 0, S, b0 * kGpb) : 0;
    for (int64_t b = b0; b < b1; ++b) {
        // ---- which events the block's granules belong to
        const int64_t g0 = b * kGpb;
        const int64_t gw0 = gofs[kc];
        const int64_t wpos = kc + 1 + lane;
        const int64_t wv = wpos <= S ? gofs[wpos] : INT64_MAX;
        int64_t kj[kGpb];
        if (ballot(wv <= g0 + kGpb - 1) != ~0ull) {
#pragma unroll
            for (int j = 0; j < kGpb; ++j) kj[j] = kc + popc64(ballot(wv <= g0 + j));
        } else {  // more than 64 events without granules in a row
#pragma unroll
            for (int j = 0; j < kGpb; ++j) kj[j] = find_event(gofs, kc, S, g0 + j);
        }
        // slots: the distinct events of the valid granules, in order
        int slot_of[kGpb];
        int64_t sk[kGpb];
        int n_ev = 0;
#pragma unroll
        for (int j = 0; j < kGpb; ++j) {
            const bool valid = g0 + j < NG;
            if (valid && (n_ev == 0 || sk[n_ev - 1] != kj[j])) {
                sk[n_ev] = kj[j];
                ++n_ev;
            }
            slot_of[j] = valid ? n_ev - 1 : -1;
        }
        // granule offset of each slot's event
        int64_t sg[kGpb];
#pragma unroll
        for (int q = 0; q < kGpb; ++q) {
            if (q < n_ev) {
                const int64_t d = sk[q] - kc - 1;
                sg[q] = d < 0 ? gw0 : (d < kWave ? __shfl(wv, (int)d) : gofs[sk[q]]);
            } else {
                sg[q] = 0;
            }
        }
        kc = sk[n_ev - 1];  // the next block starts in this event or a later one

        // ---- records into LDS (80 words per slot; all loads issued before the stores)
        {
            constexpr int kIt = (kGpb * kRecWords + kWave - 1) / kWave;
            uint64_t wd[kIt];
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int w = it * kWave + lane;
                const bool in = w < n_ev * kRecWords;
                const int q = in ? w / kRecWords : 0, off = in ? w - q * kRecWords : 0;
                const int64_t kq = q == 0 ? sk[0] : q == 1 ? sk[1] : q == 2 ? sk[2] : sk[3];
                wd[it] = recw[kq * kRecWords + off];  // always a valid address (slot 0 when out of range)
            }
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int w = it * kWave + lane;
                if (w < n_ev * kRecWords) reinterpret_cast<uint64_t *>(&st.rec[0])[w] = wd[it];
            }
        }
        wave_sync();

        // ---- this lane's event and variation
        const int gj = lane / kGran;
        const int my_slot = gj == 0 ? slot_of[0] : gj == 1 ? slot_of[1] : gj == 2 ? slot_of[2] : slot_of[3];
        const int ms = my_slot < 0 ? 0 : my_slot;
        const int64_t my_g0 = ms == 0 ? sg[0] : ms == 1 ? sg[1] : ms == 2 ? sg[2] : sg[3];
        const int my_v = (int)((g0 + gj - my_g0) * kGran) + (lane % kGran);
        const int my_nc = st.rec[ms].nc;
        const bool in_block = my_slot >= 0 && my_v < st.rec[ms].V;

        double best_s = -INFINITY, best_x = 0.0, best_y = 0.0;
        int best_v = kNoBest, best_p = kNoBest, nsol = 0;

        // ---- passes over the slots whose candidates fit the side-constant table
        int s_lo = 0;
        while (s_lo < n_ev) {
            int s_hi = s_lo, used = 0, ncmax = 0;
            int sbase[kGpb] = {0, 0, 0, 0};
            while (s_hi < n_ev) {
                const int ncq = __builtin_amdgcn_readfirstlane(st.rec[s_hi].nc);
                if (used + ncq > kSideCap) break;
#pragma unroll
                for (int q = 0; q < kGpb; ++q)
                    if (q == s_hi) sbase[q] = used;
                used += ncq;
                ncmax = ncq > ncmax ? ncq : ncmax;
                ++s_hi;
            }
            // side constants: lanes [0, used) with l+, [32, 32 + used) with l-
            {
                const int e = lane & 31;
                if (e < used) {
                    int q = s_lo;
                    while (q + 1 < s_hi && e >= (q + 1 == 1 ? sbase[1] : q + 1 == 2 ? sbase[2] : sbase[3])) ++q;
                    const int qb = q == 0 ? sbase[0] : q == 1 ? sbase[1] : q == 2 ? sbase[2] : sbase[3];
                    const int c = e - qb;
                    if (lane < 32)
                        st.okp[e] = make_side(st.rec[q].lp, st.rec[q].cand[c], st.sp[e]) ? 1 : 0;
                    else
                        st.okm[e] = make_side(st.rec[q].lm, st.rec[q].cand[c], st.sm[e]) ? 1 : 0;
                }
            }
            wave_sync();
            const bool act = in_block && my_slot >= s_lo && my_slot < s_hi;
            const int sb = ms == 0 ? sbase[0] : ms == 1 ? sbase[1] : ms == 2 ? sbase[2] : sbase[3];
            const StageRec &R = st.rec[ms];
            // valid pairings of this lane's event (for the counters)
            if (act) {
                int np = 0;
                for (int i = 0; i < my_nc; ++i)
                    for (int j = 0; j < my_nc; ++j) np += (i != j && st.okp[sb + i] && st.okm[sb + j]) ? 1 : 0;
                ++acc_var;
                acc_pair += (uint64_t)np;
            }
            // ---- draws of this lane's variation, kept in LDS so that any lane can
            // rebuild another lane's smear factors
            {
                T zl[4] = {(T)0, (T)0, (T)0, (T)0};
                if (a.smear && act) {
                    const uint64_t g = R.g;
                    gauss_block<T>(a.seed, g, (uint32_t)my_v, 0u, zl);
                    uint32_t last_blk = 0xffffffffu;
                    T zb[4];
                    for (int c = 0; c < my_nc; ++c) {
                        const uint32_t slot = 4u + (uint32_t)R.jidx[c];
                        const uint32_t blk = slot >> 2;
                        if (blk != last_blk) {
                            gauss_block<T>(a.seed, g, (uint32_t)my_v, blk, zb);
                            last_blk = blk;
                        }
                        const uint32_t ln = slot & 3u;
                        st.z[c][lane] = ln == 0 ? zb[0] : ln == 1 ? zb[1] : ln == 2 ? zb[2] : zb[3];
                    }
                } else {
                    for (int c = 0; c < kMaxC; ++c) st.z[c][lane] = (T)0;
                }
                st.zl[0][lane] = zl[0];
                st.zl[1][lane] = zl[1];
                st.zl[2][lane] = zl[2];
                st.zl[3][lane] = zl[3];
            }
            wave_sync();
            const double slp = smear(a.lep_sigma, st.zl[0][lane]);
            const double slm = smear(a.lep_sigma, st.zl[1][lane]);
            const double mx = R.met[0] + a.met_sigma * (double)st.zl[2][lane];
            const double my = R.met[1] + a.met_sigma * (double)st.zl[3][lane];
            const double Wp = (0.5 * mw2) * fast_rcp(slp) - 0.5 * slp * R.ml2p;
            const double Wm = (0.5 * mw2) * fast_rcp(slm) - 0.5 * slm * R.ml2m;
            for (int i = 0; i < ncmax; ++i) {
                const bool act_i = act && i < my_nc && st.okp[sb + i];
                SideVar A;
                A.e0 = A.z0 = 0.0;
                A.q = Conic{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (act_i) A = side_var(st.sp[sb + i], Wp, slp, smear(R.sigma[i], st.z[i][lane]), mt2_mw2);
                for (int j = 0; j < ncmax; ++j) {
                    if (j == i) continue;
                    const bool act_ij = act_i && j < my_nc && st.okm[sb + j];
                    // ---- stage 1 (own variation): eliminant quartic and its root intervals
                    SideVar Bv;
                    Bv.e0 = Bv.z0 = 0.0;
                    Conic Q{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    Brackets Bk;
                    Bk.mask = 0;
                    Bk.direct = 0;
                    Bk.signs = 0;
                    if (act_ij) {
                        Bv = side_var(st.sm[sb + j], Wm, slm, smear(R.sigma[j], st.z[j][lane]), mt2_mw2);
                        Q = reflect(Bv.q, mx, my);
                        double qc[5];
                        eliminant(A.q, Q, qc);
                        Bk = quartic_brackets<T>(qc);
                    }
                    // ---- stage 2: the wave's root intervals dealt out to lanes, 64 at a time;
                    // each result goes back to the lane that owns the variation
                    const uint64_t m0 = ballot(Bk.mask & 1), m1 = ballot(Bk.mask & 2);
                    const uint64_t m2 = ballot(Bk.mask & 4), m3 = ballot(Bk.mask & 8);
                    const int n0 = popc64(m0), n1 = popc64(m1), n2 = popc64(m2), n3 = popc64(m3);
                    const int total = n0 + n1 + n2 + n3;
                    if (total == 0) continue;
                    const int packed = Bk.mask | (Bk.direct << 4) | (Bk.signs << 5);
                    // queue positions of this lane's own intervals
                    const int pos0 = popc64(m0 & lt), pos1 = n0 + popc64(m1 & lt);
                    const int pos2 = n0 + n1 + popc64(m2 & lt), pos3 = n0 + n1 + n2 + popc64(m3 & lt);
                    const int my_p = i * my_nc + j;
                    if (Bk.mask & 1) st.queue[pos0] = lane;
                    if (Bk.mask & 2) st.queue[pos1] = lane | (1 << 6);
                    if (Bk.mask & 4) st.queue[pos2] = lane | (2 << 6);
                    if (Bk.mask & 8) st.queue[pos3] = lane | (3 << 6);
                    wave_sync();
                    for (int base = 0; base < total; base += kWave) {
                        const int t = base + lane;
                        const bool live = t < total;
                        const int qe = live ? st.queue[t] : lane;
                        const int src = qe & (kWave - 1), k = qe >> 6;
                        // the source lane's intervals and event, as plain values (no aggregate
                        // whose fields get selected by k, which would force it into scratch)
                        const Poly4 fc{from_lane(Bk.c.c0, src), from_lane(Bk.c.c1, src), from_lane(Bk.c.c2, src),
                                       from_lane(Bk.c.c3, src), from_lane(Bk.c.c4, src)};
                        const double fe1 = from_lane(Bk.e1, src), fe2 = from_lane(Bk.e2, src);
                        const double fe3 = from_lane(Bk.e3, src), fbd = from_lane(Bk.bound, src);
                        const double ff1 = from_lane(Bk.f1, src), ff2 = from_lane(Bk.f2, src);
                        const double ff3 = from_lane(Bk.f3, src);
                        const int fp = from_lane(packed, src);
                        const int s_src = from_lane(ms, src), sb_src = from_lane(sb, src);
                        const double px = from_lane(A.q.x, src), py = from_lane(A.q.y, src), pc = from_lane(A.q.c, src);
                        const double qx = from_lane(Q.x, src), qy = from_lane(Q.y, src), qcc = from_lane(Q.c, src);
                        const double ae0 = from_lane(A.e0, src), be0 = from_lane(Bv.e0, src);
                        int ok = 0;
                        double w = 0.0, x = 0.0, y = 0.0;
                        if (live) {
                            ++acc_int;
                            const double *spi = st.sp[sb_src + i];
                            const double *smj = st.sm[sb_src + j];
                            const Conic P{spi[kQxx], spi[kQxy], spi[kQyy], px, py, pc};
                            const Conic Qs{smj[kQxx], smj[kQxy], smj[kQyy], qx, qy, qcc};
                            if ((fp >> 4) & 1) {  // degree <= 2: the roots are given
                                x = kXScale * (k == 0 ? fe1 : fe2);
                            } else {
                                const double f0 = (fp & 32) ? -1.0 : 1.0, f4 = (fp & 64) ? -1.0 : 1.0;
                                const double lo = k == 0 ? -fbd : k == 1 ? fe1 : k == 2 ? fe2 : fe3;
                                const double hi = k == 0 ? fe1 : k == 1 ? fe2 : k == 2 ? fe3 : fbd;
                                const double flo = k == 0 ? f0 : k == 1 ? ff1 : k == 2 ? ff2 : ff3;
                                const double fhi = k == 0 ? ff1 : k == 1 ? ff2 : k == 2 ? ff3 : f4;
                                bool found;
                                solve_interval(fc, lo, hi, flo, fhi, k > 0 && lo < fbd, k < 3 && hi < fbd, x, found);
                            }
                            if (recover_y(P, Qs, x, y) &&
                                polish_xy(P, Qs, x, y, 4, a.polish_skip_m2) <= a.accept_m2) {
                                // the source variation's smear factors and MET, rebuilt from its draws
                                const StageRec &Rs = st.rec[s_src];
                                const T zli0 = st.zl[0][src], zli1 = st.zl[1][src];
                                const T zi = st.z[i][src], zj = st.z[j][src];
                                const double rslp = smear(a.lep_sigma, zli0), rslm = smear(a.lep_sigma, zli1);
                                const double rsi = smear(Rs.sigma[i], zi), rsj = smear(Rs.sigma[j], zj);
                                const double rmx = Rs.met[0] + a.met_sigma * (double)st.zl[2][src];
                                const double rmy = Rs.met[1] + a.met_sigma * (double)st.zl[3][src];
                                const double en = spi[kE1] * x + spi[kE2] * y + ae0;
                                const double xb = rmx - x, yb = rmy - y;
                                const double eb = smj[kE1] * xb + smj[kE2] * yb + be0;
                                if (en >= 0.0 && eb >= 0.0) {
                                    const double tx = rsi * Rs.cand[i][1] + rslp * Rs.lp[1] + x;  // top pT components
                                    const double ty = rsi * Rs.cand[i][2] + rslp * Rs.lp[2] + y;
                                    const double tbx = rsj * Rs.cand[j][1] + rslm * Rs.lm[1] + xb;
                                    const double tby = rsj * Rs.cand[j][2] + rslm * Rs.lm[2] + yb;
                                    const double zz = (double)zli0 * zli0 + (double)zli1 * zli1 +
                                                      (double)st.zl[2][src] * st.zl[2][src] +
                                                      (double)st.zl[3][src] * st.zl[3][src] + (double)zi * zi +
                                                      (double)zj * zj;
                                    w = -0.5 * zz -
                                        (fast_sqrt(tx * tx + ty * ty) + fast_sqrt(tbx * tbx + tby * tby)) * a.inv_lambda;
                                    ok = 1;
                                }
                            }
                        }
                        st.res_ok[lane] = ok;
                        st.res_w[lane] = w;
                        st.res_x[lane] = x;
                        st.res_y[lane] = y;
                        wave_sync();
                        // the owner of each interval of this round takes its result
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const int pos = kk == 0 ? pos0 : kk == 1 ? pos1 : kk == 2 ? pos2 : pos3;
                            if (!((Bk.mask >> kk) & 1) || pos < base || pos >= base + kWave) continue;
                            const int q = pos - base;
                            if (!st.res_ok[q]) continue;
                            ++nsol;
                            const double rw = st.res_w[q], rx = st.res_x[q];
                            if (better(rw, my_v, my_p, rx, best_s, best_v, best_p, best_x)) {
                                best_s = rw;
                                best_v = my_v;
                                best_p = my_p;
                                best_x = rx;
                                best_y = st.res_y[q];
                            }
                        }
                        wave_sync();
                    }
                }
            }
            wave_sync();
            s_lo = s_hi;
        }

        acc_sol += (uint64_t)nsol;
        // ---- per granule (16 lanes of one event), then per event in order
#pragma unroll
        for (int off = kGran / 2; off > 0; off >>= 1) {
            const double os = __shfl_xor(best_s, off);
            const int ov = __shfl_xor(best_v, off);
            const int op = __shfl_xor(best_p, off);
            const double ox = __shfl_xor(best_x, off);
            const double oy = __shfl_xor(best_y, off);
            if (better(os, ov, op, ox, best_s, best_v, best_p, best_x)) {
                best_s = os;
                best_v = ov;
                best_p = op;
                best_x = ox;
                best_y = oy;
            }
            nsol += __shfl_xor(nsol, off);
        }
        if ((lane % kGran) == 0) {
            st.gb_s[gj] = best_s;
            st.gb_x[gj] = best_x;
            st.gb_y[gj] = best_y;
            st.gb_v[gj] = best_v;
            st.gb_p[gj] = best_p;
            st.gb_n[gj] = nsol;
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < kGpb; ++j) {
            if (slot_of[j] < 0) continue;
            const int64_t kk = kj[j];
            if (kk != open_k) {
                flush(false);
                open_k = kk;
                open_head = (b == b0 && j == 0 && sg[0] < g0);  // started before this range
                open_nc = st.rec[slot_of[j]].nc;
                acc = Acc{-INFINITY, 0.0, 0.0, kNoBest, kNoBest, 0};
            }
            const Acc gbj{st.gb_s[j], st.gb_x[j], st.gb_y[j], st.gb_v[j], st.gb_p[j], st.gb_n[j]};
            acc_merge(acc, gbj);
        }
        wave_sync();
    }
    // the open event at the end of the range: does it continue in the next range?
    if (open_k >= 0) {
        const bool cont = gofs[open_k + 1] > b1 * kGpb;
        flush(cont);
    }
    if (lane == 0) {
        part[2 * wid] = st.headp;
        part[2 * wid + 1] = st.tailp;
    }
    // intervals and variations are counted per lane
    uint64_t ni = acc_int, nv = acc_var, npr = acc_pair, nso = acc_sol;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        ni += __shfl_xor(ni, off);
        nv += __shfl_xor(nv, off);
        npr += __shfl_xor(npr, off);
        nso += __shfl_xor(nso, off);
    }
    if (lane == 0 && wstats) {
        atomicAdd((unsigned long long *)&wstats[1], (unsigned long long)nv);
        atomicAdd((unsigned long long *)&wstats[2], (unsigned long long)npr);
        atomicAdd((unsigned long long *)&wstats[3], (unsigned long long)ni);
        atomicAdd((unsigned long long *)&wstats[4], (unsigned long long)nso);
    }
}

// Search with one wavefront per event (lanes = variations in chunks of 64,
// events taken from per-class counters by a persistent grid, the next
// event's ticket and record fetched one event ahead).  Used when every event
// has the same number of variations: then no block is shared between events
// and nothing needs merging, and this form avoids the worklist's
// indirections.
template <typename T>
__global__ __launch_bounds__(kRecoBlock, 2) void k_search_ev(const int64_t *__restrict__ count, int64_t capacity,
                                                          RecoArgs a, const StageRec *__restrict__ stage,
                                                          BestRec *__restrict__ best_out,
                                                          uint64_t *__restrict__ wstats) {
    __shared__ WaveStageEv<T> stage_all[kRecoWaves];
    __shared__ int queue_all[kRecoWaves][4 * kWave];  // stage-2 queue: source lane | interval << 6
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    WaveStageEv<T> &st = stage_all[wave];
    int *queue = queue_all[wave];
    const uint64_t lt = lanemask_lt();
    const int64_t S = clamp_count(count, capacity);
    const double mt2_mw2 = a.m_t * a.m_t - a.m_w * a.m_w;
    const double mw2 = a.m_w * a.m_w;
    uint64_t acc_var = 0, acc_pair = 0, acc_int = 0, acc_sol = 0;

    // Events are handed out by counters, not dealt round robin: the cost of an
    // event varies (root intervals, iterations), and with a static deal the
    // waves' busy times spread by a sixth of the kernel.  Blocks of class c
    // (blockIdx mod ncls, which follows the round-robin placement of blocks on
    // the XCDs) take events c, c + ncls, c + 2 ncls, ... in the order of their
    // class's counter; one counter for the whole grid serialises its atomics.
    // Lane 0 takes the next ticket one event ahead and the wave reads it at
    // the top of the next event, when the atomic has long returned; the staged
    // record of that event is loaded one event ahead as well.
    const int ncls = gridDim.x < (unsigned)kTicketClasses ? (int)gridDim.x : kTicketClasses;
    const int cls = (int)(blockIdx.x % (unsigned)ncls);
    unsigned long long *ticket = reinterpret_cast<unsigned long long *>(wstats) + kTicketWord + 16 * cls;
    const uint64_t *recw = reinterpret_cast<const uint64_t *>(stage);
    constexpr int kTail = kRecWords - kWave;
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(ticket, 1ull);
    int64_t k = cls + (int64_t)ncls * (int64_t)__shfl(tk, 0);
    uint64_t w0 = 0, w1 = 0;
    if (k < S) {
        w0 = recw[k * kRecWords + lane];
        if (lane < kTail) w1 = recw[k * kRecWords + kWave + lane];
        if (lane == 0) tk = atomicAdd(ticket, 1ull);
    }
    while (k < S) {
        {
            uint64_t *dst = reinterpret_cast<uint64_t *>(&st.rec);
            dst[lane] = w0;
            if (lane < kTail) dst[kWave + lane] = w1;
        }
        const int64_t kn = cls + (int64_t)ncls * (int64_t)__shfl(tk, 0);
        if (kn < S) {
            w0 = recw[kn * kRecWords + lane];
            if (lane < kTail) w1 = recw[kn * kRecWords + kWave + lane];
            if (lane == 0) tk = atomicAdd(ticket, 1ull);
        }
        wave_sync();
        const int nc = __builtin_amdgcn_readfirstlane(st.rec.nc);
        const bool ok = nc >= 2;
        // valid sides as wave-uniform bit masks: bit c of okp / okm when the
        // l+ / l- side with candidate c is not degenerate
        uint32_t okp = 0, okm = 0;
        if (ok) {
            // side constants: lanes [0, nc) with l+, lanes [16, 16 + nc) with l-
            bool side_ok = false;
            if (lane < nc) {
                side_ok = make_side(st.rec.lp, st.rec.cand[lane], st.sp[lane]);
            } else if (lane >= 16 && lane < 16 + nc) {
                const int c = lane - 16;
                side_ok = make_side(st.rec.lm, st.rec.cand[c], st.sm[c]);
            }
            const uint64_t okb = ballot(side_ok);
            okp = (uint32_t)okb & 0xffffu;
            okm = (uint32_t)(okb >> 16) & 0xffffu;
            wave_sync();
        }

        // ------------------------------------------------------- variations
        const int V = __builtin_amdgcn_readfirstlane(st.rec.V);
        double best_s = -INFINITY, best_x = 0.0, best_y = 0.0;
        int best_v = kNoBest, best_p = kNoBest;
        int nsol = 0;
        // ordered pairings (i, j), i != j, with both sides valid
        const int npair_valid = __popc(okp) * __popc(okm) - __popc(okp & okm);
        if (npair_valid > 0) {
            const double metx = st.rec.met[0], mety = st.rec.met[1];
            const uint64_t g = st.rec.g;
            for (int vb = 0; vb < V; vb += kWave) {
                const int v = vb + lane;
                const bool act = v < V;
                // ---- draws of this lane's variation, kept in LDS so that any lane can
                // rebuild another lane's smear factors
                {
                    T zl[4] = {(T)0, (T)0, (T)0, (T)0};
                    if (a.smear && act) {
                        gauss_block<T>(a.seed, g, (uint32_t)v, 0u, zl);
                        uint32_t last_blk = 0xffffffffu;
                        T zb[4];
                        for (int c = 0; c < nc; ++c) {
                            const uint32_t slot = 4u + (uint32_t)st.rec.jidx[c];
                            const uint32_t blk = slot >> 2;
                            if (blk != last_blk) {
                                gauss_block<T>(a.seed, g, (uint32_t)v, blk, zb);
                                last_blk = blk;
                            }
                            const uint32_t ln = slot & 3u;
                            st.z[c][lane] = ln == 0 ? zb[0] : ln == 1 ? zb[1] : ln == 2 ? zb[2] : zb[3];
                        }
                    } else {
                        for (int c = 0; c < nc; ++c) st.z[c][lane] = (T)0;
                    }
                    st.zl[0][lane] = zl[0];
                    st.zl[1][lane] = zl[1];
                    st.zl[2][lane] = zl[2];
                    st.zl[3][lane] = zl[3];
                }
                wave_sync();
                const double slp = smear(a.lep_sigma, st.zl[0][lane]);
                const double slm = smear(a.lep_sigma, st.zl[1][lane]);
                const double mx = metx + a.met_sigma * (double)st.zl[2][lane];
                const double my = mety + a.met_sigma * (double)st.zl[3][lane];
                const double Wp = (0.5 * mw2) * fast_rcp(slp) - 0.5 * slp * st.rec.ml2p;
                const double Wm = (0.5 * mw2) * fast_rcp(slm) - 0.5 * slm * st.rec.ml2m;
                for (int i = 0; i < nc; ++i) {
                    if (!((okp >> i) & 1u)) continue;
                    const double si = smear(st.rec.sigma[i], st.z[i][lane]);
                    const SideVar A = side_var(st.sp[i], Wp, slp, si, mt2_mw2);
                    for (int j = 0; j < nc; ++j) {
                        if (j == i || !((okm >> j) & 1u)) continue;
                        // ---- stage 1 (own variation): eliminant quartic and its root intervals
                        const double sj = smear(st.rec.sigma[j], st.z[j][lane]);
                        const SideVar Bv = side_var(st.sm[j], Wm, slm, sj, mt2_mw2);
                        const Conic Q = reflect(Bv.q, mx, my);
                        Brackets Bk;
                        Bk.mask = 0;
                        if (act) {
                            double qc[5];
                            eliminant(A.q, Q, qc);
                            Bk = quartic_brackets<T>(qc);
                        }
                        // ---- stage 2: the wave's root intervals dealt out to lanes, 64 at a time
                        const uint64_t m0 = ballot(Bk.mask & 1), m1 = ballot(Bk.mask & 2);
                        const uint64_t m2 = ballot(Bk.mask & 4), m3 = ballot(Bk.mask & 8);
                        const int n0 = popc64(m0), n1 = popc64(m1), n2 = popc64(m2), n3 = popc64(m3);
                        const int total = n0 + n1 + n2 + n3;
                        if (total == 0) continue;
                        const int p = i * nc + j;
                        const int packed = Bk.mask | (Bk.direct << 4) | (Bk.signs << 5);
                        // the queue: every interval 0 in lane order, then every interval 1, ...
                        if (Bk.mask & 1) queue[popc64(m0 & lt)] = lane;
                        if (Bk.mask & 2) queue[n0 + popc64(m1 & lt)] = lane | (1 << 6);
                        if (Bk.mask & 4) queue[n0 + n1 + popc64(m2 & lt)] = lane | (2 << 6);
                        if (Bk.mask & 8) queue[n0 + n1 + n2 + popc64(m3 & lt)] = lane | (3 << 6);
                        wave_sync();
                        for (int base = 0; base < total; base += kWave) {
                            const int t = base + lane;
                            const bool live = t < total;
                            const int qe = live ? queue[t] : lane;
                            const int src = qe & (kWave - 1), k = qe >> 6;
                            // the source lane's intervals, as plain values (no aggregate whose
                            // fields get selected by k, which would force it into scratch)
                            const Poly4 fc{from_lane(Bk.c.c0, src), from_lane(Bk.c.c1, src),
                                           from_lane(Bk.c.c2, src), from_lane(Bk.c.c3, src),
                                           from_lane(Bk.c.c4, src)};
                            const double fe1 = from_lane(Bk.e1, src), fe2 = from_lane(Bk.e2, src);
                            const double fe3 = from_lane(Bk.e3, src), fbd = from_lane(Bk.bound, src);
                            const double ff1 = from_lane(Bk.f1, src), ff2 = from_lane(Bk.f2, src);
                            const double ff3 = from_lane(Bk.f3, src);
                            const int fp = from_lane(packed, src);
                            const Conic P{st.sp[i][kQxx], st.sp[i][kQxy], st.sp[i][kQyy], from_lane(A.q.x, src),
                                          from_lane(A.q.y, src), from_lane(A.q.c, src)};
                            const Conic Qs{Q.xx, Q.xy, Q.yy, from_lane(Q.x, src), from_lane(Q.y, src),
                                           from_lane(Q.c, src)};
                            const double ae0 = from_lane(A.e0, src), be0 = from_lane(Bv.e0, src);
                            // accepted solutions are counted per pass with a ballot
                            bool accepted = false;
                            double x = 0.0, y = 0.0;
                            if (live) {
                                if ((fp >> 4) & 1) {  // degree <= 2: the roots are given
                                    x = kXScale * (k == 0 ? fe1 : fe2);
                                } else {
                                    const double f0 = (fp & 32) ? -1.0 : 1.0, f4 = (fp & 64) ? -1.0 : 1.0;
                                    const double lo = k == 0 ? -fbd : k == 1 ? fe1 : k == 2 ? fe2 : fe3;
                                    const double hi = k == 0 ? fe1 : k == 1 ? fe2 : k == 2 ? fe3 : fbd;
                                    const double flo = k == 0 ? f0 : k == 1 ? ff1 : k == 2 ? ff2 : ff3;
                                    const double fhi = k == 0 ? ff1 : k == 1 ? ff2 : k == 2 ? ff3 : f4;
                                    bool found;
                                    solve_interval(fc, lo, hi, flo, fhi, k > 0 && lo < fbd, k < 3 && hi < fbd, x,
                                                   found);
                                }
                                accepted = recover_y(P, Qs, x, y) &&
                                           polish_xy(P, Qs, x, y, 4, a.polish_skip_m2) <= a.accept_m2;
                            }
                            if (accepted) {
                                // the source variation's smear factors and MET, rebuilt from its draws
                                const T zli0 = st.zl[0][src], zli1 = st.zl[1][src];
                                const T zi = st.z[i][src], zj = st.z[j][src];
                                const double rslp = smear(a.lep_sigma, zli0), rslm = smear(a.lep_sigma, zli1);
                                const double rsi = smear(st.rec.sigma[i], zi), rsj = smear(st.rec.sigma[j], zj);
                                const double rmx = metx + a.met_sigma * (double)st.zl[2][src];
                                const double rmy = mety + a.met_sigma * (double)st.zl[3][src];
                                const double en = st.sp[i][kE1] * x + st.sp[i][kE2] * y + ae0;
                                const double xb = rmx - x, yb = rmy - y;
                                const double eb = st.sm[j][kE1] * xb + st.sm[j][kE2] * yb + be0;
                                accepted = en >= 0.0 && eb >= 0.0;
                                if (accepted) {
                                    // top pT components
                                    const double tx = rsi * st.rec.cand[i][1] + rslp * st.rec.lp[1] + x;
                                    const double ty = rsi * st.rec.cand[i][2] + rslp * st.rec.lp[2] + y;
                                    const double tbx = rsj * st.rec.cand[j][1] + rslm * st.rec.lm[1] + xb;
                                    const double tby = rsj * st.rec.cand[j][2] + rslm * st.rec.lm[2] + yb;
                                    const double zz = (double)zli0 * zli0 + (double)zli1 * zli1 +
                                                      (double)st.zl[2][src] * st.zl[2][src] +
                                                      (double)st.zl[3][src] * st.zl[3][src] + (double)zi * zi +
                                                      (double)zj * zj;
                                    const double w =
                                        -0.5 * zz -
                                        (fast_sqrt(tx * tx + ty * ty) + fast_sqrt(tbx * tbx + tby * tby)) * a.inv_lambda;
                                    const int vs = vb + src;
                                    if (better(w, vs, p, x, best_s, best_v, best_p, best_x)) {
                                        best_s = w;
                                        best_v = vs;
                                        best_p = p;
                                        best_x = x;
                                        best_y = y;
                                    }
                                }
                            }
                            nsol += popc64(ballot(accepted));
                        }
                        wave_sync();  // the next pairing rewrites the queue
                        acc_int += (uint64_t)total;
                    }
                }
                wave_sync();
            }
        }
        // --------------------------------------------------- wave argmax
        // better() is a total order, so any pairing of lanes that reaches all
        // of them gives every lane the maximum: four in-row DPP steps (pairs,
        // quads, eights, rows), then across rows by shuffles
        auto take = [&](double os, int ov, int op, double ox, double oy) {
            if (better(os, ov, op, ox, best_s, best_v, best_p, best_x)) {
                best_s = os;
                best_v = ov;
                best_p = op;
                best_x = ox;
                best_y = oy;
            }
        };
        take(dpp_f64<0xB1>(best_s), dpp_i32<0xB1>(best_v), dpp_i32<0xB1>(best_p), dpp_f64<0xB1>(best_x),
             dpp_f64<0xB1>(best_y));
        take(dpp_f64<0x4E>(best_s), dpp_i32<0x4E>(best_v), dpp_i32<0x4E>(best_p), dpp_f64<0x4E>(best_x),
             dpp_f64<0x4E>(best_y));
        take(dpp_f64<0x141>(best_s), dpp_i32<0x141>(best_v), dpp_i32<0x141>(best_p), dpp_f64<0x141>(best_x),
             dpp_f64<0x141>(best_y));
        take(dpp_f64<0x140>(best_s), dpp_i32<0x140>(best_v), dpp_i32<0x140>(best_p), dpp_f64<0x140>(best_x),
             dpp_f64<0x140>(best_y));
        for (int off = 16; off < kWave; off <<= 1)
            take(__shfl_xor(best_s, off), __shfl_xor(best_v, off), __shfl_xor(best_p, off), __shfl_xor(best_x, off),
                 __shfl_xor(best_y, off));
        acc_var += (uint64_t)V;
        acc_pair += (uint64_t)V * (uint64_t)npair_valid;
        acc_sol += (uint64_t)nsol;
        if (lane == 0) {
            BestRec r;
            r.score = best_s;
            r.x = best_x;
            r.y = best_y;
            r.v = best_v;
            r.p = best_p;
            r.nsol = nsol;
            r.nc = nc;
            best_out[k] = r;
        }
        wave_sync();
        k = kn;
    }
    if (lane == 0) {
        atomicAdd((unsigned long long *)&wstats[1], (unsigned long long)acc_var);
        atomicAdd((unsigned long long *)&wstats[2], (unsigned long long)acc_pair);
        atomicAdd((unsigned long long *)&wstats[3], (unsigned long long)acc_int);
        atomicAdd((unsigned long long *)&wstats[4], (unsigned long long)acc_sol);
    }
}


// One thread per search wavefront: an event that continues past the end of
// the wavefront's range is merged with the head records of the following
// ranges (in order) and its best record written.
__global__ __launch_bounds__(256) void k_fixup(const PartRec *__restrict__ part, int64_t nw,
                                               BestRec *__restrict__ best_out) {
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= nw) return;
    const PartRec t = part[2 * w + 1];
    if (t.k < 0) return;
    Acc acc{t.score, t.x, t.y, t.v, t.p, t.nsol};
    for (int64_t w2 = w + 1; w2 < nw; ++w2) {
        const PartRec h = part[2 * w2];
        if (h.k == -2) continue;  // empty range
        if (h.k != t.k) break;
        acc_merge(acc, Acc{h.score, h.x, h.y, h.v, h.p, h.nsol});
        if (!h.cont) break;
    }
    BestRec r;
    r.score = acc.s;
    r.x = acc.x;
    r.y = acc.y;
    r.v = acc.v;
    r.p = acc.p;
    r.nsol = acc.n;
    r.nc = t.nc;
    best_out[t.k] = r;
}

__global__ void k_reco_init(uint64_t *wstats) {
    if (threadIdx.x < 5) wstats[threadIdx.x] = 0;
    if (threadIdx.x < kTicketClasses) wstats[kTicketWord + 16 * threadIdx.x] = 0;
}

__device__ __forceinline__ double mass4(double E, double X, double Y, double Z) {
    const double m2 = E * E - X * X - Y * Y - Z * Z;
    return m2 > 0.0 ? sqrt(m2) : 0.0;
}

// One thread per compacted event: outputs of the chosen solution, the
// H -> bb candidate, and the RECO counters (one atomic per block).
template <typename T>
__global__ __launch_bounds__(256) void k_epilogue(EvView ev, const int64_t *__restrict__ count, int64_t capacity,
                                                  RecoArgs a, const StageRec *__restrict__ stage,
                                                  const BestRec *__restrict__ best, RecoOutView out,
                                                  hf_counters_t *__restrict__ counter, const uint64_t *wstats) {
    __shared__ uint32_t s_pass[256 / kWave];
    const int64_t S = clamp_count(count, capacity);
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool have = false;
    if (k < S) {
        const BestRec r = best[k];
        have = r.v != kNoBest;
        out.has_sol[k] = have ? 1 : 0;
        out.n_sol[k] = r.nsol;
        if (!have) {
            out.best_v[k] = -1;
            out.best_i[k] = -1;
            out.best_j[k] = -1;
            for (int q = 0; q < 3; ++q) out.nu[3 * k + q] = out.nubar[3 * k + q] = HF_NO_SOLUTION;
            out.m_t[k] = out.m_tbar[k] = out.m_wp[k] = out.m_wm[k] = out.logw[k] = HF_NO_SOLUTION;
            if (out.m_bb) out.m_bb[k] = HF_NO_SOLUTION;
        } else {
            const StageRec &rec = stage[k];
            const uint64_t g = rec.g;
            const int64_t e = (int64_t)g - ev.index_base;  // in the chunk: a solution exists
            // the r.p-th ordered pair of the candidate list
            const int nc = r.nc, ci = r.p / nc, cj = r.p % nc;
            const int jidx[2] = {rec.jidx[ci], rec.jidx[cj]};
            double lp[4], lm[4], b[4], bb[4];
            for (int q = 0; q < 4; ++q) {
                lp[q] = rec.lp[q];
                lm[q] = rec.lm[q];
                b[q] = rec.cand[ci][q];
                bb[q] = rec.cand[cj][q];
            }
            double sp[kSide], sm[kSide];
            make_side(lp, b, sp);
            make_side(lm, bb, sm);
            T zl[4] = {(T)0, (T)0, (T)0, (T)0};
            T zi = (T)0, zj = (T)0;
            if (a.smear) {
                gauss_block<T>(a.seed, g, (uint32_t)r.v, 0u, zl);
                zi = gauss_slot<T>(a.seed, g, (uint32_t)r.v, 4u + (uint32_t)jidx[0]);
                zj = gauss_slot<T>(a.seed, g, (uint32_t)r.v, 4u + (uint32_t)jidx[1]);
            }
            const double slp = smear(a.lep_sigma, zl[0]), slm = smear(a.lep_sigma, zl[1]);
            const double si = smear(rec.sigma[ci], zi), sj = smear(rec.sigma[cj], zj);
            const double mx = rec.met[0] + a.met_sigma * (double)zl[2];
            const double my = rec.met[1] + a.met_sigma * (double)zl[3];
            const double mw2 = a.m_w * a.m_w, mt2_mw2 = a.m_t * a.m_t - mw2;
            const double ml2p = rec.ml2p, ml2m = rec.ml2m;
            const SideVar A = side_var(sp, (0.5 * mw2) * fast_rcp(slp) - 0.5 * slp * ml2p, slp, si, mt2_mw2);
            const SideVar Bv = side_var(sm, (0.5 * mw2) * fast_rcp(slm) - 0.5 * slm * ml2m, slm, sj, mt2_mw2);
            const double x = r.x, y = r.y, xb = mx - x, yb = my - y;
            const double nu[4] = {sp[kE1] * x + sp[kE2] * y + A.e0, x, y, sp[kZ1] * x + sp[kZ2] * y + A.z0};
            const double nb[4] = {sm[kE1] * xb + sm[kE2] * yb + Bv.e0, xb, yb, sm[kZ1] * xb + sm[kZ2] * yb + Bv.z0};
            for (int q = 0; q < 4; ++q) {
                lp[q] *= slp;
                lm[q] *= slm;
                b[q] *= si;
                bb[q] *= sj;
            }
            out.best_v[k] = r.v;
            out.best_i[k] = (int16_t)jidx[0];
            out.best_j[k] = (int16_t)jidx[1];
            out.nu[3 * k + 0] = nu[1];
            out.nu[3 * k + 1] = nu[2];
            out.nu[3 * k + 2] = nu[3];
            out.nubar[3 * k + 0] = nb[1];
            out.nubar[3 * k + 1] = nb[2];
            out.nubar[3 * k + 2] = nb[3];
            out.m_wp[k] = mass4(lp[0] + nu[0], lp[1] + nu[1], lp[2] + nu[2], lp[3] + nu[3]);
            out.m_wm[k] = mass4(lm[0] + nb[0], lm[1] + nb[1], lm[2] + nb[2], lm[3] + nb[3]);
            out.m_t[k] = mass4(b[0] + lp[0] + nu[0], b[1] + lp[1] + nu[1], b[2] + lp[2] + nu[2], b[3] + lp[3] + nu[3]);
            out.m_tbar[k] =
                mass4(bb[0] + lm[0] + nb[0], bb[1] + lm[1] + nb[1], bb[2] + lm[2] + nb[2], bb[3] + lm[3] + nb[3]);
            out.logw[k] = r.score;
            if (out.m_bb) {
                // H -> b bbar from the remaining jets (section 4): the two leading remaining
                // b-tagged selected jets; with only one, the leading remaining untagged one joins it.
                double mbb = HF_NO_SOLUTION;
                if (a.want_mbb) {
                    const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
                    const uint32_t bi = j0 + (uint32_t)jidx[0], bj = j0 + (uint32_t)jidx[1];
                    uint32_t pick[2] = {0, 0};
                    int got = 0;
                    for (uint32_t q = j0; q < j1 && got < 2; ++q)
                        if (q != bi && q != bj && jet_sel(ev, q, a) && ev.jet_btag[q] > a.btag_min) pick[got++] = q;
                    if (got == 1)
                        for (uint32_t q = j0; q < j1 && got < 2; ++q)
                            if (q != bi && q != bj && jet_sel(ev, q, a) && !(ev.jet_btag[q] > a.btag_min))
                                pick[got++] = q;
                    if (got == 2) {
                        double p0[4], p1[4];
                        polar_to_cart(ev.jet_pt[pick[0]], ev.jet_eta[pick[0]], ev.jet_phi[pick[0]], ev.jet_e[pick[0]],
                                      p0);
                        polar_to_cart(ev.jet_pt[pick[1]], ev.jet_eta[pick[1]], ev.jet_phi[pick[1]], ev.jet_e[pick[1]],
                                      p1);
                        mbb = mass4(p0[0] + p1[0], p0[1] + p1[1], p0[2] + p1[2], p0[3] + p1[3]);
                    }
                }
                out.m_bb[k] = mbb;
            }
        }
    }
    // RECO counters: reached += S (once), passed += events with a solution
    const uint64_t m = ballot(have);
    if (lane_id() == 0) s_pass[threadIdx.x / kWave] = (uint32_t)popc64(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (int w = 0; w < 256 / kWave; ++w) tot += s_pass[w];
        if (counter && tot) atomicAdd((unsigned long long *)&counter->passed, (unsigned long long)tot);
        if (blockIdx.x == 0) {
            if (counter) atomicAdd((unsigned long long *)&counter->reached, (unsigned long long)S);
            if (out.stats) {
                atomicAdd((unsigned long long *)&out.stats[0], (unsigned long long)S);
                for (int q = 1; q < 5; ++q) atomicAdd((unsigned long long *)&out.stats[q], (unsigned long long)wstats[q]);
            }
        }
    }
}

// Persistent grid: the resident blocks of one kernel on every CU.
int resident_grid(const void *kernel, int *cache) {
    if (*cache <= 0) {
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
        if (n_cu <= 0) n_cu = 256;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kRecoBlock, 0) != hipSuccess || nb < 1) nb = 1;
        int64_t g = (int64_t)n_cu * nb;
        if (g > kMaxSearchWaves / kRecoWaves) g = kMaxSearchWaves / kRecoWaves;
        *cache = (int)g;
    }
    return *cache;
}

hipEvent_t g_time_start = nullptr, g_time_stop = nullptr;

// Workspace layout (each part 256-byte aligned): counters, BestRec[capacity],
// StageRec[capacity], granule counts int32[capacity], granule offsets
// int64[capacity + 1], tile sums int64[tiles + 1], PartRec[2 kMaxSearchWaves].
struct WsLayout {
    size_t best, stage, gcnt, gofs, tsum, part, total;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static WsLayout ws_layout(int64_t capacity) {
    const size_t c = (size_t)(capacity > 0 ? capacity : 0);
    const size_t tiles = (c + kScanTile - 1) / kScanTile + 1;
    WsLayout L;
    L.best = kWsHeader;
    L.stage = align256(L.best + c * sizeof(BestRec));
    L.gcnt = align256(L.stage + c * sizeof(StageRec));
    L.gofs = align256(L.gcnt + c * sizeof(int32_t));
    L.tsum = align256(L.gofs + (c + 1) * sizeof(int64_t));
    L.part = align256(L.tsum + (tiles + 1) * sizeof(int64_t));
    L.total = align256(L.part + 2 * (size_t)kMaxSearchWaves * sizeof(PartRec));
    return L;
}

// worklist: the packed / split schedule (per-event variation counts); else one
// wavefront per event.
template <typename T>
hipError_t launch_t(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity, const RecoArgs &a,
                    const RecoOutView &out, hf_counters_t *reco_counter, uint64_t *wstats, char *ws, bool worklist,
                    hipStream_t s) {
    const WsLayout L = ws_layout(capacity);
    BestRec *best = reinterpret_cast<BestRec *>(ws + L.best);
    StageRec *stage = reinterpret_cast<StageRec *>(ws + L.stage);
    int32_t *gcnt = reinterpret_cast<int32_t *>(ws + L.gcnt);
    int64_t *gofs = reinterpret_cast<int64_t *>(ws + L.gofs);
    int64_t *tsum = reinterpret_cast<int64_t *>(ws + L.tsum);
    PartRec *part = reinterpret_cast<PartRec *>(ws + L.part);
    const int64_t eg = capacity > 0 ? (capacity + 255) / 256 : 1;
    const int64_t sg = capacity > 0 ? (capacity + kStageEvents - 1) / kStageEvents : 1;
    if (capacity > 0) {
        const unsigned tiles = (unsigned)((capacity + kScanTile - 1) / kScanTile);
        hipLaunchKernelGGL(k_stage, dim3((unsigned)sg), dim3(256), 0, s, ev, idx, count, capacity, a, stage, gcnt,
                           best);
        if (worklist) {
            hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(256), 0, s, gcnt, count, capacity, tsum);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, count, capacity, tsum);
            hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(256), 0, s, gcnt, count, capacity, tsum, gofs);
        }
        hipError_t e1 = hipGetLastError();
        if (e1 != hipSuccess) return e1;
        if (g_time_start) {
            const hipError_t e0 = hipEventRecord(g_time_start, s);
            if (e0 != hipSuccess) return e0;
        }
        hipError_t err;
        if (!worklist) {
            // every event has the same number of variations: one wavefront per event
            static int grid_ev = 0;
            int64_t g = resident_grid(reinterpret_cast<const void *>(&k_search_ev<T>), &grid_ev);
            const int64_t need = (capacity + kRecoWaves - 1) / kRecoWaves;
            g = g < need ? g : need;
            hipLaunchKernelGGL(k_search_ev<T>, dim3((unsigned)(g < 1 ? 1 : g)), dim3(kRecoBlock), 0, s, count,
                               capacity, a, stage, best, wstats);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
            if (g_time_stop) {
                err = hipEventRecord(g_time_stop, s);
                if (err != hipSuccess) return err;
            }
        } else {
            static int grid_wl = 0;
            const int grid = resident_grid(reinterpret_cast<const void *>(&k_search<T>), &grid_wl);
            hipLaunchKernelGGL(k_search<T>, dim3(grid), dim3(kRecoBlock), 0, s, count, capacity, a, stage, gofs,
                               best, part, wstats);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
            if (g_time_stop) {
                err = hipEventRecord(g_time_stop, s);
                if (err != hipSuccess) return err;
            }
            const int64_t nw = (int64_t)grid * kRecoWaves;
            hipLaunchKernelGGL(k_fixup, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, part, nw, best);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
    }
    hipLaunchKernelGGL(k_epilogue<T>, dim3((unsigned)eg), dim3(256), 0, s, ev, count, capacity, a, stage, best, out,
                       reco_counter, wstats);
    return hipGetLastError();
}

}  // namespace

void set_reco_timing(hipEvent_t start, hipEvent_t stop) {
    g_time_start = start;
    g_time_stop = stop;
}

size_t reco_ws_bytes(int64_t capacity) { return ws_layout(capacity).total; }

hipError_t launch_reco(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity,
                       const RecoArgs &a, int precision, const RecoOutView &out, hf_counters_t *reco_counter,
                       void *ws, bool worklist, hipStream_t s) {
    uint64_t *wstats = static_cast<uint64_t *>(ws);
    hipLaunchKernelGGL(k_reco_init, dim3(1), dim3(64), 0, s, wstats);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    char *w = static_cast<char *>(ws);
    if (precision == HF_PREC_MIXED)
        return launch_t<float>(ev, idx, count, capacity, a, out, reco_counter, wstats, w, worklist, s);
    return launch_t<double>(ev, idx, count, capacity, a, out, reco_counter, wstats, w, worklist, s);
}

}  // namespace hf
