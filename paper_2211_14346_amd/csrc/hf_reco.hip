// Dileptonic ttbar kinematic reconstruction over the compacted events
// (paper section 4: W and top mass constraints for every lepton / b-jet
// pairing, over resolution-smeared pseudo-experiments, the most probable
// solution kept; the event fails the last cut when no solution exists).
//
// Kernels, in launch order.
//
// k_stage: eight lanes per compacted event; selects the leptons and b
// candidates, writes their FP64 Cartesian 4-vectors to a record and an
// empty best record.
//
// k_search_ev: persistent grid, one wavefront per event (events taken from
// per-class counters).  The wavefront copies the event's record into LDS and
// adds, per candidate and lepton side, the constants of the linear maps and
// of the conic's quadratic part.  Lanes run over the variations, 64 at a
// time.  Each lane draws its variation (Philox4x32-10 + Box-Muller in
// precision T) and, for every pairing, intersects its two conics through
// their pencil in FP64 (the degenerate member from the isolated root of the
// pencil cubic, seeded in T; its line pair; each line against the l+ conic),
// then checks each common point's residual (polishing the rare inaccurate
// one), the acceptance bound, the energies' signs and the score.  A wave
// maximum of the score, with a total-order tie-break (score, then smallest
// variation, pairing, x) where lanes tie, gives the event's winner.
// Instantiated for workgroups of one, two and four wavefronts (a launch
// choice that leaves every result unchanged; the autotuner times them).
//
// k_epilogue: one thread per event; recomputes the winner's kinematics in
// FP64 (draws recomputed bit-identically in T), writes the outputs, the
// H -> bb candidate mass, and folds the RECO counters.
//
// T = float (HF_PREC_MIXED): draws and the cubic's seed in FP32.
// T = double (HF_PREC_FP64): everything in FP64.
#include <math.h>

#include "hf_device.hpp"
#include "hf_internal.hpp"
#include "hf_reco_math.hpp"

namespace hf {
namespace {

constexpr int kMaxC = HF_MAX_CANDS;
constexpr int kNoBest = 0x7fffffff;
constexpr size_t kWsHeader = 2048;
// Event counters of the one-wavefront-per-event search: kTicketClasses of
// them at words kTicketWord + 16 c of the workspace header, each on its own
// 128-byte line.
constexpr int kTicketWord = 16;
constexpr int kTicketClasses = 8;

// Per-event result of the search, read by the epilogue.
struct BestRec {
    double score, x, y;
    int32_t v, p, nsol, nc;
};

// One compacted event as the reconstruction sees it, built by k_stage: the
// two selected leptons and the b candidates as nominal FP64 (E, px, py, pz),
// in the order of the candidate rule; nc = 0 when the lepton selection
// fails (or the id lies outside the chunk).  The used part is contiguous: a
// 14-word header, then 6 words per candidate (k_stage writes only those;
// the search kernel reads the header and three candidates ahead of time and
// the rest, for an event with more candidates, when it gets to it).
struct CandRec {
    double v[4];    // nominal (E, px, py, pz)
    double sigma;   // jet energy resolution at the nominal energy
    int32_t jidx;   // jet index within the event
    int32_t pad;
};
struct StageRec {
    double lp[4], lm[4];    // l+ and l-
    double met[2];          // nominal MET x, y
    double ml2p, ml2m;      // squared masses of l+ and l-
    uint64_t g;             // global event id (the generator's counter)
    int32_t nc, V;          // number of candidates, of variations
    CandRec cand[kMaxC];    // b candidates
};
constexpr int kRecWords = (int)(sizeof(StageRec) / 8);
constexpr int kHeadWords = 14, kCandWords = 6;
constexpr int kPrefetchWords = kHeadWords + 3 * kCandWords;  // header and three candidates
static_assert(sizeof(CandRec) == 8 * kCandWords && offsetof(StageRec, cand) == 8 * kHeadWords &&
                  kRecWords <= kPrefetchWords + kWave && kPrefetchWords <= kWave,
              "record layout");

template <typename T>
struct WaveStageEv {
    StageRec rec;
    double sp[kMaxC][kSide];  // side constants with l+
    double sm[kMaxC][kSide];  // side constants with l-
    T z[kMaxC][kWave];  // per-lane draw of each candidate
    T zl[4][kWave];     // per-lane draws of l+, l-, MET x, MET y
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

__device__ __forceinline__ bool jet_sel(const EvView &ev, uint32_t k, const RecoArgs &a) {
    return ev.jet_pt[k] > a.jet_pt_min && fabsf(ev.jet_eta[k]) < a.jet_eta_max;
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
// event take its objects eight at a time, leptons then jets, and load every
// column of an object at once; ballots restricted to the event's eight bits
// give the selection, the candidates' order and the first untagged jets, and
// each object the record needs is converted on the lane that holds it:
// candidates straight into the record, the first two selected leptons and
// the two fill jets into LDS until the charges and the candidate count are
// known.  So an event costs three dependent loads (id, offsets, columns), and
// spreading it over lanes keeps many wavefronts in flight to hide them.
constexpr int kStageLanes = 8;
constexpr int kStageEvents = 256 / kStageLanes;  // events per block

__global__ __launch_bounds__(256) void k_stage(EvView ev, const int32_t *__restrict__ idx,
                                               const int64_t *__restrict__ count, int64_t capacity, RecoArgs a,
                                               StageRec *__restrict__ stage,
                                               BestRec *__restrict__ best) {
    __shared__ double s_lv[kStageEvents][2][4];  // the first two selected leptons, by rank
    __shared__ float s_lq[kStageEvents][2];      // and their charges
    __shared__ double s_fv[kStageEvents][2][5];  // the first two untagged selected jets: 4-vector, sigma
    __shared__ int32_t s_fj[kStageEvents][2];    // and their indices
    const int lane = lane_id(), sub = lane & (kStageLanes - 1);
    const int slot = threadIdx.x / kStageLanes;
    const int shift = lane & ~(kStageLanes - 1);     // the event's first lane in the wave
    const uint32_t below = (1u << sub) - 1u;         // lanes of this event below this one
    const int64_t S = clamp_count(count, capacity);
    const int64_t k = (int64_t)blockIdx.x * kStageEvents + slot;
    if (k >= S) return;  // whole events only: the eight lanes of an event leave together
    StageRec &r = stage[k];
    const uint64_t g = (uint64_t)idx[k];
    const int64_t e = (int64_t)g - ev.index_base;
    const bool in_chunk = e >= 0 && e < ev.n;  // ids outside the chunk get no solution
    auto bits = [&](bool p) { return (uint32_t)((ballot(p) >> shift) & 0xffu); };
    const bool all = a.pair_mode == HF_PAIR_ALL_JETS;
    int nl = 0, nc = 0, nfill = 0, V = 0;
    float mx = 0.0f, my = 0.0f;
    if (in_chunk) {
        const uint32_t l0 = ev.lep_off[e], l1 = ev.lep_off[e + 1];
        const uint32_t j0 = ev.jet_off[e], j1 = ev.jet_off[e + 1];
        V = ev.n_var ? (int)ev.n_var[e] : a.n_var_uniform;
        mx = ev.met_x[e];
        my = ev.met_y[e];
        const uint32_t nlep = l1 > l0 ? l1 - l0 : 0u, nobj = nlep + (j1 > j0 ? j1 - j0 : 0u);
        const int cap = a.max_cands < kMaxC ? a.max_cands : kMaxC;
        for (uint32_t c0 = 0; c0 < nobj; c0 += kStageLanes) {
            const uint32_t o = c0 + (uint32_t)sub;
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
            const uint32_t ml = bits(lsel), mt = bits(jsel && tag), mu = bits(jsel && !tag);
            const int lrank = nl + __popc(ml & below);
            const int pos = nc + __popc(mt & below);
            const int frank = nfill + __popc(mu & below);
            const bool wl = lsel && lrank < 2, wc = jsel && tag && pos < cap, wf = jsel && !tag && frank < 2;
            if (wl || wc || wf) {
                double v[4];
                polar_to_cart(pt, eta, phi, en, v);
                if (wl) {
                    for (int c = 0; c < 4; ++c) s_lv[slot][lrank][c] = v[c];
                    s_lq[slot][lrank] = aux;
                } else {
                    const double sg = sqrt(a.jet_a * a.jet_a / (double)en + a.jet_c * a.jet_c);
                    const int32_t jx = (int32_t)(q - j0);
                    if (wc) {
                        for (int c = 0; c < 4; ++c) r.cand[pos].v[c] = v[c];
                        r.cand[pos].sigma = sg;
                        r.cand[pos].jidx = jx;
                    } else {
                        for (int c = 0; c < 4; ++c) s_fv[slot][frank][c] = v[c];
                        s_fv[slot][frank][4] = sg;
                        s_fj[slot][frank] = jx;
                    }
                }
            }
            nl += __popc(ml);
            nc = min(cap, nc + __popc(mt));
            nfill += __popc(mu);
        }
    }
    wave_sync();  // the leptons and fill jets were written by other lanes
    bool lep_ok = false;
    int pr = 0;  // rank of l+ among the two selected leptons
    if (nl == 2) {
        const float qa = s_lq[slot][0], qb = s_lq[slot][1];
        lep_ok = qa * qb < 0.0f;
        pr = qa > 0.0f ? 0 : 1;
    }
    if (!lep_ok) nc = 0;
    // ---- the record: leptons by lanes 0 and 1; fewer than two candidates: the
    // leading untagged selected jets fill, one per lane
    if (nc > 0 || (lep_ok && nfill > 0 && !all)) {
        const int nf = (all || nc >= 2) ? 0 : min(nfill, 2 - nc);
        if (sub < nf) {
            CandRec &cd = r.cand[nc + sub];
            for (int c = 0; c < 4; ++c) cd.v[c] = s_fv[slot][sub][c];
            cd.sigma = s_fv[slot][sub][4];
            cd.jidx = s_fj[slot][sub];
        }
        nc += nf;
        if (sub < 2) {
            const double *v = s_lv[slot][sub == 0 ? pr : 1 - pr];
            double *dst = sub == 0 ? r.lp : r.lm;
            for (int c = 0; c < 4; ++c) dst[c] = v[c];
            const double m2 = v[0] * v[0] - v[1] * v[1] - v[2] * v[2] - v[3] * v[3];
            if (sub == 0) r.ml2p = m2;
            else r.ml2m = m2;
        }
    }
    if (sub == 2) {
        r.g = g;
        if (in_chunk) {
            r.met[0] = (double)mx;
            r.met[1] = (double)my;
        }
        r.nc = nc;
        r.V = V;
    }
    if (sub == 3) {
        BestRec b;
        b.score = -INFINITY;
        b.x = b.y = 0.0;
        b.v = b.p = kNoBest;
        b.nsol = 0;
        b.nc = nc;
        best[k] = b;
    }
}

// ------------------------------------------------------------ search

// Search with one wavefront per event (lanes = variations in chunks of 64,
// events taken from per-class counters by a persistent grid, the next
// event's ticket and record fetched one event ahead).  NW wavefronts per
// workgroup; the launch bound (two wavefronts per SIMD) gives every size the
// same register budget.
template <typename T, int NW>
__global__ __launch_bounds__(NW * kWave, 2) void k_search_ev(const int64_t *__restrict__ count, int64_t capacity,
                                                               RecoArgs a, const StageRec *__restrict__ stage,
                                                               BestRec *__restrict__ best_out,
                                                               uint64_t *__restrict__ wstats) {
    __shared__ WaveStageEv<T> stage_all[NW];
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    WaveStageEv<T> &st = stage_all[wave];
    const int64_t S = clamp_count(count, capacity);
    const double mt2_mw2 = a.m_t * a.m_t - a.m_w * a.m_w;
    const double mw2 = a.m_w * a.m_w;
    uint64_t acc_var = 0, acc_pair = 0, acc_int = 0, acc_sol = 0;

    // Events are handed out by counters, not dealt round robin: the cost of an
    // event varies (pairings, variations, intersection points), and with a static deal the
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
    uint64_t *dst = reinterpret_cast<uint64_t *>(&st.rec);
    unsigned long long tk = 0;
    if (lane == 0) tk = atomicAdd(ticket, 1ull);
    int64_t k = cls + (int64_t)ncls * (int64_t)__shfl(tk, 0);
    uint64_t w0 = 0;
    if (k < S) {
        if (lane < kPrefetchWords) w0 = recw[k * kRecWords + lane];
        if (lane == 0) tk = atomicAdd(ticket, 1ull);
    }
    while (k < S) {
        if (lane < kPrefetchWords) dst[lane] = w0;
        wave_sync();
        // the rest of a record with more than three candidates, read now
        // (issued before the next event's prefetch, stored after it)
        const int nc = __builtin_amdgcn_readfirstlane(st.rec.nc);
        const int used = kHeadWords + kCandWords * nc;
        const bool tail = used > kPrefetchWords && kPrefetchWords + lane < used;
        uint64_t t = 0;
        if (tail) t = recw[k * kRecWords + kPrefetchWords + lane];
        const int64_t kn = cls + (int64_t)ncls * (int64_t)__shfl(tk, 0);
        if (kn < S) {
            if (lane < kPrefetchWords) w0 = recw[kn * kRecWords + lane];
            if (lane == 0) tk = atomicAdd(ticket, 1ull);
        }
        if (tail) dst[kPrefetchWords + lane] = t;
        wave_sync();
        const bool ok = nc >= 2;
        // valid sides as wave-uniform bit masks: bit c of okp / okm when the
        // l+ / l- side with candidate c is not degenerate
        uint32_t okp = 0, okm = 0;
        if (ok) {
            // side constants: lanes [0, nc) with l+, lanes [16, 16 + nc) with l-
            // (one call on per-lane operands, not one branch per lepton)
            bool side_ok = false;
            const bool minus = lane >= 16;
            const int c = lane & 15;
            if (c < nc && lane < 32)
                side_ok = make_side(minus ? st.rec.lm : st.rec.lp, st.rec.cand[c].v, minus ? st.sm[c] : st.sp[c]);
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
            // the event's counter words are wave-uniform (scalar registers), so
            // the generator's first rounds run on the scalar unit
            const uint64_t g = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(st.rec.g >> 32)) << 32) |
                               (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)st.rec.g);
            for (int vb = 0; vb < V; vb += kWave) {
                const int v = vb + lane;
                const bool act = v < V;
                // ---- draws of this lane's variation, kept in LDS so that any lane can
                // rebuild another lane's smear factors
                {
                    T zl[4] = {(T)0, (T)0, (T)0, (T)0};
                    if (a.smear && act) {
                        gauss_block<T>(a.seed, g, (uint32_t)v, 0u, zl);
                        // a candidate's slot 4 + j lies in Philox block (4 + j) / 4; each
                        // block is generated once for consecutive candidates in it.  In
                        // FP32 only the Box-Muller pairs that are used are formed; the
                        // FP64 form takes whole blocks (its pairs need more registers than
                        // the raw words held across the loop would leave)
                        uint32_t last_blk = 0xffffffffu, have = 0;
                        U4 raw{0u, 0u, 0u, 0u};
                        T zb[4] = {(T)0, (T)0, (T)0, (T)0};
                        for (int c = 0; c < nc; ++c) {
                            const uint32_t slot = 4u + (uint32_t)__builtin_amdgcn_readfirstlane(st.rec.cand[c].jidx);
                            const uint32_t blk = slot >> 2;
                            if constexpr (sizeof(T) == sizeof(float)) {
                                if (blk != last_blk) {
                                    raw = philox_block(a.seed, g, (uint32_t)v, blk);
                                    last_blk = blk;
                                    have = 0;
                                }
                                const uint32_t pr = (slot >> 1) & 1u;
                                if (!((have >> pr) & 1u)) {
                                    if (pr)
                                        box_muller(raw.z, raw.w, zb[2], zb[3]);
                                    else
                                        box_muller(raw.x, raw.y, zb[0], zb[1]);
                                    have |= 1u << pr;
                                }
                            } else {
                                if (blk != last_blk) {
                                    gauss_block<T>(a.seed, g, (uint32_t)v, blk, zb);
                                    last_blk = blk;
                                }
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
                const double zz_l = (double)st.zl[0][lane] * st.zl[0][lane] + (double)st.zl[1][lane] * st.zl[1][lane] +
                                    (double)st.zl[2][lane] * st.zl[2][lane] + (double)st.zl[3][lane] * st.zl[3][lane];
                for (int i = 0; i < nc; ++i) {
                    if (!((okp >> i) & 1u)) continue;
                    const double si = smear(st.rec.cand[i].sigma, st.z[i][lane]);
                    const SideVar A = side_var(st.sp[i], Wp, slp, si, mt2_mw2);
                    const PencilP pa = pencil_p(A.q);
                    for (int j = 0; j < nc; ++j) {
                        if (j == i || !((okm >> j) & 1u)) continue;
                        // ---- the common points of this lane's two conics (its own variation)
                        const double sj = smear(st.rec.cand[j].sigma, st.z[j][lane]);
                        const SideVar Bv = side_var(st.sm[j], Wm, slm, sj, mt2_mw2);
                        const Conic Q = reflect(Bv.q, mx, my);
                        Points4 pts;
                        pts.n = 0;
                        if (act) pts = conic_intersections<T>(A.q, pa, Q);
                        acc_int += 2 * (uint64_t)(popc64(ballot(pts.n > 0)) + popc64(ballot(pts.n > 2)));
                        const int p = i * nc + j;
                        // score terms of this variation that do not depend on the point
                        const double bxs = si * st.rec.cand[i].v[1] + slp * st.rec.lp[1];
                        const double bys = si * st.rec.cand[i].v[2] + slp * st.rec.lp[2];
                        const double bxb = sj * st.rec.cand[j].v[1] + slm * st.rec.lm[1];
                        const double byb = sj * st.rec.cand[j].v[2] + slm * st.rec.lm[2];
                        const double zzv = zz_l + (double)st.z[i][lane] * st.z[i][lane] +
                                           (double)st.z[j][lane] * st.z[j][lane];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            // points come in pairs (one line, two roots): a wave with no lane
                            // holding point k skips it
                            const bool live = k < pts.n;
                            if (!ballot(live)) break;
                            bool accepted = false;
                            if (live) {
                                double x = k == 0 ? pts.x0 : k == 1 ? pts.x1 : k == 2 ? pts.x2 : pts.x3;
                                double y = k == 0 ? pts.y0 : k == 1 ? pts.y1 : k == 2 ? pts.y2 : pts.y3;
                                if (polish_xy(A.q, Q, x, y, 4, a.polish_skip_m2) <= a.accept_m2) {
                                    const double en = st.sp[i][kE1] * x + st.sp[i][kE2] * y + A.e0;
                                    const double xb = mx - x, yb = my - y;
                                    const double eb = st.sm[j][kE1] * xb + st.sm[j][kE2] * yb + Bv.e0;
                                    accepted = en >= 0.0 && eb >= 0.0;
                                    if (accepted) {
                                        const double tx = bxs + x, ty = bys + y, tbx = bxb + xb, tby = byb + yb;
                                        const double w = -0.5 * zzv - (fast_sqrt(tx * tx + ty * ty) +
                                                                       fast_sqrt(tbx * tbx + tby * tby)) *
                                                                          a.inv_lambda;
                                        if (better(w, v, p, x, best_s, best_v, best_p, best_x)) {
                                            best_s = w;
                                            best_v = v;
                                            best_p = p;
                                            best_x = x;
                                            best_y = y;
                                        }
                                    }
                                }
                            }
                            nsol += popc64(ballot(accepted));
                        }
                    }
                }
                wave_sync();
            }
        }
        // --------------------------------------------------- wave argmax
        // The wave's top score first (a max over four in-row DPP steps --
        // pairs, quads, eights, rows -- then across rows by shuffles); the
        // lanes holding it are found by a ballot.  One such lane (the usual
        // case) is the winner.  Among several (equal scores), better() -- a
        // total order -- settles it by the same exchange pattern, with every
        // other lane set below all of them.
        double top = best_s;
        top = fmax(top, dpp_f64<0xB1>(top));
        top = fmax(top, dpp_f64<0x4E>(top));
        top = fmax(top, dpp_f64<0x141>(top));
        top = fmax(top, dpp_f64<0x140>(top));
        top = fmax(top, __shfl_xor(top, 16));
        top = fmax(top, __shfl_xor(top, 32));
        const uint64_t at_top = ballot(best_v != kNoBest && best_s == top);
        double win_s = -INFINITY, win_x = 0.0, win_y = 0.0;
        int win_v = kNoBest, win_p = kNoBest;
        if (at_top != 0) {
            if ((at_top & (at_top - 1)) != 0) {
                if (!((at_top >> lane) & 1ull)) {
                    best_s = -INFINITY;
                    best_v = kNoBest;
                    best_p = kNoBest;
                    best_x = 0.0;
                    best_y = 0.0;
                }
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
                    take(__shfl_xor(best_s, off), __shfl_xor(best_v, off), __shfl_xor(best_p, off),
                         __shfl_xor(best_x, off), __shfl_xor(best_y, off));
            }
            // the winner's record (after the tie-break every lane holds it)
            const int wl = (int)__builtin_ctzll(at_top);
            win_s = __shfl(best_s, wl);
            win_v = __shfl(best_v, wl);
            win_p = __shfl(best_p, wl);
            win_x = __shfl(best_x, wl);
            win_y = __shfl(best_y, wl);
        }
        acc_var += (uint64_t)V;
        acc_pair += (uint64_t)V * (uint64_t)npair_valid;
        acc_sol += (uint64_t)nsol;
        if (lane == 0) {
            BestRec r;
            r.score = win_s;
            r.x = win_x;
            r.y = win_y;
            r.v = win_v;
            r.p = win_p;
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
            const int jidx[2] = {rec.cand[ci].jidx, rec.cand[cj].jidx};
            double lp[4], lm[4], b[4], bb[4];
            for (int q = 0; q < 4; ++q) {
                lp[q] = rec.lp[q];
                lm[q] = rec.lm[q];
                b[q] = rec.cand[ci].v[q];
                bb[q] = rec.cand[cj].v[q];
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
            const double si = smear(rec.cand[ci].sigma, zi), sj = smear(rec.cand[cj].sigma, zj);
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
int resident_grid(const void *kernel, int block, int *cache) {
    if (*cache <= 0) {
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) n_cu = prop.multiProcessorCount;
        if (n_cu <= 0) n_cu = 256;
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess || nb < 1) nb = 1;
        *cache = n_cu * nb;
    }
    return *cache;
}

hipEvent_t g_time_start = nullptr, g_time_stop = nullptr;

// Workspace layout (each part 256-byte aligned): header (statistics and the
// search's event counters), BestRec[capacity], StageRec[capacity].
struct WsLayout {
    size_t best, stage, total;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static WsLayout ws_layout(int64_t capacity) {
    const size_t c = (size_t)(capacity > 0 ? capacity : 0);
    WsLayout L;
    L.best = kWsHeader;
    L.stage = align256(L.best + c * sizeof(BestRec));
    L.total = align256(L.stage + c * sizeof(StageRec));
    return L;
}

template <typename T, int NW>
hipError_t launch_search(const int64_t *count, int64_t capacity, const RecoArgs &a, const StageRec *stage,
                         BestRec *best, uint64_t *wstats, hipStream_t s) {
    static int grid = 0;
    int64_t g = resident_grid(reinterpret_cast<const void *>(&k_search_ev<T, NW>), NW * kWave, &grid);
    const int64_t need = (capacity + NW - 1) / NW;  // no more wavefronts than events
    g = g < need ? g : need;
    hipLaunchKernelGGL((k_search_ev<T, NW>), dim3((unsigned)(g < 1 ? 1 : g)), dim3(NW * kWave), 0, s, count,
                       capacity, a, stage, best, wstats);
    return hipGetLastError();
}

// waves: wavefronts per workgroup of the search (1, 2 or 4)
template <typename T>
hipError_t launch_t(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity, const RecoArgs &a,
                    const RecoOutView &out, hf_counters_t *reco_counter, uint64_t *wstats, char *ws, int waves,
                    hipStream_t s) {
    const WsLayout L = ws_layout(capacity);
    BestRec *best = reinterpret_cast<BestRec *>(ws + L.best);
    StageRec *stage = reinterpret_cast<StageRec *>(ws + L.stage);
    const int64_t eg = capacity > 0 ? (capacity + 255) / 256 : 1;
    const int64_t sg = capacity > 0 ? (capacity + kStageEvents - 1) / kStageEvents : 1;
    if (capacity > 0) {
        hipLaunchKernelGGL(k_stage, dim3((unsigned)sg), dim3(256), 0, s, ev, idx, count, capacity, a, stage, best);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        if (g_time_start) {
            err = hipEventRecord(g_time_start, s);
            if (err != hipSuccess) return err;
        }
        err = waves == 1 ? launch_search<T, 1>(count, capacity, a, stage, best, wstats, s)
              : waves == 2 ? launch_search<T, 2>(count, capacity, a, stage, best, wstats, s)
                           : launch_search<T, 4>(count, capacity, a, stage, best, wstats, s);
        if (err != hipSuccess) return err;
        if (g_time_stop) {
            err = hipEventRecord(g_time_stop, s);
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
                       void *ws, int waves, hipStream_t s) {
    uint64_t *wstats = static_cast<uint64_t *>(ws);
    hipLaunchKernelGGL(k_reco_init, dim3(1), dim3(64), 0, s, wstats);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    char *w = static_cast<char *>(ws);
    if (precision == HF_PREC_MIXED)
        return launch_t<float>(ev, idx, count, capacity, a, out, reco_counter, wstats, w, waves, s);
    return launch_t<double>(ev, idx, count, capacity, a, out, reco_counter, wstats, w, waves, s);
}

}  // namespace hf
