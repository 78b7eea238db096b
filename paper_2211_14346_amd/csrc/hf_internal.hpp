// Internal interfaces between the C-ABI front end (hf_api.cpp) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hf.h"

namespace hf {

// Device pointers of one chunk, passed to kernels by value.
struct EvView {
    int64_t n;
    int64_t index_base;
    const uint32_t *lep_off, *jet_off;
    const float *lep_pt, *lep_eta, *lep_phi, *lep_e, *lep_q;
    const float *jet_pt, *jet_eta, *jet_phi, *jet_e, *jet_btag;
    const float *met_x, *met_y;
    const uint16_t *n_var;
};

inline EvView make_view(const hf_events_t &e) {
    return EvView{e.n,      e.index_base, e.lep_off,  e.jet_off,  e.lep_pt,   e.lep_eta,
                  e.lep_phi, e.lep_e,     e.lep_q,    e.jet_pt,   e.jet_eta,  e.jet_phi,
                  e.jet_e,   e.jet_btag,  e.met_x,    e.met_y,    e.n_var};
}

// Cut table passed by value in the kernel argument segment.
struct CutTable {
    hf_cut_t c[HF_MAX_CUTS];
    int n;
};

// ---- selection (hf_select.hip)
int select_grid(int64_t n);
size_t select_ws_bytes(int64_t n, int n_cuts);
hipError_t launch_select(const EvView &ev, const CutTable &ct, const int32_t *order, uint8_t *survive,
                         hf_counters_t *counters, void *ws, hipStream_t s);
hipError_t launch_reorder(const hf_counters_t *counters, const CutTable &ct, int32_t *order, hipStream_t s);

// ---- compaction (hf_compact.hip)
size_t compact_ws_bytes(int64_t capacity);
hipError_t launch_compact(const uint8_t *mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                          const int32_t *map, int32_t *idx, int64_t *count, void *ws, hipStream_t s);
hipError_t launch_compact_noalloc(const uint8_t *mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                                  const int32_t *map, int32_t *idx, int64_t *count, hipStream_t s);

// ---- reconstruction (hf_reco.hip)
struct RecoArgs {
    double m_t, m_w, lambda_pt, inv_lambda;
    double accept_m2, polish_skip_m2;  // GeV^2: acceptance bound and no-polish bound on m_nu^2
    double jet_a, jet_c, lep_sigma, met_sigma;
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    uint64_t seed;
    int smear, n_var_uniform, pair_mode, max_cands, want_mbb;
};

struct RecoOutView {
    uint8_t *has_sol;
    int32_t *n_sol, *best_v;
    int16_t *best_i, *best_j;
    double *nu, *nubar;
    double *m_t, *m_tbar, *m_wp, *m_wm, *logw, *m_bb;
    uint64_t *stats;
};

size_t reco_ws_bytes(int64_t capacity);
void set_reco_timing(hipEvent_t start, hipEvent_t stop);
hipError_t launch_reco(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity,
                       const RecoArgs &a, int precision, const RecoOutView &out, hf_counters_t *reco_counter,
                       void *ws, int waves, hipStream_t s);

// ---- single-neutrino reconstruction (hf_semilep.hip)
struct SemilepArgs {
    double m_t, m_w, inv_st2, inv_sw2;  // 1 / sigma_t^2, 1 / sigma_W^2
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max;
    int topology, max_cands;
};

struct SemilepOutView {
    uint8_t *has_sol;
    int8_t *root;
    int16_t *best_j, *best_h, *best_p, *best_q;
    double *nu, *m_tl, *m_wl, *m_th, *m_wh, *chi2;
};

hipError_t launch_semilep(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity,
                          const SemilepArgs &a, const SemilepOutView &out, hf_counters_t *counter, hipStream_t s);

// ---- random draws (hf_rng.hip)
hipError_t launch_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out, int64_t n, hipStream_t s);
hipError_t launch_gauss(uint64_t seed, const int64_t *g, const int32_t *v, const int32_t *slot, int64_t n,
                        int precision, double *z, hipStream_t s);

}  // namespace hf
