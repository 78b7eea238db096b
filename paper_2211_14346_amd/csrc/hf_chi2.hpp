// Dileptonic chi^2 fit with a MET split: internal interface between the
// C-ABI front end and its kernel unit.  Not part of the public ABI.
#pragma once

#include "hf_internal.hpp"

namespace hf {

struct Chi2Args {
    double m_t, m_w, sigma_t, sigma_w, inv_st2, inv_sw2, half_range;
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    int pair_mode, max_cands, n_grid, n_refine, n_top;
};

struct Chi2OutView {
    uint8_t *has_sol;
    int8_t *root_nu, *root_nubar;
    int16_t *best_i, *best_j;
    double *nu, *nubar, *m_t, *m_tbar, *m_wp, *m_wm, *chi2, *split;
};

hipError_t launch_chi2(const EvView &ev, const int32_t *idx, const int64_t *count, int64_t capacity, const Chi2Args &a,
                       const Chi2OutView &out, hf_counters_t *counter, hipStream_t s);

}  // namespace hf
