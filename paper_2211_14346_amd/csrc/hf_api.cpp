// C-ABI front end of libhf: argument validation, error reporting and kernel
// launches.  Host code only; every device launch lives in the .hip units.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hf.h"
#include "hf_chi2.hpp"
#include "hf_internal.hpp"
#include "hf_reco_math.hpp"
#include "hf_rtc.hpp"
#include "hf_unpack.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int device_fail(const char *what, hipError_t e) {
    return fail(HF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool events_ok(const hf_events_t *ev, bool need_phi_e, const char **why) {
    if (!ev) return *why = "ev is NULL", false;
    if (ev->n < 0 || ev->n >= (int64_t)1 << 31) return *why = "n out of range [0, 2^31)", false;
    if (ev->index_base < 0 || ev->index_base + ev->n > ((int64_t)1 << 31))
        return *why = "index_base + n must lie in [0, 2^31]", false;
    if (ev->n == 0) return true;
    if (!ev->lep_off || !ev->jet_off || !ev->lep_pt || !ev->lep_eta || !ev->lep_q || !ev->jet_pt ||
        !ev->jet_eta || !ev->jet_btag || !ev->met_x || !ev->met_y)
        return *why = "a required event column is NULL", false;
    if (need_phi_e && (!ev->lep_phi || !ev->lep_e || !ev->jet_phi || !ev->jet_e))
        return *why = "phi/E columns are NULL", false;
    return true;
}

int check_cuts(const hf_cut_t *h_cuts, int n_cuts, bool *need_phi_e) {
    if (!h_cuts) return fail(HF_ERR_INVAL, "h_cuts is NULL");
    if (n_cuts < 1 || n_cuts > HF_MAX_CUTS) return fail(HF_ERR_INVAL, "n_cuts=%d outside [1, %d]", n_cuts, HF_MAX_CUTS);
    *need_phi_e = false;
    for (int c = 0; c < n_cuts; ++c) {
        const hf_cut_t &k = h_cuts[c];
        if (k.kind < HF_CUT_LEP_N_OS || k.kind > HF_CUT_JET_N_RANGE)
            return fail(HF_ERR_INVAL, "cut %d: unknown kind %d", c, k.kind);
        if (k.reserved != 0) return fail(HF_ERR_INVAL, "cut %d: reserved field must be 0", c);
        if (k.dep_mask >> n_cuts) return fail(HF_ERR_INVAL, "cut %d: dependency on a cut id >= n_cuts", c);
        if (k.dep_mask & (1ull << c)) return fail(HF_ERR_INVAL, "cut %d depends on itself", c);
        for (int q = 0; q < 8; ++q)
            if (!isfinite(k.f[q])) return fail(HF_ERR_INVAL, "cut %d: non-finite parameter f[%d]", c, q);
        if (k.kind == HF_CUT_MLL_MIN || k.kind == HF_CUT_LEP_ISO || k.kind == HF_CUT_MTW_MIN) *need_phi_e = true;
    }
    return HF_OK;
}

// ---- autotuner cache: one line per configuration, "key schedule ms_wg256 ms_wg128 ms_wg64";
// the last line for a key wins.  Read once per process from HF_AUTOTUNE_CACHE.
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::map<std::string, int> g_tune;

std::string tune_key(const hf_events_t *ev, const hf_reco_params_t *p, int64_t capacity) {
    int dev = 0;
    char name[64] = "gpu";
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        snprintf(name, sizeof name, "%s", prop.gcnArchName);
    for (char *c = name; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    int bucket = 0;
    while (bucket < 62 && ((int64_t)1 << (bucket + 1)) <= capacity) ++bucket;
    char key[256];
    snprintf(key, sizeof key, "%s|prec=%d|pair=%d|cands=%d|nvar=%s%d|cap=2^%d", name, p->precision, p->pair_mode,
             p->max_cands, ev->n_var ? "per_event" : "", ev->n_var ? 0 : p->n_var_uniform, bucket);
    return key;
}

bool valid_schedule(int s) {
    return s == HF_SCHED_AUTO || s == HF_SCHED_EVENT || s == HF_SCHED_EVENT_WG64 || s == HF_SCHED_EVENT_WG128;
}

// wavefronts per workgroup of the search for a schedule
int schedule_waves(int s) { return s == HF_SCHED_EVENT_WG64 ? 1 : s == HF_SCHED_EVENT_WG128 ? 2 : 4; }

void load_tune_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("HF_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[256];
    int sched;
    double a, b, c;
    while (fscanf(f, "%255s %d %lf %lf %lf", key, &sched, &a, &b, &c) == 5)
        if (valid_schedule(sched) && sched != HF_SCHED_AUTO) g_tune[key] = sched;
    fclose(f);
}

int tuned_schedule(const std::string &key) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    auto it = g_tune.find(key);
    return it == g_tune.end() ? HF_SCHED_AUTO : it->second;
}

void store_schedule(const std::string &key, int sched, const double ms[3]) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache();
    g_tune[key] = sched;
    const char *path = getenv("HF_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %.6f %.6f %.6f\n", key.c_str(), sched, ms[0], ms[1], ms[2]);
    fclose(f);
}

}  // namespace

extern "C" {

const char *hf_last_error(void) { return g_err.c_str(); }

const char *hf_version(void) { return "hf 0.1 gfx950"; }

size_t hf_select_workspace_size(int64_t n, int n_cuts) {
    if (n < 0 || n_cuts < 1 || n_cuts > HF_MAX_CUTS) return 0;
    return hf::select_ws_bytes(n, n_cuts);
}

int hf_select(const hf_events_t *ev, const hf_cut_t *h_cuts, int n_cuts, const int32_t *d_order,
              uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes, hipStream_t stream) {
    bool need_pe = false;
    int rc = check_cuts(h_cuts, n_cuts, &need_pe);
    if (rc != HF_OK) return rc;
    for (int c = 0; c < n_cuts; ++c)
        if (h_cuts[c].kind == HF_CUT_USER)
            return fail(HF_ERR_INVAL, "hf_select: cut %d is a user predicate; compile the chain with "
                                      "hf_chain_compile and run it with hf_chain_select", c);
    const char *why = nullptr;
    if (!events_ok(ev, need_pe, &why)) return fail(HF_ERR_INVAL, "hf_select: %s", why);
    if (!d_order || !d_counters) return fail(HF_ERR_INVAL, "hf_select: order or counters is NULL");
    if (ev->n > 0 && !d_survive) return fail(HF_ERR_INVAL, "hf_select: survive is NULL");
    const size_t need = hf::select_ws_bytes(ev->n, n_cuts);
    if (!d_ws || ws_bytes < need)
        return fail(HF_ERR_CAPACITY, "hf_select: workspace %zu bytes < %zu required", ws_bytes, need);
    hf::CutTable ct;
    memset(&ct, 0, sizeof ct);
    for (int c = 0; c < n_cuts; ++c) ct.c[c] = h_cuts[c];
    ct.n = n_cuts;
    hipError_t e = hf::launch_select(hf::make_view(*ev), ct, d_order, d_survive, d_counters, d_ws, stream);
    if (e != hipSuccess) return device_fail("hf_select launch", e);
    return HF_OK;
}

size_t hf_compact_workspace_size(int64_t capacity) {
    if (capacity < 0) return 0;
    return hf::compact_ws_bytes(capacity);
}

int hf_compact(const uint8_t *d_mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
               const int32_t *d_map, int32_t *d_idx, int64_t *d_count, void *d_ws, size_t ws_bytes,
               hipStream_t stream) {
    if (capacity < 0) return fail(HF_ERR_INVAL, "hf_compact: capacity < 0");
    if (capacity >= ((int64_t)1 << 31)) return fail(HF_ERR_CAPACITY, "hf_compact: capacity >= 2^31");
    if (!d_count) return fail(HF_ERR_INVAL, "hf_compact: count is NULL");
    if (capacity > 0 && (!d_mask || !d_idx)) return fail(HF_ERR_INVAL, "hf_compact: mask or idx is NULL");
    if (!d_map && (index_base < 0 || index_base + capacity > ((int64_t)1 << 31)))
        return fail(HF_ERR_INVAL, "hf_compact: index_base + capacity must lie in [0, 2^31]");
    const size_t need = hf::compact_ws_bytes(capacity);
    if (!d_ws || ws_bytes < need)
        return fail(HF_ERR_CAPACITY, "hf_compact: workspace %zu bytes < %zu required", ws_bytes, need);
    hipError_t e = hf::launch_compact(d_mask, capacity, d_n, index_base, d_map, d_idx, d_count, d_ws, stream);
    if (e != hipSuccess) return device_fail("hf_compact launch", e);
    return HF_OK;
}

int hf_compact_noalloc(const uint8_t *d_mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                       const int32_t *d_map, int32_t *d_idx, int64_t *d_count, hipStream_t stream) {
    if (capacity < 0) return fail(HF_ERR_INVAL, "hf_compact_noalloc: capacity < 0");
    if (capacity > HF_COMPACT_NOALLOC_MAX_ENTRIES)
        return fail(HF_ERR_CAPACITY, "hf_compact_noalloc: capacity %lld above the maximum %lld",
                    (long long)capacity, (long long)HF_COMPACT_NOALLOC_MAX_ENTRIES);
    if (!d_count) return fail(HF_ERR_INVAL, "hf_compact_noalloc: count is NULL");
    if (capacity > 0 && (!d_mask || !d_idx)) return fail(HF_ERR_INVAL, "hf_compact_noalloc: mask or idx is NULL");
    if (!d_map && (index_base < 0 || index_base + capacity > ((int64_t)1 << 31)))
        return fail(HF_ERR_INVAL, "hf_compact_noalloc: index_base + capacity must lie in [0, 2^31]");
    hipError_t e = hf::launch_compact_noalloc(d_mask, capacity, d_n, index_base, d_map, d_idx, d_count, stream);
    if (e != hipSuccess) return device_fail("hf_compact_noalloc launch", e);
    return HF_OK;
}

size_t hf_ttbar_reco_workspace_size(int64_t capacity) {
    if (capacity < 0) return 0;
    return hf::reco_ws_bytes(capacity);
}

int hf_ttbar_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                  const hf_reco_params_t *p, const hf_reco_out_t *out, hf_counters_t *d_counters, void *d_ws,
                  size_t ws_bytes, hipStream_t stream) {
    const char *why = nullptr;
    if (!events_ok(ev, true, &why)) return fail(HF_ERR_INVAL, "hf_ttbar_reco: %s", why);
    if (!p || !out) return fail(HF_ERR_INVAL, "hf_ttbar_reco: params or out is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31)) return fail(HF_ERR_INVAL, "hf_ttbar_reco: capacity out of range");
    if (!d_count) return fail(HF_ERR_INVAL, "hf_ttbar_reco: count is NULL");
    if (capacity > 0) {
        if (!d_idx || !out->has_sol || !out->n_sol || !out->best_v || !out->best_i || !out->best_j || !out->nu ||
            !out->nubar || !out->m_t || !out->m_tbar || !out->m_wp || !out->m_wm || !out->logw)
            return fail(HF_ERR_INVAL, "hf_ttbar_reco: an index or output array is NULL");
        if (p->want_mbb && !out->m_bb) return fail(HF_ERR_INVAL, "hf_ttbar_reco: want_mbb needs out->m_bb");
    }
    if (p->precision != HF_PREC_FP64 && p->precision != HF_PREC_MIXED)
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: unknown precision %d", p->precision);
    if (p->pair_mode != HF_PAIR_BTAG_FILL && p->pair_mode != HF_PAIR_ALL_JETS)
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: unknown pair_mode %d", p->pair_mode);
    if (p->max_cands < 2 || p->max_cands > HF_MAX_CANDS)
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: max_cands %d outside [2, %d]", p->max_cands, HF_MAX_CANDS);
    if (!ev->n_var && (p->n_var_uniform < 1 || p->n_var_uniform > 65535))
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: n_var_uniform %d outside [1, 65535]", p->n_var_uniform);
    if (!(p->m_t > p->m_w && p->m_w > 0.0) || !(p->lambda_pt > 0.0) || !isfinite(p->m_t))
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: masses or lambda_pt invalid");
    if (!(p->jet_a >= 0.0) || !(p->jet_c >= 0.0) || !(p->lep_sigma >= 0.0) || !(p->met_sigma >= 0.0))
        return fail(HF_ERR_INVAL, "hf_ttbar_reco: resolutions must be finite and >= 0");
    if (p->smear != 0 && p->smear != 1) return fail(HF_ERR_INVAL, "hf_ttbar_reco: smear must be 0 or 1");
    if (!valid_schedule(p->schedule)) return fail(HF_ERR_INVAL, "hf_ttbar_reco: unknown schedule %d", p->schedule);
    const size_t need = hf::reco_ws_bytes(capacity);
    if (!d_ws || ws_bytes < need)
        return fail(HF_ERR_CAPACITY, "hf_ttbar_reco: workspace %zu bytes < %zu required", ws_bytes, need);
    hf::RecoArgs a;
    a.m_t = p->m_t;
    a.m_w = p->m_w;
    a.lambda_pt = p->lambda_pt;
    a.inv_lambda = 1.0 / p->lambda_pt;
    a.accept_m2 = hf::kAcceptM2 * p->m_w * p->m_w;
    a.polish_skip_m2 = hf::kPolishSkip * a.accept_m2;
    a.jet_a = p->jet_a;
    a.jet_c = p->jet_c;
    a.lep_sigma = p->lep_sigma;
    a.met_sigma = p->met_sigma;
    a.lep_pt_min = p->lep_pt_min;
    a.lep_eta_max = p->lep_eta_max;
    a.jet_pt_min = p->jet_pt_min;
    a.jet_eta_max = p->jet_eta_max;
    a.btag_min = p->btag_min;
    a.seed = p->seed;
    a.smear = p->smear;
    a.n_var_uniform = p->n_var_uniform;
    a.pair_mode = p->pair_mode;
    a.max_cands = p->max_cands;
    a.want_mbb = p->want_mbb;
    hf::RecoOutView o{out->has_sol, out->n_sol, out->best_v, out->best_i, out->best_j, out->nu, out->nubar,
                      out->m_t,     out->m_tbar, out->m_wp,  out->m_wm,   out->logw, out->m_bb, out->stats};
    hf_counters_t *rc = (d_counters && p->reco_cut >= 0) ? d_counters + p->reco_cut : nullptr;
    int sched = p->schedule;
    if (sched == HF_SCHED_AUTO) sched = tuned_schedule(tune_key(ev, p, capacity));
    if (sched == HF_SCHED_AUTO) sched = HF_SCHED_EVENT;
    hipError_t e = hf::launch_reco(hf::make_view(*ev), d_idx, d_count, capacity, a, p->precision, o, rc, d_ws,
                                   schedule_waves(sched), stream);
    if (e != hipSuccess) return device_fail("hf_ttbar_reco launch", e);
    return HF_OK;
}

int hf_ttbar_reco_autotune(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                           hf_reco_params_t *h_params, const hf_reco_out_t *out, void *d_ws, size_t ws_bytes,
                           hipStream_t stream, double *h_ms) {
    if (!h_params || !out) return fail(HF_ERR_INVAL, "hf_ttbar_reco_autotune: params or out is NULL");
    hf_reco_params_t p = *h_params;
    hf_reco_out_t o = *out;
    o.stats = nullptr;  // the trial calls leave no trace in the statistics or counters
    const int cand[3] = {HF_SCHED_EVENT, HF_SCHED_EVENT_WG128, HF_SCHED_EVENT_WG64};
    double ms[3] = {0.0, 0.0, 0.0};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return fail(HF_ERR_DEVICE, "hf_ttbar_reco_autotune: hipEventCreate failed");
    }
    int rc = HF_OK;
    constexpr int kReps = 3;
    for (int c = 0; c < 3 && rc == HF_OK; ++c) {
        p.schedule = cand[c];
        rc = hf_ttbar_reco(ev, d_idx, d_count, capacity, &p, &o, nullptr, d_ws, ws_bytes, stream);  // warm-up
        if (rc != HF_OK) break;
        if (hipEventRecord(t0, stream) != hipSuccess) rc = fail(HF_ERR_DEVICE, "hf_ttbar_reco_autotune: record");
        for (int r = 0; r < kReps && rc == HF_OK; ++r)
            rc = hf_ttbar_reco(ev, d_idx, d_count, capacity, &p, &o, nullptr, d_ws, ws_bytes, stream);
        if (rc != HF_OK) break;
        float el = 0.0f;
        if (hipEventRecord(t1, stream) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
            hipEventElapsedTime(&el, t0, t1) != hipSuccess)
            rc = fail(HF_ERR_DEVICE, "hf_ttbar_reco_autotune: timing failed");
        ms[c] = (double)el / kReps;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc != HF_OK) return rc;
    int bi = 0;
    for (int c = 1; c < 3; ++c)
        if (ms[c] < ms[bi]) bi = c;
    const int best = cand[bi];
    h_params->schedule = best;
    if (h_ms)
        for (int c = 0; c < 3; ++c) h_ms[c] = ms[c];
    store_schedule(tune_key(ev, h_params, capacity), best, ms);
    return HF_OK;
}

int hf_chain_compile(const hf_cut_t *h_cuts, int n_cuts, const char *const *h_user_src, int n_user,
                     hf_chain_t **out) {
    if (!out) return fail(HF_ERR_INVAL, "hf_chain_compile: out is NULL");
    *out = nullptr;
    bool need_pe = false;
    int rc = check_cuts(h_cuts, n_cuts, &need_pe);
    if (rc != HF_OK) return rc;
    if (n_user < 0 || n_user > HF_MAX_CUTS)
        return fail(HF_ERR_INVAL, "hf_chain_compile: n_user %d outside [0, %d]", n_user, HF_MAX_CUTS);
    if (n_user > 0 && !h_user_src) return fail(HF_ERR_INVAL, "hf_chain_compile: user sources are NULL");
    std::vector<std::string> src;
    for (int u = 0; u < n_user; ++u) {
        if (!h_user_src[u]) return fail(HF_ERR_INVAL, "hf_chain_compile: user source %d is NULL", u);
        src.emplace_back(h_user_src[u]);
    }
    for (int c = 0; c < n_cuts; ++c) {
        if (h_cuts[c].kind == HF_CUT_USER && (h_cuts[c].i[0] < 0 || h_cuts[c].i[0] >= n_user))
            return fail(HF_ERR_INVAL, "hf_chain_compile: cut %d names user source %d outside [0, %d)", c,
                        h_cuts[c].i[0], n_user);
        if (h_cuts[c].kind == HF_CUT_USER && h_cuts[c].i[1] < 0)
            return fail(HF_ERR_INVAL, "hf_chain_compile: cut %d has a negative loop budget %d", c, h_cuts[c].i[1]);
    }
    std::vector<char> code;
    std::string lowered, log;
    if (!hf::rtc_compile(hf::chain_source(src), code, lowered, log)) {
        g_err = "hf_chain_compile: the user predicates do not compile:\n" + log;
        return HF_ERR_INVAL;
    }
    hf_chain *ch = new hf_chain;
    ch->cuts.assign(h_cuts, h_cuts + n_cuts);
    ch->n_user = n_user;
    ch->log = log;
    hipError_t e = hipModuleLoadData(&ch->module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&ch->fn, ch->module, lowered.c_str());
    if (e != hipSuccess) {
        if (ch->module) (void)hipModuleUnload(ch->module);
        delete ch;
        return device_fail("hf_chain_compile: loading the chain kernel", e);
    }
    *out = ch;
    return HF_OK;
}

namespace {

// Checks shared by the segment entry points; *items receives the number of
// survive entries (events or compacted positions) the launch writes.
int check_segment(const char *who, const hf_events_t *ev, int n_cuts, const int32_t *d_order, int pos_begin,
                  int pos_end, const int32_t *d_idx, const int64_t *d_count, int64_t capacity, uint8_t *d_survive,
                  hf_counters_t *d_counters, void *d_ws, size_t ws_bytes) {
    if (!d_order || !d_counters) return fail(HF_ERR_INVAL, "%s: order or counters is NULL", who);
    if (pos_begin < 0 || pos_begin > pos_end || pos_end > n_cuts)
        return fail(HF_ERR_INVAL, "%s: positions [%d, %d) outside [0, %d]", who, pos_begin, pos_end, n_cuts);
    if (d_idx && !d_count) return fail(HF_ERR_INVAL, "%s: d_idx given without d_count", who);
    if (capacity < 0 || capacity >= ((int64_t)1 << 31)) return fail(HF_ERR_INVAL, "%s: capacity out of range", who);
    const int64_t items = d_idx ? capacity : ev->n;
    if (items > 0 && !d_survive) return fail(HF_ERR_INVAL, "%s: survive is NULL", who);
    const size_t need = hf::select_ws_bytes(items, n_cuts);
    if (!d_ws || ws_bytes < need)
        return fail(HF_ERR_CAPACITY, "%s: workspace %zu bytes < %zu required", who, ws_bytes, need);
    return HF_OK;
}

int chain_launch(const hf_chain_t *ch, const hf_events_t *ev, const int32_t *d_order, int pos_begin, int pos_end,
                 const int32_t *d_idx, const int64_t *d_count, int64_t capacity, uint8_t *d_survive,
                 hf_counters_t *d_counters, void *d_ws, const char *who, hipStream_t stream) {
    const int n_cuts = (int)ch->cuts.size();
    hf::CutTable ct;
    memset(&ct, 0, sizeof ct);
    for (int c = 0; c < n_cuts; ++c) ct.c[c] = ch->cuts[c];
    ct.n = n_cuts;
    hf::EvView v = hf::make_view(*ev);
    const int grid = hf::select_grid(d_idx ? capacity : ev->n);
    uint64_t *partial = static_cast<uint64_t *>(d_ws);
    void *args[] = {&v, &ct, &d_order, &d_survive, &partial, &d_idx, &d_count, &capacity, &pos_begin, &pos_end};
    hipError_t e = hipModuleLaunchKernel(ch->fn, grid, 1, 1, hf::kChainBlock, 1, 1, 0, stream, args, nullptr);
    if (e != hipSuccess) return device_fail(who, e);
    e = hf::launch_select_reduce(partial, grid, n_cuts, d_counters, stream);
    if (e != hipSuccess) return device_fail(who, e);
    return HF_OK;
}

}  // namespace

int hf_chain_select(const hf_chain_t *ch, const hf_events_t *ev, const int32_t *d_order, uint8_t *d_survive,
                    hf_counters_t *d_counters, void *d_ws, size_t ws_bytes, hipStream_t stream) {
    if (!ch || !ch->fn) return fail(HF_ERR_INVAL, "hf_chain_select: chain is NULL");
    const char *why = nullptr;
    if (!events_ok(ev, true, &why)) return fail(HF_ERR_INVAL, "hf_chain_select: %s", why);
    const int n_cuts = (int)ch->cuts.size();
    int rc = check_segment("hf_chain_select", ev, n_cuts, d_order, 0, n_cuts, nullptr, nullptr, 0, d_survive,
                           d_counters, d_ws, ws_bytes);
    if (rc != HF_OK) return rc;
    return chain_launch(ch, ev, d_order, 0, n_cuts, nullptr, nullptr, 0, d_survive, d_counters, d_ws,
                        "hf_chain_select launch", stream);
}

int hf_chain_select_segment(const hf_chain_t *ch, const hf_events_t *ev, const int32_t *d_order, int pos_begin,
                            int pos_end, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                            uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes,
                            hipStream_t stream) {
    if (!ch || !ch->fn) return fail(HF_ERR_INVAL, "hf_chain_select_segment: chain is NULL");
    const char *why = nullptr;
    if (!events_ok(ev, true, &why)) return fail(HF_ERR_INVAL, "hf_chain_select_segment: %s", why);
    int rc = check_segment("hf_chain_select_segment", ev, (int)ch->cuts.size(), d_order, pos_begin, pos_end, d_idx,
                           d_count, capacity, d_survive, d_counters, d_ws, ws_bytes);
    if (rc != HF_OK) return rc;
    return chain_launch(ch, ev, d_order, pos_begin, pos_end, d_idx, d_count, capacity, d_survive, d_counters, d_ws,
                        "hf_chain_select_segment launch", stream);
}

int hf_select_segment(const hf_events_t *ev, const hf_cut_t *h_cuts, int n_cuts, const int32_t *d_order,
                      int pos_begin, int pos_end, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                      uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes,
                      hipStream_t stream) {
    bool need_pe = false;
    int rc = check_cuts(h_cuts, n_cuts, &need_pe);
    if (rc != HF_OK) return rc;
    for (int c = 0; c < n_cuts; ++c)
        if (h_cuts[c].kind == HF_CUT_USER)
            return fail(HF_ERR_INVAL, "hf_select_segment: cut %d is a user predicate; use hf_chain_select_segment", c);
    const char *why = nullptr;
    if (!events_ok(ev, need_pe, &why)) return fail(HF_ERR_INVAL, "hf_select_segment: %s", why);
    rc = check_segment("hf_select_segment", ev, n_cuts, d_order, pos_begin, pos_end, d_idx, d_count, capacity,
                       d_survive, d_counters, d_ws, ws_bytes);
    if (rc != HF_OK) return rc;
    hf::CutTable ct;
    memset(&ct, 0, sizeof ct);
    for (int c = 0; c < n_cuts; ++c) ct.c[c] = h_cuts[c];
    ct.n = n_cuts;
    hipError_t e = hf::launch_select_segment(hf::make_view(*ev), ct, d_order, pos_begin, pos_end, d_idx, d_count,
                                             capacity, d_survive, d_counters, d_ws, stream);
    if (e != hipSuccess) return device_fail("hf_select_segment launch", e);
    return HF_OK;
}

const char *hf_chain_log(const hf_chain_t *ch) { return ch ? ch->log.c_str() : ""; }

void hf_chain_destroy(hf_chain_t *ch) {
    if (!ch) return;
    if (ch->module) (void)hipModuleUnload(ch->module);
    delete ch;
}

int hf_dilep_chi2_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                       const hf_chi2_params_t *p, const hf_chi2_out_t *out, hf_counters_t *d_counters,
                       hipStream_t stream) {
    const char *why = nullptr;
    if (!events_ok(ev, true, &why)) return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: %s", why);
    if (!p || !out) return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: params or out is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31))
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: capacity out of range");
    if (!d_count) return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: count is NULL");
    if (capacity > 0 && (!d_idx || !out->has_sol || !out->root_nu || !out->root_nubar || !out->best_i ||
                         !out->best_j || !out->nu || !out->nubar || !out->m_t || !out->m_tbar || !out->m_wp ||
                         !out->m_wm || !out->chi2 || !out->split))
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: an index or output array is NULL");
    if (p->pair_mode != HF_PAIR_BTAG_FILL && p->pair_mode != HF_PAIR_ALL_JETS)
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: unknown pair_mode %d", p->pair_mode);
    if (p->max_cands < 2 || p->max_cands > HF_MAX_CANDS)
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: max_cands %d outside [2, %d]", p->max_cands, HF_MAX_CANDS);
    if (p->n_grid < 2 || p->n_grid > 129 || p->n_refine < 0 || p->n_refine > 8)
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: grid n_grid %d / n_refine %d out of range", p->n_grid,
                    p->n_refine);
    if (!(p->half_range > 0.0) || !isfinite(p->half_range))
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: half_range must be finite and > 0");
    if (!(p->m_t > p->m_w && p->m_w > 0.0) || !isfinite(p->m_t))
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: masses invalid");
    if (!(p->sigma_t > 0.0) || !(p->sigma_w > 0.0) || !isfinite(p->sigma_t) || !isfinite(p->sigma_w))
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: widths must be finite and > 0");
    if (p->n_top != 0 && p->n_top != 1 && p->n_top != 2)
        return fail(HF_ERR_INVAL, "hf_dilep_chi2_reco: n_top %d is not 1 or 2", p->n_top);
    hf::Chi2Args a;
    a.m_t = p->m_t;
    a.m_w = p->m_w;
    a.sigma_t = p->sigma_t;
    a.sigma_w = p->sigma_w;
    a.inv_st2 = 1.0 / (p->sigma_t * p->sigma_t);
    a.inv_sw2 = 1.0 / (p->sigma_w * p->sigma_w);
    a.half_range = p->half_range;
    a.lep_pt_min = p->lep_pt_min;
    a.lep_eta_max = p->lep_eta_max;
    a.jet_pt_min = p->jet_pt_min;
    a.jet_eta_max = p->jet_eta_max;
    a.btag_min = p->btag_min;
    a.pair_mode = p->pair_mode;
    a.max_cands = p->max_cands;
    a.n_grid = p->n_grid;
    a.n_top = p->n_top == 1 ? 1 : 2;
    a.n_refine = p->n_refine;
    hf::Chi2OutView o{out->has_sol, out->root_nu, out->root_nubar, out->best_i, out->best_j, out->nu, out->nubar,
                      out->m_t,     out->m_tbar,  out->m_wp,       out->m_wm,   out->chi2,   out->split};
    hf_counters_t *rc = (d_counters && p->reco_cut >= 0) ? d_counters + p->reco_cut : nullptr;
    hipError_t e = hf::launch_chi2(hf::make_view(*ev), d_idx, d_count, capacity, a, o, rc, stream);
    if (e != hipSuccess) return device_fail("hf_dilep_chi2_reco launch", e);
    return HF_OK;
}

size_t hf_unpack_workspace_size(int64_t n) { return n < 0 ? 0 : hf::unpack_ws_bytes(n); }

int hf_unpack_events(int64_t n, const uint8_t *d_lep_cnt, const uint8_t *d_jet_cnt, int64_t n_lep, int64_t n_jet,
                     const int8_t *d_lep_q8, const uint8_t *d_jet_btag8, uint32_t *d_lep_off, uint32_t *d_jet_off,
                     float *d_lep_q, float *d_jet_btag, void *d_ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(HF_ERR_INVAL, "hf_unpack_events: n out of range [0, 2^31)");
    if (n_lep < 0 || n_jet < 0 || n_lep >= ((int64_t)1 << 32) || n_jet >= ((int64_t)1 << 32))
        return fail(HF_ERR_INVAL, "hf_unpack_events: object counts out of range [0, 2^32)");
    if (!d_lep_off || !d_jet_off || (n > 0 && (!d_lep_cnt || !d_jet_cnt)) || (n_lep > 0 && (!d_lep_q8 || !d_lep_q)) ||
        (n_jet > 0 && (!d_jet_btag8 || !d_jet_btag)))
        return fail(HF_ERR_INVAL, "hf_unpack_events: a pointer is NULL");
    if (((uintptr_t)d_lep_cnt | (uintptr_t)d_jet_cnt) & 15u)
        return fail(HF_ERR_INVAL, "hf_unpack_events: the count arrays must be 16-byte aligned");
    const size_t need = hf::unpack_ws_bytes(n);
    if (!d_ws || ws_bytes < need)
        return fail(HF_ERR_CAPACITY, "hf_unpack_events: workspace %zu bytes < %zu required", ws_bytes, need);
    hipError_t e = hf::launch_unpack(n, d_lep_cnt, d_jet_cnt, n_lep, n_jet, d_lep_q8, d_jet_btag8, d_lep_off,
                                     d_jet_off, d_lep_q, d_jet_btag, d_ws, stream);
    if (e != hipSuccess) return device_fail("hf_unpack_events launch", e);
    return HF_OK;
}

int hf_semilep_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                    const hf_semilep_params_t *p, const hf_semilep_out_t *out, hf_counters_t *d_counters,
                    hipStream_t stream) {
    const char *why = nullptr;
    if (!events_ok(ev, true, &why)) return fail(HF_ERR_INVAL, "hf_semilep_reco: %s", why);
    if (!p || !out) return fail(HF_ERR_INVAL, "hf_semilep_reco: params or out is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31))
        return fail(HF_ERR_INVAL, "hf_semilep_reco: capacity out of range");
    if (!d_count) return fail(HF_ERR_INVAL, "hf_semilep_reco: count is NULL");
    if (capacity > 0 && (!d_idx || !out->has_sol || !out->root || !out->best_j || !out->best_h || !out->best_p ||
                         !out->best_q || !out->nu || !out->m_tl || !out->m_wl || !out->m_th || !out->m_wh ||
                         !out->chi2))
        return fail(HF_ERR_INVAL, "hf_semilep_reco: an index or output array is NULL");
    if (p->topology != HF_TOPO_TCHAN && p->topology != HF_TOPO_WT && p->topology != HF_TOPO_TTSEMI)
        return fail(HF_ERR_INVAL, "hf_semilep_reco: unknown topology %d", p->topology);
    if (p->max_cands < 1 || p->max_cands > HF_MAX_CANDS)
        return fail(HF_ERR_INVAL, "hf_semilep_reco: max_cands %d outside [1, %d]", p->max_cands, HF_MAX_CANDS);
    if (!(p->m_t > p->m_w && p->m_w > 0.0) || !isfinite(p->m_t))
        return fail(HF_ERR_INVAL, "hf_semilep_reco: masses invalid");
    if (!(p->sigma_t > 0.0) || !(p->sigma_w > 0.0) || !isfinite(p->sigma_t) || !isfinite(p->sigma_w))
        return fail(HF_ERR_INVAL, "hf_semilep_reco: widths must be finite and > 0");
    if (p->reserved != 0) return fail(HF_ERR_INVAL, "hf_semilep_reco: reserved field must be 0");
    hf::SemilepArgs a;
    a.m_t = p->m_t;
    a.m_w = p->m_w;
    a.inv_st2 = 1.0 / (p->sigma_t * p->sigma_t);
    a.inv_sw2 = 1.0 / (p->sigma_w * p->sigma_w);
    a.lep_pt_min = p->lep_pt_min;
    a.lep_eta_max = p->lep_eta_max;
    a.jet_pt_min = p->jet_pt_min;
    a.jet_eta_max = p->jet_eta_max;
    a.topology = p->topology;
    a.max_cands = p->max_cands;
    hf::SemilepOutView o{out->has_sol, out->root, out->best_j, out->best_h, out->best_p, out->best_q, out->nu,
                         out->m_tl,    out->m_wl, out->m_th,   out->m_wh,   out->chi2};
    hf_counters_t *rc = (d_counters && p->reco_cut >= 0) ? d_counters + p->reco_cut : nullptr;
    hipError_t e = hf::launch_semilep(hf::make_view(*ev), d_idx, d_count, capacity, a, o, rc, stream);
    if (e != hipSuccess) return device_fail("hf_semilep_reco launch", e);
    return HF_OK;
}

int hf_reco_timing_events(hipEvent_t start, hipEvent_t stop) {
    if ((start == nullptr) != (stop == nullptr)) return fail(HF_ERR_INVAL, "hf_reco_timing_events: one event is NULL");
    hf::set_reco_timing(start, stop);
    return HF_OK;
}

int hf_philox_blocks(const uint32_t *d_ctr, uint64_t seed, uint32_t *d_out, int64_t n, hipStream_t stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(HF_ERR_INVAL, "hf_philox_blocks: n out of range");
    if (n > 0 && (!d_ctr || !d_out)) return fail(HF_ERR_INVAL, "hf_philox_blocks: NULL pointer");
    hipError_t e = hf::launch_philox(d_ctr, seed, d_out, n, stream);
    if (e != hipSuccess) return device_fail("hf_philox_blocks launch", e);
    return HF_OK;
}

int hf_gauss_draws(uint64_t seed, const int64_t *d_g, const int32_t *d_v, const int32_t *d_slot, int64_t n,
                   int precision, double *d_z, hipStream_t stream) {
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(HF_ERR_INVAL, "hf_gauss_draws: n out of range");
    if (n > 0 && (!d_g || !d_v || !d_slot || !d_z)) return fail(HF_ERR_INVAL, "hf_gauss_draws: NULL pointer");
    if (precision != HF_PREC_FP64 && precision != HF_PREC_MIXED)
        return fail(HF_ERR_INVAL, "hf_gauss_draws: unknown precision %d", precision);
    hipError_t e = hf::launch_gauss(seed, d_g, d_v, d_slot, n, precision, d_z, stream);
    if (e != hipSuccess) return device_fail("hf_gauss_draws launch", e);
    return HF_OK;
}

int hf_reorder_stats(const hf_counters_t *h_counters, const hf_cut_t *h_cuts, int n_cuts, int32_t *h_order) {
    if (!h_counters || !h_cuts || !h_order) return fail(HF_ERR_INVAL, "hf_reorder_stats: NULL argument");
    if (n_cuts < 1 || n_cuts > HF_MAX_CUTS) return fail(HF_ERR_INVAL, "hf_reorder_stats: n_cuts out of range");
    double rank[HF_MAX_CUTS];
    for (int c = 0; c < n_cuts; ++c) {
        const hf_counters_t &k = h_counters[c];
        const double p = k.reached ? (double)k.passed / (double)k.reached : 1.0;
        const double cost = k.reached ? (double)k.cost / (double)k.reached : 0.0;
        const double rej = 1.0 - p;
        rank[c] = cost / (rej > 1e-9 ? rej : 1e-9);
        if (h_cuts[c].dep_mask >> n_cuts) return fail(HF_ERR_INVAL, "hf_reorder_stats: dependency out of range");
    }
    int32_t order[HF_MAX_CUTS];
    uint64_t placed = 0;
    for (int pos = 0; pos < n_cuts; ++pos) {
        int best = -1;
        for (int c = 0; c < n_cuts; ++c) {
            if ((placed >> c) & 1ull) continue;
            if (h_cuts[c].dep_mask & ~placed) continue;
            if (best < 0 || rank[c] < rank[best]) best = c;
        }
        if (best < 0) return fail(HF_ERR_INVAL, "hf_reorder_stats: cyclic dependencies");
        order[pos] = best;
        placed |= 1ull << best;
    }
    memcpy(h_order, order, sizeof(int32_t) * (size_t)n_cuts);
    return HF_OK;
}

int hf_reorder_device(const hf_counters_t *d_counters, const hf_cut_t *h_cuts, int n_cuts, int32_t *d_order,
                      hipStream_t stream) {
    if (!d_counters || !h_cuts || !d_order) return fail(HF_ERR_INVAL, "hf_reorder_device: NULL argument");
    if (n_cuts < 1 || n_cuts > HF_MAX_CUTS) return fail(HF_ERR_INVAL, "hf_reorder_device: n_cuts out of range");
    uint64_t placed = 0;
    for (int c = 0; c < n_cuts; ++c)
        if (h_cuts[c].dep_mask >> n_cuts) return fail(HF_ERR_INVAL, "hf_reorder_device: dependency out of range");
    // a placement exists for any ranks iff the dependencies are acyclic
    for (int pos = 0; pos < n_cuts; ++pos) {
        int pick = -1;
        for (int c = 0; c < n_cuts && pick < 0; ++c)
            if (!((placed >> c) & 1ull) && !(h_cuts[c].dep_mask & ~placed)) pick = c;
        if (pick < 0) return fail(HF_ERR_INVAL, "hf_reorder_device: cyclic dependencies");
        placed |= 1ull << pick;
    }
    hf::CutTable ct;
    memset(&ct, 0, sizeof ct);
    for (int c = 0; c < n_cuts; ++c) ct.c[c] = h_cuts[c];
    ct.n = n_cuts;
    hipError_t e = hf::launch_reorder(d_counters, ct, d_order, stream);
    if (e != hipSuccess) return device_fail("hf_reorder_device launch", e);
    return HF_OK;
}

}  // extern "C"
