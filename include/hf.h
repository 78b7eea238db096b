/*
 * hf.h -- C ABI of the MI355X (gfx950) hot path of a HEP-Frame-style
 * analysis: a chain of per-event cuts with adaptive ordering, on-device
 * compaction of the surviving events, and the dileptonic ttbar kinematic
 * reconstruction that ends the chain.
 *
 * Paper: A. Pereira, A. Onofre, A. Proenca, "HEP-Frame: an Efficient Tool for
 * Big Data Applications at the LHC", arXiv:2211.14346.
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless their name starts with h_ (host).
 *     Structures passed by pointer (hf_events_t, hf_reco_params_t,
 *     hf_reco_out_t, hf_cut_t arrays) live in host memory and are read before
 *     the call returns; the device pointers they hold must stay valid until
 *     the queued work has finished.
 *   - Device work is queued on the given stream and the call returns without
 *     waiting.  No entry point allocates, frees or synchronises; scratch
 *     memory is passed in as a workspace whose size the matching
 *     *_workspace_size query reports (hf_compact_noalloc alone uses a fixed
 *     array the library holds).  Every entry point may be recorded into
 *     a HIP graph (no memset nodes, no host reads of device data).
 *   - The caller owns all memory.  Concurrent calls that share outputs,
 *     counters or workspace race.
 *   - Return value: HF_OK, or a negative HF_ERR_* code; no work is queued
 *     when an error is returned.  hf_last_error() gives a message for the
 *     last error raised on the calling host thread.
 *   - Energies and momenta are in GeV.  Events are stored as structure of
 *     arrays: per-object float32 columns in a ragged (CSR) layout, objects of
 *     each event sorted by descending pT.
 */
#ifndef HF_H
#define HF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HF_OK 0
#define HF_ERR_INVAL (-1)       /* malformed argument (null pointer, size, enum) */
#define HF_ERR_CAPACITY (-2)    /* workspace or output smaller than required */
#define HF_ERR_DEVICE (-3)      /* the HIP runtime reported an error */
#define HF_ERR_UNSUPPORTED (-4) /* valid request this build does not implement */

#define HF_MAX_CUTS 32
#define HF_MAX_CANDS 12
#define HF_NO_SOLUTION (-9999.0) /* value of every float output without a solution */

/* One chunk of events (section 3: the per-event variables the cuts read).
 * Objects of event e are [lep_off[e], lep_off[e+1]) and
 * [jet_off[e], jet_off[e+1]) in the column arrays.  lep_q is the charge
 * (+1 or -1); jet_btag is the b-tag discriminant (tagged when above the
 * threshold).  n_var optionally gives a per-event variation count (1..65535);
 * when NULL every event uses hf_reco_params_t.n_var_uniform.  index_base is
 * the global id of event 0: it keys the random streams and is added to the
 * compaction output.  Capacity limits: n < 2^31, index_base + n < 2^31. */
typedef struct hf_events {
    int64_t n;
    int64_t index_base;
    const uint32_t *lep_off, *jet_off; /* [n+1] */
    const float *lep_pt, *lep_eta, *lep_phi, *lep_e, *lep_q;
    const float *jet_pt, *jet_eta, *jet_phi, *jet_e, *jet_btag;
    const float *met_x, *met_y; /* [n] */
    const uint16_t *n_var;      /* [n] or NULL */
} hf_events_t;

/* Cut kinds (section 3: each cut is a boolean predicate of one event;
 * section 6.1: the HL-LHC selection).  Object selection inside a cut is
 * pT > pt_min and |eta| < eta_max (strict); a jet is b-tagged when
 * btag > btag_min.  Parameters:
 *   HF_CUT_LEP_N_OS     f = {pt_min, eta_max}             i = {n_exact, opposite_sign}
 *   HF_CUT_JET_N_MIN    f = {pt_min, eta_max}             i = {n_min}
 *   HF_CUT_BTAG_N_MIN   f = {pt_min, eta_max, btag_min}   i = {n_min}
 *   HF_CUT_BTAG_N_EQ    f = {pt_min, eta_max, btag_min}   i = {n_exact}
 *   HF_CUT_MET_MIN      f = {met_min}                     (E_T^miss > met_min)
 *   HF_CUT_MLL_MIN      f = {pt_min, eta_max, mll_min}    (two leading selected leptons)
 *   HF_CUT_FWD_JET_VETO f = {pt_min, abs_eta_lo, abs_eta_hi} (fails on a jet in [lo, hi))
 *   HF_CUT_LEP_ISO      f = {lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, dr_min}
 *                       (every selected lepton at Delta R >= dr_min from every
 *                        selected jet; Delta R = sqrt(Delta eta^2 + Delta phi^2))
 *   HF_CUT_RECO         the kinematic reconstruction (section 4: last cut);
 *                       hf_select skips it, hf_ttbar_reco or hf_semilep_reco
 *                       fills its counters.
 *   HF_CUT_MTW_MIN      f = {lep_pt_min, lep_eta_max, mtw_min}
 *                       (W transverse mass of the leading selected lepton and
 *                        the missing momentum, M_T^2 = 2 (pT_l MET - pT_l . MET),
 *                        above mtw_min; fails without a selected lepton;
 *                        section 6.1)
 *   HF_CUT_USER         a user predicate compiled at run time by
 *                       hf_chain_compile; i = {index of its source, loop
 *                       budget (0: HF_USER_LOOP_BUDGET)}
 *   HF_CUT_JET_N_RANGE  f = {pt_min, abs_eta_lo, abs_eta_hi}  i = {n_min, n_max}
 *                       (the number of jets with pT > pt_min and
 *                        abs_eta_lo <= |eta| < abs_eta_hi lies in
 *                        [n_min, n_max]; section 6.1: jet counts in the
 *                        central Region I and the forward Regions II, III) */
enum {
    HF_CUT_LEP_N_OS = 0,
    HF_CUT_JET_N_MIN = 1,
    HF_CUT_BTAG_N_MIN = 2,
    HF_CUT_BTAG_N_EQ = 3,
    HF_CUT_MET_MIN = 4,
    HF_CUT_MLL_MIN = 5,
    HF_CUT_FWD_JET_VETO = 6,
    HF_CUT_LEP_ISO = 7,
    HF_CUT_RECO = 8,
    HF_CUT_MTW_MIN = 9,
    HF_CUT_USER = 10,
    HF_CUT_JET_N_RANGE = 11
};

/* A cut of the chain.  Its id is its index in the cut table.  Bit j of
 * dep_mask means cut j must come earlier in any order (section 5.2:
 * reordering respects the dependencies between cuts). */
typedef struct hf_cut {
    int32_t kind;
    int32_t reserved; /* must be 0 */
    uint64_t dep_mask;
    float f[8];
    int32_t i[4];
} hf_cut_t;

/* Per-cut counters, indexed by cut id, accumulated (+=) by every call.
 * For the cut at position k of the order: reached = events that survived
 * positions 0..k-1, passed = events that also pass position k, cost = device
 * clock cycles spent evaluating it, summed over wavefronts (section 5.2: the
 * filter ratio and the measured time of each cut drive the reordering). */
typedef struct hf_counters {
    uint64_t reached, passed, cost;
} hf_counters_t;

/* ---------------------------------------------------------------- errors */

/* Message of the last error raised on this host thread ("" if none). */
const char *hf_last_error(void);

/* Library version string. */
const char *hf_version(void);

/* ------------------------------------------------------------- selection */

/* Workspace bytes hf_select needs for n events and n_cuts cuts. */
size_t hf_select_workspace_size(int64_t n, int n_cuts);

/* Evaluate the cut chain on every event of ev (sections 3 and 5.2).
 *   h_cuts[n_cuts]  cut table (host), 1 <= n_cuts <= HF_MAX_CUTS;
 *   d_order[n_cuts] device int32: cut ids in evaluation order (a permutation;
 *                   ids out of range are skipped); kept on the device so that
 *                   a recorded graph picks up a new order without re-recording;
 *   d_survive[n]    out: 1 if the event passes every non-RECO cut, else 0;
 *   d_counters      in/out: hf_counters_t[n_cuts], accumulated;
 *   d_ws, ws_bytes  workspace of at least hf_select_workspace_size(n, n_cuts).
 * An event stops at its first failed cut; a wavefront whose 64 events have
 * all failed skips the remaining cuts and their loads.  Errors: HF_ERR_INVAL
 * for null pointers, n < 0 or a bad cut table; HF_ERR_CAPACITY for a short
 * workspace. */
int hf_select(const hf_events_t *ev, const hf_cut_t *h_cuts, int n_cuts, const int32_t *d_order,
              uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes,
              hipStream_t stream);

/* ------------------------------------------------------------ compaction */

/* Workspace bytes hf_compact needs for up to `capacity` mask entries. */
size_t hf_compact_workspace_size(int64_t capacity);

/* Indices of the set entries of a byte mask, in ascending order (section 3:
 * the events passing all cuts form the filtered output).
 *   d_mask[capacity]  1 = keep, 0 = drop (any nonzero byte keeps);
 *   d_n               device int64 holding the number of mask entries to use
 *                     (clamped to capacity), or NULL to use all of them; lets
 *                     the count produced by an earlier call drive this one;
 *   d_map             device int32[capacity] or NULL: the output for entry e is
 *                     d_map[e] if given, else index_base + e;
 *   d_idx[capacity]   out: the kept indices, ascending;
 *   d_count           out: device int64, number of kept entries.
 * Errors: HF_ERR_INVAL for null pointers or capacity < 0; HF_ERR_CAPACITY
 * for a short workspace or capacity >= 2^31. */
int hf_compact(const uint8_t *d_mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
               const int32_t *d_map, int32_t *d_idx, int64_t *d_count, void *d_ws, size_t ws_bytes,
               hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hf_compact
 * with the workspace held by the library instead of passed in.  Same
 * arguments, semantics and errors as hf_compact without d_ws and ws_bytes;
 * capacity is limited to HF_COMPACT_NOALLOC_MAX_ENTRIES (HF_ERR_CAPACITY
 * above it).  The workspace is a fixed device array of about 256 KiB per
 * GPU, resolved on the first call with each device current and kept until
 * the process ends; the call allocates and frees nothing.  The stream must
 * belong to the current device.  Every call on one GPU shares that array:
 * calls whose work overlaps on one GPU (other streams, other host threads)
 * race and must be ordered by the caller. */
#define HF_COMPACT_NOALLOC_MAX_ENTRIES ((int64_t)1 << 28)
int hf_compact_noalloc(const uint8_t *d_mask, int64_t capacity, const int64_t *d_n, int64_t index_base,
                       const int32_t *d_map, int32_t *d_idx, int64_t *d_count, hipStream_t stream);

/* ------------------------------------------------------- reconstruction */

#define HF_PREC_FP64 0  /* every step in FP64 */
#define HF_PREC_MIXED 1 /* the Box-Muller transcendentals of the draws and the
                           closed-form seed of the pencil cubic's isolated root in
                           FP32 (refined in FP64); kinematic staging, smear
                           factors, linear maps, the pencil and its line pair,
                           polish and scores in FP64 (FP32 staging and smearing
                           miss the 1e-4 agreement with the FP64 oracle on
                           near-tangent solutions) */
#define HF_PAIR_BTAG_FILL 0 /* b candidates: tagged selected jets in input order
                               (descending pT), at most max_cands, filled up to two
                               with the leading untagged selected jets */
#define HF_PAIR_ALL_JETS 1  /* b candidates: every selected jet (at most max_cands) */

/* Reconstruction parameters (section 4; the resolution model and the choice
 * rule are the readings listed in the design notes).  m_t and m_w are the
 * top and W masses of the constraints (172.5 and 80.4 GeV in the paper);
 * lambda_pt scales the top-pT term of the score.  Each variation scales
 * every component of a 4-vector by max(1 + sigma z, 0.01) with z a standard
 * normal: jets sigma = sqrt(jet_a^2 / E + jet_c^2) at the nominal energy,
 * leptons sigma = lep_sigma; MET components are shifted by met_sigma z.
 * smear = 0 gives every variation z = 0.  Random streams: Philox4x32-10
 * keyed by seed, counter (global event id, variation, block).  reco_cut is
 * the id of the RECO cut whose counters the call updates (-1: none).
 * schedule is a launch choice that leaves every result unchanged: the
 * search runs one wavefront per event (lanes over its variations) on a
 * persistent grid, in workgroups of four (HF_SCHED_EVENT), two
 * (HF_SCHED_EVENT_WG128) or one (HF_SCHED_EVENT_WG64) wavefronts, eight
 * wavefronts per CU in every case.  HF_SCHED_AUTO takes the choice that
 * hf_ttbar_reco_autotune stored for this configuration in the file named by
 * HF_AUTOTUNE_CACHE, if any, else HF_SCHED_EVENT.  (The value 2 named a
 * worklist schedule that was slower on every workload and is rejected.) */
#define HF_SCHED_AUTO 0
#define HF_SCHED_EVENT 1
#define HF_SCHED_EVENT_WG64 3
#define HF_SCHED_EVENT_WG128 4

typedef struct hf_reco_params {
    double m_t, m_w, lambda_pt;
    double jet_a, jet_c, lep_sigma, met_sigma;
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    int32_t reco_cut;
    uint64_t seed;
    int32_t smear, n_var_uniform, precision, pair_mode, max_cands, want_mbb;
    int32_t schedule, reserved;
} hf_reco_params_t;

/* Outputs, structure of arrays over the compacted positions [0, capacity);
 * entries at positions >= *d_count are left untouched.  nu and nubar hold
 * (px, py, pz) per position ([capacity][3]).  best_i/best_j are the jet
 * indices (within the event) paired with l+ and l-; best_v the variation.
 * n_sol counts the accepted solutions over all variations and pairings.
 * Masses are recomputed from the chosen solution; logw is its score; m_bb
 * (may be NULL) is the mass of the two leading remaining b jets.  Positions
 * without a solution get has_sol = 0, best_* = -1 and HF_NO_SOLUTION in every
 * float output.  stats (may be NULL) accumulates 5 uint64 counts: events,
 * variations, pairings solved, real common points of the pairings' two
 * conics found, accepted solutions. */
typedef struct hf_reco_out {
    uint8_t *has_sol;
    int32_t *n_sol, *best_v;
    int16_t *best_i, *best_j;
    double *nu, *nubar;
    double *m_t, *m_tbar, *m_wp, *m_wm, *logw, *m_bb;
    uint64_t *stats;
} hf_reco_out_t;

/* Workspace bytes hf_ttbar_reco needs for `capacity` compacted events. */
size_t hf_ttbar_reco_workspace_size(int64_t capacity);

/* Dileptonic ttbar kinematic reconstruction of the compacted events
 * (section 4): for each event d_idx[k] (global id, k < *d_count <= capacity),
 * every variation and every ordered pairing of two b candidates (the first
 * with l+, the second with l-), solve the two-neutrino system from the W and
 * top mass constraints (the common points of two conics in the neutrino's
 * transverse momentum, up to four), keep the solution
 * with the highest score, and mark the event as passing the RECO cut when at
 * least one solution exists.  Updates d_counters[reco_cut] (reached += count,
 * passed += events with a solution).  Errors: HF_ERR_INVAL for null pointers,
 * bad enums or parameters; HF_ERR_CAPACITY for a short workspace. */
int hf_ttbar_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                  const hf_reco_params_t *h_params, const hf_reco_out_t *out, hf_counters_t *d_counters,
                  void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Autotuner for the launch of hf_ttbar_reco (section 5: the framework
 * adapts its execution to the hardware and the workload).  Runs the same
 * reconstruction once per candidate schedule (HF_SCHED_EVENT,
 * HF_SCHED_EVENT_WG128, HF_SCHED_EVENT_WG64) after a warm-up, times each
 * with HIP events on `stream`, writes the fastest into h_params->schedule
 * and, when the
 * environment variable HF_AUTOTUNE_CACHE names a file, appends the choice
 * under this configuration's key (device, precision, pairing mode, variation
 * layout, capacity bucket) so that later HF_SCHED_AUTO calls in any process
 * use it.  The outputs are those of an ordinary call; counters and stats are
 * not updated.  Synchronises `stream` (not for graph capture).
 *   h_ms: NULL or double[3], receives the measured milliseconds per call of
 *         HF_SCHED_EVENT, HF_SCHED_EVENT_WG128 and HF_SCHED_EVENT_WG64.
 * Errors: those of hf_ttbar_reco; HF_ERR_DEVICE if timing fails. */
int hf_ttbar_reco_autotune(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                           hf_reco_params_t *h_params, const hf_reco_out_t *out, void *d_ws, size_t ws_bytes,
                           hipStream_t stream, double *h_ms);

/* Instrumentation: from the next call on, hf_ttbar_reco records `start` just
 * before and `stop` just after its search kernel (the kernel that intersects
 * the conics), on the stream of the call, so that the caller can time that
 * kernel alone with hipEventElapsedTime.  Both NULL switches it off.  The
 * events are created and owned by the caller and must outlive the calls that
 * record them.  Process-wide setting; calls from several threads race.
 * Errors: HF_ERR_INVAL if exactly one of the two is NULL. */
int hf_reco_timing_events(hipEvent_t start, hipEvent_t stop);

/* One segment of a cut chain (section 5.2: heavy cuts placed late in the
 * pipeline process fewer events): the cuts at positions [pos_begin, pos_end)
 * of d_order, over all events of the chunk (d_idx == NULL; d_survive[n]
 * indexed by event) or over the compacted global ids
 * d_idx[0, min(*d_count, capacity)) (d_survive[capacity] indexed by
 * position; an id outside the chunk fails without being counted).  Running
 * positions [0, s) over all events, compacting, then [s, n_cuts) over the
 * compacted ids (hf_compact with d_map = d_idx carries the ids forward)
 * gives the same survivors and counters as one hf_select, with the later
 * cuts evaluated by densely packed wavefronts.  Counters accumulate as in
 * hf_select.  Workspace: hf_select_workspace_size(d_idx ? capacity : n,
 * n_cuts).  Errors: those of hf_select; HF_ERR_INVAL unless
 * 0 <= pos_begin <= pos_end <= n_cuts, or for d_idx without d_count or a
 * capacity outside [0, 2^31). */
int hf_select_segment(const hf_events_t *ev, const hf_cut_t *h_cuts, int n_cuts, const int32_t *d_order,
                      int pos_begin, int pos_end, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                      uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes,
                      hipStream_t stream);

/* ------------------------------------------------------------- ingest */

/* Workspace bytes hf_unpack_events needs for n events. */
size_t hf_unpack_workspace_size(int64_t n);

/* Rebuild the offsets and the charge and b-tag columns of hf_events_t from a
 * packed transfer format, so that a chunk crosses the host link in fewer
 * bytes (section 3: many events are loaded and processed at once; the
 * loading is overlapped with the processing).  In: per-event lepton and jet
 * counts as bytes d_lep_cnt[n], d_jet_cnt[n] (16-byte aligned), charges as
 * signed bytes d_lep_q8[n_lep], b-tags as bytes d_jet_btag8[n_jet].  Out:
 * d_lep_off[n + 1], d_jet_off[n + 1] (exclusive prefix sums of the counts),
 * d_lep_q[n_lep], d_jet_btag[n_jet] (the bytes as float32).  The other
 * columns travel as float32 unchanged.  Byte and integer work: the result
 * equals the unpacked columns exactly; the counts must sum to n_lep and
 * n_jet, both below 2^32.  Asynchronous, allocates nothing.  Errors:
 * HF_ERR_INVAL for null pointers, sizes out of range or misaligned counts;
 * HF_ERR_CAPACITY for a short workspace. */
int hf_unpack_events(int64_t n, const uint8_t *d_lep_cnt, const uint8_t *d_jet_cnt, int64_t n_lep, int64_t n_jet,
                     const int8_t *d_lep_q8, const uint8_t *d_jet_btag8, uint32_t *d_lep_off, uint32_t *d_jet_off,
                     float *d_lep_q, float *d_jet_btag, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------ user-defined cuts */

/* A cut chain with user predicates (section 3: the user registers each cut
 * of the pipeline as a function of one event that returns a boolean).  Each
 * HF_CUT_USER cut names one source h_user_src[i[0]]: the body of a C function
 * of one event that returns nonzero when the event passes, written against
 * these accessors (float values of the event's columns; an index outside
 * the event's list reads 0):
 *   n_lep(), n_jet()                      object counts (int)
 *   lep_pt(i) lep_eta(i) lep_phi(i) lep_e(i) lep_q(i)
 *   jet_pt(i) jet_eta(i) jet_phi(i) jet_e(i) jet_btag(i)
 *   met_x(), met_y()
 * plus the C math functions and local variables, loops and conditionals,
 * e.g. "int n = 0; for (int k = 0; k < n_jet(); ++k) n += fabsf(jet_eta(k))
 * >= 2.5f; return n >= 1;".  Arithmetic is compiled without contraction
 * (-ffp-contract=off).  Loops are bounded: every iteration of a for, while
 * or do-while loop spends one unit of the cut's budget for the event (the
 * cut's i[1], or HF_USER_LOOP_BUDGET when it is 0) -- a for loop as an
 * iteration starts, a while or do-while loop when its condition lets
 * another iteration run -- and a predicate that would run past its budget
 * stops and fails the event, so no predicate can hang the chain kernel.
 * goto is not accepted; recursion (through lambdas) is not bounded.
 *
 * hf_chain_compile generates the chain kernel with the user predicates
 * inlined, compiles it for the current device with hipRTC and loads it
 * (this call allocates: the code object; it is a set-up call, not one to
 * record into a graph).  h_cuts[n_cuts] may mix built-in kinds and
 * HF_CUT_USER; n_user sources are given.  *out receives the chain, owned by
 * the caller (hf_chain_destroy); on failure *out is NULL and the compiler's
 * messages are in hf_last_error().
 * Errors: HF_ERR_INVAL for malformed cut tables, a user index outside
 * [0, n_user), a negative loop budget, a NULL source or a source that does
 * not compile;
 * HF_ERR_DEVICE if loading the code fails. */
typedef struct hf_chain hf_chain_t;

/* Default loop budget of a user predicate, iterations per event. */
#define HF_USER_LOOP_BUDGET 65536

int hf_chain_compile(const hf_cut_t *h_cuts, int n_cuts, const char *const *h_user_src, int n_user,
                     hf_chain_t **out);

/* hf_select for a compiled chain: the same kernel structure, order,
 * counters, survive mask and workspace (hf_select_workspace_size(n, n_cuts));
 * every event column must be present.  Asynchronous, allocates nothing, may
 * be recorded into a HIP graph.  Errors: those of hf_select. */
int hf_chain_select(const hf_chain_t *chain, const hf_events_t *ev, const int32_t *d_order, uint8_t *d_survive,
                    hf_counters_t *d_counters, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* hf_select_segment for a compiled chain. */
int hf_chain_select_segment(const hf_chain_t *chain, const hf_events_t *ev, const int32_t *d_order, int pos_begin,
                            int pos_end, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                            uint8_t *d_survive, hf_counters_t *d_counters, void *d_ws, size_t ws_bytes,
                            hipStream_t stream);

/* The compiler's messages for the chain ("" if none). */
const char *hf_chain_log(const hf_chain_t *chain);

/* Releases the chain's code object.  NULL is ignored. */
void hf_chain_destroy(hf_chain_t *chain);

/* ------------------------------------- single-neutrino reconstruction */

#define HF_TOPO_TCHAN 0  /* t-channel single top: one top (j l nu), one W (l nu) */
#define HF_TOPO_WT 1     /* Wt, semileptonic: one top (j l nu), W (l nu) and W (p q) */
#define HF_TOPO_TTSEMI 2 /* semileptonic ttbar: tops (j l nu) and (h p q), W (l nu) and W (p q) */

/* Parameters of the chi^2 reconstruction (section 6.2, Eq. (chi2)): m_t and
 * m_w are the central masses (172.5 and 80.4 GeV in the paper), sigma_t and
 * sigma_w the widths (11.5 and 7.5 GeV).  The lepton is the leading one with
 * pT > lep_pt_min and |eta| < lep_eta_max; the candidate jets are the jets
 * with pT > jet_pt_min and |eta| < jet_eta_max, in input (pT) order, at most
 * max_cands (1..HF_MAX_CANDS).  reco_cut is the id of the RECO cut whose
 * counters the call updates (-1: none); reserved must be 0. */
typedef struct hf_semilep_params {
    double m_t, m_w, sigma_t, sigma_w;
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max;
    int32_t topology, max_cands, reco_cut, reserved;
} hf_semilep_params_t;

/* Outputs, structure of arrays over the compacted positions [0, capacity);
 * positions >= *d_count are left untouched.  root: 0 (minus sign) or 1 (plus
 * sign) root of the neutrino p_z quadratic, 2 when its discriminant is
 * negative and the real part was taken.  best_j: the jet of the leptonic top;
 * best_h: the b jet of the hadronic top (semileptonic ttbar); best_p < best_q:
 * the jets of the two-jet W (Wt, semileptonic ttbar); -1 where the topology
 * has no such jet.  Jet indices are within the event.  nu: (px, py, pz) of the
 * neutrino ([capacity][3]).  m_tl, m_wl: leptonic top and W masses; m_th,
 * m_wh: hadronic top and W masses (HF_NO_SOLUTION where absent); chi2: the
 * minimum.  Positions without a solution (no selected lepton, fewer jets than
 * the topology needs, an id outside the chunk) get has_sol = 0, -1 indices
 * and HF_NO_SOLUTION in every float output. */
typedef struct hf_semilep_out {
    uint8_t *has_sol;
    int8_t *root;
    int16_t *best_j, *best_h, *best_p, *best_q;
    double *nu;
    double *m_tl, *m_wl, *m_th, *m_wh, *chi2;
} hf_semilep_out_t;

/* Single-neutrino kinematic reconstruction of the compacted events
 * (section 6.2): for each event d_idx[k] (global id, k < *d_count <=
 * capacity), the missing transverse momentum is the neutrino's transverse
 * momentum and its p_z solves (l + nu)^2 = m_W^2 for a massless neutrino:
 *   p_z = (mu pz_l -/+ E_l sqrt(mu^2 - a pT^2)) / a,
 *   mu = (m_W^2 - m_l^2)/2 + px_l px + py_l py,  a = E_l^2 - pz_l^2,
 * or mu pz_l / a when the discriminant is negative.  Every assignment of
 * distinct candidate jets to the topology's tops and W bosons, with every p_z
 * candidate, is scored by Eq. (chi2) and the smallest chi^2 is kept (ties:
 * the first in the order root, j, h, p, q).  Every step runs in FP64 on the
 * device.  Updates d_counters[reco_cut] (reached += count, passed += events
 * with a solution).  Allocates nothing; no workspace.  Errors: HF_ERR_INVAL
 * for null pointers, an unknown topology, max_cands outside
 * [1, HF_MAX_CANDS], non-positive widths or masses with m_t <= m_w. */
int hf_semilep_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                    const hf_semilep_params_t *h_params, const hf_semilep_out_t *out, hf_counters_t *d_counters,
                    hipStream_t stream);

/* --------------------------- dileptonic chi^2 fit with a MET split */

/* Parameters of the chi^2 fit of the dileptonic final state (section 6.2):
 * the masses and widths of Eq. (chi2) (172.5, 80.4, 11.5, 7.5 GeV in the
 * paper); leptons and b candidates as for hf_ttbar_reco (pair_mode,
 * max_cands in [2, HF_MAX_CANDS], the selection thresholds); the split
 * search: n_grid in [2, 129] points per axis over [-half_range, half_range]
 * (GeV, > 0), n_refine in [0, 8] refinements; reco_cut as for hf_ttbar_reco;
 * n_top the number of top quarks of Eq. (chi2): 2 (or 0) for ttbar, 1 for
 * Wt, whose second W comes from the hard process (section 6.2: one top and
 * two W bosons in Wt events). */
typedef struct hf_chi2_params {
    double m_t, m_w, sigma_t, sigma_w, half_range;
    float lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    int32_t pair_mode, max_cands, n_grid, n_refine, reco_cut, n_top;
} hf_chi2_params_t;

/* Outputs over the compacted positions [0, capacity) (positions >= *d_count
 * untouched): root_nu, root_nubar as hf_semilep_out_t's root; best_i, best_j
 * the b jets (indices within the event) of the l+ and l- sides; nu, nubar
 * (px, py, pz) [capacity][3]; the top and W masses; chi2 the minimum; split
 * the offset (u, v) of nu_T from MET/2 [capacity][2].  With one top, the
 * side without it has best_* = -1 and HF_NO_SOLUTION as its top mass.  No
 * solution (fewer than two opposite-sign leptons, fewer candidates than
 * tops, an id outside the chunk): has_sol = 0, -1 indices, HF_NO_SOLUTION
 * floats. */
typedef struct hf_chi2_out {
    uint8_t *has_sol;
    int8_t *root_nu, *root_nubar;
    int16_t *best_i, *best_j;
    double *nu, *nubar;
    double *m_t, *m_tbar, *m_wp, *m_wm, *chi2, *split;
} hf_chi2_out_t;

/* The chi^2 fit of the dileptonic final state (section 6.2): E_T^miss is
 * split between the two neutrinos, nu_T = MET/2 + (u, v) and
 * nubar_T = MET/2 - (u, v); each neutrino's p_z follows from its W mass as
 * in hf_semilep_reco; every ordered pairing of two b candidates (the first
 * with l+) and every pair of p_z candidates is scored by Eq. (chi2) with two
 * tops and two W (n_top = 1: every candidate forms the top with l+, then
 * with l-, and Eq. (chi2) has that top and both W).  (u, v) is searched on
 * an n_grid x n_grid grid, then
 * refined n_refine times on a 5 x 5 grid centred on the best point with a
 * quarter of the previous step (a refined point must be strictly better).
 * Ties go to the first grid point, then pairing, then roots.  FP64 on the
 * device.  Updates d_counters[reco_cut].  Allocates nothing.  Errors:
 * HF_ERR_INVAL for null pointers or parameters out of range. */
int hf_dilep_chi2_reco(const hf_events_t *ev, const int32_t *d_idx, const int64_t *d_count, int64_t capacity,
                       const hf_chi2_params_t *h_params, const hf_chi2_out_t *out, hf_counters_t *d_counters,
                       hipStream_t stream);

/* -------------------------------------------------------- random draws */

/* The variation draws the reconstruction uses (paper section 5.3 draws its
 * pseudo-experiment numbers from Mersenne Twister; here a counter-based
 * Philox4x32-10, Salmon et al. SC'11, so any implementation reproduces them).
 * hf_philox_blocks: raw generator output, d_out[k][0..3] =
 * Philox4x32-10(counter d_ctr[k][0..3], key (seed low, seed high)).
 * hf_gauss_draws: standard normal of Gaussian slot d_slot[k] for variation
 * d_v[k] of global event d_g[k], computed exactly as the reconstruction does
 * in the given precision (HF_PREC_MIXED: FP32, HF_PREC_FP64), widened to
 * double.  Slot s uses Philox block s/4 (counter = (g low, g high, v, s/4));
 * lanes (0,1) and (2,3) of a block are Box-Muller pairs with
 * u = (top 24 bits + 1/2) / 2^24, r = sqrt(-2 ln u_first),
 * z = r cos(2 pi u_second) for the even lane, r sin(...) for the odd one.
 * Errors: HF_ERR_INVAL for null pointers, n < 0 or a bad precision. */
int hf_philox_blocks(const uint32_t *d_ctr, uint64_t seed, uint32_t *d_out, int64_t n, hipStream_t stream);
int hf_gauss_draws(uint64_t seed, const int64_t *d_g, const int32_t *d_v, const int32_t *d_slot, int64_t n,
                   int precision, double *d_z, hipStream_t stream);

/* ------------------------------------------------------- cut reordering */

/* New cut order from accumulated counters (section 5.2: cuts that reject
 * more events and cost less go first, respecting dependencies; the user's
 * order is the starting point).  Host only.  For each cut: pass rate
 * p = passed/reached (1 if never reached), per-event cost c = cost/reached
 * (0 if never reached), rank r = c / max(1 - p, 1e-9).  Cuts are placed one
 * at a time: among those whose dependencies are all placed, the smallest
 * rank first, ties to the lower id.  For independent cuts this minimises the
 * expected cost sum_k c_k prod_{m<k} p_m.
 *   h_counters[n_cuts], h_cuts[n_cuts] in; h_order[n_cuts] out.
 * Errors: HF_ERR_INVAL for null pointers, n_cuts out of range or cyclic
 * dependencies (h_order is left unchanged). */
int hf_reorder_stats(const hf_counters_t *h_counters, const hf_cut_t *h_cuts, int n_cuts, int32_t *h_order);

/* The same rule on the device: reads d_counters and writes d_order on
 * `stream`, so that a step recorded into a HIP graph reorders its own cuts
 * for the next step without a host round trip (section 5.2's reordering
 * during the run).  Produces exactly the order hf_reorder_stats gives for
 * the same counters.  Asynchronous; allocates nothing.
 *   d_counters[n_cuts] device in; h_cuts[n_cuts] host in (dependencies);
 *   d_order[n_cuts] device out (also the order the next hf_select reads).
 * Errors: HF_ERR_INVAL for null pointers, n_cuts out of range, dependencies
 * out of range or cyclic (checked on the host at the call). */
int hf_reorder_device(const hf_counters_t *d_counters, const hf_cut_t *h_cuts, int n_cuts, int32_t *d_order,
                      hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HF_H */
