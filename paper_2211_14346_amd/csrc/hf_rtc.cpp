// Run-time compilation of cut chains with user predicates (paper section 3:
// the user's cuts are functions of one event returning a boolean).  The
// chain kernel of hf_cuts.hpp is a template over the evaluator of user
// predicates; a chain with user cuts instantiates it with the predicates
// inlined, through hipRTC, so that they run inside the same wavefront-level
// early-exit loop as the built-in cuts.  Host code.
#include <stdio.h>

#include <string>
#include <vector>

#include <hip/hiprtc.h>

#include "hf_rtc.hpp"

namespace hf {

namespace {

// Stand-ins for the host headers the shared device headers include: hipRTC
// has the device runtime built in but none of these files, and the host
// declarations in them only need the type names.
const char *const kStandInNames[] = {"hip/hip_runtime.h", "hip/hip_runtime_api.h", "stddef.h"};
const char *const kStandInSources[] = {
    "#pragma once\n#include <hip/hip_runtime_api.h>\n",
    "#pragma once\ntypedef int hipError_t;\ntypedef struct ihipStream_t *hipStream_t;\n"
    "typedef struct ihipEvent_t *hipEvent_t;\n",
    "#pragma once\n"};

// Accessors of a user predicate over the event being evaluated (hf_ev, hf_e)
// and its object ranges.
const char *kAccessors =
    "#define n_lep() ((int)hf_nl)\n"
    "#define n_jet() ((int)hf_nj)\n"
    "#define lep_pt(i) hf::user_col(hf_ev.lep_pt, hf_l0, hf_nl, (i))\n"
    "#define lep_eta(i) hf::user_col(hf_ev.lep_eta, hf_l0, hf_nl, (i))\n"
    "#define lep_phi(i) hf::user_col(hf_ev.lep_phi, hf_l0, hf_nl, (i))\n"
    "#define lep_e(i) hf::user_col(hf_ev.lep_e, hf_l0, hf_nl, (i))\n"
    "#define lep_q(i) hf::user_col(hf_ev.lep_q, hf_l0, hf_nl, (i))\n"
    "#define jet_pt(i) hf::user_col(hf_ev.jet_pt, hf_j0, hf_nj, (i))\n"
    "#define jet_eta(i) hf::user_col(hf_ev.jet_eta, hf_j0, hf_nj, (i))\n"
    "#define jet_phi(i) hf::user_col(hf_ev.jet_phi, hf_j0, hf_nj, (i))\n"
    "#define jet_e(i) hf::user_col(hf_ev.jet_e, hf_j0, hf_nj, (i))\n"
    "#define jet_btag(i) hf::user_col(hf_ev.jet_btag, hf_j0, hf_nj, (i))\n"
    "#define met_x() (hf_ev.met_x[hf_e])\n"
    "#define met_y() (hf_ev.met_y[hf_e])\n";

// Loops of a user predicate spend one unit of its budget per iteration: a
// for loop as an iteration starts, a while or do-while loop when its
// condition lets another iteration run.  Past the budget the loop stops and
// the predicate fails the event, so a predicate always ends.  goto (the one
// other way to loop without recursion) does not compile.
const char *kLoopBudget =
    "#define for(...) for (__VA_ARGS__) if (--*hf_budget < 0) { *hf_over = true; break; } else\n"
    "#define while(...) while ((__VA_ARGS__) && (--*hf_budget >= 0 || (*hf_over = true, false)))\n"
    "#define goto hf_user_cuts_may_not_use_goto\n";
const char *kLoopBudgetEnd = "#undef for\n#undef while\n#undef goto\n";

}  // namespace

std::string chain_source(const std::vector<std::string> &user_src) {
    // pi as the host's math.h defines it (hipRTC has no math.h)
    std::string s = "#define M_PI 3.14159265358979323846\n#include \"hf_cuts.hpp\"\n\nnamespace hf_user {\n\n";
    s += kAccessors;
    for (size_t u = 0; u < user_src.size(); ++u) {
        char head[640];
        snprintf(head, sizeof head,
                 "\n__device__ __forceinline__ bool body_%zu(const hf::EvView &hf_ev, int64_t hf_e, int64_t *hf_budget,\n"
                 "                                         bool *hf_over) {\n"
                 "    const uint32_t hf_l0 = hf_ev.lep_off[hf_e], hf_nl = hf_ev.lep_off[hf_e + 1] - hf_l0;\n"
                 "    const uint32_t hf_j0 = hf_ev.jet_off[hf_e], hf_nj = hf_ev.jet_off[hf_e + 1] - hf_j0;\n"
                 "    (void)hf_nl;\n    (void)hf_nj;\n    (void)hf_budget;\n    (void)hf_over;\n",
                 u);
        s += head;
        s += kLoopBudget;
        snprintf(head, sizeof head, "#line 1 \"user_cut_%zu\"\n", u);
        s += head;
        s += user_src[u];
        s += "\n#line 1 \"hf_user_chain_tail\"\n";
        s += kLoopBudgetEnd;
        snprintf(head, sizeof head,
                 "}\n__device__ __forceinline__ bool cut_%zu(const hf::EvView &hf_ev, int64_t hf_e, int32_t budget) {\n"
                 "    int64_t b = budget > 0 ? budget : HF_USER_LOOP_BUDGET;\n    bool over = false;\n"
                 "    const bool r = body_%zu(hf_ev, hf_e, &b, &over);\n    return r && !over;\n}\n",
                 u, u);
        s += head;
    }
    s += "\nstruct Cuts {\n    __device__ static bool eval(int u, const hf::EvView &ev, int64_t e, int32_t budget) {\n"
         "        switch (u) {\n";
    for (size_t u = 0; u < user_src.size(); ++u) {
        char c[96];
        snprintf(c, sizeof c, "        case %zu: return cut_%zu(ev, e, budget);\n", u, u);
        s += c;
    }
    s += "        default: return false;\n        }\n    }\n};\n\n}  // namespace hf_user\n";
    return s;
}

bool rtc_compile(const std::string &src, std::vector<char> &code, std::string &lowered, std::string &log) {
    std::vector<const char *> names, texts;
    for (int k = 0; k < kRtcHeaderCount; ++k) {
        names.push_back(kRtcHeaderNames[k]);
        texts.push_back(kRtcHeaderSources[k]);
    }
    for (int k = 0; k < 3; ++k) {
        names.push_back(kStandInNames[k]);
        texts.push_back(kStandInSources[k]);
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "hf_user_chain.hip", (int)names.size(), texts.data(),
                            names.data()) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return false;
    }
    const char *expr = "hf::k_select_t<hf_user::Cuts>";
    hiprtcAddNameExpression(prog, expr);
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "--offload-arch=gfx950";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = std::string("--offload-arch=") + prop.gcnArchName;
    const char *opts[] = {arch.c_str(), "-O3", "-std=c++17", "-ffp-contract=off", "-Werror=return-type",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    log.assign(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    while (!log.empty() && log.back() == '\0') log.pop_back();
    bool ok = r == HIPRTC_SUCCESS;
    if (ok) {
        const char *low = nullptr;
        size_t cs = 0;
        ok = hiprtcGetLoweredName(prog, expr, &low) == HIPRTC_SUCCESS && low &&
             hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
        if (ok) {
            lowered = low;
            code.resize(cs);
            ok = hiprtcGetCode(prog, code.data()) == HIPRTC_SUCCESS;
        }
    }
    hiprtcDestroyProgram(&prog);
    return ok;
}

}  // namespace hf
