// Run-time compiled cut chains (user predicates): internal interfaces between
// the C-ABI front end, the hipRTC driver and the selection unit.  Host code.
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hf.h"
#include "hf_internal.hpp"

namespace hf {

// Threads per block of the chain kernel (kSelBlock of hf_cuts.hpp).
constexpr int kChainBlock = 256;

// Folds the chain kernel's per-block partial counter rows into counters.
hipError_t launch_select_reduce(const uint64_t *partial, int grid, int n_cuts, hf_counters_t *counters,
                                hipStream_t s);

// One segment of a chain (positions [pos_begin, pos_end) of the order) over
// all events (idx == nullptr) or over compacted ids (hf_select_segment).
hipError_t launch_select_segment(const EvView &ev, const CutTable &ct, const int32_t *order, int pos_begin,
                                 int pos_end, const int32_t *idx, const int64_t *count, int64_t capacity,
                                 uint8_t *survive, hf_counters_t *counters, void *ws, hipStream_t s);

// The device sources a generated chain kernel includes, embedded at build
// time: header names as the generated source and the headers include them,
// and their text.
extern const int kRtcHeaderCount;
extern const char *const kRtcHeaderNames[];
extern const char *const kRtcHeaderSources[];

// Generated source of a chain kernel with the given user predicate bodies.
std::string chain_source(const std::vector<std::string> &user_src);

// Compiles `src` for the current device; returns true and the code object
// on success; `log` receives the compiler's messages either way.
bool rtc_compile(const std::string &src, std::vector<char> &code, std::string &lowered, std::string &log);

}  // namespace hf

struct hf_chain {
    std::vector<hf_cut_t> cuts;
    int n_user = 0;
    std::string log;
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;
};
