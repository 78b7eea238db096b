// Ingest from the packed transfer format: internal interface between the
// C-ABI front end and its kernel unit.  Not part of the public ABI.
#pragma once

#include "hf_internal.hpp"

namespace hf {

size_t unpack_ws_bytes(int64_t n);
hipError_t launch_unpack(int64_t n, const uint8_t *lc, const uint8_t *jc, int64_t n_lep, int64_t n_jet,
                         const int8_t *q8, const uint8_t *b8, uint32_t *loff, uint32_t *joff, float *q, float *b,
                         void *ws, hipStream_t s);

}  // namespace hf
