/*
 * orc_events.h -- the oracle's view of one chunk of events (FP64 columns
 * widened exactly from the float32 inputs) and the signature of a user
 * predicate.  TEST INFRASTRUCTURE ONLY (see hf_oracle.c).
 */
#ifndef ORC_EVENTS_H
#define ORC_EVENTS_H

#include <stdint.h>

typedef struct {
    int64_t n;
    int64_t index_base;
    const uint32_t *lep_off, *jet_off;
    const double *lep_pt, *lep_eta, *lep_phi, *lep_e, *lep_q;
    const double *jet_pt, *jet_eta, *jet_phi, *jet_e, *jet_btag;
    const double *met_x, *met_y;
    const int32_t *n_var; /* per event, or NULL */
} orc_events;

/* A user cut: nonzero when event e passes. */
/* A compiled user predicate of one event; budget: the most loop iterations
 * it may run for the event (it fails the event beyond that). */
typedef int (*orc_user_fn)(const orc_events *ev, int64_t e, int32_t budget);

#endif
