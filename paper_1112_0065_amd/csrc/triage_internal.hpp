// Internal interface of the triage network used by the streaming server.
#pragma once

#include <vector>

#include "search_internal.hpp"

namespace dd {

// Scores (probability that an event is astrophysical) for n events of one
// series block [ndm][nout] (uint16) with boxcar widths W; stream-ordered.
// series block [ndm][nout] (uint16), pk_ws its find_peaks workspace, d_events
// device events.  Synchronises s.
dedisp_status triage_score_events(triage_model m, const void* series_u16, const void* pk_ws, int ndm,
                                  int64_t nout, const Widths& W, const dedisp_event* d_events, int64_t n,
                                  std::vector<float>* scores, hipStream_t s);

}  // namespace dd
