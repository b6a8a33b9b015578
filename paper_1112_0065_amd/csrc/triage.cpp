// Triage network scoring hook of the streaming server.
#include "triage_internal.hpp"

namespace dd {

dedisp_status triage_score_events(triage_model m, const void* series_u16, int ndm, int64_t nout,
                                  const Widths& W, const dedisp_event* events, int64_t n,
                                  std::vector<float>* scores, hipStream_t s) {
    (void)m; (void)series_u16; (void)ndm; (void)nout; (void)W; (void)events; (void)n; (void)s;
    scores->clear();
    return fail(DEDISP_ERR_UNSUPPORTED, "no triage network in this build");
}

}  // namespace dd
