// Candidate export and baseband-dump triggers (host code).
//
// The introduction's case for real-time processing names two payoffs:
// immediate follow-up of significant events, and triggered dumps of the
// full-resolution baseband data, which cannot be stored continuously but can
// be held briefly in a buffer and written out when an event merits it.  The
// clusters of dedisp_cluster_events are the events; this file turns them into
// (a) a plain-text candidate list and (b) the raw-sample windows a baseband
// buffer should dump: the samples that fed the candidate's dedispersed span
// in every channel, over the candidate's whole DM range.
#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <unordered_map>
#include <vector>

#include "dedisp_internal.hpp"

using dd::fail;

extern "C" dedisp_status dedisp_write_candidates(const char* path, const dedisp_cluster* clusters,
                                                 int64_t n, const double* dm_list, int32_t ndm,
                                                 const int32_t* widths, int32_t nwidths,
                                                 double tsamp, int64_t t_offset, int32_t beam) {
    if (!path || (n > 0 && (!clusters || !dm_list || !widths)))
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (n < 0 || ndm < 1 || nwidths < 1 || !(tsamp > 0))
        return fail(DEDISP_ERR_INVALID_ARG, "need n >= 0, ndm >= 1, nwidths >= 1, tsamp > 0");
    for (int64_t k = 0; k < n; ++k) {
        const dedisp_cluster& c = clusters[k];
        if (c.dm_idx < 0 || c.dm_idx >= ndm || c.width_idx < 0 || c.width_idx >= nwidths)
            return fail(DEDISP_ERR_INVALID_ARG, "cluster %lld indexes outside the DM or width list",
                        static_cast<long long>(k));
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(DEDISP_ERR_INVALID_ARG, "cannot open %s for writing", path);
    std::fprintf(f,
                 "# snr t_peak time_s dm dm_idx width width_idx n_members t_lo t_hi dm_lo dm_hi "
                 "beam\n");
    for (int64_t k = 0; k < n; ++k) {
        const dedisp_cluster& c = clusters[k];
        const int64_t t = c.t_peak + t_offset;
        std::fprintf(f,
                     "%.9g %" PRId64 " %.17g %.17g %d %d %d %d %" PRId64 " %" PRId64 " %d %d %d\n",
                     static_cast<double>(c.snr), t, static_cast<double>(t) * tsamp,
                     dm_list[c.dm_idx], c.dm_idx, widths[c.width_idx], c.width_idx, c.n_members,
                     c.t_lo + t_offset, c.t_hi + t_offset, c.dm_lo, c.dm_hi, beam);
    }
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    if (!ok) return fail(DEDISP_ERR_INVALID_ARG, "write to %s failed", path);
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_trigger_windows(const dedisp_cluster* clusters, int64_t n,
                                                const int32_t* delays, int32_t ndm,
                                                int32_t nchans, float snr_min,
                                                int32_t min_members, int64_t pad, int64_t nsamps,
                                                dedisp_trigger* out, int64_t capacity,
                                                int64_t* n_out) {
    if (!n_out || (n > 0 && (!clusters || !delays)) || (capacity > 0 && !out))
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (n < 0 || ndm < 1 || nchans < 1 || pad < 0 || nsamps < 1 || capacity < 0)
        return fail(DEDISP_ERR_INVALID_ARG, "bad sizes");
    *n_out = 0;
    // per trial: smallest and largest delay over the channels
    std::vector<int32_t> dmin(ndm), dmax(ndm);
    for (int d = 0; d < ndm; ++d) {
        const int32_t* row = delays + static_cast<int64_t>(d) * nchans;
        dmin[d] = *std::min_element(row, row + nchans);
        dmax[d] = *std::max_element(row, row + nchans);
    }
    std::vector<dedisp_trigger> w;
    for (int64_t k = 0; k < n; ++k) {
        const dedisp_cluster& c = clusters[k];
        if (!(c.snr >= snr_min) || c.n_members < min_members) continue;
        if (c.dm_lo < 0 || c.dm_hi >= ndm || c.dm_lo > c.dm_hi || c.t_lo > c.t_hi)
            return fail(DEDISP_ERR_INVALID_ARG, "cluster %lld has bad ranges",
                        static_cast<long long>(k));
        int32_t lo = dmin[c.dm_lo], hi = dmax[c.dm_lo];
        for (int d = c.dm_lo + 1; d <= c.dm_hi; ++d) {
            lo = std::min(lo, dmin[d]);
            hi = std::max(hi, dmax[d]);
        }
        const int64_t s = std::max<int64_t>(0, c.t_lo + lo - pad);
        const int64_t e = std::min<int64_t>(nsamps, c.t_hi + hi + pad + 1);
        if (s >= e) continue;
        w.push_back(dedisp_trigger{s, e, c.snr, static_cast<int32_t>(k), 1});
    }
    std::sort(w.begin(), w.end(), [](const dedisp_trigger& a, const dedisp_trigger& b) {
        return a.start != b.start ? a.start < b.start : a.cluster < b.cluster;
    });
    // merge overlapping or touching windows; keep the strongest cluster
    std::vector<dedisp_trigger> m;
    for (const dedisp_trigger& t : w) {
        if (!m.empty() && t.start <= m.back().end) {
            dedisp_trigger& b = m.back();
            b.end = std::max(b.end, t.end);
            if (t.snr > b.snr || (t.snr == b.snr && t.cluster < b.cluster)) {
                b.snr = t.snr;
                b.cluster = t.cluster;
            }
            b.n_clusters += 1;
        } else {
            m.push_back(t);
        }
    }
    *n_out = static_cast<int64_t>(m.size());
    const int64_t k = std::min<int64_t>(capacity, *n_out);
    std::copy(m.begin(), m.begin() + k, out);
    if (*n_out > capacity)
        return fail(DEDISP_ERR_CAPACITY, "%lld windows, capacity %lld",
                    static_cast<long long>(*n_out), static_cast<long long>(capacity));
    dd::clear_error();
    return DEDISP_OK;
}

// Candidate selection for the triage network: per-width non-maximum
// suppression.  Within one boxcar width w, events are visited from the
// highest S/N down (ties: lower DM, earlier t_peak, lower index); an event
// is kept unless a kept event of the same width lies within dm_half trials
// and t_half_per_width * w samples of it (both strict).  Kept events are
// bucketed on a grid of dm_half x t_half * w cells, so each test looks at
// the 3 x 3 neighbouring cells only: O(n log n) for the sort, O(n) tests.
extern "C" dedisp_status dedisp_candidates_nms(const dedisp_event* events, int64_t n,
                                               const int32_t* widths, int32_t nwidths,
                                               int32_t dm_half, int32_t t_half_per_width,
                                               int64_t* keep_out, int64_t* n_keep) {
    if (!n_keep || (n > 0 && (!events || !keep_out)) || !widths)
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (n < 0 || nwidths < 1 || dm_half < 1 || t_half_per_width < 1)
        return fail(DEDISP_ERR_INVALID_ARG, "need n >= 0, nwidths >= 1, dm_half >= 1, t_half >= 1");
    for (int64_t i = 0; i < n; ++i)
        if (events[i].width_idx < 0 || events[i].width_idx >= nwidths || widths[events[i].width_idx] < 1)
            return fail(DEDISP_ERR_INVALID_ARG, "event %lld has no valid width", static_cast<long long>(i));
    std::vector<int64_t> order(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) order[static_cast<size_t>(i)] = i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        const dedisp_event& x = events[a];
        const dedisp_event& y = events[b];
        if (x.width_idx != y.width_idx) return x.width_idx < y.width_idx;
        if (x.snr != y.snr) return x.snr > y.snr;
        if (x.dm_idx != y.dm_idx) return x.dm_idx < y.dm_idx;
        if (x.t_peak != y.t_peak) return x.t_peak < y.t_peak;
        return a < b;
    });
    std::vector<int64_t> keep;
    std::unordered_map<uint64_t, std::vector<int64_t>> grid;
    auto floordiv = [](int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    auto key = [](int64_t cd, int64_t ct) {
        return (static_cast<uint64_t>(cd) << 40) ^ static_cast<uint64_t>(ct & ((int64_t(1) << 40) - 1));
    };
    int32_t cur_w = -1;
    for (int64_t i : order) {
        const dedisp_event& e = events[i];
        if (e.width_idx != cur_w) {
            grid.clear();
            cur_w = e.width_idx;
        }
        const int64_t tw = static_cast<int64_t>(t_half_per_width) * widths[e.width_idx];
        const int64_t cd = floordiv(e.dm_idx, dm_half), ct = floordiv(e.t_peak, tw);
        bool suppressed = false;
        for (int64_t a = cd - 1; a <= cd + 1 && !suppressed; ++a)
            for (int64_t b = ct - 1; b <= ct + 1 && !suppressed; ++b) {
                auto it = grid.find(key(a, b));
                if (it == grid.end()) continue;
                for (int64_t j : it->second) {
                    const dedisp_event& k = events[j];
                    if (std::llabs(static_cast<long long>(k.dm_idx) - e.dm_idx) < dm_half &&
                        std::llabs(static_cast<long long>(k.t_peak - e.t_peak)) < tw) {
                        suppressed = true;
                        break;
                    }
                }
            }
        if (suppressed) continue;
        grid[key(cd, ct)].push_back(i);
        keep.push_back(i);
    }
    std::sort(keep.begin(), keep.end());
    std::copy(keep.begin(), keep.end(), keep_out);
    *n_keep = static_cast<int64_t>(keep.size());
    dd::clear_error();
    return DEDISP_OK;
}
