// Multi-beam batch: all beams of a multibeam receiver (13 feed horns at
// Parkes, paper section 1) dedispersed by one persistent launch, followed by
// each beam's boxcar / sigma-cut / peak-finding chain, the whole sequence
// captured once in a HIP graph and replayed per batch.
//
// The graph is re-captured whenever a beam's input, output, event buffer,
// capacity or length changes.  Counters the persistent kernel pops work from
// are cleared by a kernel inside the graph (no memset nodes).
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "dedisp_internal.hpp"
#include "search_internal.hpp"

using dd::fail;

struct dedisp_batch_s {
    std::vector<dedisp_plan> plans;
    int nbeams = 0;
    dd::Widths W{};
    uint32_t kmant = 0;
    int kexp2 = 0;
    int out_u16 = 1;
    dd::TileConfig cfg{};
    int nl = 12;
    size_t lds = 0;
    int grid = 0;
    int nq = 8;
    dd::BeamArgs* d_beams = nullptr;
    unsigned long long* d_counters = nullptr;
    int64_t* h_totals = nullptr;   // pinned
    dd::BeamArgs* h_beams = nullptr;   // pinned descriptor staging
    std::vector<void*> words, pk_ws;
    std::vector<size_t> words_bytes, pk_bytes;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // optional stages (dedisp_batch_set_stages)
    int rfi_min = 0;                    // 0: no coincidence mask
    uint32_t rfi_kmant = 0;
    int rfi_kexp2 = 0;
    int bl_radius = 0;                  // 0: no baseline removal
    void* rfi_ws = nullptr;
    size_t rfi_ws_bytes = 0;
    void* d_mask = nullptr;
    size_t mask_bytes = 0;
    std::vector<void*> flat;
    std::vector<size_t> flat_bytes;
    // capture key
    std::vector<const void*> k_in, k_out, k_ev;
    std::vector<int64_t> k_nsamps, k_cap;
    int captures = 0;
};

namespace dd {

// Enqueue on `s`: descriptor upload (from pinned h_beams), repack of every
// item, one persistent dedispersion over all items, then each item's
// boxcar / sigma-cut / peak chain and the D2H copy of its event count.
hipError_t launch_multi(const MultiItem* items, int n, const Widths& W, uint32_t kmant, int kexp2,
                        int out_u16, const TileConfig& cfg, int nl, size_t lds, int grid, int nq,
                        BeamArgs* h_beams, BeamArgs* d_beams, unsigned long long* d_counters,
                        hipStream_t s, int bl_radius, int bl_offset) {
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const MultiItem& it = items[i];
        const int64_t nout = it.nsamps - it.plan->max_delay;
        h_beams[i] = beam_args(it.plan, static_cast<const uint2*>(it.words), repack_words(it.nsamps),
                               nout, it.out, cfg);
        if (!h_beams[i].offs) return hipErrorInvalidValue;   // table not built for this shape
        h_beams[i].item_begin = total;
        total += h_beams[i].n_items;
    }
    hipError_t e = hipMemcpyAsync(d_beams, h_beams, sizeof(BeamArgs) * n, hipMemcpyHostToDevice, s);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = launch_repack(items[i].in, items[i].nsamps, items[i].plan->nchans,
                          static_cast<uint2*>(items[i].words), repack_words(items[i].nsamps), s,
                          items[i].mask, items[i].mask_n);
    if (e == hipSuccess)
        e = launch_dedisperse_persistent(d_beams, n, total, nl, out_u16, cfg, lds, d_counters, nq,
                                         grid, s);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const MultiItem& it = items[i];
        const dedisp_plan_s* p = it.plan;
        int64_t nout = it.nsamps - p->max_delay;
        const void* series = it.out;
        if (it.flat) {
            // baseline removal between dedispersion and the search: the
            // search runs on the nout - 2R samples of the flattened series
            e = launch_baseline(it.out, out_u16, p->ndm, nout, bl_radius, bl_offset, it.flat,
                                out_u16, s);
            if (e != hipSuccess) break;
            series = it.flat;
            nout -= 2 * static_cast<int64_t>(bl_radius);
        }
        const PeaksLayout lay = peaks_layout(p->ndm, nout, W);
        const PeaksWs ws = peaks_ws(it.pk_ws, lay);
        e = launch_peaks_count(series, out_u16, p->ndm, nout, W, lay, ws, kmant, kexp2, s);
        if (e == hipSuccess && it.capacity > 0)
            e = launch_peaks_write(series, out_u16, p->ndm, nout, W, lay, ws, it.events, it.capacity, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(it.h_total, ws.total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    }
    return e;
}

int batch_grid(int nl, int out_u16, const TileConfig& cfg, size_t lds, int device, int nq) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    const int per_cu = persistent_blocks_per_cu(nl, out_u16, cfg, lds);
    if (cus < 1 || per_cu < 1) return 0;
    return ((cus * per_cu + nq - 1) / nq) * nq;
}

}  // namespace dd

namespace {

void release_graph(dedisp_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

dedisp_status ensure(void*& ptr, size_t& have, size_t need) {
    if (have >= need && ptr) return DEDISP_OK;
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    have = 0;
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "batch buffer of %zu bytes: %s", need, hipGetErrorString(e));
    have = need;
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status dedisp_batch_create(const dedisp_plan* plans, int32_t nbeams,
                                             const int32_t* widths, int32_t nwidths,
                                             float snr_thresh, dedisp_out_type out_type,
                                             const char* tune_cache_path, dedisp_batch* out) {
    if (!out || !plans || nbeams < 1 || nbeams > 1024)
        return fail(DEDISP_ERR_INVALID_ARG, "need 1..1024 plans and an output handle");
    *out = nullptr;
    if (out_type != DEDISP_OUT_I32 && out_type != DEDISP_OUT_U16)
        return fail(DEDISP_ERR_INVALID_ARG, "bad out_type");
    dd::Widths W;
    dedisp_status st = dd::check_widths_public(widths, nwidths, INT64_C(1) << 20, &W);
    if (st != DEDISP_OK) return st;
    uint32_t km;
    int ke;
    st = dd::split_threshold_public(snr_thresh, &km, &ke);
    if (st != DEDISP_OK) return st;
    const int nl = dd::levels_for(plans[0] ? plans[0]->nchans : 4);
    for (int i = 0; i < nbeams; ++i) {
        if (!plans[i]) return fail(DEDISP_ERR_INVALID_ARG, "plan %d is NULL", i);
        if (dd::levels_for(plans[i]->nchans) != nl)
            return fail(DEDISP_ERR_UNSUPPORTED, "beams need the same counter width (nchans %d vs %d)",
                        plans[i]->nchans, plans[0]->nchans);
        if (plans[i]->device != plans[0]->device)
            return fail(DEDISP_ERR_INVALID_ARG, "all plans must be on one device");
    }
    dedisp_batch_s* b = new (std::nothrow) dedisp_batch_s;
    if (!b) return fail(DEDISP_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->plans.assign(plans, plans + nbeams);
    b->nbeams = nbeams;
    b->W = W;
    b->kmant = km;
    b->kexp2 = ke;
    b->out_u16 = out_type == DEDISP_OUT_U16;
    b->nl = nl;
    b->cfg = dd::tuned_or_default(plans[0], tune_cache_path, b->out_u16);
    for (int i = 0; i < nbeams; ++i) b->lds = std::max(b->lds, dd::tile_lds_bytes(plans[i], b->cfg));
    if (b->lds > 160 * 1024) {
        delete b;
        return fail(DEDISP_ERR_UNSUPPORTED, "LDS tile of %zu bytes too large", b->lds);
    }
    b->grid = dd::batch_grid(nl, b->out_u16, b->cfg, b->lds, plans[0]->device, b->nq);
    if (b->grid < 1) {
        delete b;
        return fail(DEDISP_ERR_HIP, "occupancy query of the persistent kernel failed");
    }
    for (int i = 0; i < nbeams; ++i) {
        dedisp_status sto = DEDISP_OK;
        if (!dd::offset_table(plans[i], b->cfg, true, &sto)) {
            delete b;
            return sto;
        }
    }
    hipError_t e = hipSuccess;
    b->words.assign(nbeams, nullptr);
    b->pk_ws.assign(nbeams, nullptr);
    b->flat.assign(nbeams, nullptr);
    b->flat_bytes.assign(nbeams, 0);
    b->words_bytes.assign(nbeams, 0);
    b->pk_bytes.assign(nbeams, 0);
    e = hipMalloc(&b->d_beams, sizeof(dd::BeamArgs) * nbeams);
    if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(unsigned long long) * b->nq);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_totals, sizeof(int64_t) * nbeams, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(&b->h_beams, sizeof(dd::BeamArgs) * nbeams, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        dedisp_batch_destroy(b);
        return fail(DEDISP_ERR_HIP, "batch setup failed: %s", hipGetErrorString(e));
    }
    *out = b;
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_batch_destroy(dedisp_batch b) {
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "batch is NULL");
    release_graph(b);
    for (void* p : b->words)
        if (p) (void)hipFree(p);
    for (void* p : b->pk_ws)
        if (p) (void)hipFree(p);
    for (void* p : b->flat)
        if (p) (void)hipFree(p);
    if (b->rfi_ws) (void)hipFree(b->rfi_ws);
    if (b->d_mask) (void)hipFree(b->d_mask);
    if (b->d_beams) (void)hipFree(b->d_beams);
    if (b->d_counters) (void)hipFree(b->d_counters);
    if (b->h_totals) (void)hipHostFree(b->h_totals);
    if (b->h_beams) (void)hipHostFree(b->h_beams);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_batch_info(dedisp_batch b, dedisp_tile* tile, int32_t* grid,
                                           int32_t* captures) {
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "batch is NULL");
    if (tile) *tile = dedisp_tile{b->cfg.dms_per_block, b->cfg.groups, b->cfg.stage_chans};
    if (grid) *grid = b->grid;
    if (captures) *captures = b->captures;
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_batch_set_stages(dedisp_batch b, float rfi_k_sigma,
                                                 int32_t rfi_min_beams, int32_t baseline_radius) {
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "batch is NULL");
    uint32_t km = 0;
    int ke = 0;
    if (rfi_k_sigma != 0.0f) {
        dedisp_status st = dd::split_threshold_public(rfi_k_sigma, &km, &ke);
        if (st != DEDISP_OK) return st;
        if (rfi_min_beams < 1 || rfi_min_beams > b->nbeams || b->nbeams > 64)
            return fail(DEDISP_ERR_INVALID_ARG, "min_beams %d outside [1, %d] (at most 64 beams)",
                        rfi_min_beams, b->nbeams);
        for (int i = 1; i < b->nbeams; ++i)
            if (b->plans[i]->nchans != b->plans[0]->nchans)
                return fail(DEDISP_ERR_INVALID_ARG, "the coincidence mask needs one channel count");
    }
    if (baseline_radius < 0 || baseline_radius > 8192)
        return fail(DEDISP_ERR_INVALID_ARG, "baseline radius %d outside [0, 8192]", baseline_radius);
    if (baseline_radius > 0)
        for (int i = 0; i < b->nbeams; ++i)
            if (b->out_u16 && 6 * b->plans[i]->nchans > 65535)
                return fail(DEDISP_ERR_UNSUPPORTED, "uint16 baseline output needs 6 nchans <= 65535");
    b->rfi_min = rfi_k_sigma != 0.0f ? rfi_min_beams : 0;
    b->rfi_kmant = km;
    b->rfi_kexp2 = ke;
    b->bl_radius = baseline_radius;
    release_graph(b);   // the next execute captures the new sequence
    dd::clear_error();
    return DEDISP_OK;
}

namespace {

dedisp_status capture(dedisp_batch_s* b, const uint8_t* const* in, const int64_t* nsamps,
                      void* const* out, dedisp_event* const* events, const int64_t* capacity) {
    release_graph(b);
    int64_t n_common = nsamps[0];
    for (int i = 1; i < b->nbeams; ++i) n_common = std::min(n_common, nsamps[i]);
    const uint8_t* mask = b->rfi_min ? static_cast<const uint8_t*>(b->d_mask) : nullptr;
    std::vector<dd::MultiItem> items(b->nbeams);
    for (int i = 0; i < b->nbeams; ++i)
        items[i] = dd::MultiItem{b->plans[i], in[i], nsamps[i], b->words[i], out[i], b->pk_ws[i],
                                 events[i], capacity[i], &b->h_totals[i], mask, n_common,
                                 b->bl_radius ? b->flat[i] : nullptr};
    DD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (mask)
        e = dd::launch_rfi_mask(in, b->nbeams, b->plans[0]->nchans, n_common, b->rfi_kmant,
                                b->rfi_kexp2, b->rfi_min, static_cast<uint8_t*>(b->d_mask),
                                b->rfi_ws, b->cap);
    if (e == hipSuccess)
        e = dd::launch_multi(items.data(), b->nbeams, b->W, b->kmant, b->kexp2, b->out_u16, b->cfg,
                             b->nl, b->lds, b->grid, b->nq, b->h_beams, b->d_beams, b->d_counters,
                             b->cap, b->bl_radius, 3 * b->plans[0]->nchans);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(DEDISP_ERR_HIP, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    DD_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->captures++;
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status dedisp_batch_execute(dedisp_batch b, const uint8_t* const* in_2bit,
                                              const int64_t* nsamps, void* const* out,
                                              dedisp_event* const* events, const int64_t* capacity,
                                              int64_t* n_events, dedisp_stream stream) {
    if (!b || !in_2bit || !nsamps || !out || !events || !capacity || !n_events)
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    const int w_max = b->W.w[b->W.n - 1];
    for (int i = 0; i < b->nbeams; ++i) {
        const dedisp_plan_s* p = b->plans[i];
        if (!in_2bit[i] || !out[i] || capacity[i] < 0 || (capacity[i] > 0 && !events[i]))
            return fail(DEDISP_ERR_INVALID_ARG, "beam %d: NULL buffer or negative capacity", i);
        if (nsamps[i] - p->max_delay - 2 * static_cast<int64_t>(b->bl_radius) - w_max + 1 < 1)
            return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "beam %d: %lld samples", i,
                        static_cast<long long>(nsamps[i]));
        if ((nsamps[i] - p->max_delay + 16384 + w_max) * 4 >= (int64_t(1) << 31))
            return fail(DEDISP_ERR_UNSUPPORTED, "beam %d too long", i);
    }
    bool changed = !b->exec || b->k_in.size() != static_cast<size_t>(b->nbeams);
    for (int i = 0; i < b->nbeams && !changed; ++i)
        changed = b->k_in[i] != in_2bit[i] || b->k_out[i] != out[i] || b->k_ev[i] != events[i] ||
                  b->k_nsamps[i] != nsamps[i] || b->k_cap[i] != capacity[i];
    if (changed) {
        for (int i = 0; i < b->nbeams; ++i) {
            const dedisp_plan_s* p = b->plans[i];
            const int64_t nout = nsamps[i] - p->max_delay;
            dedisp_status st = ensure(b->words[i], b->words_bytes[i],
                                      static_cast<size_t>(p->nchans) * dd::repack_words(nsamps[i]) * sizeof(uint2));
            if (st != DEDISP_OK) return st;
            const int64_t nsearch = nout - 2 * static_cast<int64_t>(b->bl_radius);
            st = ensure(b->pk_ws[i], b->pk_bytes[i], dd::peaks_layout(p->ndm, nsearch, b->W).bytes);
            if (st != DEDISP_OK) return st;
            if (b->bl_radius) {
                st = ensure(b->flat[i], b->flat_bytes[i],
                            static_cast<size_t>(p->ndm) * nsearch * (b->out_u16 ? 2 : 4));
                if (st != DEDISP_OK) return st;
            }
        }
        if (b->rfi_min) {
            int64_t n_common = nsamps[0];
            for (int i = 1; i < b->nbeams; ++i) n_common = std::min(n_common, nsamps[i]);
            dedisp_status st = ensure(b->rfi_ws, b->rfi_ws_bytes, dd::rfi_mask_ws_bytes(b->nbeams, n_common));
            if (st != DEDISP_OK) return st;
            st = ensure(b->d_mask, b->mask_bytes, static_cast<size_t>(n_common));
            if (st != DEDISP_OK) return st;
        }
        dedisp_status st = capture(b, in_2bit, nsamps, out, events, capacity);
        if (st != DEDISP_OK) return st;
        b->k_in.assign(in_2bit, in_2bit + b->nbeams);
        b->k_out.assign(out, out + b->nbeams);
        b->k_ev.assign(reinterpret_cast<const void* const*>(events),
                       reinterpret_cast<const void* const*>(events) + b->nbeams);
        b->k_nsamps.assign(nsamps, nsamps + b->nbeams);
        b->k_cap.assign(capacity, capacity + b->nbeams);
    }
    DD_HIP(hipGraphLaunch(b->exec, stream));
    DD_HIP(hipStreamSynchronize(stream));
    dedisp_status st = DEDISP_OK;
    for (int i = 0; i < b->nbeams; ++i) {
        n_events[i] = b->h_totals[i];
        if (n_events[i] > capacity[i]) st = DEDISP_ERR_CAPACITY;
    }
    if (st != DEDISP_OK) return fail(st, "a beam found more events than its capacity");
    dd::clear_error();
    return DEDISP_OK;
}
