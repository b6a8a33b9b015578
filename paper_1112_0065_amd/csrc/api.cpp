// extern "C" entry points of the search chain: argument validation and
// kernel launches.  No entry point throws or aborts; every failure becomes a
// dedisp_status with a message for dedisp_last_error().
#include <cmath>
#include <cstring>
#include <mutex>

#include "dedisp_internal.hpp"
#include "search_internal.hpp"

namespace {

using dd::fail;

dedisp_status check_widths(const int32_t* widths, int32_t nwidths, int64_t nout, dd::Widths* W) {
    if (!widths || nwidths < 1 || nwidths > dd::kMaxWidths)
        return fail(DEDISP_ERR_INVALID_ARG, "need 1..%d widths", dd::kMaxWidths);
    for (int i = 0; i < nwidths; ++i) {
        if (widths[i] < 1) return fail(DEDISP_ERR_INVALID_ARG, "width %d < 1", widths[i]);
        if (i && widths[i] <= widths[i - 1])
            return fail(DEDISP_ERR_INVALID_ARG, "widths must be strictly increasing");
        W->w[i] = widths[i];
    }
    W->n = nwidths;
    const int w_max = widths[nwidths - 1];
    if (w_max > 32768) return fail(DEDISP_ERR_UNSUPPORTED, "widest boxcar %d > 32768", w_max);
    if (nout - w_max + 1 < 1)
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "series of %lld samples shorter than width %d",
                    static_cast<long long>(nout), w_max);
    // the search kernels address a series row (plus one segment's halo) with
    // 32-bit byte offsets
    if ((nout + 16384 + w_max) * 4 >= (int64_t(1) << 31))
        return fail(DEDISP_ERR_UNSUPPORTED, "series of %lld samples: rows must stay below 2^31 bytes",
                    static_cast<long long>(nout));
    return DEDISP_OK;
}

bool valid_type(dedisp_out_type t) { return t == DEDISP_OUT_I32 || t == DEDISP_OUT_U16; }

// The exact binary value of a positive float threshold: k = kmant * 2^kexp2,
// kmant odd.
dedisp_status split_threshold(float k, uint32_t* kmant, int* kexp2) {
    if (!std::isfinite(k) || !(k > 0.0f) || k > 1.0e6f)
        return fail(DEDISP_ERR_INVALID_ARG, "snr_thresh must be finite and in (0, 1e6]");
    int e = 0;
    const float m = std::frexp(k, &e);               // k = m * 2^e, m in [0.5, 1)
    uint32_t im = static_cast<uint32_t>(std::ldexp(m, 24));  // exact: 24-bit significand
    int ex = e - 24;
    while ((im & 1u) == 0u) {
        im >>= 1;
        ++ex;
    }
    *kmant = im;
    *kexp2 = ex;
    return DEDISP_OK;
}

}  // namespace

namespace dd {

dedisp_status split_threshold_public(float k, uint32_t* kmant, int* kexp2) {
    return split_threshold(k, kmant, kexp2);
}

dedisp_status check_widths_public(const int32_t* widths, int32_t nwidths, int64_t nout, Widths* W) {
    return check_widths(widths, nwidths, nout, W);
}

dedisp_status check_exec(dedisp_plan p, const void* workspace, int64_t nsamps) {
    if (!p || !workspace) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (nsamps <= p->max_delay)
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps=%lld <= max_delay=%lld",
                    static_cast<long long>(nsamps), static_cast<long long>(p->max_delay));
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(DEDISP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    int dev = -1;
    DD_HIP(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(DEDISP_ERR_INVALID_ARG, "current device %d differs from the plan's %d", dev,
                    p->device);
    return DEDISP_OK;
}

dedisp_status repack(dedisp_plan p, const uint8_t* in, int64_t nsamps, void* workspace,
                     hipStream_t stream) {
    dedisp_status st = check_exec(p, workspace, nsamps);
    if (st != DEDISP_OK) return st;
    if (!in) return fail(DEDISP_ERR_INVALID_ARG, "NULL input");
    DD_HIP(launch_repack(in, nsamps, p->nchans, static_cast<uint2*>(workspace),
                         repack_words(nsamps), stream));
    return DEDISP_OK;
}

dedisp_status execute_repacked(dedisp_plan p, const void* workspace, int64_t nsamps, void* out,
                               dedisp_out_type out_type, const TileConfig& cfg,
                               hipStream_t stream) {
    dedisp_status st = check_exec(p, workspace, nsamps);
    if (st != DEDISP_OK) return st;
    if (!out) return fail(DEDISP_ERR_INVALID_ARG, "NULL output");
    if (!valid_type(out_type)) return fail(DEDISP_ERR_INVALID_ARG, "bad out_type");
    st = launch_dedisperse(p, static_cast<const uint2*>(workspace), repack_words(nsamps),
                           nsamps - p->max_delay, out, out_type == DEDISP_OUT_U16, cfg, stream);
    if (st == DEDISP_OK) clear_error();
    return st;
}

dedisp_status execute_with_tile(dedisp_plan p, const uint8_t* in, int64_t nsamps, void* out,
                                dedisp_out_type out_type, void* workspace, const TileConfig& cfg,
                                hipStream_t stream) {
    if (!p || !in || !out || !workspace) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!valid_type(out_type)) return fail(DEDISP_ERR_INVALID_ARG, "bad out_type");
    dedisp_status st = repack(p, in, nsamps, workspace, stream);
    if (st != DEDISP_OK) return st;
    return execute_repacked(p, workspace, nsamps, out, out_type, cfg, stream);
}

}  // namespace dd

extern "C" dedisp_status dedisp_execute(dedisp_plan p, const uint8_t* in, int64_t nsamps,
                                        void* out, dedisp_out_type out_type, void* workspace,
                                        dedisp_stream stream) {
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    return dd::execute_with_tile(p, in, nsamps, out, out_type, workspace,
                                 dd::default_tile_config(p), stream);
}

namespace {

// (dms_per_block, groups) pairs with compiled kernels, times the stage sizes.
const int kShapes[][2] = {{4, 1}, {8, 1}, {16, 1}, {32, 1}, {4, 2}, {8, 2}, {16, 2}};
const int kStages[] = {8, 16, 32};

}  // namespace

extern "C" int32_t dedisp_tile_candidates(dedisp_tile* out, int32_t cap) {
    int32_t n = 0;
    for (const auto& sh : kShapes)
        for (int st : kStages) {
            if (out && n < cap) out[n] = dedisp_tile{sh[0], sh[1], st};
            ++n;
        }
    return n;
}

extern "C" dedisp_status dedisp_default_tile(dedisp_plan p, dedisp_tile* out) {
    if (!p || !out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    const dd::TileConfig c = dd::default_tile_config(p);
    *out = dedisp_tile{c.dms_per_block, c.groups, c.stage_chans};
    return DEDISP_OK;
}

namespace {

dedisp_status tile_from(const dedisp_tile* tile, dedisp_plan p, dd::TileConfig* cfg) {
    if (!tile) {
        *cfg = dd::default_tile_config(p);
        return DEDISP_OK;
    }
    bool ok = false;
    for (const auto& sh : kShapes)
        ok |= sh[0] == tile->dms_per_block && sh[1] == tile->groups;
    if (!ok || tile->stage_chans < 4 || tile->stage_chans > 128 || tile->stage_chans % 4)
        return fail(DEDISP_ERR_INVALID_ARG, "unsupported tile (%d, %d, %d)", tile->dms_per_block,
                    tile->groups, tile->stage_chans);
    *cfg = dd::TileConfig{tile->dms_per_block, tile->groups, tile->stage_chans};
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status dedisp_execute_tile(dedisp_plan p, const uint8_t* in, int64_t nsamps,
                                             void* out, dedisp_out_type out_type, void* workspace,
                                             const dedisp_tile* tile, dedisp_stream stream) {
    if (!p || !tile) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    dd::TileConfig cfg;
    dedisp_status st = tile_from(tile, p, &cfg);
    if (st != DEDISP_OK) return st;
    return dd::execute_with_tile(p, in, nsamps, out, out_type, workspace, cfg, stream);
}

extern "C" dedisp_status dedisp_repack(dedisp_plan p, const uint8_t* in, int64_t nsamps,
                                       void* workspace, dedisp_stream stream) {
    dedisp_status st = dd::repack(p, in, nsamps, workspace, stream);
    if (st == DEDISP_OK) dd::clear_error();
    return st;
}

extern "C" dedisp_status dedisp_execute_repacked(dedisp_plan p, const void* workspace,
                                                 int64_t nsamps, void* out,
                                                 dedisp_out_type out_type, const dedisp_tile* tile,
                                                 dedisp_stream stream) {
    if (!p) return fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    dd::TileConfig cfg;
    dedisp_status st = tile_from(tile, p, &cfg);
    if (st != DEDISP_OK) return st;
    return dd::execute_repacked(p, workspace, nsamps, out, out_type, cfg, stream);
}

extern "C" dedisp_status boxcar_filter(const void* in, dedisp_out_type in_type, int32_t ndm,
                                       int64_t nout, const int32_t* widths, int32_t nwidths,
                                       int32_t dm_first, int32_t dm_count, int32_t* out,
                                       dedisp_stream stream) {
    if (!in || !out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!valid_type(in_type)) return fail(DEDISP_ERR_INVALID_ARG, "bad in_type");
    if (ndm < 1 || nout < 1) return fail(DEDISP_ERR_INVALID_ARG, "need ndm >= 1 and nout >= 1");
    if (dm_first < 0 || dm_count < 1 || dm_first + static_cast<int64_t>(dm_count) > ndm || dm_count > 65535)
        return fail(DEDISP_ERR_INVALID_ARG, "DM range [%d, %d+%d) outside [0, %d)", dm_first,
                    dm_first, dm_count, ndm);
    dd::Widths W;
    dedisp_status st = check_widths(widths, nwidths, nout, &W);
    if (st != DEDISP_OK) return st;
    DD_HIP(dd::launch_boxcar(in, in_type == DEDISP_OUT_U16, ndm, nout, W, dm_first, dm_count, out,
                             stream));
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status baseline_remove(const void* in, dedisp_out_type in_type, int32_t ndm,
                                         int64_t nout, int32_t radius, int32_t offset, void* out,
                                         dedisp_out_type out_type, dedisp_stream stream) {
    if (!in || !out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!valid_type(in_type) || !valid_type(out_type))
        return fail(DEDISP_ERR_INVALID_ARG, "bad in_type or out_type");
    if (ndm < 1 || ndm > 65535) return fail(DEDISP_ERR_INVALID_ARG, "need 1 <= ndm <= 65535");
    if (radius < 0 || radius > 8192)
        return fail(DEDISP_ERR_INVALID_ARG, "radius %d outside [0, 8192]", radius);
    if (nout - 2 * static_cast<int64_t>(radius) < 1)
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "series of %lld samples, window of %d",
                    static_cast<long long>(nout), 2 * radius + 1);
    if ((nout + 8192 + 2 * static_cast<int64_t>(radius) + 1) * 4 >= (int64_t(1) << 31))
        return fail(DEDISP_ERR_UNSUPPORTED, "series rows must stay below 2^31 bytes");
    DD_HIP(dd::launch_baseline(in, in_type == DEDISP_OUT_U16, ndm, nout, radius, offset, out,
                               out_type == DEDISP_OUT_U16, stream));
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" size_t find_peaks_workspace_bytes(int32_t ndm, int64_t nout, const int32_t* widths,
                                             int32_t nwidths) {
    dd::Widths W;
    if (ndm < 1 || ndm > 65535 || check_widths(widths, nwidths, nout, &W) != DEDISP_OK) return 0;
    return dd::peaks_layout(ndm, nout, W).bytes;
}

namespace {

// The peak finder over a workspace of ws_cap bytes (0: the caller sized it
// with find_peaks_workspace_bytes).
dedisp_status find_peaks_impl(const void* in, dedisp_out_type in_type, int32_t ndm, int64_t nout,
                              const int32_t* widths, int32_t nwidths, float snr_thresh,
                              dedisp_event* events, int64_t capacity, int64_t* n_events,
                              void* workspace, size_t ws_cap, hipStream_t stream) {
    if (!in || !n_events || !workspace || (capacity > 0 && !events))
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (capacity < 0) return fail(DEDISP_ERR_INVALID_ARG, "capacity < 0");
    if (!valid_type(in_type)) return fail(DEDISP_ERR_INVALID_ARG, "bad in_type");
    if (ndm < 1 || ndm > 65535 || nout < 1)
        return fail(DEDISP_ERR_INVALID_ARG, "need 1 <= ndm <= 65535 and nout >= 1");
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(DEDISP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    dd::Widths W;
    dedisp_status st = check_widths(widths, nwidths, nout, &W);
    if (st != DEDISP_OK) return st;
    uint32_t kmant = 0;
    int kexp2 = 0;
    st = split_threshold(snr_thresh, &kmant, &kexp2);
    if (st != DEDISP_OK) return st;
    const dd::PeaksLayout lay = dd::peaks_layout(ndm, nout, W);
    if (ws_cap && lay.bytes > ws_cap)
        return fail(DEDISP_ERR_UNSUPPORTED,
                    "%d series of %lld samples need %zu bytes of workspace; the static scratch "
                    "holds %zu", ndm, static_cast<long long>(nout), lay.bytes, ws_cap);
    const dd::PeaksWs ws = dd::peaks_ws(workspace, lay);
    const int u16 = in_type == DEDISP_OUT_U16;
    DD_HIP(dd::launch_peaks_count(in, u16, ndm, nout, W, lay, ws, kmant, kexp2, stream));
    int64_t total = 0;
    DD_HIP(hipMemcpyAsync(&total, ws.total, sizeof total, hipMemcpyDeviceToHost, stream));
    DD_HIP(hipStreamSynchronize(stream));
    *n_events = total;
    if (total > 0 && capacity > 0) {
        DD_HIP(dd::launch_peaks_write(in, u16, ndm, nout, W, lay, ws, events, capacity, stream));
        DD_HIP(hipStreamSynchronize(stream));
    }
    if (total > capacity)
        return fail(DEDISP_ERR_CAPACITY, "%lld events found, capacity %lld",
                    static_cast<long long>(total), static_cast<long long>(capacity));
    dd::clear_error();
    return DEDISP_OK;
}

// Workspace of find_peaks_noalloc: a static device array, one per GPU the
// library runs on (each holds it until the process ends).  Host code never
// passes its name to a kernel: the name is a host-side stand-in; the device
// address comes from hipGetSymbolAddress, taken once per device on the first
// call with that device current.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

dedisp_status scratch_address(void** out) {
    int dev = -1;
    DD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(DEDISP_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DEDISP_ERR_HIP, "address of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DEDISP_OK;
}

}  // namespace

extern "C" dedisp_status find_peaks(const void* in, dedisp_out_type in_type, int32_t ndm,
                                    int64_t nout, const int32_t* widths, int32_t nwidths,
                                    float snr_thresh, dedisp_event* events, int64_t capacity,
                                    int64_t* n_events, void* workspace, dedisp_stream stream) {
    return find_peaks_impl(in, in_type, ndm, nout, widths, nwidths, snr_thresh, events, capacity,
                           n_events, workspace, 0, stream);
}

extern "C" dedisp_status find_peaks_noalloc(const void* in, dedisp_out_type in_type, int32_t ndm,
                                            int64_t nout, const int32_t* widths, int32_t nwidths,
                                            float snr_thresh, dedisp_event* events,
                                            int64_t capacity, int64_t* n_events,
                                            dedisp_stream stream) {
    void* ws = nullptr;
    const dedisp_status st = scratch_address(&ws);
    if (st != DEDISP_OK) return st;
    return find_peaks_impl(in, in_type, ndm, nout, widths, nwidths, snr_thresh, events, capacity,
                           n_events, ws, kScratchBytes, stream);
}

extern "C" dedisp_status find_peaks_read_stats(const void* workspace, int32_t ndm, int64_t nout,
                                               const int32_t* widths, int32_t nwidths,
                                               int64_t* s1, uint64_t* s2_lo, uint64_t* s2_hi,
                                               int64_t* thr, dedisp_stream stream) {
    if (!workspace || ndm < 1 || ndm > 65535) return fail(DEDISP_ERR_INVALID_ARG, "bad argument");
    dd::Widths W;
    dedisp_status st = check_widths(widths, nwidths, nout, &W);
    if (st != DEDISP_OK) return st;
    const dd::PeaksLayout lay = dd::peaks_layout(ndm, nout, W);
    const dd::PeaksWs ws = dd::peaks_ws(const_cast<void*>(workspace), lay);
    const size_t n = static_cast<size_t>(lay.nseries);
    if (s1) DD_HIP(hipMemcpyAsync(s1, ws.s1, n * 8, hipMemcpyDeviceToHost, stream));
    if (s2_lo) DD_HIP(hipMemcpyAsync(s2_lo, ws.s2lo, n * 8, hipMemcpyDeviceToHost, stream));
    if (s2_hi) DD_HIP(hipMemcpyAsync(s2_hi, ws.s2hi, n * 8, hipMemcpyDeviceToHost, stream));
    if (thr) DD_HIP(hipMemcpyAsync(thr, ws.thr, n * 8, hipMemcpyDeviceToHost, stream));
    DD_HIP(hipStreamSynchronize(stream));
    dd::clear_error();
    return DEDISP_OK;
}
