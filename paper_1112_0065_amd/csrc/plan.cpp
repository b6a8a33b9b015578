// Plan: argument validation, the DM delay table and per-block skews.
//
// Section 2.2 of the paper: each trial DM integrates every channel shifted by
// a frequency- and DM-dependent delay.  The table is evaluated on the host in
// IEEE double with one rounding per operation (this file is compiled with
// -ffp-contract=off so no multiply-add is fused), in the order
//   fc = f_top + c*df;  a = 1/(fc*fc) - 1/(f_top*f_top);  x = ((K*DM)*a)/tsamp
// and rounded half away from zero (C round()).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "dedisp_internal.hpp"

namespace {

constexpr double kDispersionConst = 4.148808e3;  // s MHz^2 pc^-1 cm^3

thread_local std::string g_last_error;

int64_t delay_entry(double f_top, double df, double tsamp, double dm, int c) {
    const double fc = f_top + static_cast<double>(c) * df;
    const double a = 1.0 / (fc * fc) - 1.0 / (f_top * f_top);
    const double x = ((kDispersionConst * dm) * a) / tsamp;
    return static_cast<int64_t>(std::round(x));
}

}  // namespace

namespace dd {

dedisp_status fail(dedisp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace dd

extern "C" const char* dedisp_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* dedisp_version(void) { return "dedisp-gfx950 0.1"; }

extern "C" dedisp_status dedisp_plan_create(int32_t nchans, double f_top, double df,
                                            double tsamp, const double* dm_list,
                                            int32_t ndm, dedisp_plan* plan_out) {
    using dd::fail;
    if (!plan_out) return fail(DEDISP_ERR_INVALID_ARG, "plan_out is NULL");
    *plan_out = nullptr;
    if (nchans < 4 || nchans % 4 != 0 || nchans > 21844)
        return fail(DEDISP_ERR_INVALID_ARG,
                    "nchans=%d must be a multiple of 4 in [4, 21844]", nchans);
    if (!std::isfinite(f_top) || !std::isfinite(df) || !(df < 0.0))
        return fail(DEDISP_ERR_INVALID_ARG, "need finite f_top and df < 0");
    const double f_low = f_top + static_cast<double>(nchans - 1) * df;
    if (!(f_low > 0.0))
        return fail(DEDISP_ERR_INVALID_ARG, "lowest channel frequency %g <= 0", f_low);
    if (!std::isfinite(tsamp) || !(tsamp > 0.0))
        return fail(DEDISP_ERR_INVALID_ARG, "tsamp must be > 0");
    if (ndm < 1 || !dm_list) return fail(DEDISP_ERR_INVALID_ARG, "need ndm >= 1 and a DM list");
    for (int d = 0; d < ndm; ++d) {
        if (!std::isfinite(dm_list[d]) || dm_list[d] < 0.0)
            return fail(DEDISP_ERR_INVALID_ARG, "dm_list[%d] is negative or not finite", d);
        if (d && dm_list[d] < dm_list[d - 1])
            return fail(DEDISP_ERR_INVALID_ARG, "dm_list must be non-decreasing (index %d)", d);
    }

    dedisp_plan_s* p = new (std::nothrow) dedisp_plan_s;
    if (!p) return fail(DEDISP_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->nchans = nchans;
    p->ndm = ndm;
    p->f_top = f_top;
    p->df = df;
    p->tsamp = tsamp;
    p->dm_list.assign(dm_list, dm_list + ndm);
    p->delays.resize(static_cast<size_t>(ndm) * nchans);
    int64_t mx = 0;
    for (int d = 0; d < ndm; ++d)
        for (int c = 0; c < nchans; ++c) {
            const int64_t v = delay_entry(f_top, df, tsamp, dm_list[d], c);
            if (v < 0 || v > (int64_t(1) << 30)) {
                delete p;
                return fail(DEDISP_ERR_UNSUPPORTED, "delay %lld out of range",
                            static_cast<long long>(v));
            }
            p->delays[static_cast<size_t>(d) * nchans + c] = static_cast<int32_t>(v);
            if (v > mx) mx = v;
        }
    p->max_delay = mx;

    // Per DM-block skew: max over channels of the spread, in 32-sample words,
    // between the block's first and last trial.
    const int sizes[dedisp_plan_s::kNumDmBlock] = {4, 8, 16, 32};
    std::vector<std::vector<int32_t>> skews(dedisp_plan_s::kNumDmBlock);
    for (int k = 0; k < dedisp_plan_s::kNumDmBlock; ++k) {
        const int nd = sizes[k];
        const int nblk = (ndm + nd - 1) / nd;
        skews[k].resize(nblk);
        int32_t smax = 0;
        for (int b = 0; b < nblk; ++b) {
            const int dlo = b * nd;
            const int dhi = std::min(ndm, dlo + nd) - 1;
            int32_t s = 0;
            for (int c = 0; c < nchans; ++c) {
                const int32_t lo = p->delays[static_cast<size_t>(dlo) * nchans + c] >> 5;
                const int32_t hi = p->delays[static_cast<size_t>(dhi) * nchans + c] >> 5;
                s = std::max(s, hi - lo);
            }
            skews[k][b] = s;
            smax = std::max(smax, s);
        }
        p->skew_max[k] = smax;
    }

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess)
        e = hipMalloc(&p->d_delays, p->delays.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_delays, p->delays.data(), p->delays.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice);
    for (int k = 0; k < dedisp_plan_s::kNumDmBlock && e == hipSuccess; ++k) {
        e = hipMalloc(&p->d_skew[k], skews[k].size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(p->d_skew[k], skews[k].data(), skews[k].size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        dedisp_plan_destroy(p);
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "device setup of the plan failed: %s", hipGetErrorString(e));
    }
    dd::apply_env_cache(p);
    {
        dedisp_status st = DEDISP_OK;
        if (!dd::offset_table(p, dd::default_tile_config(p), true, &st)) {
            dedisp_plan_destroy(p);
            return st;
        }
    }
    *plan_out = p;
    dd::clear_error();
    return DEDISP_OK;
}

namespace dd {

const uint32_t* offset_table(const dedisp_plan_s* p, const TileConfig& cfg, bool build,
                             dedisp_status* st) {
    if (st) *st = DEDISP_OK;
    std::lock_guard<std::mutex> lock(p->tab_mu);
    for (const auto& t : p->tabs)
        if (t.dms == cfg.dms_per_block && t.groups == cfg.groups && t.stage == cfg.stage_chans)
            return t.d;
    if (!build) {
        if (st) *st = fail(DEDISP_ERR_INVALID_ARG, "no offset table for tile (%d, %d, %d)",
                           cfg.dms_per_block, cfg.groups, cfg.stage_chans);
        return nullptr;
    }
    const int k = dm_block_index(cfg.dms_per_block);
    if (k < 0 || cfg.groups < 1 || cfg.stage_chans < 4) {
        if (st) *st = fail(DEDISP_ERR_INVALID_ARG, "unsupported tile configuration");
        return nullptr;
    }
    const int nc = p->nchans;
    // quads (16-byte copies of two consecutive words) per LDS row
    const int64_t pitch = 64 * cfg.groups + p->skew_max[k];
    std::vector<uint32_t> h(static_cast<size_t>(p->ndm) * nc);
    for (int d = 0; d < p->ndm; ++d) {
        const int blk = d / cfg.dms_per_block;
        const int32_t* row = &p->delays[static_cast<size_t>(d) * nc];
        const int32_t* lo = &p->delays[static_cast<size_t>(blk) * cfg.dms_per_block * nc];
        for (int c = 0; c < nc; ++c) {
            const int64_t quads = (c % cfg.stage_chans) * pitch + (row[c] >> 5) - (lo[c] >> 5);
            const int64_t bytes = quads * 16;
            if (quads < 0 || (bytes << 5) >= (int64_t(1) << 32)) {
                if (st) *st = fail(DEDISP_ERR_UNSUPPORTED, "LDS offset out of range");
                return nullptr;
            }
            h[static_cast<size_t>(d) * nc + c] =
                static_cast<uint32_t>(bytes << 5) | static_cast<uint32_t>(row[c] & 31);
        }
    }
    // upload on a private stream and wait for it, so that a launch on any
    // stream afterwards sees the whole table
    uint32_t* dptr = nullptr;
    hipStream_t up = nullptr;
    hipError_t e = hipMalloc(&dptr, h.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&up, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dptr, h.data(), h.size() * sizeof(uint32_t), hipMemcpyHostToDevice, up);
    if (e == hipSuccess) e = hipStreamSynchronize(up);
    if (up) (void)hipStreamDestroy(up);
    if (e != hipSuccess) {
        if (dptr) (void)hipFree(dptr);
        if (st)
            *st = fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                       "offset table upload failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    p->tabs.push_back({cfg.dms_per_block, cfg.groups, cfg.stage_chans, dptr});
    return dptr;
}

void drop_offset_tables(const dedisp_plan_s* p, const std::vector<TileConfig>& keep) {
    std::lock_guard<std::mutex> lock(p->tab_mu);
    std::vector<dedisp_plan_s::OffsetTable> kept;
    for (const auto& t : p->tabs) {
        bool k = false;
        for (const TileConfig& c : keep)
            k = k || (t.dms == c.dms_per_block && t.groups == c.groups && t.stage == c.stage_chans);
        if (k)
            kept.push_back(t);
        else
            (void)hipFree(t.d);
    }
    p->tabs.swap(kept);
}

std::vector<TileConfig> offset_table_shapes(const dedisp_plan_s* p) {
    std::lock_guard<std::mutex> lock(p->tab_mu);
    std::vector<TileConfig> v;
    for (const auto& t : p->tabs) v.push_back(TileConfig{t.dms, t.groups, t.stage});
    return v;
}

}  // namespace dd

extern "C" dedisp_status dedisp_plan_destroy(dedisp_plan p) {
    if (!p) return dd::fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    for (const auto& t : p->tabs) (void)hipFree(t.d);
    p->tabs.clear();
    if (p->d_delays) (void)hipFree(p->d_delays);
    for (int k = 0; k < dedisp_plan_s::kNumDmBlock; ++k)
        if (p->d_skew[k]) (void)hipFree(p->d_skew[k]);
    delete p;
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_plan_info(dedisp_plan p, int32_t* nchans, int32_t* ndm,
                                          int64_t* max_delay) {
    if (!p) return dd::fail(DEDISP_ERR_INVALID_ARG, "plan is NULL");
    if (nchans) *nchans = p->nchans;
    if (ndm) *ndm = p->ndm;
    if (max_delay) *max_delay = p->max_delay;
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_plan_copy_delays(dedisp_plan p, int32_t* host_out) {
    if (!p || !host_out) return dd::fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    std::memcpy(host_out, p->delays.data(), p->delays.size() * sizeof(int32_t));
    return DEDISP_OK;
}

extern "C" size_t dedisp_workspace_bytes(dedisp_plan p, int64_t nsamps) {
    if (!p || nsamps <= 0) return 0;
    return static_cast<size_t>(p->nchans) * static_cast<size_t>(dd::repack_words(nsamps)) *
           sizeof(uint2);
}
