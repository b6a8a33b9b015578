// Subband (two-stage) dedispersion.
//
// Section 2.2 calls its brute-force method the "direct" algorithm; the usual
// cheaper one splits the band into nsub subbands of S channels, dedisperses
// each subband on a coarse DM grid, and then dedisperses the subband series
// on the fine grid with each subband's own arrival delay:
//
//   stage 1  sub[s][q][t] = sum_{c' < S} x[c0 + c'][t + dsub[s][q][c']]
//            (subband s as a filterbank of its own: top frequency
//            f_top + c0 * df, c0 = s * S; coarse trial q = the middle fine
//            trial of group q, groups of G consecutive fine trials);
//   stage 2  out[d][t] = sum_s sub[s][q(d)][t + delay[d][c0(s)]].
//
// All sums are exact integers.  The result is the direct sum with an
// effective delay delay[d][c0] + dsub[s][q(d)][c - c0] per channel; its error
// against the direct delay grows with the subband width and the DM distance
// to the group's middle trial.
//
// Design.  Stage 1 is the library's bit-sliced dedispersion kernel, run once
// per subband on the common channel-major bit-plane copy of the input (each
// subband is a block of rows), writing uint16 series.  Stage 2 is a gather
// of nsub values per output: a block takes one trial group and a tile of
// 1024 output samples, stages the group's rows of up to 8 subbands at a time
// in LDS (the tile plus the spread of the group's subband delays), and sums
// them in registers for every trial of the group -- the LDS rows are shared
// by the G trials.  Stage 1 does ncoarse * nchans adds per sample instead of
// ndm * nchans; stage 2 adds ndm * nsub.
#include <algorithm>
#include <climits>
#include <vector>

#include "dedisp_internal.hpp"

namespace {

constexpr int kS2Threads = 256;
constexpr int kS2Tile = 1024;        // output samples per block (4 per thread)
constexpr int kS2PerThread = kS2Tile / kS2Threads;
constexpr int kMaxGroup = 16;        // fine trials per coarse trial
// LDS per block: rows of a few subbands at a time; 16 KiB (several blocks per
// CU) ran stage 2 a fifth faster than 64 KiB, 8-12 KiB no faster
constexpr int kS2LdsBytes = 16 * 1024;

// Block (tile, group q): out[d][t] for the group's trials and t in the tile.
// sub: uint16 series of subband s at sub + ncoarse * (s * nsamps - cum[s]),
// rows of nsamps - maxd[s] samples (the stage-1 output of each subband).
// lo[q][s]: smallest delay[d][c0(s)] over the group.  The samples
// [t0 + lo, t0 + lo + row_len) of subband sc0 + k are staged in LDS row k with
// 16-byte loads from the 16-byte boundary at or before the first one; that
// sample sits at LDS index mis (0..7) of the row, and mis is folded into the
// trials' read offsets, which are block-uniform and come from scalar loads of
// the delay tables, so that all reads of a subband issue back to back.  Chunks that reach past the row end load sample by
// sample (positions past it read as 0; they only feed outputs past nout).
constexpr int kS2MaxChunk = 16;

template <int GM, bool OUT16>
__global__ __launch_bounds__(kS2Threads) void subband_sum_kernel(
    const uint16_t* __restrict__ sub, const int64_t* __restrict__ cum,
    const int32_t* __restrict__ maxd, const int32_t* __restrict__ inter,
    const int32_t* __restrict__ lo, int nsub, int ncoarse, int ndm, int group, int64_t nsamps,
    int64_t nout, int row_len, int row_stride, int chunk, void* __restrict__ out) {
    extern __shared__ uint4 rows_raw[];
    uint16_t* rows = reinterpret_cast<uint16_t*>(rows_raw);
    const int q = blockIdx.y;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kS2Tile;
    const int d0 = q * group;
    const int gq = min(group, ndm - d0);
    const int tid = threadIdx.x;
    uint32_t acc[GM][kS2PerThread];
#pragma unroll
    for (int g = 0; g < GM; ++g)
#pragma unroll
        for (int j = 0; j < kS2PerThread; ++j) acc[g][j] = 0;

    for (int sc0 = 0; sc0 < nsub; sc0 += chunk) {
        const int nsc = min(chunk, nsub - sc0);
        for (int k = 0; k < nsc; ++k) {
            const int s = sc0 + k;
            const int64_t nrow = nsamps - maxd[s];
            const uint16_t* row = sub + static_cast<int64_t>(ncoarse) * (s * nsamps - cum[s]) +
                                  static_cast<int64_t>(q) * nrow;
            const int64_t base = t0 + lo[static_cast<int64_t>(q) * nsub + s];
            const uint16_t* first = row + base;
            const int mis = static_cast<int>((reinterpret_cast<uintptr_t>(first) >> 1) & 7);
            const uint16_t* a0 = first - mis;                 // 16-byte aligned
            const int nchunk = (mis + row_len + 7) >> 3;
            const int64_t valid = nrow - base + mis;           // a0[i] is in the row for i < valid
            uint16_t* dst = rows + k * row_stride;
            for (int c = tid; c < nchunk; c += kS2Threads) {
                const int64_t i0 = static_cast<int64_t>(c) * 8;
                if (i0 + 8 <= valid) {
                    reinterpret_cast<uint4*>(dst)[c] = *reinterpret_cast<const uint4*>(a0 + i0);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        dst[i0 + e] = (i0 + e >= mis && i0 + e < valid) ? a0[i0 + e] : static_cast<uint16_t>(0);
                }
            }
        }
        __syncthreads();
        for (int k = 0; k < nsc; ++k) {
            // read offsets (uniform: scalar loads); trials past the group's
            // end repeat its last one and are never written
            const int s = sc0 + k;
            const int64_t nrow = nsamps - maxd[s];
            const int64_t lo_qs = lo[static_cast<int64_t>(q) * nsub + s];
            const uint16_t* first = sub + static_cast<int64_t>(ncoarse) * (s * nsamps - cum[s]) +
                                    static_cast<int64_t>(q) * nrow + t0 + lo_qs;
            const int mis = static_cast<int>((reinterpret_cast<uintptr_t>(first) >> 1) & 7);
            const uint16_t* src = rows + k * row_stride + tid;
            int off[GM];
#pragma unroll
            for (int g = 0; g < GM; ++g)
                off[g] = inter[static_cast<int64_t>(d0 + min(g, gq - 1)) * nsub + s] -
                         static_cast<int>(lo_qs) + mis;
            uint32_t v[GM][kS2PerThread];
#pragma unroll
            for (int g = 0; g < GM; ++g)
#pragma unroll
                for (int j = 0; j < kS2PerThread; ++j) v[g][j] = src[off[g] + j * kS2Threads];
#pragma unroll
            for (int g = 0; g < GM; ++g)
#pragma unroll
                for (int j = 0; j < kS2PerThread; ++j) acc[g][j] += v[g][j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < GM; ++g) {
#pragma unroll
        for (int j = 0; j < kS2PerThread; ++j) {
            const int64_t t = t0 + tid + j * kS2Threads;
            if (g < gq && t < nout) {
                const int64_t o = static_cast<int64_t>(d0 + g) * nout + t;
                if (OUT16) static_cast<uint16_t*>(out)[o] = static_cast<uint16_t>(acc[g][j]);
                else static_cast<int32_t*>(out)[o] = static_cast<int32_t>(acc[g][j]);
            }
        }
    }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct dedisp_subband_s {
    dedisp_plan base = nullptr;      // the caller's plan (fine trials); not owned
    int nsub = 0, group = 0, S = 0, ncoarse = 0;
    std::vector<dedisp_plan> sub;    // per subband: S channels, coarse trials
    std::vector<int32_t> maxd;       // per subband: its plan's max delay
    std::vector<int64_t> cum;        // prefix sums of maxd
    int64_t loss = 0;                // nsamps - nout
    int span = 0;                    // largest spread of a group's subband delays
    int32_t* d_inter = nullptr;      // [ndm][nsub] delay[d][c0(s)]
    int32_t* d_lo = nullptr;         // [ncoarse][nsub]
    int32_t* d_maxd = nullptr;
    int64_t* d_cum = nullptr;
};

namespace {

using dd::fail;

void free_subband(dedisp_subband_s* b) {
    for (dedisp_plan p : b->sub)
        if (p) (void)dedisp_plan_destroy(p);
    if (b->d_inter) (void)hipFree(b->d_inter);
    if (b->d_lo) (void)hipFree(b->d_lo);
    if (b->d_maxd) (void)hipFree(b->d_maxd);
    if (b->d_cum) (void)hipFree(b->d_cum);
    delete b;
}

size_t words_bytes(const dedisp_subband_s* b, int64_t nsamps) {
    return align256(static_cast<size_t>(b->base->nchans) * dd::repack_words(nsamps) * sizeof(uint2));
}

size_t series_bytes(const dedisp_subband_s* b, int64_t nsamps) {
    size_t n = 0;
    for (int s = 0; s < b->nsub; ++s)
        n += static_cast<size_t>(b->ncoarse) * static_cast<size_t>(nsamps - b->maxd[s]);
    return n * 2;
}

}  // namespace

extern "C" dedisp_status dedisp_subband_create(dedisp_plan plan, int32_t nsub, int32_t group,
                                               dedisp_subband* out) {
    if (!plan || !out) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    const int nchans = plan->nchans, ndm = plan->ndm;
    if (nsub < 1 || nchans % nsub || (nchans / nsub) % 4)
        return fail(DEDISP_ERR_INVALID_ARG,
                    "nsub=%d must divide nchans=%d into subbands of a multiple of 4 channels", nsub,
                    nchans);
    if (group < 1 || group > kMaxGroup)
        return fail(DEDISP_ERR_INVALID_ARG, "group=%d outside [1, %d]", group, kMaxGroup);
    auto* b = new dedisp_subband_s;
    b->base = plan;
    b->nsub = nsub;
    b->group = group;
    b->S = nchans / nsub;
    b->ncoarse = (ndm + group - 1) / group;
    std::vector<double> coarse(b->ncoarse);
    for (int q = 0; q < b->ncoarse; ++q) {
        const int size = std::min(group, ndm - q * group);
        coarse[q] = plan->dm_list[q * group + (size - 1) / 2];
    }
    b->sub.assign(nsub, nullptr);
    for (int s = 0; s < nsub; ++s) {
        const double ftop_s = plan->f_top + static_cast<double>(s * b->S) * plan->df;
        const dedisp_status st =
            dedisp_plan_create(b->S, ftop_s, plan->df, plan->tsamp, coarse.data(), b->ncoarse, &b->sub[s]);
        if (st != DEDISP_OK) {
            free_subband(b);
            return st;
        }
    }
    // Stage 1 sums few channels per output, so its best tile shape differs
    // from the direct sum's: tune it (bit-exact candidates only) on the
    // subband with the largest delays and use it wherever its LDS tile fits.
    int ref = 0;
    for (int s = 1; s < nsub; ++s)
        if (b->sub[s]->max_delay > b->sub[ref]->max_delay) ref = s;
    dedisp_tile best{};
    int32_t rejected = 0;
    const int64_t tune_n = std::max<int64_t>(int64_t(1) << 17, b->sub[ref]->max_delay + (int64_t(1) << 15));
    if (dedisp_autotune(b->sub[ref], tune_n, DEDISP_OUT_U16, nullptr, &best, &rejected) == DEDISP_OK) {
        const dd::TileConfig c{best.dms_per_block, best.groups, best.stage_chans};
        for (int s = 0; s < nsub; ++s)
            if (s != ref && dd::tile_lds_bytes(b->sub[s], c) <= 160 * 1024)
                b->sub[s]->tuned.store((c.dms_per_block << 16) | (c.groups << 8) | c.stage_chans);
    }
    for (int s = 0; s < nsub; ++s) {
        dedisp_status tst = DEDISP_OK;
        if (!dd::offset_table(b->sub[s], dd::default_tile_config(b->sub[s]), true, &tst)) {
            free_subband(b);
            return tst;
        }
    }
    b->maxd.resize(nsub);
    b->cum.resize(nsub);
    int64_t run = 0;
    for (int s = 0; s < nsub; ++s) {
        b->maxd[s] = static_cast<int32_t>(b->sub[s]->max_delay);
        b->cum[s] = run;
        run += b->maxd[s];
    }
    std::vector<int32_t> inter(static_cast<size_t>(ndm) * nsub), lo(static_cast<size_t>(b->ncoarse) * nsub);
    for (int d = 0; d < ndm; ++d)
        for (int s = 0; s < nsub; ++s) {
            const int32_t v = plan->delays[static_cast<size_t>(d) * nchans + s * b->S];
            inter[static_cast<size_t>(d) * nsub + s] = v;
            b->loss = std::max<int64_t>(b->loss, static_cast<int64_t>(v) + b->maxd[s]);
        }
    for (int q = 0; q < b->ncoarse; ++q)
        for (int s = 0; s < nsub; ++s) {
            int32_t mn = INT32_MAX, mx = INT32_MIN;
            for (int d = q * group; d < std::min(ndm, (q + 1) * group); ++d) {
                mn = std::min(mn, inter[static_cast<size_t>(d) * nsub + s]);
                mx = std::max(mx, inter[static_cast<size_t>(d) * nsub + s]);
            }
            lo[static_cast<size_t>(q) * nsub + s] = mn;
            b->span = std::max(b->span, mx - mn);
        }
    if (static_cast<int64_t>(kS2Tile + b->span + 16) * 2 > kS2LdsBytes) {
        free_subband(b);
        return fail(DEDISP_ERR_UNSUPPORTED,
                    "a group's subband delays spread over %d samples: use smaller groups", b->span);
    }
    hipError_t e = hipMalloc(&b->d_inter, inter.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&b->d_lo, lo.size() * 4);
    if (e == hipSuccess) e = hipMalloc(&b->d_maxd, static_cast<size_t>(nsub) * 4);
    if (e == hipSuccess) e = hipMalloc(&b->d_cum, static_cast<size_t>(nsub) * 8);
    if (e == hipSuccess) e = hipMemcpy(b->d_inter, inter.data(), inter.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_lo, lo.data(), lo.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_maxd, b->maxd.data(), static_cast<size_t>(nsub) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_cum, b->cum.data(), static_cast<size_t>(nsub) * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_subband(b);
        return fail(e == hipErrorOutOfMemory ? DEDISP_ERR_OUT_OF_MEMORY : DEDISP_ERR_HIP,
                    "subband tables: %s", hipGetErrorString(e));
    }
    *out = b;
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_subband_info(dedisp_subband b, int64_t* max_delay,
                                             int32_t* ncoarse, int32_t* span, dedisp_tile* tile) {
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (max_delay) *max_delay = b->loss;
    if (ncoarse) *ncoarse = b->ncoarse;
    if (span) *span = b->span;
    if (tile) {
        int ref = 0;
        for (int s = 1; s < b->nsub; ++s)
            if (b->sub[s]->max_delay > b->sub[ref]->max_delay) ref = s;
        const dd::TileConfig c = dd::default_tile_config(b->sub[ref]);
        *tile = dedisp_tile{c.dms_per_block, c.groups, c.stage_chans};
    }
    return DEDISP_OK;
}

extern "C" size_t dedisp_subband_workspace_bytes(dedisp_subband b, int64_t nsamps) {
    if (!b || nsamps <= b->loss) return 0;
    return words_bytes(b, nsamps) + series_bytes(b, nsamps);
}

extern "C" dedisp_status dedisp_subband_execute(dedisp_subband b, const uint8_t* in, int64_t nsamps,
                                                void* out, dedisp_out_type out_type, void* workspace,
                                                dedisp_stream stream) {
    if (!b || !in || !out || !workspace) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (out_type != DEDISP_OUT_I32 && out_type != DEDISP_OUT_U16)
        return fail(DEDISP_ERR_INVALID_ARG, "bad out_type");
    if (nsamps <= b->loss)
        return fail(DEDISP_ERR_TOO_FEW_SAMPLES, "nsamps=%lld <= subband max delay %lld",
                    static_cast<long long>(nsamps), static_cast<long long>(b->loss));
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(DEDISP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const dedisp_plan_s* p = b->base;
    int dev = -1;
    DD_HIP(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(DEDISP_ERR_INVALID_ARG, "current device %d differs from the plan's %d", dev,
                    p->device);
    const int64_t nwords = dd::repack_words(nsamps);
    uint2* words = static_cast<uint2*>(workspace);
    uint16_t* series = reinterpret_cast<uint16_t*>(static_cast<char*>(workspace) + words_bytes(b, nsamps));
    DD_HIP(dd::launch_repack(in, nsamps, p->nchans, words, nwords, stream));
    for (int s = 0; s < b->nsub; ++s) {
        const dedisp_plan_s* sp = b->sub[s];
        uint16_t* dst = series + static_cast<int64_t>(b->ncoarse) * (s * nsamps - b->cum[s]);
        const dedisp_status st = dd::launch_dedisperse(sp, words + static_cast<int64_t>(s) * b->S * nwords,
                                                       nwords, nsamps - b->maxd[s], dst, 1,
                                                       dd::default_tile_config(sp), stream);
        if (st != DEDISP_OK) return st;
    }
    const int64_t nout = nsamps - b->loss;
    const int row_len = kS2Tile + b->span;
    const int row_stride = (row_len + 7 + 7) & ~7;        // room for the leading misalignment
    const int chunk = std::max(1, std::min(kS2MaxChunk, kS2LdsBytes / (row_stride * 2)));
    const dim3 grid(static_cast<unsigned>((nout + kS2Tile - 1) / kS2Tile), static_cast<unsigned>(b->ncoarse));
    const size_t lds = static_cast<size_t>(chunk) * row_stride * 2;
    const bool u16 = out_type == DEDISP_OUT_U16;
#define DD_S2(GM_)                                                                             \
    if (b->group <= GM_) {                                                                     \
        if (u16)                                                                               \
            hipLaunchKernelGGL((subband_sum_kernel<GM_, true>), grid, dim3(kS2Threads), lds,   \
                               stream, series, b->d_cum, b->d_maxd, b->d_inter, b->d_lo,      \
                               b->nsub, b->ncoarse, p->ndm, b->group, nsamps, nout, row_len,   \
                               row_stride, chunk, out);                                                    \
        else                                                                                   \
            hipLaunchKernelGGL((subband_sum_kernel<GM_, false>), grid, dim3(kS2Threads), lds,  \
                               stream, series, b->d_cum, b->d_maxd, b->d_inter, b->d_lo,      \
                               b->nsub, b->ncoarse, p->ndm, b->group, nsamps, nout, row_len,   \
                               row_stride, chunk, out);                                                    \
    } else
    DD_S2(1) DD_S2(2) DD_S2(4) DD_S2(8) DD_S2(16) {}
#undef DD_S2
    DD_HIP(hipGetLastError());
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_subband_destroy(dedisp_subband b) {
    if (!b) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    free_subband(b);
    return DEDISP_OK;
}
