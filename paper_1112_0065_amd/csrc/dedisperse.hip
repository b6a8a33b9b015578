// Brute-force incoherent dedispersion (paper section 2.2):
//     out[d][t] = sum_c x[c][t + delay[d][c]],   0 <= t < nout.
//
// Design for gfx950 (integer gather-sum, no contraction, so no MFMA):
//   * input is the channel-major bit-plane copy made by repack.hip: 32
//     samples of one channel per {lo, hi} word pair;
//   * a block owns a tile of `ND` consecutive DM trials x T = 2048*G output
//     samples; its four waves each own ND/4 trials, every lane owns G
//     32-sample groups (lane-strided, so LDS reads are conflict-free);
//   * channels are streamed in stages of CS channels: the block copies, per
//     channel, the skewed window of words all its trials need into LDS
//     (one coalesced load shared by the ND trials);
//   * per (trial, channel) a lane reads two words per group, aligns them to
//     the trial's delay with one funnel shift per plane, and adds the 32
//     2-bit samples into a bit-sliced counter with carry-save adder trees:
//     about 8 bit-operations add 32 samples (see gen_csa.py);
//   * after the last stage the counter planes are transposed to integers in
//     registers and written once (int32 or uint16).
// The result is exact; its order of additions is irrelevant (integers).
#include "bitslice.hpp"
#include "dedisp_internal.hpp"

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

template <int NL, int N>
__device__ __forceinline__ void csa_add(uint32_t (&a)[NL], const uint32_t (&lo)[N],
                                        const uint32_t (&hi)[N]);

#define DD_CSA_SPEC(NL_, N_)                                                                   \
    template <>                                                                                \
    __device__ __forceinline__ void csa_add<NL_, N_>(uint32_t (&a)[NL_], const uint32_t (&lo)[N_], \
                                                     const uint32_t (&hi)[N_]) {               \
        csa_add_##N_##_##NL_(a, lo, hi);                                                       \
    }
DD_CSA_SPEC(12, 4) DD_CSA_SPEC(12, 8) DD_CSA_SPEC(12, 16) DD_CSA_SPEC(12, 32)
DD_CSA_SPEC(16, 4) DD_CSA_SPEC(16, 8) DD_CSA_SPEC(16, 16) DD_CSA_SPEC(16, 32)
#undef DD_CSA_SPEC

// Accumulate channels [c, c+N) of the current stage for one trial into the
// counters of its G groups.
template <int NL, int G, int N>
__device__ __forceinline__ void accumulate_chunk(uint32_t (&acc)[G][NL], const uint2* lds,
                                                 const int32_t* __restrict__ drow,
                                                 const int32_t* __restrict__ dlo_row, int c,
                                                 int cl, int stride, int lane) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        uint32_t lo[N], hi[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const int dl = drow[c + k];
            const int rel = (dl >> 5) - (dlo_row[c + k] >> 5);
            const uint32_t r = static_cast<uint32_t>(dl & 31);
            const uint2* p = lds + (cl + k) * stride + rel + lane + 64 * g;
            const uint2 w0 = p[0];
            const uint2 w1 = p[1];
            lo[k] = bs::funnel(w1.x, w0.x, r);
            hi[k] = bs::funnel(w1.y, w0.y, r);
        }
        csa_add<NL, N>(acc[g], lo, hi);
    }
}

template <int NL, int NDW, int G, bool OUT16>
__global__ __launch_bounds__(kThreads) void dedisperse_kernel(
    const uint2* __restrict__ words, int64_t nwords, int nchans, int ndm, int64_t nout,
    const int32_t* __restrict__ delays, const int32_t* __restrict__ skew, int stage_chans,
    int n_dm_blocks, int n_items, void* __restrict__ out) {
    constexpr int ND = NDW * kWaves;
    constexpr int T = 2048 * G;
    extern __shared__ uint2 lds[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // XCD-aware order: hardware deals consecutive blocks round-robin to the 8
    // XCDs; give each XCD a contiguous run of (time tile, DM block) items with
    // the DM block fastest, so blocks resident on one XCD share input words in
    // its L2.
    const int per_xcd = gridDim.x / 8;
    const int item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (item >= n_items) return;
    const int tile = item / n_dm_blocks;
    const int dblk = item % n_dm_blocks;
    const int64_t T0 = static_cast<int64_t>(tile) * T;
    const int d_lo = dblk * ND;
    const int stride = T / 32 + 1 + skew[dblk];
    const int64_t w_base = T0 >> 5;
    const int32_t* dlo_row = delays + static_cast<int64_t>(d_lo) * nchans;

    uint32_t acc[NDW][G][NL];
#pragma unroll
    for (int i = 0; i < NDW; ++i)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int l = 0; l < NL; ++l) acc[i][g][l] = 0u;

#pragma unroll 1
    for (int c0 = 0; c0 < nchans; c0 += stage_chans) {
        const int cs = min(stage_chans, nchans - c0);
        // Stage fill: channel cl gets words [w_base + (delay[d_lo][c] >> 5), +stride).
        for (int cl = wave; cl < cs; cl += kWaves) {
            const int c = c0 + cl;
            const int64_t w0 = w_base + (dlo_row[c] >> 5);
            const uint2* src = words + static_cast<int64_t>(c) * nwords;
            uint2* dst = lds + cl * stride;
            for (int i = lane; i < stride; i += 64) {
                const int64_t w = w0 + i;
                dst[i] = w < nwords ? src[w] : make_uint2(0u, 0u);
            }
        }
        __syncthreads();

#pragma unroll
        for (int i = 0; i < NDW; ++i) {
            const int d = d_lo + wave + kWaves * i;
            if (d < ndm) {
                const int32_t* drow = delays + static_cast<int64_t>(d) * nchans;
                int cl = 0;
#pragma unroll 1
                for (; cl + 16 <= cs; cl += 16)
                    accumulate_chunk<NL, G, 16>(acc[i], lds, drow, dlo_row, c0 + cl, cl, stride, lane);
                if (cl + 8 <= cs) {
                    accumulate_chunk<NL, G, 8>(acc[i], lds, drow, dlo_row, c0 + cl, cl, stride, lane);
                    cl += 8;
                }
                if (cl + 4 <= cs)
                    accumulate_chunk<NL, G, 4>(acc[i], lds, drow, dlo_row, c0 + cl, cl, stride, lane);
            }
        }
        __syncthreads();
    }

    // Write: counters -> integers, one 32-sample group per lane and group.
#pragma unroll
    for (int i = 0; i < NDW; ++i) {
        const int d = d_lo + wave + kWaves * i;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t t = T0 + 32 * (lane + 64 * g);
            if (d >= ndm || t >= nout) continue;
            uint32_t r[16];
            bs::planes_to_pairs<NL>(acc[i][g], r);
            const int64_t row = static_cast<int64_t>(d) * nout;
            const bool full = t + 32 <= nout;
            if (OUT16) {
                uint16_t* o = static_cast<uint16_t*>(out) + row + t;
                if (full && ((row + t) & 1) == 0) {
                    uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        o32[q] = (r[2 * q] & 0xFFFFu) | (r[2 * q + 1] << 16);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        o32[8 + q] = (r[2 * q] >> 16) | (r[2 * q + 1] & 0xFFFF0000u);
                } else {
                    const int n = static_cast<int>(min<int64_t>(32, nout - t));
#pragma unroll
                    for (int b = 0; b < 32; ++b)
                        if (b < n) o[b] = static_cast<uint16_t>(b < 16 ? r[b] : (r[b - 16] >> 16));
                }
            } else {
                int32_t* o = static_cast<int32_t*>(out) + row + t;
                if (full && ((row + t) & 3) == 0) {
                    int4* o4 = reinterpret_cast<int4*>(o);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        o4[q] = make_int4(r[4 * q] & 0xFFFF, r[4 * q + 1] & 0xFFFF,
                                          r[4 * q + 2] & 0xFFFF, r[4 * q + 3] & 0xFFFF);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        o4[4 + q] = make_int4(r[4 * q] >> 16, r[4 * q + 1] >> 16,
                                              r[4 * q + 2] >> 16, r[4 * q + 3] >> 16);
                } else {
                    const int n = static_cast<int>(min<int64_t>(32, nout - t));
#pragma unroll
                    for (int b = 0; b < 32; ++b)
                        if (b < n) o[b] = static_cast<int32_t>(b < 16 ? (r[b] & 0xFFFFu) : (r[b - 16] >> 16));
                }
            }
        }
    }
}

template <int NL, int NDW, int G, bool OUT16>
hipError_t launch_cfg(const dedisp_plan_s* p, const uint2* words, int64_t nwords, int64_t nout,
                      void* out, int stage_chans, hipStream_t s) {
    constexpr int ND = NDW * kWaves;
    constexpr int T = 2048 * G;
    const int k = dd::dm_block_index(ND);
    const int n_time_tiles = static_cast<int>((nout + T - 1) / T);
    const int n_dm_blocks = (p->ndm + ND - 1) / ND;
    const size_t lds = static_cast<size_t>(stage_chans) * (T / 32 + 1 + p->skew_max[k]) * sizeof(uint2);
    auto kern = dedisperse_kernel<NL, NDW, G, OUT16>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const int64_t n_items = static_cast<int64_t>(n_time_tiles) * n_dm_blocks;
    if (n_items > (int64_t(1) << 30)) return hipErrorInvalidValue;
    const int64_t nblocks = 8 * ((n_items + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(nblocks)), dim3(kThreads), lds, s, words,
                       nwords, p->nchans, p->ndm, nout, p->d_delays, p->d_skew[k], stage_chans,
                       n_dm_blocks, static_cast<int>(n_items), out);
    return hipGetLastError();
}

}  // namespace

namespace dd {

TileConfig default_tile_config(const dedisp_plan_s* p) {
    (void)p;
    return TileConfig{16, 2, 32};
}

dedisp_status launch_dedisperse(const dedisp_plan_s* p, const uint2* words, int64_t nwords,
                                int64_t nout, void* out, int out_u16, const TileConfig& cfg,
                                hipStream_t s) {
    const int k = dm_block_index(cfg.dms_per_block);
    if (k < 0 || cfg.stage_chans < 4 || cfg.stage_chans % 4 || cfg.groups < 1 || cfg.groups > 2)
        return fail(DEDISP_ERR_INVALID_ARG, "unsupported tile configuration");
    const int T = 2048 * cfg.groups;
    const size_t lds = static_cast<size_t>(cfg.stage_chans) * (T / 32 + 1 + p->skew_max[k]) * sizeof(uint2);
    if (lds > 160 * 1024)
        return fail(DEDISP_ERR_UNSUPPORTED,
                    "DM block of %d trials spans %d words of skew: LDS tile of %zu bytes too large",
                    cfg.dms_per_block, p->skew_max[k], lds);
    const int nl = levels_for(p->nchans);
    hipError_t e = hipErrorInvalidValue;
#define DD_DISPATCH(NL_, NDW_, G_)                                                               \
    if (nl == NL_ && cfg.dms_per_block == NDW_ * kWaves && cfg.groups == G_) {                  \
        e = out_u16 ? launch_cfg<NL_, NDW_, G_, true>(p, words, nwords, nout, out, cfg.stage_chans, s) \
                    : launch_cfg<NL_, NDW_, G_, false>(p, words, nwords, nout, out, cfg.stage_chans, s); \
    }
    DD_DISPATCH(12, 1, 1) DD_DISPATCH(12, 2, 1) DD_DISPATCH(12, 4, 1) DD_DISPATCH(12, 8, 1)
    DD_DISPATCH(12, 1, 2) DD_DISPATCH(12, 2, 2) DD_DISPATCH(12, 4, 2)
    DD_DISPATCH(16, 1, 1) DD_DISPATCH(16, 2, 1) DD_DISPATCH(16, 4, 1) DD_DISPATCH(16, 8, 1)
    DD_DISPATCH(16, 1, 2) DD_DISPATCH(16, 2, 2) DD_DISPATCH(16, 4, 2)
#undef DD_DISPATCH
    if (e != hipSuccess)
        return fail(e == hipErrorInvalidValue ? DEDISP_ERR_UNSUPPORTED : DEDISP_ERR_HIP,
                    "dedispersion launch failed: %s", hipGetErrorString(e));
    return DEDISP_OK;
}

}  // namespace dd
