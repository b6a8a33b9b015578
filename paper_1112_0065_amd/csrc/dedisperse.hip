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
//     (one coalesced load shared by the ND trials), as 16-byte quads that
//     each hold two consecutive words (every word is stored twice);
//   * per (trial, channel) a lane reads one aligned quad per group (one
//     ds_read_b128, which moves about 1.5x the bytes per clock of the two
//     8-byte reads of unaligned word pairs) at an LDS offset taken from the
//     plan's per-tile-shape offset table (one scalar load per channel; the
//     table also carries the shift within the word), aligns the two words
//     to the trial's delay with one funnel shift per plane, and adds the 32
//     2-bit samples into a bit-sliced counter with carry-save adder trees:
//     8 channels at a time into a 5-level low counter (2 bit-operations per
//     input plane, see gen_csa.py), whose carry-out plane waits for the next
//     8 channels' so that the two ripple through the upper levels once;
//   * after the last stage the counter planes are transposed to integers in
//     registers and written once (int32 or uint16).
// The result is exact; its order of additions is irrelevant (integers).
#include <algorithm>

#include "bitslice.hpp"
#include "dedisp_internal.hpp"

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
// L2 bytes of LDS-offset rows that one group of DM blocks may occupy: a
// quarter of an XCD's 4 MiB L2, the rest holding the input windows and the
// blocks' delay rows (one row per block).
constexpr int64_t kItemGroupBytes = int64_t(1) << 20;

// Read-only tables (delays, skews, beam descriptors) are read through the
// constant address space: the loads stay scalar even after the output stores
// of an earlier work item, which would otherwise force them onto the vector
// memory path in the persistent kernel.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)p;
}

// Word-wise copy of a descriptor out of the constant address space.
__device__ __forceinline__ dd::BeamArgs load_beam(cptr<dd::BeamArgs> p) {
    static_assert(sizeof(dd::BeamArgs) % 4 == 0, "descriptor size");
    constexpr int n = sizeof(dd::BeamArgs) / 4;
    const cptr<uint32_t> w = (cptr<uint32_t>)p;
    uint32_t tmp[n];
#pragma unroll
    for (int i = 0; i < n; ++i) tmp[i] = w[i];
    dd::BeamArgs a;
    __builtin_memcpy(&a, tmp, sizeof a);
    return a;
}

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

// Low counter of 5 levels per chunk (see gen_csa.py): the chunk's carry-out
// plane of weight 32 waits in `pend` for the next chunk's, and the two enter
// the upper levels together -- one ripple per two chunks instead of one per
// chunk.
template <int NL, int N>
__device__ __forceinline__ uint32_t csa_low(uint32_t (&a)[NL], const uint32_t (&lo)[N],
                                            const uint32_t (&hi)[N]) {
    if constexpr (N == 8)
        return csa5_add_8<NL>(a, lo, hi);
    else
        return csa5_add_4<NL>(a, lo, hi);
}

// Accumulate channels [c, c+N) of the current stage for one trial into the
// counters of its G groups.
// The trial's offset-table row gives, per channel, the LDS byte offset of the
// channel's first needed quad (bits 5 and up) and the funnel shift (bits 0-4,
// which is all the shift instruction reads).  A quad is a 16-byte aligned
// copy of two consecutive words, so each (trial, channel, group) is one
// aligned 16-byte LDS read.
template <int NL, int G, int N, bool ODD>
__device__ __forceinline__ void accumulate_chunk(uint32_t (&acc)[G][NL], uint32_t (&pend)[G],
                                                 const char* lds_lane, cptr<uint32_t> trow, int c) {
    uint32_t e[N];
#pragma unroll
    for (int k = 0; k < N; ++k) e[k] = trow[c + k];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // all N reads first, then the shifts: the reads' latencies overlap
        uint4 w[N];
#pragma unroll
        for (int k = 0; k < N; ++k)
            w[k] = *reinterpret_cast<const uint4*>(lds_lane + (e[k] >> 5) + 1024 * g);
        uint32_t lo[N], hi[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            lo[k] = bs::funnel(w[k].z, w[k].x, e[k]);
            hi[k] = bs::funnel(w[k].w, w[k].y, e[k]);
        }
        const uint32_t cy = csa_low<NL, N>(acc[g], lo, hi);
        if (ODD)
            bs::carry_in2<NL, 5>(acc[g], pend[g], cy);
        else
            pend[g] = cy;
    }
}

// One chunk, completing a pair of carry-outs when it is the second of two.
template <int NL, int G, int N>
__device__ __forceinline__ void chunk(uint32_t (&acc)[G][NL], uint32_t (&pend)[G], int k,
                                      const char* lds_lane, cptr<uint32_t> trow, int c) {
    if (k & 1)
        accumulate_chunk<NL, G, N, true>(acc, pend, lds_lane, trow, c);
    else
        accumulate_chunk<NL, G, N, false>(acc, pend, lds_lane, trow, c);
}

// Asynchronous copy of one LDS stage: channels [c0, c0 + cs) of the block's
// window, channel cl into row `cl` (a.pitch quads of 16 bytes).  Quad j of a
// row holds the words j and j + 1 of the window that starts at word
// w_base + (delay[d_lo][c] >> 5): stride - 1 quads cover the `stride` words,
// cut at the end of the channel's words (what lies beyond only feeds output
// samples past nout, which are never stored).  Each lane copies one quad,
// global -> LDS directly (16 bytes from an 8-byte aligned word address); the
// copies complete asynchronously: the caller waits for them before the
// barrier that publishes the stage.
__device__ __forceinline__ void fill_stage(const dd::BeamArgs& a, cptr<int32_t> dlo_row,
                                           int64_t w_base, int stride, int c0, int cs,
                                           char* __restrict__ lds, int lane, int wave) {
    for (int cl = wave; cl < cs; cl += kWaves) {
        const int c = c0 + cl;
        const int64_t w0 = w_base + (dlo_row[c] >> 5);
        // words of the row from w0 on: > 0 (w0 < nsamps / 32 + 1 < nwords) and
        // below 2^31, so the bound is 32-bit scalar arithmetic (a 64-bit
        // signed compare would go through vector registers)
        const int avail = static_cast<int>(a.nwords - w0);
        const int nq = min(avail, stride) - 1;
        // uniform source row; each lane adds its own 8-byte word offset
        const uint2* src = a.words + static_cast<int64_t>(c) * a.nwords + w0;
        char* dst = lds + cl * a.pitch * 16;
        // full batches of 64 quads need no per-lane check; only the last,
        // partial one (if any) compares lanes
        int i = 0;
        for (; i + 64 <= nq; i += 64)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + i + lane),
                                             (__attribute__((address_space(3))) void*)(dst + 16 * i), 16, 0, 0);
        if (i < nq && lane < nq - i)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + i + lane),
                                             (__attribute__((address_space(3))) void*)(dst + 16 * i), 16, 0, 0);
    }
}

// One stage: start the copy of the next stage into `nxt` (if any), then add
// this stage's channels from `cur`.  The two buffers are passed as restrict
// pointers so the compiler knows the LDS reads do not wait on the copy.
template <int NL, int NDW, int G>
__device__ __forceinline__ void run_stage(const dd::BeamArgs& a, uint32_t (&acc)[NDW][G][NL],
                                          uint32_t (&pend)[NDW][G], int kbase,
                                          cptr<int32_t> dlo_row, int64_t w_base, int stride,
                                          int c0, int stage_chans, int d_lo,
                                          const char* __restrict__ cur, char* __restrict__ nxt,
                                          bool more, int lane, int wave) {
    const int cs = min(stage_chans, a.nchans - c0);
    if (more)
        fill_stage(a, dlo_row, w_base, stride, c0 + stage_chans,
                   min(stage_chans, a.nchans - c0 - stage_chans), nxt, lane, wave);
#pragma unroll
    for (int i = 0; i < NDW; ++i) {
        const int d = d_lo + wave + kWaves * i;
        if (d < a.ndm) {
            const cptr<uint32_t> trow = as_const(a.offs) + static_cast<int64_t>(d) * a.nchans;
            int cl = 0, k = kbase;
            // 8-channel steps: fewer live registers than 16, more resident waves
#pragma unroll 1
            for (; cl + 8 <= cs; cl += 8, ++k)
                chunk<NL, G, 8>(acc[i], pend[i], k, cur + 16 * lane, trow, c0 + cl);
            if (cl + 4 <= cs) chunk<NL, G, 4>(acc[i], pend[i], k, cur + 16 * lane, trow, c0 + cl);
        }
    }
}

// One stage of exactly 8 channels: start the copy of the next stage, then add
// this stage's 8-channel chunk for every trial.  SECOND: the chunk is the
// second of a pair (its carry-out joins the first one's).
template <int NL, int NDW, int G, bool SECOND>
__device__ __forceinline__ void stage8(const dd::BeamArgs& a, uint32_t (&acc)[NDW][G][NL],
                                       uint32_t (&pend)[NDW][G], cptr<int32_t> dlo_row,
                                       int64_t w_base, int stride, int c0, int d_lo,
                                       const char* __restrict__ cur, char* __restrict__ nxt,
                                       bool more, int lane, int wave) {
    if (more) fill_stage(a, dlo_row, w_base, stride, c0 + 8, 8, nxt, lane, wave);
#pragma unroll
    for (int i = 0; i < NDW; ++i) {
        // a trial past the last one (a short last DM block) repeats the last
        // trial's offsets, so the code has no branch; its sums are never stored
        const int d = min(d_lo + wave + kWaves * i, a.ndm - 1);
        const cptr<uint32_t> trow = as_const(a.offs) + static_cast<int64_t>(d) * a.nchans;
        accumulate_chunk<NL, G, 8, SECOND>(acc[i], pend[i], cur + 16 * lane, trow, c0);
        // The trial's sums must exist here (an empty statement that reads and
        // writes them): the compiler may not sink the adds past the next
        // stage's barrier, where every trial's quads would be live at once.
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int l = 0; l < NL; ++l) asm volatile("" : "+v"(acc[i][g][l]));
            asm volatile("" : "+v"(pend[i][g]));
        }
    }
}

// One work item: DM block `dblk` x time tile `tile` of one beam.
//
// The LDS holds two stage buffers of `stage_chans` rows each; stage s lives in
// buffer s & 1, so channel c sits in row c mod (2 * stage_chans) -- the row
// the offset table assumes.  While the waves work on stage s, the copy of
// stage s + 1 into the other buffer is in flight.
template <int NL, int NDW, int G, bool OUT16, bool S8>
__device__ __forceinline__ void process_item(const dd::BeamArgs& a, int tile, int dblk,
                                             int stage_chans, char* lds, int lane, int wave) {
    constexpr int ND = NDW * kWaves;
    constexpr int T = 2048 * G;
    const int64_t T0 = static_cast<int64_t>(tile) * T;
    const int d_lo = dblk * ND;
    // words this block needs per channel row (<= a.pitch + 1)
    const int stride = a.tile_words + as_const(a.skew)[dblk];
    const int64_t w_base = T0 >> 5;
    const cptr<int32_t> dlo_row = as_const(a.delays) + static_cast<int64_t>(d_lo) * a.nchans;
    const int nst = (a.nchans + stage_chans - 1) / stage_chans;

    uint32_t acc[NDW][G][NL];
    uint32_t pend[NDW][G];
#pragma unroll
    for (int i = 0; i < NDW; ++i)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            pend[i][g] = 0u;
#pragma unroll
            for (int l = 0; l < NL; ++l) acc[i][g][l] = 0u;
        }
    int kbase = 0;   // chunks added so far (the same for every trial)

    fill_stage(a, dlo_row, w_base, stride, 0, min(stage_chans, a.nchans), lds, lane, wave);
    const int64_t half = static_cast<int64_t>(stage_chans) * a.pitch * 16;   // bytes
    if (S8) {
        // stages of 8 channels, every one full: pairs of stages, the first in
        // buffer 0 and the second in buffer 1, so the pairing of carry-outs
        // and the buffers are fixed in the code
        int st = 0;
#pragma unroll 1
        for (; st + 1 < nst; st += 2) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            stage8<NL, NDW, G, false>(a, acc, pend, dlo_row, w_base, stride, 8 * st, d_lo, lds,
                                      lds + half, true, lane, wave);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            stage8<NL, NDW, G, true>(a, acc, pend, dlo_row, w_base, stride, 8 * st + 8, d_lo,
                                     lds + half, lds, st + 2 < nst, lane, wave);
        }
        kbase = st;
        if (st < nst) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            stage8<NL, NDW, G, false>(a, acc, pend, dlo_row, w_base, stride, 8 * st, d_lo, lds,
                                      lds + half, false, lane, wave);
            kbase = nst;
        }
    }
#pragma unroll 1
    for (int st = 0; st < (S8 ? 0 : nst); ++st) {
        const int c0 = st * stage_chans;
        // this wave's copies of stage st are done; after the barrier every
        // wave's are, and every wave has finished stage st - 1, whose buffer
        // the copy of stage st + 1 now overwrites
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        run_stage<NL, NDW, G>(a, acc, pend, kbase, dlo_row, w_base, stride, c0, stage_chans, d_lo,
                              (st & 1) ? lds + half : lds, (st & 1) ? lds : lds + half,
                              st + 1 < nst, lane, wave);
        const int cs = min(stage_chans, a.nchans - c0);
        kbase += cs / 8 + ((cs & 4) ? 1 : 0);
    }
    // an odd number of chunks leaves one carry-out waiting
    if (kbase & 1) {
#pragma unroll
        for (int i = 0; i < NDW; ++i)
#pragma unroll
            for (int g = 0; g < G; ++g) bs::carry_in1<NL, 5>(acc[i][g], pend[i][g]);
    }

    // Write: counters -> integers, one 32-sample group per lane and group.
#pragma unroll
    for (int i = 0; i < NDW; ++i) {
        const int d = d_lo + wave + kWaves * i;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t t = T0 + 32 * (lane + 64 * g);
            if (d >= a.ndm || t >= a.nout) continue;
            uint32_t r[16];
            bs::planes_to_pairs<NL>(acc[i][g], r);
            const int64_t row = static_cast<int64_t>(d) * a.nout;
            const bool full = t + 32 <= a.nout;
            if (OUT16) {
                uint16_t* o = static_cast<uint16_t*>(a.out) + row + t;
                if (full && ((row + t) & 1) == 0) {
                    uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        o32[q] = (r[2 * q] & 0xFFFFu) | (r[2 * q + 1] << 16);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        o32[8 + q] = (r[2 * q] >> 16) | (r[2 * q + 1] & 0xFFFF0000u);
                } else {
                    const int n = static_cast<int>(min<int64_t>(32, a.nout - t));
#pragma unroll
                    for (int b = 0; b < 32; ++b)
                        if (b < n) o[b] = static_cast<uint16_t>(b < 16 ? r[b] : (r[b - 16] >> 16));
                }
            } else {
                int32_t* o = static_cast<int32_t*>(a.out) + row + t;
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
                    const int n = static_cast<int>(min<int64_t>(32, a.nout - t));
#pragma unroll
                    for (int b = 0; b < 32; ++b)
                        if (b < n) o[b] = static_cast<int32_t>(b < 16 ? (r[b] & 0xFFFFu) : (r[b - 16] >> 16));
                }
            }
        }
    }
}

// Work items go in groups of a.dm_group DM blocks: inside a group the DM
// block varies fastest, then the time tile.  The group's offset rows then stay
// in L2 while its time tiles go by, and the DM blocks of one time tile, whose
// input windows overlap, run together.
__device__ __forceinline__ void item_coords(const dd::BeamArgs& a, int64_t item, int* tile,
                                            int* dblk) {
    const int64_t n_tt = a.n_items / a.n_dm_blocks;
    const int64_t per_group = static_cast<int64_t>(a.dm_group) * n_tt;
    const int g = static_cast<int>(item / per_group);
    const int64_t rem = item - g * per_group;
    const int gs = min(a.dm_group, a.n_dm_blocks - g * a.dm_group);
    *tile = static_cast<int>(rem / gs);
    *dblk = g * a.dm_group + static_cast<int>(rem % gs);
}

template <int NL, int NDW, int G, bool OUT16>
__global__ __launch_bounds__(kThreads) void dedisperse_kernel(dd::BeamArgs a, int stage_chans,
                                                              int n_items) {
    extern __shared__ uint4 lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: hardware deals consecutive blocks round-robin to the 8
    // XCDs; give each XCD a contiguous run of (time tile, DM block) items with
    // the DM block fastest, so blocks resident on one XCD share input words in
    // its L2.
    const int per_xcd = gridDim.x / 8;
    const int item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (item >= n_items) return;
    int tile, dblk;
    item_coords(a, item, &tile, &dblk);
    if (stage_chans == 8 && (a.nchans & 7) == 0)
        process_item<NL, NDW, G, OUT16, true>(a, tile, dblk, 8, reinterpret_cast<char*>(lds), lane,
                                              wave);
    else
        process_item<NL, NDW, G, OUT16, false>(a, tile, dblk, stage_chans,
                                               reinterpret_cast<char*>(lds), lane, wave);
}

// Persistent form over the work items of several beams: blocks pop items
// from `nq` queues (block b serves queue b % nq; queue q owns the contiguous
// item range [q*total/nq, (q+1)*total/nq)), so that the blocks of one XCD work
// through neighbouring (beam, time tile, DM block) items.  Every block leaves
// once its queue is drained.
// The 12-level, 16-trial, one-group shape (the survey's) asks for 5 waves
// per SIMD: the item queue's extra scalars would otherwise spill into enough
// vector registers to leave 4 (the compiler then spills two per-item values
// to scratch instead).
template <int NL, int NDW, int G>
constexpr int persistent_min_waves() {
    return (NL == 12 && NDW == 4 && G == 1) ? 5 : 1;
}

template <int NL, int NDW, int G, bool OUT16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(persistent_min_waves<NL, NDW, G>())))
void dedisperse_persistent_kernel(
    const dd::BeamArgs* __restrict__ beams, int nbeams, int64_t total, int stage_chans,
    unsigned long long* __restrict__ counters, int nq) {
    extern __shared__ uint4 lds[];
    __shared__ long long item_sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = blockIdx.x % nq;
    const int64_t q_lo = total * q / nq;
    const int64_t q_hi = total * (q + 1) / nq;
    for (;;) {
        if (threadIdx.x == 0) item_sh = static_cast<long long>(q_lo + atomicAdd(&counters[q], 1ull));
        __syncthreads();
        // The popped item is uniform over the block: keep it (and all that is
        // derived from it: beam, delay rows, skew) in scalar registers.
        const unsigned long long raw = static_cast<unsigned long long>(item_sh);
        const int64_t item = static_cast<int64_t>(
            (static_cast<unsigned long long>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(raw >> 32))) << 32) |
            static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(raw))));
        __syncthreads();
        if (item >= q_hi) break;
        const cptr<dd::BeamArgs> cb = as_const(beams);
        int b = 0;
        while (b + 1 < nbeams && item >= cb[b + 1].item_begin) ++b;
        const dd::BeamArgs a = load_beam(cb + b);
        const int64_t local = item - a.item_begin;
        int tile, dblk;
        item_coords(a, local, &tile, &dblk);
        if (stage_chans == 8 && (a.nchans & 7) == 0)
            process_item<NL, NDW, G, OUT16, true>(a, tile, dblk, 8, reinterpret_cast<char*>(lds),
                                                  lane, wave);
        else
            process_item<NL, NDW, G, OUT16, false>(a, tile, dblk, stage_chans,
                                                   reinterpret_cast<char*>(lds), lane, wave);
    }
}

__global__ void zero_counters_kernel(unsigned long long* c, int n) {
    if (static_cast<int>(threadIdx.x) < n) c[threadIdx.x] = 0ull;
}

template <int NL, int NDW, int G, bool OUT16>
hipError_t launch_cfg(const dd::BeamArgs& a, int stage_chans, size_t lds, hipStream_t s) {
    auto kern = dedisperse_kernel<NL, NDW, G, OUT16>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    if (a.n_items > (int64_t(1) << 30)) return hipErrorInvalidValue;
    const int64_t nblocks = 8 * ((a.n_items + 7) / 8);
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(nblocks)), dim3(kThreads), lds, s, a,
                       stage_chans, static_cast<int>(a.n_items));
    return hipGetLastError();
}

template <int NL, int NDW, int G, bool OUT16>
hipError_t launch_persistent_cfg(const dd::BeamArgs* beams, int nbeams, int64_t total,
                                 int stage_chans, size_t lds, unsigned long long* counters, int nq,
                                 int grid, hipStream_t s) {
    auto kern = dedisperse_persistent_kernel<NL, NDW, G, OUT16>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, counters, nq);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, beams, nbeams, total, stage_chans,
                       counters, nq);
    return hipGetLastError();
}

template <int NL, int NDW, int G, bool OUT16>
int occupancy_cfg(size_t lds) {
    auto kern = dedisperse_persistent_kernel<NL, NDW, G, OUT16>;
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, kThreads, lds) != hipSuccess) return 0;
    return n;
}

}  // namespace

namespace dd {


int tile_pitch(const dedisp_plan_s* p, const TileConfig& cfg) {
    // quads per LDS row: one fewer than the words a row covers
    const int k = dm_block_index(cfg.dms_per_block);
    return k < 0 ? 0 : 2048 * cfg.groups / 32 + p->skew_max[k];
}

size_t tile_lds_bytes(const dedisp_plan_s* p, const TileConfig& cfg) {
    // two stage buffers of stage_chans rows of 16-byte quads
    return 2 * static_cast<size_t>(cfg.stage_chans) * tile_pitch(p, cfg) * sizeof(uint4);
}

BeamArgs beam_args(const dedisp_plan_s* p, const uint2* words, int64_t nwords, int64_t nout,
                   void* out, const TileConfig& cfg) {
    const int k = dm_block_index(cfg.dms_per_block);
    BeamArgs a{};
    a.words = words;
    a.nwords = nwords;
    a.nchans = p->nchans;
    a.ndm = p->ndm;
    a.nout = nout;
    a.delays = p->d_delays;
    a.offs = offset_table(p, cfg, false);
    a.skew = k >= 0 ? p->d_skew[k] : nullptr;
    a.out = out;
    a.n_dm_blocks = (p->ndm + cfg.dms_per_block - 1) / cfg.dms_per_block;
    // groups whose LDS-offset rows (4 bytes per trial and channel) fill about
    // kItemGroupBytes of L2
    const int64_t rows = static_cast<int64_t>(cfg.dms_per_block) * p->nchans * 4;
    a.dm_group = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(a.n_dm_blocks, kItemGroupBytes / rows)));
    const int64_t T = 2048 * cfg.groups;
    a.tile_words = static_cast<int>(T / 32 + 1);
    a.pitch = tile_pitch(p, cfg);
    a.item_begin = 0;
    a.n_items = ((nout + T - 1) / T) * a.n_dm_blocks;
    return a;
}

#define DD_SHAPES(X)                                                                   \
    X(12, 1, 1) X(12, 2, 1) X(12, 4, 1) X(12, 8, 1) X(12, 1, 2) X(12, 2, 2) X(12, 4, 2)   \
    X(16, 1, 1) X(16, 2, 1) X(16, 4, 1) X(16, 8, 1) X(16, 1, 2) X(16, 2, 2) X(16, 4, 2)

dedisp_status launch_dedisperse(const dedisp_plan_s* p, const uint2* words, int64_t nwords,
                                int64_t nout, void* out, int out_u16, const TileConfig& cfg,
                                hipStream_t s) {
    const int k = dm_block_index(cfg.dms_per_block);
    if (k < 0 || cfg.stage_chans < 4 || cfg.stage_chans % 4 || cfg.groups < 1 || cfg.groups > 2)
        return fail(DEDISP_ERR_INVALID_ARG, "unsupported tile configuration");
    const size_t lds = tile_lds_bytes(p, cfg);
    if (lds > 160 * 1024)
        return fail(DEDISP_ERR_UNSUPPORTED,
                    "DM block of %d trials spans %d words of skew: LDS tile of %zu bytes too large",
                    cfg.dms_per_block, p->skew_max[k], lds);
    const int nl = levels_for(p->nchans);
    dedisp_status st = DEDISP_OK;
    if (!offset_table(p, cfg, true, &st)) return st;
    const BeamArgs a = beam_args(p, words, nwords, nout, out, cfg);
    hipError_t e = hipErrorInvalidValue;
#define DD_DISPATCH(NL_, NDW_, G_)                                                    \
    if (nl == NL_ && cfg.dms_per_block == NDW_ * kWaves && cfg.groups == G_)          \
        e = out_u16 ? launch_cfg<NL_, NDW_, G_, true>(a, cfg.stage_chans, lds, s)     \
                    : launch_cfg<NL_, NDW_, G_, false>(a, cfg.stage_chans, lds, s);
    DD_SHAPES(DD_DISPATCH)
#undef DD_DISPATCH
    if (e != hipSuccess)
        return fail(e == hipErrorInvalidValue ? DEDISP_ERR_UNSUPPORTED : DEDISP_ERR_HIP,
                    "dedispersion launch failed: %s", hipGetErrorString(e));
    return DEDISP_OK;
}

hipError_t launch_dedisperse_persistent(const BeamArgs* d_beams, int nbeams, int64_t total,
                                        int nl, int out_u16, const TileConfig& cfg, size_t lds,
                                        unsigned long long* d_counters, int nq, int grid,
                                        hipStream_t s) {
    hipError_t e = hipErrorInvalidValue;
#define DD_DISPATCH(NL_, NDW_, G_)                                                              \
    if (nl == NL_ && cfg.dms_per_block == NDW_ * kWaves && cfg.groups == G_)                    \
        e = out_u16 ? launch_persistent_cfg<NL_, NDW_, G_, true>(d_beams, nbeams, total,        \
                          cfg.stage_chans, lds, d_counters, nq, grid, s)                        \
                    : launch_persistent_cfg<NL_, NDW_, G_, false>(d_beams, nbeams, total,       \
                          cfg.stage_chans, lds, d_counters, nq, grid, s);
    DD_SHAPES(DD_DISPATCH)
#undef DD_DISPATCH
    return e;
}

int persistent_blocks_per_cu(int nl, int out_u16, const TileConfig& cfg, size_t lds) {
    int n = 0;
#define DD_DISPATCH(NL_, NDW_, G_)                                                   \
    if (nl == NL_ && cfg.dms_per_block == NDW_ * kWaves && cfg.groups == G_)         \
        n = out_u16 ? occupancy_cfg<NL_, NDW_, G_, true>(lds) : occupancy_cfg<NL_, NDW_, G_, false>(lds);
    DD_SHAPES(DD_DISPATCH)
#undef DD_DISPATCH
    return n;
}

}  // namespace dd
