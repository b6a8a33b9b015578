// Boxcar matched filter, exact sigma-cut and peak finding (paper section 2.3).
//
// Boxcars come from a running sum: B_w[t] = P[t+w] - P[t] with P the prefix
// sum of a dedispersed series (the leading window; every width shares the
// valid length n_bx = nout - w_max + 1).  A block owns one (DM, segment of
// L start positions); it scans its window of the series in LDS with a
// wave-shuffle prefix sum -- only differences of P are used, so a segment
// needs no carry from the segments before it -- and evaluates every width
// from that one scan.  All boxcar arithmetic is uint32 modular (exact, since
// each B_w < 2^31).
//
// The sigma-cut is decided in integers: per (width, DM) series the exact sums
// S1 = sum B and S2 = sum B^2 give D = n S2 - S1^2, and a sample is above the
// cut iff B >= B_thr = ceil((S1 + isqrt(floor(k^2 D)) + 1) / n), k being the
// exact binary value of the float threshold (128/256-bit integer helpers).
//
// Events (section 2.3: each maximal run of above-cut samples of one series
// is one event) are compacted deterministically: count run starts per
// (width, DM, segment), exclusive scan, then write each event at its offset
// -- the output order is (width, DM, t_start) without any sort.  Only the
// (DM, segment)s whose largest boxcar reaches the cut are counted, and only
// those with events are written: both passes work through lists of them.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dedisp_internal.hpp"
#include "intmath.hpp"
#include "search_internal.hpp"

namespace {

constexpr int kThreads = 256;
// ----------------------------------------------------------------------------
// Block-level helpers.
// ----------------------------------------------------------------------------

// Exclusive prefix of one value per thread over the block (uint32, modular).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wave_tot[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < wave; ++i) base += wave_tot[i];
    __syncthreads();
    return base + x - v;
}

// Fill pl[0..n) with the running sum of the series values s[first + i]
// (values outside [0, nout) count as 0): pl[i] = sum_{k<i} s[first+k].
// Loads and LDS reads are issued in batches of kBatch per thread so that
// their latencies overlap.
constexpr int kBatch = 12;
// Word 3 of a raw (unstrided) buffer resource on gfx9-family GPUs: 32-bit
// data format, no swizzle; loads are range-checked against the byte count.
constexpr int kRowRsrcWord3 = 0x00020000;

// One sample of a series row through a buffer resource whose range is the
// row: offsets outside it (negative ones wrap to huge) read as 0.
__device__ __forceinline__ uint32_t row_load(__amdgpu_buffer_rsrc_t rs, int byte_off, uint16_t*) {
    return __builtin_amdgcn_raw_buffer_load_b16(rs, byte_off, 0, 0);
}
__device__ __forceinline__ uint32_t row_load(__amdgpu_buffer_rsrc_t rs, int byte_off, int32_t*) {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0);
}

template <typename T>
__device__ void load_prefix(const T* __restrict__ row, int64_t nout, int64_t first, int n,
                            uint32_t* pl, uint32_t* wave_tot, uint32_t* vmax = nullptr) {
    // coalesced load of the raw values into pl[1..n); the launchers keep a
    // row (and first + n) below 2^31 bytes
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(row), 0, static_cast<int>(nout * static_cast<int64_t>(sizeof(T))), kRowRsrcWord3);
    const int off0 = static_cast<int>(first) * static_cast<int>(sizeof(T));
    uint32_t m = 0;
    // full batches (every index below n - 1) store without checks; the last,
    // partial one checks each index
    int base = threadIdx.x;
    for (; base + (kBatch - 1) * kThreads < n - 1; base += kBatch * kThreads) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
            v[k] = row_load(rs, off0 + (base + k * kThreads) * static_cast<int>(sizeof(T)),
                            static_cast<T*>(nullptr));
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            pl[base + k * kThreads + 1] = v[k];
            m = max(m, v[k]);
        }
    }
    if (base < n - 1) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = base + k * kThreads;
            v[k] = row_load(rs, off0 + i * static_cast<int>(sizeof(T)), static_cast<T*>(nullptr));
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = base + k * kThreads;
            if (i < n - 1) {
                pl[i + 1] = v[k];
                m = max(m, v[k]);
            }
        }
    }
    if (vmax) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = max(m, static_cast<uint32_t>(__shfl_xor(m, o, 64)));
    }
    __syncthreads();
    // after the barrier, which orders them after the caller's clearing of
    // *vmax; the barrier at the end orders them before its readers
    if (vmax && (threadIdx.x & 63) == 0) atomicMax(vmax, m);
    // each thread scans a contiguous chunk (odd chunk stride: no bank conflicts)
    const int chunk = (((n - 1) + kThreads - 1) / kThreads) | 1;
    const int lo = 1 + threadIdx.x * chunk;
    const int hi = min(n, lo + chunk);
    // full batches without checks, then one checked remainder batch
    const int full_end = lo + ((max(hi - lo, 0)) / kBatch) * kBatch;
    uint32_t sum = 0;
    for (int i0 = lo; i0 < full_end; i0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = pl[i0 + k];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) sum += v[k];
    }
    if (full_end < hi) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = full_end + k < hi ? pl[full_end + k] : 0u;
#pragma unroll
        for (int k = 0; k < kBatch; ++k) sum += v[k];
    }
    const uint32_t scan_base = block_exclusive_scan(sum, wave_tot);
    uint32_t run = scan_base;
    for (int i0 = lo; i0 < full_end; i0 += kBatch) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = pl[i0 + k];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            run += v[k];
            pl[i0 + k] = run;
        }
    }
    if (full_end < hi) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = full_end + k < hi ? pl[full_end + k] : 0u;
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            run += v[k];
            if (full_end + k < hi) pl[full_end + k] = run;
        }
    }
    if (threadIdx.x == 0) pl[0] = 0u;
    __syncthreads();
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ----------------------------------------------------------------------------
// Kernels.
// ----------------------------------------------------------------------------

// Materialised boxcars for a DM sub-range (tests and inspection).
template <typename T>
__global__ __launch_bounds__(kThreads) void boxcar_kernel(const T* __restrict__ in, int64_t nout,
                                                          int64_t nbx, dd::Widths W, int dm_first,
                                                          int L, int32_t* __restrict__ out,
                                                          int dm_count) {
    extern __shared__ uint32_t pl[];
    __shared__ uint32_t wave_tot[kThreads / 64];
    const int d = dm_first + blockIdx.y;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * L;
    const int n = L + W.w[W.n - 1] + 1;
    load_prefix(in + static_cast<int64_t>(d) * nout, nout, s0 - 1, n, pl, wave_tot);
    for (int i = threadIdx.x; i < L; i += kThreads) {
        const int64_t t = s0 + i;
        if (t >= nbx) break;
        const uint32_t p0 = pl[i + 1];
        for (int wi = 0; wi < W.n; ++wi)
            out[(static_cast<int64_t>(wi) * dm_count + blockIdx.y) * nbx + t] =
                static_cast<int32_t>(pl[i + 1 + W.w[wi]] - p0);
    }
}

// Baseline (red-noise) removal by a running mean (section 2.3, first
// paragraph), streamed: out[t] = s[t + R] - floor(W(t) / (2R + 1)) + offset,
// W(t) = sum_{j=t}^{t+2R} s[j], integer and exact.  One wave walks kBlSeg
// outputs of one row, 64 consecutive outputs per row of a step (lane l takes
// t = tc + 64 i + l, so every load is coalesced).  The window slides:
// W(t + 1) - W(t) = s[t + 2R + 1] - s[t], so W(t) is W(t0) plus an exclusive
// wave prefix (DPP scan) of those differences -- one scan per row of 64
// outputs, every sample loaded once by the front cursor (and again, from
// cache, by the middle and back ones), no halo re-read.  Integers modulo 2^32
// are exact as every window sum is below 2^31; the division is the
// multiply-shift below.  The loads of the next step are in flight while a
// step is computed.
constexpr int kBlSeg = 16384;       // outputs per wave
constexpr int kBlRows = 16;         // rows of 64 outputs per step
constexpr int kBlStep = 64 * kBlRows;

// Inclusive prefix sum over the 64 lanes of a wave: shifts within each row
// of 16 lanes, then the row totals carried across rows.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, true));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, true));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, true));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, true));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xA, 0xF, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xC, 0xF, false));
    return x;
}

// Two uint16 values packed in a 32-bit word.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// c + the two 16-bit halves of v (one v_dot2_u32_u16 with the vector (1, 1)).
__device__ __forceinline__ uint32_t add_halves(uint32_t v, uint32_t c) {
    const u16x2 one = {1, 1};
    return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, v), one, c, false);
}

// The same running sums of a uint16 series window, for rows of a multiple of
// 4 samples from an 8-byte aligned series, without the LDS passes of the
// scan.  The window is read from a = first rounded down to a multiple of 4
// (and not below 0) in kRounds rounds of 1024 samples; in round i thread t
// takes samples a + 4(256 i + t) .. + 3 with one 8-byte load (every load lies
// wholly inside the row or wholly past its end, where it reads 0).  The
// thread sums its four (two packed 16-bit dot products), a DPP scan per
// round gives the wave's prefix, one DPP scan of the 36 wave totals in
// (round, wave) order gives the block's, and each group of four running
// sums goes to LDS with one 16-byte store.  The samples
// between a and first and past the window enter the sums too: only
// differences of the running sums are used, and the largest value only gates
// the fast path, so both stay exact.  lds needs kRunWords words.
// Returns ps with ps[i] - ps[j] = the sum of s[first + j .. first + i).
constexpr int kRounds = 9;
constexpr int kRunWords = 4 + 4 * kThreads * kRounds;

__device__ __forceinline__ const uint32_t* load_prefix_runs(const uint16_t* __restrict__ row,
                                                            int64_t nout, int64_t first, uint32_t* lds,
                                                            uint32_t* round_tot, uint32_t* vmax) {
    // first >= -1; the window of the first segment (first = -1) starts at 0
    // with shift -1 (its sample -1 counts as 0)
    const int64_t a = first < 0 ? 0 : first - (first & 3);
    const int shift = static_cast<int>(first - a);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(row), 0, static_cast<int>(nout * 2), kRowRsrcWord3);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int off0 = static_cast<int>(a) * 2 + static_cast<int>(threadIdx.x) * 8;
    uint32_t v[2 * kRounds];
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(rs, off0 + i * (8 * kThreads), 0, 0);
        v[2 * i] = x[0];
        v[2 * i + 1] = x[1];
    }
    u16x2 m2 = {0, 0};
    uint32_t excl[kRounds];
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        m2 = __builtin_elementwise_max(m2, __builtin_elementwise_max(__builtin_bit_cast(u16x2, v[2 * i]),
                                                                     __builtin_bit_cast(u16x2, v[2 * i + 1])));
        const uint32_t c = add_halves(v[2 * i + 1], add_halves(v[2 * i], 0u));
        const uint32_t incl = wave_incl_scan(c);
        excl[i] = incl - c;
        if (lane == 63) round_tot[i * (kThreads / 64) + wave] = incl;
    }
    uint32_t m = max(static_cast<uint32_t>(m2.x), static_cast<uint32_t>(m2.y));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, static_cast<uint32_t>(__shfl_xor(m, o, 64)));
    __syncthreads();
    // after the barrier (ordered after the caller's clearing of *vmax) and
    // before the final one (ordered before its readers)
    if (lane == 0) atomicMax(vmax, m);
    // The block's prefix before (round i, wave w) is the exclusive scan of
    // the wave totals in (round, wave) order: lane 4 i + w of every wave
    // scans them, and each wave reads its rounds' entries.
    const uint32_t tv = lane < kRounds * (kThreads / 64) ? round_tot[lane] : 0u;
    const uint32_t tin = wave_incl_scan(tv);
    const uint32_t tex = tin - tv;
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const uint32_t pre = static_cast<uint32_t>(
            __builtin_amdgcn_readlane(static_cast<int>(tex), i * (kThreads / 64) + wave));
        const uint32_t run = pre + excl[i];
        // lds[3 + k] = sum of s[a .. a + k): sample a + 4g + j ends at 4 + 4g + j
        const uint32_t w0 = run + (v[2 * i] & 0xFFFFu);
        const uint32_t w1 = add_halves(v[2 * i], run);
        const uint32_t w2 = w1 + (v[2 * i + 1] & 0xFFFFu);
        const uint32_t w3 = add_halves(v[2 * i + 1], w1);
        *reinterpret_cast<uint4*>(lds + 4 + 4 * (i * kThreads + threadIdx.x)) = make_uint4(w0, w1, w2, w3);
    }
    if (threadIdx.x == 0) {
        lds[2] = 0u;
        lds[3] = 0u;
    }
    __syncthreads();
    return lds + 3 + shift;
}

template <typename T>
__device__ __forceinline__ void bl_load(__amdgpu_buffer_rsrc_t rs, int64_t tc, int lane, int radius,
                                        uint32_t (&b)[kBlRows], uint32_t (&f)[kBlRows],
                                        uint32_t (&m)[kBlRows]) {
    const int sz = static_cast<int>(sizeof(T));
    const int base = static_cast<int>(tc) + lane;
#pragma unroll
    for (int i = 0; i < kBlRows; ++i) {
        b[i] = row_load(rs, (base + 64 * i) * sz, static_cast<T*>(nullptr));
        f[i] = row_load(rs, (base + 64 * i + 2 * radius + 1) * sz, static_cast<T*>(nullptr));
        m[i] = row_load(rs, (base + 64 * i + radius) * sz, static_cast<T*>(nullptr));
    }
}

template <typename T, typename U>
__global__ __launch_bounds__(kThreads) void baseline_kernel(const T* __restrict__ in, int ndm,
                                                            int64_t nout, int64_t nres, int radius,
                                                            int offset, int64_t nseg, uint64_t magic,
                                                            int shift, U* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    // the wave's item, in scalar registers (so is everything derived from
    // it, the row's buffer resource included: the loads need it uniform)
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int64_t item = static_cast<int64_t>(blockIdx.x) * (kThreads / 64) + wave;
    if (item >= static_cast<int64_t>(ndm) * nseg) return;   // whole waves
    const int d = static_cast<int>(item / nseg);
    const int64_t t0 = (item % nseg) * kBlSeg;
    const int64_t t1 = min<int64_t>(t0 + kBlSeg, nres);
    const T* row = in + static_cast<int64_t>(d) * nout;
    // a row stays below 2^31 bytes; offsets past it read as 0
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(row), 0, static_cast<int>(nout * static_cast<int64_t>(sizeof(T))), kRowRsrcWord3);
    const int sz = static_cast<int>(sizeof(T));
    const int win = 2 * radius + 1;
    // front start: the sum of s[t0 .. t0 + 2R]
    uint32_t acc = 0;
    for (int base = static_cast<int>(t0) + lane; base < static_cast<int>(t0) + win; base += kBatch * 64) {
        uint32_t v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = base + k * 64;
            v[k] = i < static_cast<int>(t0) + win ? row_load(rs, i * sz, static_cast<T*>(nullptr)) : 0u;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) acc += v[k];
    }
    // W(t0): the sum of s[t0 .. t0 + 2R]
    uint32_t wcur = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(wave_incl_scan(acc)), 63));
    U* o = out + static_cast<int64_t>(d) * nres;
    uint32_t b[kBlRows], f[kBlRows], m[kBlRows];
    bl_load<T>(rs, t0, lane, radius, b, f, m);
    for (int64_t tc = t0; tc < t1; tc += kBlStep) {
        uint32_t nb[kBlRows], nf[kBlRows], nm[kBlRows];
        bl_load<T>(rs, tc + kBlStep, lane, radius, nb, nf, nm);   // next step, in flight
#pragma unroll
        for (int i = 0; i < kBlRows; ++i) {
            const uint32_t delta = f[i] - b[i];        // W(t + 1) - W(t)
            const uint32_t incl = wave_incl_scan(delta);
            const uint32_t sum = wcur + incl - delta;   // W(t)
            // floor(sum / win) as a multiply and shift (exact for sum < 2^31)
            const uint32_t mean = static_cast<uint32_t>((static_cast<uint64_t>(sum) * magic) >> shift);
            const int64_t t = tc + 64 * i + lane;
            if (t < t1) o[t] = static_cast<U>(static_cast<int32_t>(m[i]) - static_cast<int32_t>(mean) + offset);
            wcur += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), 63));
        }
#pragma unroll
        for (int i = 0; i < kBlRows; ++i) {
            b[i] = nb[i];
            f[i] = nf[i];
            m[i] = nm[i];
        }
    }
}

// Pass 1: per (width, DM, segment) partial sums of B and B^2 and the largest B.
// Per thread and width at most L/256 <= 32 positions are summed in registers.
// When every B of the block's window is below 2^26 (the largest raw value
// times w_max says so) a 64-bit square sum cannot overflow even after the
// 64-lane reduction; otherwise the sums are carried as 128-bit values.
template <bool SMALL>
__device__ __forceinline__ void width_sums(const uint32_t* pl, int npos, int w, uint64_t* s1_out,
                                           u128* s2_out, uint32_t* mx_out) {
    uint64_t s1 = 0, lo = 0, hi = 0;
    uint32_t mx = 0;
    for (int i = threadIdx.x; i < npos; i += kThreads) {
        const uint32_t b = pl[i + 1 + w] - pl[i + 1];
        s1 += b;
        const uint64_t sq = static_cast<uint64_t>(b) * b;   // one v_mad_u64_u32 when SMALL
        lo += sq;
        if (!SMALL) hi += lo < sq ? 1u : 0u;
        mx = max(mx, b);
    }
    s1 = wave_sum_u64(s1);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(mx, o, 64)));
    if (SMALL) {
        *s2_out = wave_sum_u64(lo);
    } else {
        const uint64_t a = wave_sum_u64(lo & 0xFFFFFFFFull);
        const uint64_t b = wave_sum_u64(lo >> 32);
        const uint64_t c = wave_sum_u64(hi);
        *s2_out = static_cast<u128>(a) + (static_cast<u128>(b) << 32) + (static_cast<u128>(c) << 64);
    }
    *s1_out = s1;
    *mx_out = mx;
}

// Positions per thread in the fast path of a full segment.
constexpr int kPerThread = 32;

// Row stride, in values, of the per-width rows in the fast path's block
// reductions through LDS: the 16 lanes of one width read 16 consecutive
// values, and the next width's lanes start 16 banks further on for 4-byte
// values (32 for 8-byte ones).
constexpr int kRedStride = kThreads + 16;

// Sum / maximum over the 16 lanes of a DPP row (every lane gets it): swaps
// of neighbours and of pairs within each quad, then rotations by 4 and 8.
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x, int ctrl_sel) {
    switch (ctrl_sel) {
        case 0: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0xB1, 0xF, 0xF, false));
        case 1: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x4E, 0xF, 0xF, false));
        case 2: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x124, 0xF, 0xF, false));
        default: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x128, 0xF, 0xF, false));
    }
}
__device__ __forceinline__ uint64_t row_sum_u64(uint64_t v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint64_t o = (static_cast<uint64_t>(dpp_u32(static_cast<uint32_t>(v >> 32), c)) << 32) |
                           dpp_u32(static_cast<uint32_t>(v), c);
        v += o;
    }
    return v;
}
__device__ __forceinline__ uint32_t row_max_u32(uint32_t v) {
#pragma unroll
    for (int c = 0; c < 4; ++c) v = max(v, dpp_u32(v, c));
    return v;
}

// Fast path of a full segment with small values and NW (compile-time)
// widths: positions outer, widths inner, every partial sum in registers, then
// one block reduction through LDS (which the running sums no longer need).
template <int NW>
__device__ __forceinline__ void stats_full_nw(const uint32_t* ps, uint32_t* pl, const dd::Widths& W,
                                              const dd::PeaksWs& ws, int64_t idx0, int64_t stride) {
    uint64_t s2[NW];
    uint32_t mx[NW];
    int woff[NW];
#pragma unroll
    for (int wi = 0; wi < NW; ++wi) {
        mx[wi] = 0;
        s2[wi] = 0;
        woff[wi] = W.w[wi];
    }
    const uint32_t* base = ps + 1 + threadIdx.x;
#pragma unroll 8
    for (int j = 0; j < kPerThread; ++j) {
        const uint32_t p0 = base[j * kThreads];
#pragma unroll
        for (int wi = 0; wi < NW; ++wi) {
            const uint32_t b = base[j * kThreads + woff[wi]] - p0;
            s2[wi] += static_cast<uint64_t>(b) * b;
            mx[wi] = max(mx[wi], b);
        }
    }
    // Sum of the segment's boxcars by telescoping: with P the running sums,
    //   sum_{j<L} (P[j+1+w] - P[j+1]) = sum_{k=1..w} (P[L+k] - P[k]),
    // each term D(k) a sum of L samples (below 2^32 by the caller's check).
    // (After the main loop, so that its registers are free there.)  Lane l
    // of a wave takes k = k0 + l, 64 consecutive values, and a DPP scan of
    // D's two 16-bit halves (each below 2^22 over 64 lanes) gives their
    // inclusive prefix.  Lane wi < NW keeps width wi's sum: it takes the
    // prefix at lane w - k0, clamped to 63 (every k of the wave when
    // k0 + 63 <= w), and nothing when w < k0.
    constexpr int L = kPerThread * kThreads;
    const int lane = threadIdx.x & 63;
    int myw = 0;   // this lane's width (lanes >= NW: none)
#pragma unroll
    for (int wi = 0; wi < NW; ++wi)
        if (lane == wi) myw = woff[wi];
    uint64_t s1 = 0;
    for (int k0 = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) & ~63) + 1;
         k0 <= woff[NW - 1]; k0 += kThreads) {
        const int k = k0 + lane;
        const int kc = min(k, woff[NW - 1]);   // k past the widest width reads in range, counts 0
        const uint32_t dk = k <= woff[NW - 1] ? ps[L + kc] - ps[kc] : 0u;
        const uint32_t lo = wave_incl_scan(dk & 0xFFFFu);
        const uint32_t hi = wave_incl_scan(dk >> 16);
        const int l = myw - k0;
        const int src = min(max(l, 0), 63);
        const uint32_t glo = static_cast<uint32_t>(__shfl(static_cast<int>(lo), src, 64));
        const uint32_t ghi = static_cast<uint32_t>(__shfl(static_cast<int>(hi), src, 64));
        if (l >= 0) s1 += static_cast<uint64_t>(glo) + (static_cast<uint64_t>(ghi) << 16);
    }
    __syncthreads();   // the running sums are no longer needed: reuse pl
    // Per width, thread (wi, l) = 16 wi + l takes partials l, l+16, ..., of
    // width wi (rows of kRedStride values: the next width's 16 lanes start
    // on other banks), then the 16 lanes of the width, one DPP row, sum
    // their values; lane 16 wi ends with width wi's total.
    const int t = threadIdx.x;
    uint64_t* r = reinterpret_cast<uint64_t*>(pl);
#pragma unroll
    for (int wi = 0; wi < NW; ++wi) r[wi * kRedStride + t] = s2[wi];
    __syncthreads();
    uint64_t acc = 0;
    if (t < NW * 16) {
        const uint64_t* q = r + (t / 16) * kRedStride + (t % 16);
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += q[16 * k];
    }
    acc = row_sum_u64(acc);
    __syncthreads();
    // maxima, and the sums (one per wave and width)
    uint32_t* rm = pl + 2 * NW * kRedStride;
#pragma unroll
    for (int wi = 0; wi < NW; ++wi) rm[wi * kRedStride + t] = mx[wi];
    if (lane < NW) r[(t >> 6) * NW + lane] = s1;
    __syncthreads();
    uint64_t a1 = 0;
    uint32_t am = 0;
    if (t < NW * 16) {
        const uint32_t* qm = rm + (t / 16) * kRedStride + (t % 16);
#pragma unroll
        for (int k = 0; k < 16; ++k) am = max(am, qm[16 * k]);
        if ((t & 15) == 0) {
#pragma unroll
            for (int v = 0; v < kThreads / 64; ++v) a1 += r[v * NW + (t >> 4)];
        }
    }
    am = row_max_u32(am);
    // every global write after the last barrier (a barrier would wait for
    // them)
    if (t < NW * 16 && (t & 15) == 0) {
        const int64_t i = idx0 + (t >> 4) * stride;
        ws.part_s2lo[i] = acc;
        ws.part_s2hi[i] = 0u;   // below 2^63 (see the caller)
        ws.part_s1[i] = a1;
        ws.part_max[i] = am;
    }
}

template <typename T, int NW>
__global__ __launch_bounds__(kThreads) void boxcar_stats_kernel(const T* __restrict__ in,
                                                                int64_t nout, int64_t nbx,
                                                                dd::Widths W, int L, int nseg,
                                                                int runs, dd::PeaksWs ws) {
    // the dynamic LDS as 16-byte elements, so that its base is 16-byte
    // aligned (16-byte LDS accesses in the window loads)
    extern __shared__ uint4 pl16[];
    uint32_t* pl = reinterpret_cast<uint32_t*>(pl16);
    __shared__ uint32_t wave_tot[kThreads / 64];
    __shared__ __attribute__((aligned(16))) uint32_t round_tot[kRounds * (kThreads / 64)];
    __shared__ uint64_t red1[kThreads / 64][dd::kMaxWidths];
    __shared__ u128 red2[kThreads / 64][dd::kMaxWidths];
    __shared__ uint32_t redm[kThreads / 64][dd::kMaxWidths];
    __shared__ uint32_t vmax;
    const int d = blockIdx.y;
    const int seg = blockIdx.x;
    const int64_t s0 = static_cast<int64_t>(seg) * L;
    const int w_max = W.w[W.n - 1];
    const int n = L + w_max + 1;
    if (threadIdx.x == 0) vmax = 0;
    // the window's running sums: ps[i] - ps[j] = sum of s[s0 - 1 + j .. s0 - 1 + i)
    const uint32_t* ps = pl;
    if constexpr (std::is_same<T, uint16_t>::value) {
        if (runs)
            ps = load_prefix_runs(in + static_cast<int64_t>(d) * nout, nout, s0 - 1, pl, round_tot, &vmax);
        else
            load_prefix(in + static_cast<int64_t>(d) * nout, nout, s0 - 1, n, pl, wave_tot, &vmax);
    } else {
        load_prefix(in + static_cast<int64_t>(d) * nout, nout, s0 - 1, n, pl, wave_tot, &vmax);
    }
    const int npos = static_cast<int>(min<int64_t>(L, nbx - s0));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t bmax = static_cast<uint64_t>(vmax) * static_cast<uint64_t>(w_max);
    // every boxcar below 2^26: a wave's 64-bit square sum (at most 64 x 32
    // squares below 2^52) cannot overflow
    const bool small = bmax < (uint64_t(1) << 26);
    // full fast path: a whole segment whose square sum, over all its
    // kPerThread * 256 = 2^13 positions, stays below 2^13 * 2^50 = 2^63 (every
    // boxcar below 2^25), and every sum of L consecutive samples below 2^32
    // (for the telescoped S1)
    const bool full = bmax < (uint64_t(1) << 25) && npos == kPerThread * kThreads &&
                      vmax < (1u << 19) && L == kPerThread * kThreads;
    constexpr int NWS = NW > 0 ? NW : 1;
    if (NW > 0 && full) {
        // partial of width wi at idx0 + wi * stride
        stats_full_nw<NWS>(ps, pl, W, ws, static_cast<int64_t>(d) * nseg + seg,
                           static_cast<int64_t>(gridDim.y) * nseg);
        return;
    }
    for (int wi = 0; wi < W.n; ++wi) {
        uint64_t s1;
        u128 s2;
        uint32_t mx;
        if (small)
            width_sums<true>(ps, npos, W.w[wi], &s1, &s2, &mx);
        else
            width_sums<false>(ps, npos, W.w[wi], &s1, &s2, &mx);
        if (lane == 0) {
            red1[wave][wi] = s1;
            red2[wave][wi] = s2;
            redm[wave][wi] = mx;
        }
    }
    __syncthreads();
    if (threadIdx.x < W.n) {
        const int wi = threadIdx.x;
        uint64_t s1 = 0;
        u128 s2 = 0;
        uint32_t mx = 0;
        for (int v = 0; v < kThreads / 64; ++v) {
            s1 += red1[v][wi];
            s2 += red2[v][wi];
            mx = max(mx, redm[v][wi]);
        }
        const int64_t idx = (static_cast<int64_t>(wi) * gridDim.y + d) * nseg + seg;
        ws.part_s1[idx] = s1;
        ws.part_s2lo[idx] = static_cast<uint64_t>(s2);
        ws.part_s2hi[idx] = static_cast<uint64_t>(s2 >> 64);
        ws.part_max[idx] = mx;
    }
}

// Pass 2: exact sums, D and B_thr per (width, DM) series, kSerPerBlock
// series per block.  A series' partials are contiguous (series-major), so the
// block stages a chunk of segments of all its series in LDS with loads that
// every thread issues at once (one memory round trip per chunk); thread t then
// adds series t's entries.  The sums are exact integers: their order is free.
constexpr int kSerPerBlock = 64;
constexpr int kSerChunk = 32;   // segments per staged chunk: 3 x 64 x 32 x 8 B = 48 KiB
__global__ __launch_bounds__(kThreads) void series_threshold_kernel(int nseries, int nseg,
                                                                    int64_t nbx, uint32_t kmant,
                                                                    int kexp2, dd::PeaksWs ws) {
    __shared__ uint64_t st1[kSerPerBlock * kSerChunk];
    __shared__ uint64_t st2lo[kSerPerBlock * kSerChunk];
    __shared__ uint64_t st2hi[kSerPerBlock * kSerChunk];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ws.nlist[0] = 0u;   // the mark and count passes append to the work lists
        ws.nlist[1] = 0u;
    }
    const int s0 = blockIdx.x * kSerPerBlock;
    const int ns = min(kSerPerBlock, nseries - s0);
    const int t = threadIdx.x;
    uint64_t s1 = 0;
    u128 s2 = 0;
    for (int c0 = 0; c0 < nseg; c0 += kSerChunk) {
        const int nc = min(kSerChunk, nseg - c0);
        const int n = ns * nc;
        constexpr int kPer = kSerPerBlock * kSerChunk / kThreads;
        uint64_t v1[kPer], vlo[kPer], vhi[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = t + k * kThreads;
            const int64_t idx = static_cast<int64_t>(s0 + i / nc) * nseg + c0 + i % nc;
            const bool in = i < n;
            v1[k] = in ? ws.part_s1[idx] : 0;
            vlo[k] = in ? ws.part_s2lo[idx] : 0;
            vhi[k] = in ? ws.part_s2hi[idx] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = t + k * kThreads;
            if (i < n) {
                st1[i] = v1[k];
                st2lo[i] = vlo[k];
                st2hi[i] = vhi[k];
            }
        }
        __syncthreads();
        if (t < ns) {
            for (int k = 0; k < nc; ++k) {
                const int i = t * nc + k;
                s1 += st1[i];
                s2 += static_cast<u128>(st2lo[i]) | (static_cast<u128>(st2hi[i]) << 64);
            }
        }
        __syncthreads();   // the next chunk overwrites the staging arrays
    }
    if (t >= ns) return;
    const int s = s0 + t;
    ws.s1[s] = s1;
    ws.s2lo[s] = static_cast<uint64_t>(s2);
    ws.s2hi[s] = static_cast<uint64_t>(s2 >> 64);
    u128 d = 0;
    const int64_t thr = cut_level(static_cast<uint64_t>(nbx), s1, s2, kmant, kexp2, &d);
    if (thr < 0) {
        ws.thr[s] = -1;
        ws.thr32[s] = 0xFFFFFFFFu;
        ws.sqrt_d[s] = 0.0;
        return;
    }
    ws.thr[s] = thr;
    ws.thr32[s] = thr > 0xFFFFFFFFll ? 0xFFFFFFFFu : static_cast<uint32_t>(thr);
    ws.sqrt_d[s] = sqrt(u128_to_double(d));
}

// Pass 3a: one thread per (DM, segment).  A segment where, for some width,
// the largest boxcar reaches the series' cut goes on the count work list;
// every other segment gets zero run starts for all widths here.
__global__ __launch_bounds__(kThreads) void mark_kernel(int ndm, int nseg, int nw, dd::PeaksWs ws) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (idx >= static_cast<int64_t>(ndm) * nseg) return;
    const int d = static_cast<int>(idx / nseg);
    bool any = false;
    for (int wi = 0; wi < nw; ++wi)
        any |= ws.part_max[static_cast<int64_t>(wi) * ndm * nseg + idx] >= ws.thr32[wi * ndm + d];
    if (any) {
        ws.list[atomicAdd(&ws.nlist[0], 1u)] = static_cast<uint32_t>(idx);
    } else {
        for (int wi = 0; wi < nw; ++wi) ws.counts[static_cast<int64_t>(wi) * ndm * nseg + idx] = 0;
    }
}

// Pass 3b: number of run starts per (width, DM, segment) of the listed
// segments (a fixed grid of blocks works through the list).  Segments with
// any start go on the write list.
template <typename T>
__global__ __launch_bounds__(kThreads) void peaks_count_kernel(const T* __restrict__ in, int ndm,
                                                               int64_t nout, int64_t nbx,
                                                               dd::Widths W, int L, int nseg,
                                                               dd::PeaksWs ws) {
    extern __shared__ uint32_t pl[];
    __shared__ uint32_t wave_tot[kThreads / 64];
    __shared__ uint32_t cnt[dd::kMaxWidths];
    const uint32_t nitems = ws.nlist[0];
    const int lane = threadIdx.x & 63;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int64_t idx = ws.list[item];
        const int d = static_cast<int>(idx / nseg);
        const int seg = static_cast<int>(idx % nseg);
        const int64_t s0 = static_cast<int64_t>(seg) * L;
        const int n = L + W.w[W.n - 1] + 1;
        if (threadIdx.x < dd::kMaxWidths) cnt[threadIdx.x] = 0;
        load_prefix(in + static_cast<int64_t>(d) * nout, nout, s0 - 1, n, pl, wave_tot);
        const int npos = static_cast<int>(min<int64_t>(L, nbx - s0));
        for (int wi = 0; wi < W.n; ++wi) {
            const uint32_t thr = ws.thr32[wi * ndm + d];
            if (ws.part_max[(static_cast<int64_t>(wi) * ndm + d) * nseg + seg] < thr) continue;
            const int w = W.w[wi];
            uint32_t c = 0;
            for (int i0 = threadIdx.x; i0 < npos; i0 += 4 * kThreads) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int i = i0 + k * kThreads;
                    if (i < npos) {
                        const bool above = pl[i + 1 + w] - pl[i + 1] >= thr;
                        const bool prev = (s0 + i > 0) && (pl[i + w] - pl[i] >= thr);
                        c += (above && !prev) ? 1u : 0u;
                    }
                }
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
            if (lane == 0 && c) atomicAdd(&cnt[wi], c);
        }
        __syncthreads();
        if (threadIdx.x < W.n)
            ws.counts[(static_cast<int64_t>(threadIdx.x) * ndm + d) * nseg + seg] = cnt[threadIdx.x];
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int wi = 0; wi < W.n; ++wi) tot += cnt[wi];
            if (tot) ws.list2[atomicAdd(&ws.nlist[1], 1u)] = static_cast<uint32_t>(idx);
        }
        __syncthreads();   // pl and cnt are reused by the next item
    }
}

// Exclusive scan of counts (uint32) into offsets (int64): three small kernels.
constexpr int kScanChunk = 4096;

__global__ __launch_bounds__(kThreads) void scan_chunks_kernel(const uint32_t* __restrict__ counts,
                                                               int64_t n, int64_t* __restrict__ offs,
                                                               int64_t* __restrict__ chunk_tot) {
    __shared__ uint32_t wave_tot[kThreads / 64];
    __shared__ int64_t carry;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * kScanChunk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < kScanChunk; base += kThreads) {
        const int64_t i = c0 + base + threadIdx.x;
        const uint32_t v = i < n ? counts[i] : 0u;
        const uint32_t ex = block_exclusive_scan(v, wave_tot);
        const int64_t cur = carry;
        if (i < n) offs[i] = cur + ex;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry = cur + ex + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_tot[blockIdx.x] = carry;
}

// Exclusive scan of the chunk totals in place (one block; 64-bit sums).
__global__ __launch_bounds__(kThreads) void scan_totals_kernel(int64_t* __restrict__ chunk_tot,
                                                               int nchunks,
                                                               int64_t* __restrict__ total) {
    __shared__ int64_t wave_tot[kThreads / 64];
    __shared__ int64_t carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nchunks; base += kThreads) {
        const int i = base + static_cast<int>(threadIdx.x);
        const int64_t v = i < nchunks ? chunk_tot[i] : 0;
        int64_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wave_tot[wave] = x;
        __syncthreads();
        int64_t before = carry;
        for (int w = 0; w < wave; ++w) before += wave_tot[w];
        if (i < nchunks) chunk_tot[i] = before + x - v;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry = before + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kThreads) void scan_add_kernel(int64_t* __restrict__ offs, int64_t n,
                                                            const int64_t* __restrict__ chunk_tot) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) offs[i] += chunk_tot[i / kScanChunk];
}

// Walk the run that starts at t with boxcar value b and write its event
// record.  Positions whose boxcar the block's running sums cover (local index
// below `lim`, running sums pl relative to s0) are read from LDS, kWalk at a
// time (the reads do not depend on each other); a run that goes on past them
// continues on the series in global memory with the sliding-window update,
// again loading kWalk positions' samples at once.
constexpr int kWalk = 16;

template <typename T>
__device__ __forceinline__ void write_event(const T* __restrict__ row, int64_t nbx, int w, int wi, int d,
                                            int64_t t, uint32_t b, uint32_t thr, uint64_t s1, double sqrt_d,
                                            dedisp_event* __restrict__ out, const uint32_t* pl,
                                            int64_t s0, int lim) {
    int64_t te = t, tp = t;
    uint32_t cur = b, best = b;
    bool open = true;                       // the run has not ended yet
    int64_t u = t;                          // last position of the run so far
    while (open && u + 1 < nbx && u + 1 - s0 < lim) {
        uint32_t bb[kWalk];
#pragma unroll
        for (int k = 0; k < kWalk; ++k) {
            const int64_t j = u + 1 + k - s0;
            bb[k] = (j < lim && u + 1 + k < nbx) ? pl[j + 1 + w] - pl[j + 1] : 0u;
        }
        int k = 0;
        for (; k < kWalk; ++k) {
            const int64_t v = u + 1 + k;
            if (v >= nbx || v - s0 >= lim) break;   // leave the LDS window: continue below
            if (bb[k] < thr) {
                open = false;
                break;
            }
            cur = bb[k];
            te = v;
            if (cur > best) {
                best = cur;
                tp = v;
            }
        }
        u += k;
    }
    while (open && u + 1 < nbx) {
        uint32_t add[kWalk], sub[kWalk];
#pragma unroll
        for (int k = 0; k < kWalk; ++k) {
            const bool in = u + 1 + k < nbx;    // then u + k + w <= nout - 1
            add[k] = in ? static_cast<uint32_t>(row[u + k + w]) : 0u;
            sub[k] = in ? static_cast<uint32_t>(row[u + k]) : 0u;
        }
        int k = 0;
        for (; k < kWalk; ++k) {
            if (u + 1 + k >= nbx) break;
            const uint32_t nb = cur + add[k] - sub[k];
            if (nb < thr) {
                open = false;
                break;
            }
            cur = nb;
            te = u + 1 + k;
            if (nb > best) {
                best = nb;
                tp = te;
            }
        }
        u += k;
        if (k < kWalk) break;
    }
    const int64_t lval = static_cast<int64_t>(nbx) * best - static_cast<int64_t>(s1);
    dedisp_event ev;
    ev.width_idx = wi;
    ev.dm_idx = d;
    ev.t_start = t;
    ev.t_end = te;
    ev.t_peak = tp;
    ev.b_peak = static_cast<int32_t>(best);
    ev.snr = static_cast<float>(static_cast<double>(lval) / sqrt_d);
    *out = ev;
}

// The same walk done by a whole wave, 64 consecutive positions per step.
// Inside the LDS window a lane takes its position's boxcar from the running
// sums; beyond it, the boxcars follow from the last one by a wave prefix sum
// of the add/subtract pairs.  The run goes on through the lanes before the
// first one whose boxcar is below the cut (a ballot); the peak is the largest
// boxcar, the earliest on ties, as in the walk above, so both give the same
// event.  Arguments are uniform over the wave; lane 0 writes the event.
template <typename T>
__device__ __forceinline__ void write_event_wave(const T* __restrict__ row, int64_t nbx, int w, int wi,
                                                 int d, int64_t t, uint32_t b, uint32_t thr, uint64_t s1,
                                                 double sqrt_d, dedisp_event* __restrict__ out,
                                                 const uint32_t* pl, int64_t s0, int lim, int lane) {
    int64_t te = t, tp = t;
    uint32_t cur = b, best = b;
    bool open = true;
    int64_t u = t;   // last position of the run so far
    while (open && u + 1 < nbx) {
        const int64_t v = u + 1 + lane;
        bool valid;
        uint32_t bb = 0u;
        if (u + 1 - s0 < lim) {
            // validity falls from true to false at most once along the lanes
            valid = v < nbx && v - s0 < lim;
            if (valid) {
                const int j = static_cast<int>(v - s0);
                bb = pl[j + 1 + w] - pl[j + 1];
            }
        } else {
            valid = v < nbx;   // then u + lane + w <= nout - 1
            const uint32_t delta =
                valid ? static_cast<uint32_t>(row[u + lane + w]) - static_cast<uint32_t>(row[u + lane]) : 0u;
            bb = cur + wave_incl_scan(delta);
        }
        const uint64_t below = __ballot(valid && bb < thr);
        const uint64_t stop = below | __ballot(!valid);
        const int nlive = stop ? __builtin_ctzll(stop) : 64;
        if (nlive > 0) {
            uint32_t m = lane < nlive ? bb : 0u;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) m = max(m, static_cast<uint32_t>(__shfl_xor(m, o, 64)));
            if (m > best) {
                best = m;
                tp = u + 1 + __builtin_ctzll(__ballot(lane < nlive && bb == m));
            }
            cur = static_cast<uint32_t>(__shfl(bb, nlive - 1, 64));
            te = u + nlive;
        }
        // the run ends at a position below the cut; leaving the window or the
        // data does not end it
        if (nlive < 64 && ((below >> nlive) & 1u)) open = false;
        u += nlive;
    }
    if (lane == 0) {
        const int64_t lval = static_cast<int64_t>(nbx) * best - static_cast<int64_t>(s1);
        dedisp_event ev;
        ev.width_idx = wi;
        ev.dm_idx = d;
        ev.t_start = t;
        ev.t_end = te;
        ev.t_peak = tp;
        ev.b_peak = static_cast<int32_t>(best);
        ev.snr = static_cast<float>(static_cast<double>(lval) / sqrt_d);
        *out = ev;
    }
}

// Pass 4: write the events of segments that have any.  The run starts of a
// (width, DM, segment) are collected in LDS (any order), ranked by position
// (they are few), and each is expanded by one thread at offset + rank;
// segments with very many starts use block-wide scans in position order.
constexpr int kMaxStarts = 1024;

// The events of one listed (DM, segment).
template <typename T>
__device__ __forceinline__ void write_segment(const T* __restrict__ in, int ndm, int64_t nout, int64_t nbx,
                              const dd::Widths& W, int L, int nseg, const dd::PeaksWs& ws,
                              dedisp_event* __restrict__ events, int64_t capacity, int d, int seg,
                              uint32_t* pl, uint32_t* wave_tot, int* starts, int* nstart_p,
                              uint32_t* slab_total_p) {
    int& nstart = *nstart_p;
    uint32_t& slab_total = *slab_total_p;
    const int64_t s0 = static_cast<int64_t>(seg) * L;
    const int n = L + W.w[W.n - 1] + 1;
    const T* row = in + static_cast<int64_t>(d) * nout;
    load_prefix(row, nout, s0 - 1, n, pl, wave_tot);
    const int npos = static_cast<int>(min<int64_t>(L, nbx - s0));

    // Every width at once when all the segment's run starts fit the list:
    // width wi's starts fill starts[base[wi] .. base[wi] + count[wi]) (the
    // counts are known from the count pass), one pass over the positions
    // finds them, and then all runs of all widths are walked concurrently.
    __shared__ uint32_t wb[dd::kMaxWidths + 1], wc[dd::kMaxWidths], wfill[dd::kMaxWidths];
    __shared__ uint32_t wthr[dd::kMaxWidths];
    if (threadIdx.x < W.n) {
        const int wi = threadIdx.x;
        wc[wi] = ws.counts[(static_cast<int64_t>(wi) * ndm + d) * nseg + seg];
        wthr[wi] = ws.thr32[wi * ndm + d];
        wfill[wi] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int wi = 0; wi < W.n; ++wi) {
            wb[wi] = b;
            b += wc[wi];
        }
        wb[W.n] = b;
    }
    __syncthreads();
    const uint32_t total = wb[W.n];
    if (total <= static_cast<uint32_t>(kMaxStarts)) {
        // width outer (uniform), four positions per step: as in the count pass
        for (int wi = 0; wi < W.n; ++wi) {
            if (wc[wi] == 0) continue;
            const int w = W.w[wi];
            const uint32_t thr = wthr[wi];
            for (int i0 = threadIdx.x; i0 < npos; i0 += 4 * kThreads) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + q * kThreads;
                    if (i < npos) {
                        const bool above = pl[i + 1 + w] - pl[i + 1] >= thr;
                        const bool prev = (s0 + i > 0) && (pl[i + w] - pl[i] >= thr);
                        if (above && !prev) {
                            const uint32_t k = atomicAdd(&wfill[wi], 1u);
                            if (k < wc[wi]) starts[wb[wi] + k] = i;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // one run per wave: its rank among its width's starts, then its walk
        const int lane = threadIdx.x & 63;
        for (uint32_t k = threadIdx.x >> 6; k < total; k += kThreads / 64) {
            int wi = 0;
            while (wb[wi + 1] <= k) ++wi;
            const int i = starts[k];
            uint32_t rank = 0;
            for (uint32_t q = wb[wi] + lane; q < wb[wi + 1]; q += 64) rank += starts[q] < i;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) rank += __shfl_xor(rank, o, 64);
            const int64_t cidx = (static_cast<int64_t>(wi) * ndm + d) * nseg + seg;
            const int64_t e = ws.offs[cidx] + rank;
            const int w = W.w[wi];
            const int sidx = wi * ndm + d;
            if (e < capacity)
                write_event_wave(row, nbx, w, wi, d, s0 + i, pl[i + 1 + w] - pl[i + 1], wthr[wi],
                                 ws.s1[sidx], ws.sqrt_d[sidx], &events[e], pl, s0, n - 1 - w, lane);
        }
        return;
    }

    for (int wi = 0; wi < W.n; ++wi) {
        const int64_t cidx = (static_cast<int64_t>(wi) * ndm + d) * nseg + seg;
        const uint32_t cnt = ws.counts[cidx];
        if (cnt == 0) continue;
        const int sidx = wi * ndm + d;
        const uint32_t thr = ws.thr32[sidx];
        const int w = W.w[wi];
        const int64_t off = ws.offs[cidx];
        const uint64_t s1 = ws.s1[sidx];
        const double sq = ws.sqrt_d[sidx];
        const int lim = n - 1 - w;   // local positions whose boxcar the running sums cover
        if (cnt <= kMaxStarts) {
            if (threadIdx.x == 0) nstart = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < npos; i += kThreads) {
                const uint32_t b = pl[i + 1 + w] - pl[i + 1];
                const bool prev = (s0 + i > 0) && (pl[i + w] - pl[i] >= thr);
                if (b >= thr && !prev) {
                    const int k = atomicAdd(&nstart, 1);
                    if (k < kMaxStarts) starts[k] = i;
                }
            }
            __syncthreads();
            const int m = min(nstart, kMaxStarts);
            for (int k = threadIdx.x; k < m; k += kThreads) {
                const int i = starts[k];
                int rank = 0;
                for (int q = 0; q < m; ++q) rank += starts[q] < i;
                const int64_t e = off + rank;
                if (e < capacity)
                    write_event(row, nbx, w, wi, d, s0 + i, pl[i + 1 + w] - pl[i + 1], thr, s1, sq, &events[e],
                                pl, s0, lim);
            }
            __syncthreads();
        } else {
            int64_t rank = off;
            for (int base = 0; base < npos; base += kThreads) {
                const int i = base + threadIdx.x;
                bool start = false;
                uint32_t b = 0;
                if (i < npos) {
                    b = pl[i + 1 + w] - pl[i + 1];
                    const bool prev = (s0 + i > 0) && (pl[i + w] - pl[i] >= thr);
                    start = b >= thr && !prev;
                }
                const uint32_t ex = block_exclusive_scan(start ? 1u : 0u, wave_tot);
                if (start && rank + ex < capacity)
                    write_event(row, nbx, w, wi, d, s0 + i, b, thr, s1, sq, &events[rank + ex], pl, s0,
                                lim);
                if (threadIdx.x == kThreads - 1) slab_total = ex + (start ? 1u : 0u);
                __syncthreads();
                rank += slab_total;
                __syncthreads();
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void peaks_write_kernel(const T* __restrict__ in, int ndm,
                                                               int64_t nout, int64_t nbx,
                                                               dd::Widths W, int L, int nseg,
                                                               dd::PeaksWs ws,
                                                               dedisp_event* __restrict__ events,
                                                               int64_t capacity) {
    extern __shared__ uint32_t pl[];
    __shared__ uint32_t wave_tot[kThreads / 64];
    __shared__ int starts[kMaxStarts];
    __shared__ int nstart;
    __shared__ uint32_t slab_total;
    const uint32_t nitems = ws.nlist[1];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int64_t idx = ws.list2[item];
        write_segment(in, ndm, nout, nbx, W, L, nseg, ws, events, capacity,
                      static_cast<int>(idx / nseg), static_cast<int>(idx % nseg), pl, wave_tot,
                      starts, &nstart, &slab_total);
        __syncthreads();   // LDS is reused by the next item
    }
}

}  // namespace

namespace dd {

int segment_length(int w_max) {
    // LDS holds L + w_max + 1 running sums.
    int L = 8192;
    while (L > 256 && static_cast<int64_t>(L + w_max + 1) * 4 > 60 * 1024) L >>= 1;
    return L;
}

// Blocks of the list-driven count and write passes (a few per CU).
constexpr int64_t kListBlocks = 2048;

size_t peaks_lds_bytes(int L, int w_max) { return static_cast<size_t>(L + w_max + 1) * 4; }

hipError_t set_lds_limit(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

hipError_t launch_boxcar(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                         int dm_first, int dm_count, int32_t* out, hipStream_t s) {
    (void)ndm;
    const int w_max = W.w[W.n - 1];
    const int64_t nbx = nout - w_max + 1;
    const int L = segment_length(w_max);
    const size_t lds = peaks_lds_bytes(L, w_max);
    const dim3 grid(static_cast<unsigned>((nbx + L - 1) / L), static_cast<unsigned>(dm_count));
    if (in_u16) {
        set_lds_limit(reinterpret_cast<const void*>(boxcar_kernel<uint16_t>), lds);
        hipLaunchKernelGGL(boxcar_kernel<uint16_t>, grid, dim3(kThreads), lds, s,
                           static_cast<const uint16_t*>(in), nout, nbx, W, dm_first, L, out, dm_count);
    } else {
        set_lds_limit(reinterpret_cast<const void*>(boxcar_kernel<int32_t>), lds);
        hipLaunchKernelGGL(boxcar_kernel<int32_t>, grid, dim3(kThreads), lds, s,
                           static_cast<const int32_t*>(in), nout, nbx, W, dm_first, L, out, dm_count);
    }
    return hipGetLastError();
}

hipError_t launch_baseline(const void* in, int in_u16, int ndm, int64_t nout, int radius,
                           int offset, void* out, int out_u16, hipStream_t s) {
    const int64_t nres = nout - 2 * static_cast<int64_t>(radius);
    // floor(n / w) = (n * M) >> k with k = 31 + ceil(log2 w), M = ceil(2^k / w):
    // writing M w = 2^k + e (0 <= e < w), n M / 2^k = n / w + n e / (w 2^k), and
    // n e < 2^31 * 2^ceil(log2 w) = 2^k for n < 2^31, so the extra term stays
    // below 1/w and cannot carry past the next integer; n M < 2^63.
    const uint32_t win = 2u * static_cast<uint32_t>(radius) + 1u;
    int lg = 0;
    while ((1u << lg) < win) ++lg;
    const int shift = 31 + lg;
    const uint64_t magic = ((uint64_t(1) << shift) + win - 1) / win;
    const int64_t nseg = (nres + kBlSeg - 1) / kBlSeg;
    const int64_t waves = static_cast<int64_t>(ndm) * nseg;
    const dim3 grid(static_cast<unsigned>((waves + kThreads / 64 - 1) / (kThreads / 64)));
#define DD_BL(T, U)                                                                            \
    hipLaunchKernelGGL((baseline_kernel<T, U>), grid, dim3(kThreads), 0, s,                     \
                       static_cast<const T*>(in), ndm, nout, nres, radius, offset, nseg, magic, \
                       shift, static_cast<U*>(out));
    if (in_u16 && out_u16) DD_BL(uint16_t, uint16_t)
    else if (in_u16) DD_BL(uint16_t, int32_t)
    else if (out_u16) DD_BL(int32_t, uint16_t)
    else DD_BL(int32_t, int32_t)
#undef DD_BL
    return hipGetLastError();
}

template <typename T, int NW>
hipError_t launch_stats_t(const void* in, int64_t nout, const Widths& W, const PeaksLayout& lay,
                          const PeaksWs& ws, dim3 grid, size_t lds, hipStream_t s) {
    // contiguous-run window loads (uint16 only): rows of a multiple of 4
    // samples from an 8-byte aligned series, and a window that the runs cover
    const int w_max = W.w[W.n - 1];
    const int runs = std::is_same<T, uint16_t>::value && nout % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(in) % 8 == 0 && lay.L + w_max + 1 + 3 <= 4 * kThreads * kRounds;
    if (runs) lds = std::max(lds, static_cast<size_t>(kRunWords) * 4);
    auto kern = boxcar_stats_kernel<T, NW>;
    hipError_t e = set_lds_limit(reinterpret_cast<const void*>(kern), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), lds, s, static_cast<const T*>(in), nout, lay.nbx,
                       W, lay.L, lay.nseg, runs, ws);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stats_w(const void* in, int64_t nout, const Widths& W, const PeaksLayout& lay,
                          const PeaksWs& ws, dim3 grid, size_t lds, hipStream_t s) {
    // the register fast path reuses the running-sum area (L + w_max + 1 words)
    // for its reduction (3 * NW * kRedStride words)
    const int w_max = W.w[W.n - 1];
    const int nw = (lay.L == kPerThread * kThreads && W.n <= 16 &&
                    3 * W.n * kRedStride <= lay.L + w_max + 1) ? W.n : 0;
    switch (nw) {
#define DD_NW(N) case N: return launch_stats_t<T, N>(in, nout, W, lay, ws, grid, lds, s);
        DD_NW(1) DD_NW(2) DD_NW(3) DD_NW(4) DD_NW(5) DD_NW(6) DD_NW(7) DD_NW(8)
        DD_NW(9) DD_NW(10) DD_NW(11) DD_NW(12) DD_NW(13) DD_NW(14) DD_NW(15) DD_NW(16)
#undef DD_NW
        default: return launch_stats_t<T, 0>(in, nout, W, lay, ws, grid, lds, s);
    }
}

hipError_t launch_stats(const void* in, int in_u16, int64_t nout, const Widths& W,
                        const PeaksLayout& lay, const PeaksWs& ws, dim3 grid, size_t lds,
                        hipStream_t s) {
    return in_u16 ? launch_stats_w<uint16_t>(in, nout, W, lay, ws, grid, lds, s)
                  : launch_stats_w<int32_t>(in, nout, W, lay, ws, grid, lds, s);
}

PeaksLayout peaks_layout(int ndm, int64_t nout, const Widths& W) {
    PeaksLayout lay{};
    const int w_max = W.w[W.n - 1];
    lay.nbx = nout - w_max + 1;
    lay.L = segment_length(w_max);
    lay.nseg = static_cast<int>((lay.nbx + lay.L - 1) / lay.L);
    lay.nseries = static_cast<int64_t>(W.n) * ndm;
    lay.ncounts = lay.nseries * lay.nseg;
    lay.nchunks = static_cast<int>((lay.ncounts + kScanChunk - 1) / kScanChunk);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    lay.o_part_s1 = take(lay.ncounts * 8);
    lay.o_part_s2lo = take(lay.ncounts * 8);
    lay.o_part_s2hi = take(lay.ncounts * 8);
    lay.o_part_max = take(lay.ncounts * 4);
    lay.o_s1 = take(lay.nseries * 8);
    lay.o_s2lo = take(lay.nseries * 8);
    lay.o_s2hi = take(lay.nseries * 8);
    lay.o_thr = take(lay.nseries * 8);
    lay.o_thr32 = take(lay.nseries * 4);
    lay.o_sqrt_d = take(lay.nseries * 8);
    lay.o_counts = take(lay.ncounts * 4);
    lay.o_offs = take(lay.ncounts * 8);
    lay.o_chunk = take(static_cast<size_t>(lay.nchunks) * 8);
    lay.o_total = take(8);
    lay.o_list = take(static_cast<size_t>(ndm) * lay.nseg * 4);
    lay.o_list2 = take(static_cast<size_t>(ndm) * lay.nseg * 4);
    lay.o_nlist = take(8);
    lay.bytes = off;
    return lay;
}

PeaksWs peaks_ws(void* base, const PeaksLayout& lay) {
    char* b = static_cast<char*>(base);
    PeaksWs ws;
    ws.part_s1 = reinterpret_cast<uint64_t*>(b + lay.o_part_s1);
    ws.part_s2lo = reinterpret_cast<uint64_t*>(b + lay.o_part_s2lo);
    ws.part_s2hi = reinterpret_cast<uint64_t*>(b + lay.o_part_s2hi);
    ws.part_max = reinterpret_cast<uint32_t*>(b + lay.o_part_max);
    ws.s1 = reinterpret_cast<uint64_t*>(b + lay.o_s1);
    ws.s2lo = reinterpret_cast<uint64_t*>(b + lay.o_s2lo);
    ws.s2hi = reinterpret_cast<uint64_t*>(b + lay.o_s2hi);
    ws.thr = reinterpret_cast<int64_t*>(b + lay.o_thr);
    ws.thr32 = reinterpret_cast<uint32_t*>(b + lay.o_thr32);
    ws.sqrt_d = reinterpret_cast<double*>(b + lay.o_sqrt_d);
    ws.counts = reinterpret_cast<uint32_t*>(b + lay.o_counts);
    ws.offs = reinterpret_cast<int64_t*>(b + lay.o_offs);
    ws.chunk_tot = reinterpret_cast<int64_t*>(b + lay.o_chunk);
    ws.total = reinterpret_cast<int64_t*>(b + lay.o_total);
    ws.list = reinterpret_cast<uint32_t*>(b + lay.o_list);
    ws.list2 = reinterpret_cast<uint32_t*>(b + lay.o_list2);
    ws.nlist = reinterpret_cast<uint32_t*>(b + lay.o_nlist);
    return ws;
}

hipError_t launch_scan_u32(const uint32_t* counts, int64_t n, int64_t* offs, int64_t* chunk_tot,
                           int64_t* total, hipStream_t s) {
    const int nchunks = static_cast<int>((n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(nchunks), dim3(kThreads), 0, s, counts, n, offs,
                       chunk_tot);
    hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(kThreads), 0, s, chunk_tot, nchunks, total);
    hipLaunchKernelGGL(scan_add_kernel, dim3(static_cast<unsigned>((n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, offs, n, chunk_tot);
    return hipGetLastError();
}

int64_t scan_chunk_count(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

hipError_t launch_peaks_count(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                              const PeaksLayout& lay, const PeaksWs& ws, uint32_t kmant, int kexp2,
                              hipStream_t s) {
    const int w_max = W.w[W.n - 1];
    const size_t lds = peaks_lds_bytes(lay.L, w_max);
    const dim3 grid(static_cast<unsigned>(lay.nseg), static_cast<unsigned>(ndm));
    hipError_t e = launch_stats(in, in_u16, nout, W, lay, ws, grid, lds, s);
    if (e != hipSuccess) return e;
    const int nser = static_cast<int>(lay.nseries);
    hipLaunchKernelGGL(series_threshold_kernel, dim3((nser + kSerPerBlock - 1) / kSerPerBlock), dim3(kThreads),
                       0, s, nser, lay.nseg, lay.nbx, kmant, kexp2, ws);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nblk = static_cast<int64_t>(ndm) * lay.nseg;
    hipLaunchKernelGGL(mark_kernel, dim3(static_cast<unsigned>((nblk + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, ndm, lay.nseg, W.n, ws);
    const dim3 wgrid(static_cast<unsigned>(std::min<int64_t>(nblk, kListBlocks)));
    if (in_u16) {
        set_lds_limit(reinterpret_cast<const void*>(peaks_count_kernel<uint16_t>), lds);
        hipLaunchKernelGGL(peaks_count_kernel<uint16_t>, wgrid, dim3(kThreads), lds, s,
                           static_cast<const uint16_t*>(in), ndm, nout, lay.nbx, W, lay.L, lay.nseg,
                           ws);
    } else {
        set_lds_limit(reinterpret_cast<const void*>(peaks_count_kernel<int32_t>), lds);
        hipLaunchKernelGGL(peaks_count_kernel<int32_t>, wgrid, dim3(kThreads), lds, s,
                           static_cast<const int32_t*>(in), ndm, nout, lay.nbx, W, lay.L, lay.nseg,
                           ws);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(lay.nchunks), dim3(kThreads), 0, s, ws.counts,
                       lay.ncounts, ws.offs, ws.chunk_tot);
    hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(kThreads), 0, s, ws.chunk_tot, lay.nchunks, ws.total);
    hipLaunchKernelGGL(scan_add_kernel, dim3(static_cast<unsigned>((lay.ncounts + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, ws.offs, lay.ncounts, ws.chunk_tot);
    return hipGetLastError();
}

hipError_t launch_peaks_write(const void* in, int in_u16, int ndm, int64_t nout, const Widths& W,
                              const PeaksLayout& lay, const PeaksWs& ws, dedisp_event* events,
                              int64_t capacity, hipStream_t s) {
    const int w_max = W.w[W.n - 1];
    const size_t lds = peaks_lds_bytes(lay.L, w_max);
    const dim3 grid(static_cast<unsigned>(
        std::min<int64_t>(static_cast<int64_t>(ndm) * lay.nseg, kListBlocks)));
    if (in_u16) {
        set_lds_limit(reinterpret_cast<const void*>(peaks_write_kernel<uint16_t>), lds);
        hipLaunchKernelGGL(peaks_write_kernel<uint16_t>, grid, dim3(kThreads), lds, s,
                           static_cast<const uint16_t*>(in), ndm, nout, lay.nbx, W, lay.L, lay.nseg,
                           ws, events, capacity);
    } else {
        set_lds_limit(reinterpret_cast<const void*>(peaks_write_kernel<int32_t>), lds);
        hipLaunchKernelGGL(peaks_write_kernel<int32_t>, grid, dim3(kThreads), lds, s,
                           static_cast<const int32_t*>(in), ndm, nout, lay.nbx, W, lay.L, lay.nseg,
                           ws, events, capacity);
    }
    return hipGetLastError();
}

}  // namespace dd
