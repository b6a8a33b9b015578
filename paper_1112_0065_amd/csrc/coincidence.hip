// Multibeam coincidence RFI mask (paper section 2.1).
//
// Interference is not localised on the sky: the 13 beams of the multibeam
// receiver serve as reference antennas for one another.  The paper's method is
// a transform of the multibeam time series: for each sample the beams are
// tested against a signal-to-noise threshold and the sample is flagged as
// interference when enough of them exceed it (its example: 3 sigma in 4 or
// more of the 13 beams), giving a boolean mask.
//
// Readings taken here: the per-beam series is the zero-DM series z_b[t] =
// sum_c x_b[c][t] of the beam's 2-bit samples over the common sample range;
// mean and sigma are the population statistics of z_b over that range, from
// exact integer sums; exceeding k sigma means the strict S/N > k, decided exactly
// as in the sigma-cut (z >= ceil((S1 + isqrt(floor(k^2 D)) + 1) / n)).
//
// Kernels: zero-DM sums straight from the packed bytes (popcounts of the two
// bit-planes of each 32-bit word), per-block partial sums, one thread per beam
// for the exact cut level, and one thread per sample for the vote.  All of it
// is bound by the one read of the packed input.
#include <algorithm>

#include "dedisp_internal.hpp"
#include "intmath.hpp"
#include "search_internal.hpp"

namespace {

constexpr int kCThreads = 256;
constexpr int kStatBlock = 8192;   // samples per partial-sum block

// Level sum of the sixteen 2-bit fields of a word: bit 0s count once, bit 1s twice.
__device__ __forceinline__ uint32_t level_sum(uint32_t w) {
    return static_cast<uint32_t>(__builtin_popcount(w & 0x55555555u)) +
           2u * static_cast<uint32_t>(__builtin_popcount(w & 0xAAAAAAAAu));
}

// 1024 channels (256 bytes per sample): 16 lanes per sample, one 16-byte load
// each, 4 samples per wave and step; a 16-lane reduction finishes each sum.
__global__ __launch_bounds__(kCThreads) void zero_dm_256_kernel(const uint8_t* __restrict__ in,
                                                                int64_t nsamps,
                                                                int32_t* __restrict__ z) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kCThreads + threadIdx.x) >> 6;
    const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * kCThreads) >> 6;
    const int sub = lane >> 4;      // sample within the step
    const int part = lane & 15;     // 16-byte part of the sample
    for (int64_t t0 = wave * 4; t0 < nsamps; t0 += nwaves * 4) {
        const int64_t t = t0 + sub;
        uint32_t s = 0;
        if (t < nsamps) {
            const uint4 v = *reinterpret_cast<const uint4*>(in + t * 256 + part * 16);
            s = level_sum(v.x) + level_sum(v.y) + level_sum(v.z) + level_sum(v.w);
        }
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 16);
        if (part == 0 && t < nsamps) z[t] = static_cast<int32_t>(s);
    }
}

// Any nchans (multiple of 4): one thread per sample, whole words then the
// remaining bytes.
__global__ __launch_bounds__(kCThreads) void zero_dm_any_kernel(const uint8_t* __restrict__ in,
                                                                int64_t nsamps, int bps,
                                                                int32_t* __restrict__ z) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kCThreads + threadIdx.x;
    if (t >= nsamps) return;
    const uint8_t* p = in + t * bps;
    uint32_t s = 0;
    int i = 0;
    if ((reinterpret_cast<uintptr_t>(p) & 3) == 0)
        for (; i + 4 <= bps; i += 4) s += level_sum(*reinterpret_cast<const uint32_t*>(p + i));
    for (; i < bps; ++i) s += level_sum(p[i]);
    z[t] = static_cast<int32_t>(s);
}

// Partial S1 and S2 of blocks of kStatBlock samples: grid (nblocks, nbeams).
// z <= 3*nchans < 2^16, so S2 of up to 2^31 samples fits 64 bits.
__global__ __launch_bounds__(kCThreads) void zero_dm_stats_kernel(const int32_t* __restrict__ z,
                                                                  int64_t nsamps, int nblk,
                                                                  uint64_t* __restrict__ p1,
                                                                  uint64_t* __restrict__ p2) {
    __shared__ uint64_t r1[kCThreads / 64], r2[kCThreads / 64];
    const int b = blockIdx.y;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kStatBlock;
    const int32_t* zb = z + static_cast<int64_t>(b) * nsamps;
    uint64_t a1 = 0, a2 = 0;
    for (int i = threadIdx.x; i < kStatBlock; i += kCThreads) {
        const int64_t t = t0 + i;
        if (t < nsamps) {
            const uint64_t v = static_cast<uint32_t>(zb[t]);
            a1 += v;
            a2 += v * v;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        r1[threadIdx.x >> 6] = a1;
        r2[threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s1 = 0, s2 = 0;
        for (int w = 0; w < kCThreads / 64; ++w) {
            s1 += r1[w];
            s2 += r2[w];
        }
        p1[static_cast<int64_t>(b) * nblk + blockIdx.x] = s1;
        p2[static_cast<int64_t>(b) * nblk + blockIdx.x] = s2;
    }
}

// One thread per beam: exact sums and the cut level (thr[b] = -1: D == 0,
// the beam never votes).  Thread 0 also clears the masked-sample counter.
__global__ void zero_dm_threshold_kernel(int nbeams, int nblk, int64_t nsamps, uint32_t kmant,
                                         int kexp2, const uint64_t* __restrict__ p1,
                                         const uint64_t* __restrict__ p2,
                                         int64_t* __restrict__ thr,
                                         unsigned long long* __restrict__ count) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) *count = 0ull;
    if (b >= nbeams) return;
    uint64_t s1 = 0;
    u128 s2 = 0;
    for (int g = 0; g < nblk; ++g) {
        s1 += p1[static_cast<int64_t>(b) * nblk + g];
        s2 += p2[static_cast<int64_t>(b) * nblk + g];
    }
    thr[b] = cut_level(static_cast<uint64_t>(nsamps), s1, s2, kmant, kexp2, nullptr);
}

// One thread per sample: votes of the beams and the mask byte.
__global__ __launch_bounds__(kCThreads) void coincidence_vote_kernel(
    const int32_t* __restrict__ z, int64_t nsamps, int nbeams, int min_beams,
    const int64_t* __restrict__ thr, uint8_t* __restrict__ mask,
    unsigned long long* __restrict__ count) {
    __shared__ unsigned long long bc;
    if (threadIdx.x == 0) bc = 0ull;
    __syncthreads();
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kCThreads + threadIdx.x;
    if (t < nsamps) {
        int votes = 0;
        for (int b = 0; b < nbeams; ++b) {
            const int64_t th = thr[b];
            votes += (th >= 0 && static_cast<int64_t>(z[static_cast<int64_t>(b) * nsamps + t]) >= th) ? 1 : 0;
        }
        const bool m = votes >= min_beams;
        mask[t] = m ? 1 : 0;
        if (m) atomicAdd(&bc, 1ull);
    }
    __syncthreads();
    if (threadIdx.x == 0 && bc) atomicAdd(count, bc);
}

struct CoincLayout {
    size_t o_z, o_p1, o_p2, o_thr, o_count, bytes;
    int nblk;
};

CoincLayout coinc_layout(int nbeams, int64_t nsamps) {
    CoincLayout l{};
    l.nblk = static_cast<int>((nsamps + kStatBlock - 1) / kStatBlock);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    l.o_z = take(static_cast<size_t>(nbeams) * nsamps * 4);
    l.o_p1 = take(static_cast<size_t>(nbeams) * l.nblk * 8);
    l.o_p2 = take(static_cast<size_t>(nbeams) * l.nblk * 8);
    l.o_thr = take(static_cast<size_t>(nbeams) * 8);
    l.o_count = take(8);
    l.bytes = off;
    return l;
}

bool coinc_args_ok(int32_t nbeams, int32_t nchans, int64_t nsamps) {
    return nbeams >= 1 && nbeams <= 64 && nchans >= 4 && nchans % 4 == 0 && nchans <= 21844 &&
           nsamps >= 1 && nsamps < (int64_t(1) << 31);
}

}  // namespace

namespace {

// Masked samples take the mean level 1.5 in every channel: levels 1 and 2 in
// alternate channels (byte 0x99: channels 4k and 4k + 2 at level 1, 4k + 1
// and 4k + 3 at level 2).  One thread per (beam, sample); flagged samples are
// rare, so the write is a short loop over the sample's bytes.
struct BeamPtrs {
    uint8_t* p[64];
};

__global__ __launch_bounds__(kCThreads) void rfi_apply_kernel(BeamPtrs beams, int nbeams,
                                                              int64_t nsamps, int bytes_per_sample,
                                                              const uint8_t* __restrict__ mask) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kCThreads + threadIdx.x;
    if (i >= nsamps * nbeams) return;
    const int b = static_cast<int>(i / nsamps);
    const int64_t t = i - static_cast<int64_t>(b) * nsamps;
    if (!mask[t]) return;
    uint8_t* row = beams.p[b] + t * bytes_per_sample;
    if ((bytes_per_sample & 15) == 0 && (reinterpret_cast<uintptr_t>(row) & 15) == 0) {
        const uint4 v = make_uint4(0x99999999u, 0x99999999u, 0x99999999u, 0x99999999u);
        for (int k = 0; k < bytes_per_sample / 16; ++k) reinterpret_cast<uint4*>(row)[k] = v;
    } else {
        for (int k = 0; k < bytes_per_sample; ++k) row[k] = 0x99;
    }
}

}  // namespace

namespace dd {

size_t rfi_mask_ws_bytes(int nbeams, int64_t nsamps) { return coinc_layout(nbeams, nsamps).bytes; }

hipError_t launch_rfi_mask(const uint8_t* const* ins, int nbeams, int nchans, int64_t nsamps,
                           uint32_t kmant, int kexp2, int min_beams, uint8_t* mask, void* workspace,
                           hipStream_t stream) {
    const CoincLayout l = coinc_layout(nbeams, nsamps);
    char* w = static_cast<char*>(workspace);
    int32_t* z = reinterpret_cast<int32_t*>(w + l.o_z);
    uint64_t* p1 = reinterpret_cast<uint64_t*>(w + l.o_p1);
    uint64_t* p2 = reinterpret_cast<uint64_t*>(w + l.o_p2);
    int64_t* thr = reinterpret_cast<int64_t*>(w + l.o_thr);
    unsigned long long* count = reinterpret_cast<unsigned long long*>(w + l.o_count);
    const int bps = nchans / 4;
    for (int b = 0; b < nbeams; ++b) {
        int32_t* zb = z + static_cast<int64_t>(b) * nsamps;
        if (bps == 256 && (reinterpret_cast<uintptr_t>(ins[b]) & 15) == 0) {
            const int64_t waves = std::min<int64_t>((nsamps + 3) / 4, 256 * 64);
            hipLaunchKernelGGL(zero_dm_256_kernel, dim3(static_cast<unsigned>((waves + 3) / 4)),
                               dim3(kCThreads), 0, stream, ins[b], nsamps, zb);
        } else {
            hipLaunchKernelGGL(zero_dm_any_kernel,
                               dim3(static_cast<unsigned>((nsamps + kCThreads - 1) / kCThreads)),
                               dim3(kCThreads), 0, stream, ins[b], nsamps, bps, zb);
        }
    }
    hipLaunchKernelGGL(zero_dm_stats_kernel, dim3(l.nblk, nbeams), dim3(kCThreads), 0, stream, z,
                       nsamps, l.nblk, p1, p2);
    hipLaunchKernelGGL(zero_dm_threshold_kernel, dim3(1), dim3(64), 0, stream, nbeams, l.nblk,
                       nsamps, kmant, kexp2, p1, p2, thr, count);
    hipLaunchKernelGGL(coincidence_vote_kernel,
                       dim3(static_cast<unsigned>((nsamps + kCThreads - 1) / kCThreads)),
                       dim3(kCThreads), 0, stream, z, nsamps, nbeams, min_beams, thr, mask, count);
    return hipGetLastError();
}

const unsigned long long* rfi_mask_count(const void* workspace, int nbeams, int64_t nsamps) {
    return reinterpret_cast<const unsigned long long*>(static_cast<const char*>(workspace) +
                                                       coinc_layout(nbeams, nsamps).o_count);
}

hipError_t launch_rfi_apply(uint8_t* const* beams, int nbeams, int nchans, int64_t nsamps,
                            const uint8_t* mask, hipStream_t stream) {
    if (nbeams < 1 || nbeams > 64) return hipErrorInvalidValue;
    BeamPtrs ptrs{};
    for (int b = 0; b < nbeams; ++b) ptrs.p[b] = beams[b];
    const int64_t n = nsamps * nbeams;
    hipLaunchKernelGGL(rfi_apply_kernel, dim3(static_cast<unsigned>((n + kCThreads - 1) / kCThreads)),
                       dim3(kCThreads), 0, stream, ptrs, nbeams, nsamps, nchans / 4, mask);
    return hipGetLastError();
}

}  // namespace dd

extern "C" size_t dedisp_rfi_mask_workspace_bytes(int32_t nbeams, int64_t nsamps) {
    if (nbeams < 1 || nbeams > 64 || nsamps < 1 || nsamps >= (int64_t(1) << 31)) return 0;
    return coinc_layout(nbeams, nsamps).bytes;
}

extern "C" dedisp_status dedisp_rfi_mask(const uint8_t* const* in_2bit, int32_t nbeams,
                                         int32_t nchans, int64_t nsamps, float k_sigma,
                                         int32_t min_beams, uint8_t* mask, int64_t* n_masked,
                                         void* workspace, dedisp_stream stream) {
    using dd::fail;
    if (!in_2bit || !mask || !n_masked || !workspace)
        return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!coinc_args_ok(nbeams, nchans, nsamps))
        return fail(DEDISP_ERR_INVALID_ARG,
                    "need 1 <= nbeams <= 64, nchans a multiple of 4 in [4, 21844], 1 <= nsamps < 2^31");
    if (min_beams < 1) return fail(DEDISP_ERR_INVALID_ARG, "min_beams must be >= 1");
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(DEDISP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    for (int b = 0; b < nbeams; ++b)
        if (!in_2bit[b]) return fail(DEDISP_ERR_INVALID_ARG, "beam %d input is NULL", b);
    uint32_t kmant = 0;
    int kexp2 = 0;
    dedisp_status st = dd::split_threshold_public(k_sigma, &kmant, &kexp2);
    if (st != DEDISP_OK) return st;
    DD_HIP(dd::launch_rfi_mask(in_2bit, nbeams, nchans, nsamps, kmant, kexp2, min_beams, mask,
                               workspace, stream));
    unsigned long long total = 0;
    DD_HIP(hipMemcpyAsync(&total, dd::rfi_mask_count(workspace, nbeams, nsamps), sizeof total,
                          hipMemcpyDeviceToHost, stream));
    DD_HIP(hipStreamSynchronize(stream));
    *n_masked = static_cast<int64_t>(total);
    dd::clear_error();
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_rfi_mask_read_stats(const void* workspace, int32_t nbeams,
                                                    int64_t nsamps, int32_t* zero_dm,
                                                    int64_t* thr, dedisp_stream stream) {
    using dd::fail;
    if (!workspace || nbeams < 1 || nbeams > 64 || nsamps < 1 || nsamps >= (int64_t(1) << 31))
        return fail(DEDISP_ERR_INVALID_ARG, "bad arguments");
    const CoincLayout l = coinc_layout(nbeams, nsamps);
    const char* w = static_cast<const char*>(workspace);
    if (zero_dm)
        DD_HIP(hipMemcpyAsync(zero_dm, w + l.o_z, static_cast<size_t>(nbeams) * nsamps * 4,
                              hipMemcpyDeviceToHost, stream));
    if (thr)
        DD_HIP(hipMemcpyAsync(thr, w + l.o_thr, static_cast<size_t>(nbeams) * 8,
                              hipMemcpyDeviceToHost, stream));
    DD_HIP(hipStreamSynchronize(stream));
    return DEDISP_OK;
}

extern "C" dedisp_status dedisp_rfi_apply(uint8_t* const* beams_2bit, int32_t nbeams,
                                          int32_t nchans, int64_t nsamps, const uint8_t* mask,
                                          dedisp_stream stream) {
    using dd::fail;
    if (!beams_2bit || !mask) return fail(DEDISP_ERR_INVALID_ARG, "NULL argument");
    if (!coinc_args_ok(nbeams, nchans, nsamps))
        return fail(DEDISP_ERR_INVALID_ARG,
                    "need 1 <= nbeams <= 64, nchans a multiple of 4 in [4, 21844], 1 <= nsamps < 2^31");
    for (int b = 0; b < nbeams; ++b)
        if (!beams_2bit[b]) return fail(DEDISP_ERR_INVALID_ARG, "beam %d is NULL", b);
    DD_HIP(dd::launch_rfi_apply(beams_2bit, nbeams, nchans, nsamps, mask, stream));
    dd::clear_error();
    return DEDISP_OK;
}
