// Ingest of 2-bit filterbank data (paper section 1: one time series per
// channel, 2 bits per sample), turned into the channel-major bit-plane layout
// the dedispersion kernel reads.
//
// Input : time-major bytes, channel c of sample t in bits 2(c%4) of byte
//         t*nchans/4 + c/4.
// Output: words[c*nwords + j] = {lo, hi}: bit b of lo/hi is bit 0/1 of the
//         level of sample 32j+b of channel c.  Samples >= nsamps and the two
//         trailing words are zero.
//
// One block moves a tile of 64 samples x 256 channels: a coalesced load into
// LDS, then each wave turns one 4-byte column (16 channels x 64 samples) into
// bit-planes with wave ballots -- bit k of every lane's word at once.
// The kernel is HBM-bound: it reads and writes nsamps*nchans/4 bytes each.
#include "dedisp_internal.hpp"

namespace {

constexpr int kTileT = 64;      // samples per tile (one wave64 ballot)
constexpr int kTileC = 256;     // channels per tile = 64 bytes per row

__global__ __launch_bounds__(256) void repack_2bit_kernel(const uint8_t* __restrict__ in,
                                                          int64_t nsamps, int nchans,
                                                          uint2* __restrict__ words,
                                                          int64_t nwords, int vec16) {
    __shared__ uint32_t tile[kTileT][kTileC / 16 + 1];  // padded row: no bank conflicts
    const int tid = threadIdx.x;
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kTileT;
    const int c0 = blockIdx.y * kTileC;
    const int row_bytes = nchans >> 2;

    {   // load 64 rows x 64 bytes: thread -> (row, 16-byte chunk)
        const int row = tid >> 2;
        const int q = tid & 3;
        const int64_t t = t0 + row;
        const int byte0 = (c0 >> 2) + q * 16;
        uint32_t v[4] = {0u, 0u, 0u, 0u};
        if (t < nsamps && byte0 < row_bytes) {
            const uint8_t* src = in + t * row_bytes + byte0;
            const int nb = min(16, row_bytes - byte0);
            if (vec16 && nb == 16) {
                const uint4 x = *reinterpret_cast<const uint4*>(src);
                v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
            } else {
                for (int i = 0; i < nb; ++i) v[i >> 2] |= static_cast<uint32_t>(src[i]) << (8 * (i & 3));
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) tile[row][q * 4 + i] = v[i];
    }
    __syncthreads();

    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t j = t0 >> 5;  // first of the two 32-sample words this tile fills
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        const int col = wave * 4 + k;
        const int cbase = c0 + col * 16;
        if (cbase >= nchans) break;
        const uint32_t x = tile[lane][col];
        uint64_t mylo = 0, myhi = 0;
#pragma unroll
        for (int ch = 0; ch < 16; ++ch) {
            const uint64_t lo = __ballot((x >> (2 * ch)) & 1u);
            const uint64_t hi = __ballot((x >> (2 * ch + 1)) & 1u);
            if (lane == ch) { mylo = lo; myhi = hi; }
        }
        const int c = cbase + lane;
        if (lane < 16 && c < nchans) {
            uint2* dst = words + static_cast<int64_t>(c) * nwords + j;
            dst[0] = make_uint2(static_cast<uint32_t>(mylo), static_cast<uint32_t>(myhi));
            dst[1] = make_uint2(static_cast<uint32_t>(mylo >> 32), static_cast<uint32_t>(myhi >> 32));
            if (j + 2 == nwords - 2) {   // last tile: clear the two trailing words
                dst[2] = make_uint2(0u, 0u);
                dst[3] = make_uint2(0u, 0u);
            }
        }
    }
}

}  // namespace

namespace dd {

hipError_t launch_repack(const uint8_t* in, int64_t nsamps, int nchans, uint2* words,
                         int64_t nwords, hipStream_t s) {
    const int64_t tiles_t = (nsamps + kTileT - 1) / kTileT;
    if (nwords != 2 * tiles_t + 2) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(tiles_t), static_cast<unsigned>((nchans + kTileC - 1) / kTileC));
    const int vec16 = ((nchans >> 2) % 16 == 0) && (reinterpret_cast<uintptr_t>(in) % 16 == 0);
    hipLaunchKernelGGL(repack_2bit_kernel, grid, dim3(256), 0, s, in, nsamps, nchans, words,
                       nwords, vec16);
    return hipGetLastError();
}

}  // namespace dd
