// Ingest of 2-bit filterbank data (paper section 1: one time series per
// channel, 2 bits per sample), turned into the channel-major bit-plane layout
// the dedispersion kernel reads.
//
// Input : time-major bytes, channel c of sample t in bits 2(c%4) of byte
//         t*nchans/4 + c/4.
// Output: words[c*nwords + j] = {lo, hi}: bit b of lo/hi is bit 0/1 of the
//         level of sample 32j+b of channel c.  Samples >= nsamps and the two
//         trailing words are zero.  With a coincidence mask, samples t < mask_n
//         with mask[t] != 0 are read as the mean level of every channel.
//
// One block covers a tile of 512 samples x 256 channels (64 bytes per input
// row, 16 output words per channel).  The input rows are staged in LDS with
// 16-byte loads.  Each wave then takes 16-channel columns of 64-sample
// sub-tiles: lane b holds the 32-bit word of sample b (16 channels x 2 bits),
// and a 32 x 32 bit transpose within each half-wave (five swizzle-and-mask
// stages) leaves in lane k the plane (k & 1) of channel k >> 1 for the half's
// 32 samples -- one output word.  The words go to an LDS output tile, from
// which every channel row is written as 128 contiguous bytes.  The kernel is
// bound by HBM: it reads and writes nsamps*nchans/4 bytes each.
#include <algorithm>

#include "dedisp_internal.hpp"

namespace {

constexpr int kTileT = 512;               // samples per tile
constexpr int kTileC = 256;               // channels per tile = 64 bytes per row
constexpr int kTileW = kTileT / 32;       // output words per channel per tile
constexpr int kOutStride = 2 * kTileW + 2;  // uint32 per channel in the output tile

// One stage of the 32 x 32 bit transpose across the lanes of a half-wave:
// lanes l and l ^ J exchange the J-bit blocks that the mask M selects.
template <int J, uint32_t M>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, int lane) {
    const uint32_t y = static_cast<uint32_t>(
        __builtin_amdgcn_ds_swizzle(static_cast<int>(x), 0x1F | (J << 10)));
    if (lane & J) return x ^ (((y >> J) ^ x) & M);
    return x ^ ((((x >> J) ^ y) & M) << J);
}

constexpr int kInStride = kTileC / 16 + 1;               // uint32 per staged input row
constexpr int kBufWords = kTileT * kInStride;              // = kTileC * kOutStride
static_assert(kBufWords == kTileC * kOutStride, "input and output tiles share one buffer");
constexpr int kPerWave = (kTileT / 64) * (kTileC / 16) / 4;   // (sub-tile, column) pairs per wave

__global__ __launch_bounds__(256) void repack_2bit_kernel(const uint8_t* __restrict__ in,
                                                          int64_t nsamps, int nchans,
                                                          uint2* __restrict__ words,
                                                          int64_t nwords, int64_t ntiles, int vec16,
                                                          int st16, const uint8_t* __restrict__ mask,
                                                          int64_t mask_n, int ncx) {
    // the input tile, then (after every wave holds its words) the output tile
    __shared__ uint32_t buf[kBufWords];
    const int tid = threadIdx.x;
    // Blocks are dealt to the 8 XCDs in turn (block b to XCD b % 8).  Renumber
    // them so that each XCD takes one contiguous run of (tile, channel tile)
    // items: the channel tiles of a sample range, which share the 128-byte
    // lines of the input rows, then read them through one L2.
    const int nb = static_cast<int>(gridDim.x);
    const int b = static_cast<int>(blockIdx.x);
    const int per = nb >> 3;
    const int rem = nb & 7;
    const int xcd = b & 7;
    const int item = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + (b >> 3);
    const int c0 = (item % ncx) * kTileC;
    const int64_t tile = item / ncx;
    const int row_bytes = nchans >> 2;
    if (tile >= ntiles) return;
    const int64_t t0 = tile * kTileT;

    // 1. 512 rows x 64 bytes: thread -> (row, 16-byte chunk), 8 chunks each
    for (int r = tid; r < kTileT * 4; r += 256) {
        const int row = r >> 2;
        const int q = r & 3;
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
            // a flagged sample reads as the mean level in every channel
            // (byte 0x99: levels 1, 2, 1, 2), as the coincidence mask's
            // application writes it
            if (mask && t < mask_n && mask[t]) {
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = 0u;
                for (int i = 0; i < nb; ++i) v[i >> 2] |= 0x99u << (8 * (i & 3));
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[row * kInStride + q * 4 + i] = v[i];
    }
    __syncthreads();

    // 2. each wave takes the (sub-tile, column) pairs g = wave + 4n; lane b
    //    holds sample b of the sub-tile
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;      // half-wave: samples 0-31 or 32-63 of the sub-tile
    const int k = lane & 31;
    uint32_t xs[kPerWave];
#pragma unroll
    for (int n = 0; n < kPerWave; ++n) {
        const int g = wave + 4 * n;
        xs[n] = buf[(64 * (g / (kTileC / 16)) + lane) * kInStride + g % (kTileC / 16)];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < kPerWave; ++n) {
        const int g = wave + 4 * n;
        const int sub = g / (kTileC / 16);
        const int col = g % (kTileC / 16);
        if (c0 + col * 16 >= nchans) continue;
        uint32_t x = xs[n];
        x = transpose_stage<16, 0x0000FFFFu>(x, lane);
        x = transpose_stage<8, 0x00FF00FFu>(x, lane);
        x = transpose_stage<4, 0x0F0F0F0Fu>(x, lane);
        x = transpose_stage<2, 0x33333333u>(x, lane);
        x = transpose_stage<1, 0x55555555u>(x, lane);
        // lane k: plane k & 1 of channel col*16 + (k >> 1), word 2*sub + h
        buf[(col * 16 + (k >> 1)) * kOutStride + 2 * (2 * sub + h) + (k & 1)] = x;
    }
    __syncthreads();

    // 3. every channel row: 16 words = 128 contiguous bytes, two words per store
    const int64_t j0 = t0 >> 5;
    for (int r = tid; r < kTileC * (kTileW / 2); r += 256) {
        const int cl = r / (kTileW / 2);
        const int m = r % (kTileW / 2);
        const int c = c0 + cl;
        const int64_t j = j0 + 2 * m;
        if (c >= nchans || j >= nwords) continue;
        const uint32_t* src = buf + cl * kOutStride + 4 * m;
        uint2* dst = words + static_cast<int64_t>(c) * nwords + j;
        if (st16) {
            *reinterpret_cast<uint4*>(dst) = make_uint4(src[0], src[1], src[2], src[3]);
        } else {
            dst[0] = make_uint2(src[0], src[1]);
            dst[1] = make_uint2(src[2], src[3]);
        }
    }
    // The tiles cover the data words (nwords - 2 of them, an even number);
    // when the last tile ends there, it also writes the two trailing zero
    // words of its rows (no tile of its own for them).
    const int64_t jz = (tile + 1) * kTileW;
    if (tile == ntiles - 1 && jz < nwords) {   // then jz + 2 == nwords
        for (int cl = tid; cl < kTileC; cl += 256) {
            const int c = c0 + cl;
            if (c >= nchans) continue;
            uint2* dst = words + static_cast<int64_t>(c) * nwords + jz;
            dst[0] = make_uint2(0u, 0u);
            dst[1] = make_uint2(0u, 0u);
        }
    }
}

}  // namespace

namespace dd {

// Tiles cover the data words; the last one also writes the two trailing
// words: every word of every channel row is written once (zeros past the
// last sample).
hipError_t launch_repack(const uint8_t* in, int64_t nsamps, int nchans, uint2* words,
                         int64_t nwords, hipStream_t s, const uint8_t* mask, int64_t mask_n) {
    if (nwords != repack_words(nsamps) || nwords % 2) return hipErrorInvalidValue;
    const int64_t tiles_t = (nwords - 2 + kTileW - 1) / kTileW;   // nwords - 2 >= 2 data words
    const int ncx = (nchans + kTileC - 1) / kTileC;
    const int64_t nblocks = tiles_t * ncx;    // one block per (tile, channel tile)
    if (nblocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(nblocks));
    const int vec16 = ((nchans >> 2) % 16 == 0) && (reinterpret_cast<uintptr_t>(in) % 16 == 0);
    const int st16 = reinterpret_cast<uintptr_t>(words) % 16 == 0;
    hipLaunchKernelGGL(repack_2bit_kernel, grid, dim3(256), 0, s, in, nsamps, nchans, words,
                       nwords, tiles_t, vec16, st16, mask, mask ? mask_n : 0, ncx);
    return hipGetLastError();
}

}  // namespace dd
