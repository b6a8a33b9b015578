// Triage network kernels: candidate tiles, a 4-layer bfloat16 CNN forward and
// backward pass, and Adam.
//
// The paper's section 2.1 names radio-frequency interference as the main
// source of false events.  This network scores (DM, time) candidate tiles so
// that interference can be rejected; the plain S/N detector remains the
// fallback.  Layout: activations NHWC bfloat16 (channels innermost, 64 bytes
// per pixel), float32 accumulation.  The 32->32 convolutions (forward and
// input gradient) are implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, gfx950's double-K form: M = pixels, N = 32
// output channels, K = 9 taps x 32 input channels = 288, one tap per step);
// the weight gradient is a GEMM over pixels (M = 32, N = 32 per tap,
// K = pixels, 32 per step) on the same instruction,
// reduced across blocks in a fixed order (no float atomics: training is
// reproducible bit for bit).  The 1->32 first layer (K = 9) runs on VALU.
#include <cstdint>

#include "triage_kernels.hpp"

namespace tk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

// Eight consecutive bf16 values (16 bytes, 16-byte aligned).
__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ bf16x8 pack8(const uint16_t (&v)[8]) {
    const uint4 u = make_uint4(v[0] | (static_cast<uint32_t>(v[1]) << 16),
                               v[2] | (static_cast<uint32_t>(v[3]) << 16),
                               v[4] | (static_cast<uint32_t>(v[5]) << 16),
                               v[6] | (static_cast<uint32_t>(v[7]) << 16));
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x4 load4(const uint16_t* p) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    bf16x4 r;
    r[0] = static_cast<short>(v.x & 0xFFFF);
    r[1] = static_cast<short>(v.x >> 16);
    r[2] = static_cast<short>(v.y & 0xFFFF);
    r[3] = static_cast<short>(v.y >> 16);
    return r;
}

// ---------------------------------------------------------------------------
// Candidate tiles: one block of 256 threads (one per column) per (event, row).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void tiles_kernel(const uint16_t* __restrict__ series, int ndm,
                                                    int64_t nout, int64_t nbx, TileWidths W,
                                                    const dedisp_event* __restrict__ events,
                                                    const uint64_t* __restrict__ s1,
                                                    const double* __restrict__ sqrt_d,
                                                    uint16_t* __restrict__ tiles) {
    const int e = blockIdx.x;
    const int r = blockIdx.y;
    const int j = threadIdx.x;
    const dedisp_event ev = events[e];
    const int w = W.w[ev.width_idx];
    int d0 = ev.dm_idx - 32;
    d0 = min(max(d0, 0), max(ndm - 64, 0));
    int64_t t0 = ev.t_peak - 128 * static_cast<int64_t>(w);
    t0 = min(max(t0, int64_t(0)), max(nbx - 255 * static_cast<int64_t>(w) - 1, int64_t(0)));
    const int d = d0 + r;
    float v = 0.0f;
    const int64_t t = t0 + static_cast<int64_t>(j) * w;
    if (d < ndm && t < nbx) {
        const int sidx = ev.width_idx * ndm + d;
        const double sq = sqrt_d[sidx];
        if (sq > 0.0) {
            const uint16_t* row = series + static_cast<int64_t>(d) * nout + t;
            uint32_t b = 0;
            for (int k = 0; k < w; ++k) b += row[k];
            const int64_t lval = nbx * static_cast<int64_t>(b) - static_cast<int64_t>(s1[sidx]);
            v = static_cast<float>(static_cast<double>(lval) / sq);
        }
    }
    tiles[(static_cast<int64_t>(e) * 64 + r) * 256 + j] = f2bf(v);
}

// ---------------------------------------------------------------------------
// Layer 1: 1 -> 32 channels, 3x3, pad 1, + bias, ReLU; VALU.
// ---------------------------------------------------------------------------
// The weights and biases are read through the constant address space, so
// they load into scalar registers (uniform over the block) and every
// multiply-add takes its weight as a scalar operand.
__global__ __launch_bounds__(256) void conv1_fwd_kernel(const uint16_t* __restrict__ x, int N,
                                                        const uint16_t* __restrict__ w1b,
                                                        const float* __restrict__ b1,
                                                        uint16_t* __restrict__ a) {
    typedef const __attribute__((address_space(4))) uint16_t* cw_t;
    typedef const __attribute__((address_space(4))) float* cb_t;
    const cw_t wc = (cw_t)w1b;
    const cb_t bc = (cb_t)b1;
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t npix = static_cast<int64_t>(N) * 64 * 256;
    if (p >= npix) return;
    const int xx = static_cast<int>(p & 255);
    const int yy = static_cast<int>((p >> 8) & 63);
    const int64_t n = p >> 14;
    float in[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int y2 = yy + t / 3 - 1, x2 = xx + t % 3 - 1;
        in[t] = (y2 >= 0 && y2 < 64 && x2 >= 0 && x2 < 256) ? bf2f(x[(n * 64 + y2) * 256 + x2]) : 0.0f;
    }
    uint32_t packed[kCH / 2];
#pragma unroll
    for (int c = 0; c < kCH; c += 2) {
        float z0 = bc[c], z1 = bc[c + 1];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            z0 += bf2f(wc[c * 9 + t]) * in[t];
            z1 += bf2f(wc[(c + 1) * 9 + t]) * in[t];
        }
        packed[c / 2] = static_cast<uint32_t>(f2bf(fmaxf(z0, 0.0f))) |
                        (static_cast<uint32_t>(f2bf(fmaxf(z1, 0.0f))) << 16);
    }
    uint4* dst = reinterpret_cast<uint4*>(a + p * kCH);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        dst[q] = make_uint4(packed[4 * q], packed[4 * q + 1], packed[4 * q + 2], packed[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// 32 -> 32 convolution as an implicit GEMM on MFMA.  One wave = 32 pixels of
// one image row x 32 output channels (2 x 2 tiles of 16 x 16), K = 288 in 9
// steps of 32 (one tap, all 32 input channels, per step).
// MODE 0: out = bf16(ReLU(acc + bias)); MODE 1: out = acc (float32).
// wt: [co][tap][ci] bf16 (forward) or the flipped, transposed kernel for the
// input gradient.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(64) void conv32_mfma_kernel(const uint16_t* __restrict__ x, int N, int H,
                                                         int W, const uint16_t* __restrict__ wt,
                                                         const float* __restrict__ bias,
                                                         void* __restrict__ out) {
    const int lane = threadIdx.x;
    const int segs = W / 32;
    const int64_t blk = blockIdx.x;
    const int xs = static_cast<int>(blk % segs) * 32;
    const int y = static_cast<int>((blk / segs) % H);
    const int64_t n = blk / (static_cast<int64_t>(segs) * H);
    const int row = lane & 15;       // A row (pixel) / B column (channel) within a tile
    const int kq = lane >> 4;        // which 4-element K slice
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, make_uint4(0u, 0u, 0u, 0u));
    // one tap (all 32 input channels) per step: lane slice kq holds channels
    // 8 kq .. 8 kq + 7 of its pixel (A) and of its output channel's tap (B),
    // one 16-byte load each
    const int ci0 = 8 * kq;
#pragma unroll 3
    for (int tap = 0; tap < 9; ++tap) {
        const int y2 = y + tap / 3 - 1;
        bf16x8 afr[2], bfr[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int x2 = xs + 16 * rt + row + tap % 3 - 1;
            const bool ok = y2 >= 0 && y2 < H && x2 >= 0 && x2 < W;
            afr[rt] = ok ? load8(x + ((n * H + y2) * W + x2) * kCH + ci0) : zero8;
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) bfr[ct] = load8(wt + ((16 * ct + row) * 9 + tap) * kCH + ci0);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[rt], bfr[ct], acc[rt][ct], 0, 0, 0);
    }
    // D[i][c]: lane holds rows 4*kq + j (pixels), column row (channel)
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xo = xs + 16 * rt + 4 * kq + j;
                const int co = 16 * ct + row;
                const int64_t o = ((n * H + y) * W + xo) * kCH + co;
                if (MODE == 0)
                    static_cast<uint16_t*>(out)[o] = f2bf(fmaxf(acc[rt][ct][j] + bias[co], 0.0f));
                else
                    static_cast<float*>(out)[o] = acc[rt][ct][j];
            }
}

// ---------------------------------------------------------------------------
// 2x2 max-pool (first maximum in raster order) with the winner's index.
// ---------------------------------------------------------------------------
// One thread per (pooled pixel, group of 8 channels): four 16-byte loads of
// the window, one 16-byte store of the maxima and one 8-byte store of the
// winners (the first of equal maxima); the block's pooled row from its index.
__global__ __launch_bounds__(256) void maxpool_fwd_kernel(const uint16_t* __restrict__ a, int N, int H,
                                                          int W, uint16_t* __restrict__ p,
                                                          uint8_t* __restrict__ idx) {
    const int H2 = H / 2, W2 = W / 2;
    const int bpr = (4 * W2 + 255) / 256;   // blocks per pooled row
    const int64_t row = blockIdx.x / bpr;   // n * H2 + y2
    if (row >= static_cast<int64_t>(N) * H2) return;
    const int j = static_cast<int>(blockIdx.x % bpr) * 256 + static_cast<int>(threadIdx.x);
    if (j >= 4 * W2) return;
    const int x2 = j >> 2, c0 = 8 * (j & 3);
    const int y2 = static_cast<int>(row % H2);
    const int64_t n = row / H2;
    uint4 win[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int y = 2 * y2 + (k >> 1), x = 2 * x2 + (k & 1);
        win[k] = *reinterpret_cast<const uint4*>(a + ((n * H + y) * W + x) * kCH + c0);
    }
    uint32_t ow[4];
    uint32_t iw[2] = {0u, 0u};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t w = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 2 * q + h;
            float best = -1.0f;
            uint32_t bi = 0, bv = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t word = q == 0 ? win[k].x : q == 1 ? win[k].y : q == 2 ? win[k].z : win[k].w;
                const uint32_t v = (word >> (16 * h)) & 0xFFFFu;
                const float f = bf2f(static_cast<uint16_t>(v));
                if (k == 0 || f > best) {
                    best = f;
                    bi = static_cast<uint32_t>(k);
                    bv = v;
                }
            }
            w |= bv << (16 * h);
            iw[c >> 2] |= bi << (8 * (c & 3));
        }
        ow[q] = w;
    }
    const int64_t o = (row * W2 + x2) * kCH + c0;
    *reinterpret_cast<uint4*>(p + o) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
    *reinterpret_cast<uint2*>(idx + o) = make_uint2(iw[0], iw[1]);
}

// Global average over the 4x16 map, then the 32 -> 1 linear layer: one block
// of 64 threads per tile, thread (half, channel) summing 32 of the 64
// positions (consecutive channels: coalesced), then the halves and the
// channels' products in a fixed order.
__global__ __launch_bounds__(64) void gap_fc_fwd_kernel(const uint16_t* __restrict__ p4, int N,
                                                        const float* __restrict__ wf,
                                                        const float* __restrict__ bf, float* __restrict__ g,
                                                        float* __restrict__ logits) {
    __shared__ float hs[2][kCH];
    __shared__ float prod[kCH];
    const int n = blockIdx.x;
    if (n >= N) return;
    const int c = threadIdx.x & (kCH - 1), h = threadIdx.x >> 5;
    float s = 0.0f;
    for (int q = 32 * h; q < 32 * h + 32; ++q) s += bf2f(p4[(static_cast<int64_t>(n) * 64 + q) * kCH + c]);
    hs[h][c] = s;
    __syncthreads();
    if (threadIdx.x < kCH) {
        const float gc = (hs[0][c] + hs[1][c]) * (1.0f / 64.0f);
        g[n * kCH + c] = gc;
        prod[c] = gc * wf[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float lg = bf[0];
        for (int k = 0; k < kCH; ++k) lg += prod[k];
        logits[n] = lg;
    }
}

// Loss (mean binary cross-entropy with logits) and d loss / d logit; one block.
__global__ __launch_bounds__(256) void bce_kernel(const float* __restrict__ logits,
                                                  const float* __restrict__ labels, int N,
                                                  float* __restrict__ dlogit, float* __restrict__ loss) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int n = threadIdx.x; n < N; n += 256) {
        const float z = logits[n], y = labels[n];
        s += fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
        dlogit[n] = (1.0f / (1.0f + expf(-z)) - y) / static_cast<float>(N);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (static_cast<int>(threadIdx.x) < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / static_cast<float>(N);
}

// Linear + average backward: gradients of wf, bf.  One block: thread
// (slice, channel) sums the tiles of its slice (every 8th), the 33rd column
// being the bias, then the 8 slices in order.
__global__ __launch_bounds__(512) void fc_bwd_kernel(const float* __restrict__ dlogit,
                                                     const float* __restrict__ g, int N,
                                                     const float* __restrict__ wf, float* __restrict__ gwf,
                                                     float* __restrict__ gbf) {
    __shared__ float sl[8][kCH + 1];
    const int c = threadIdx.x % 64, q = threadIdx.x / 64;   // c < 33 used
    if (c <= kCH) {
        float s = 0.0f;
        for (int n = q; n < N; n += 8) s += dlogit[n] * (c < kCH ? g[n * kCH + c] : 1.0f);
        sl[q][c] = s;
    }
    __syncthreads();
    if (threadIdx.x <= kCH) {
        float s = 0.0f;
        for (int k = 0; k < 8; ++k) s += sl[k][threadIdx.x];
        if (threadIdx.x < kCH)
            gwf[threadIdx.x] = s;
        else
            gbf[0] = s;
    }
}

__global__ void gap_bwd_kernel(const float* __restrict__ dlogit, const float* __restrict__ wf, int N,
                               float* __restrict__ dp4) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(N) * 64 * kCH) return;
    const int c = static_cast<int>(i % kCH);
    const int64_t n = i / (64 * kCH);
    dp4[i] = dlogit[n] * wf[c] * (1.0f / 64.0f);
}

// Max-pool backward + ReLU mask, rounded to bf16: dz = bf16(dA * (a > 0)).
// One thread per (pixel, group of 8 channels): 16-byte loads and stores of
// the activations and gradients, the block's image row from its index (the
// divisions are per block, in scalar registers).
__global__ __launch_bounds__(256) void pool_relu_bwd_kernel(const float* __restrict__ dp,
                                                            const uint8_t* __restrict__ idx,
                                                            const uint16_t* __restrict__ a, int N,
                                                            int H, int W, uint16_t* __restrict__ dz) {
    const int bpr = (4 * W + 255) / 256;   // blocks per image row
    const int64_t row = blockIdx.x / bpr;  // n * H + y
    if (row >= static_cast<int64_t>(N) * H) return;
    const int j = static_cast<int>(blockIdx.x % bpr) * 256 + static_cast<int>(threadIdx.x);
    if (j >= 4 * W) return;
    const int x = j >> 2, c0 = 8 * (j & 3);
    const int y = static_cast<int>(row % H);
    const int64_t n = row / H;
    const int64_t i = (row * W + x) * kCH + c0;
    const int64_t pi = ((n * (H / 2) + y / 2) * (W / 2) + x / 2) * kCH + c0;
    const uint8_t k = static_cast<uint8_t>(((y & 1) << 1) | (x & 1));
    const uint2 iw = *reinterpret_cast<const uint2*>(idx + pi);
    const float4 d0 = *reinterpret_cast<const float4*>(dp + pi);
    const float4 d1 = *reinterpret_cast<const float4*>(dp + pi + 4);
    const uint4 av = *reinterpret_cast<const uint4*>(a + i);
    const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
    uint32_t ow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t w = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = 2 * q + h;
            const uint8_t win = static_cast<uint8_t>(((c < 4 ? iw.x : iw.y) >> (8 * (c & 3))) & 0xFFu);
            float v = win == k ? dv[c] : 0.0f;
            if (!(bf2f(static_cast<uint16_t>(aw[q] >> (16 * h))) > 0.0f)) v = 0.0f;
            w |= static_cast<uint32_t>(f2bf(v)) << (16 * h);
        }
        ow[q] = w;
    }
    *reinterpret_cast<uint4*>(dz + i) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
}

// Weight gradient of a 32 -> 32 layer for one tap, over `rows` consecutive
// image rows per block: dW_tap[co][ci] = sum_pixels dz[p][co] x[p + tap][ci].
// MFMA with M = co, N = ci, K = pixels (32 per step).  Writes one partial per
// block: part[blk][tap][co][ci].
__global__ __launch_bounds__(64) void wgrad32_mfma_kernel(const uint16_t* __restrict__ x,
                                                          const uint16_t* __restrict__ dz, int N,
                                                          int H, int W, int rows,
                                                          float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int tap = blockIdx.y;
    const int ky = tap / 3 - 1, kx = tap % 3 - 1;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows;
    const int64_t nrows = static_cast<int64_t>(N) * H;
    const int idx16 = lane & 15;
    const int kq = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t rr = r0; rr < min(r0 + rows, nrows); ++rr) {
        const int y = static_cast<int>(rr % H);
        const int64_t n = rr / H;
        const int y2 = y + ky;
        const bool yok = y2 >= 0 && y2 < H;
        for (int x0 = 0; x0 < W; x0 += 32) {
            bf16x8 afr[2], bfr[2];
            // A[co][k = pixel]: 8 consecutive pixels of one output channel
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int co = 16 * rt + idx16;
                uint16_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = dz[((n * H + y) * W + x0 + 8 * kq + j) * kCH + co];
                afr[rt] = pack8(v);
            }
            // B[k = pixel][ci]: shifted input
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int ci = 16 * ct + idx16;
                uint16_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int x2 = x0 + 8 * kq + j + kx;
                    const bool ok = yok && x2 >= 0 && x2 < W;
                    v[j] = ok ? x[((n * H + y2) * W + x2) * kCH + ci] : uint16_t(0);
                }
                bfr[ct] = pack8(v);
            }
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[rt], bfr[ct], acc[rt][ct], 0, 0, 0);
        }
    }
    float* dst = part + (static_cast<int64_t>(blockIdx.x) * 9 + tap) * kCH * kCH;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                dst[(16 * rt + 4 * kq + j) * kCH + 16 * ct + idx16] = acc[rt][ct][j];
}

// Layer-1 (Cin = 1) weight and bias gradient partials on MFMA over `rows`
// image rows per block: M = co, N = the 9 taps and a column of ones (the bias;
// columns 10-15 are zero), K = pixels (32 per step).  Writes part[blk][co * 9 +
// tap] (288 values) and part[blk][288 + co].
__global__ __launch_bounds__(64) void wgrad1_mfma_kernel(const uint16_t* __restrict__ x,
                                                         const uint16_t* __restrict__ dz, int N,
                                                         int H, int W, int rows,
                                                         float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int idx16 = lane & 15;
    const int kq = lane >> 4;
    const int col = idx16;   // B column: tap (< 9), bias (9), zero (> 9)
    const int ky = col / 3 - 1, kx = col % 3 - 1;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows;
    const int64_t nrows = static_cast<int64_t>(N) * H;
    constexpr uint16_t kOne = 0x3F80;   // bf16 1.0
    f32x4 acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t rr = r0; rr < min(r0 + rows, nrows); ++rr) {
        const int y = static_cast<int>(rr % H);
        const int64_t n = rr / H;
        const int y2 = y + ky;
        const bool yok = col < 9 && y2 >= 0 && y2 < H;
        for (int x0 = 0; x0 < W; x0 += 32) {
            bf16x8 afr[2];
            // A[co][k = pixel]: 8 consecutive pixels of one output channel
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int co = 16 * rt + idx16;
                uint16_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = dz[((n * H + y) * W + x0 + 8 * kq + j) * kCH + co];
                afr[rt] = pack8(v);
            }
            // B[k = pixel][col]: the input shifted by the tap, or ones
            uint16_t v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x2 = x0 + 8 * kq + j + kx;
                const bool ok = yok && x2 >= 0 && x2 < W;
                v[j] = ok ? x[(n * H + y2) * W + x2] : (col == 9 ? kOne : uint16_t(0));
            }
            const bf16x8 bfr = pack8(v);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[rt], bfr, acc[rt], 0, 0, 0);
        }
    }
    // D[co][col]: lane holds co = 16 rt + 4 kq + j, column idx16
    float* dst = part + static_cast<int64_t>(blockIdx.x) * 320;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 16 * rt + 4 * kq + j;
            if (col < 9)
                dst[co * 9 + col] = acc[rt][j];
            else if (col == 9)
                dst[288 + co] = acc[rt][j];
        }
}

// Bias gradient partials of a 32-channel layer over `rows` image rows per
// block: part[blk][co] = sum of dz[p][co] over the block's pixels, in 8 slices
// of pixels (32 consecutive channels per slice and pixel: coalesced), then the
// slices in order.
__global__ __launch_bounds__(256) void bias_parts_kernel(const uint16_t* __restrict__ dz, int N, int H,
                                                         int W, int rows, float* __restrict__ part) {
    __shared__ float sl[8][kCH];
    const int co = threadIdx.x & (kCH - 1), q = threadIdx.x >> 5;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows;
    const int64_t nrows = static_cast<int64_t>(N) * H;
    const int64_t p0 = r0 * W, p1 = min(r0 + rows, nrows) * W;
    float acc = 0.0f;
    for (int64_t p = p0 + q; p < p1; p += 8) acc += bf2f(dz[p * kCH + co]);
    sl[q][co] = acc;
    __syncthreads();
    if (threadIdx.x < kCH) {
        float t = 0.0f;
        for (int k = 0; k < 8; ++k) t += sl[k][threadIdx.x];
        part[static_cast<int64_t>(blockIdx.x) * kCH + threadIdx.x] = t;
    }
}

// out[i] = sum over the parts b of part[b * stride + i], i < n, in a fixed
// order: slice s of kRedSlices adds its contiguous range of parts in order
// (first kernel, one thread per (i, s)), then the slices are added in order.
__global__ void reduce_slices_kernel(const float* __restrict__ part, int nparts, int stride, int n,
                                     float* __restrict__ red) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    if (i >= n) return;
    const int b0 = static_cast<int>(static_cast<int64_t>(nparts) * sl / kRedSlices);
    const int b1 = static_cast<int>(static_cast<int64_t>(nparts) * (sl + 1) / kRedSlices);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[static_cast<int64_t>(b) * stride + i];
    red[static_cast<int64_t>(sl) * n + i] = s;
}

__global__ void reduce_final_kernel(const float* __restrict__ red, int n, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int k = 0; k < kRedSlices; ++k) s += red[static_cast<int64_t>(k) * n + i];
    out[i] = s;
}

// dW (layout [tap][co][ci]) -> the master layout [co][ci][ky][kx].
__global__ void wgrad_to_master_kernel(const float* __restrict__ d_tap, float* __restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kCH * kCH * 9) return;
    const int tap = i % 9, ci = (i / 9) % kCH, co = i / (9 * kCH);
    g[i] = d_tap[(tap * kCH + co) * kCH + ci];
}

// Adam on float32 master weights.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies of the convolution weights in the kernels' layouts.
__global__ void derive_weights_kernel(const float* __restrict__ master, Offsets off,
                                      uint16_t* __restrict__ w1b, uint16_t* __restrict__ wfwd,
                                      uint16_t* __restrict__ wdg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kCH * 9) w1b[i] = f2bf(master[off.w[0] + i]);   // [co][tap]
    const int per = kCH * 9 * kCH;
    if (i >= 3 * per) return;
    const int l = i / per;          // layers 2..4 -> 0..2
    const int r = i % per;          // master index within [co][ci][ky][kx]
    const int tap = r % 9, ci = (r / 9) % kCH, co = r / (9 * kCH);
    const uint16_t b = f2bf(master[off.w[l + 1] + r]);
    wfwd[l * per + (co * 9 + tap) * kCH + ci] = b;            // [co][tap][ci]
    wdg[l * per + (ci * 9 + (8 - tap)) * kCH + co] = b;       // [ci][flipped tap][co]
}

__global__ void sigmoid_kernel(const float* __restrict__ z, int n, float* __restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = 1.0f / (1.0f + expf(-z[i]));
}

__global__ void finite_check_kernel(const float* __restrict__ a, int n, int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(a[i])) atomicAdd(bad, 1);
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

static inline unsigned blocks(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

hipError_t launch_tiles(const uint16_t* series, int ndm, int64_t nout, int64_t nbx, const TileWidths& W,
                        const dedisp_event* events, int nev, const uint64_t* s1, const double* sqrt_d,
                        uint16_t* tiles, hipStream_t s) {
    if (nev <= 0) return hipSuccess;
    hipLaunchKernelGGL(tiles_kernel, dim3(nev, 64), dim3(256), 0, s, series, ndm, nout, nbx, W, events,
                       s1, sqrt_d, tiles);
    return hipGetLastError();
}

hipError_t launch_derive(const float* master, const Offsets& off, uint16_t* w1b, uint16_t* wfwd,
                         uint16_t* wdg, hipStream_t s) {
    hipLaunchKernelGGL(derive_weights_kernel, dim3(blocks(3 * kCH * 9 * kCH, 256)), dim3(256), 0, s, master,
                       off, w1b, wfwd, wdg);
    return hipGetLastError();
}

hipError_t launch_forward(const Net& net, const uint16_t* tiles, int N, hipStream_t s) {
    const int64_t pix1 = static_cast<int64_t>(N) * 64 * 256;
    hipLaunchKernelGGL(conv1_fwd_kernel, dim3(blocks(pix1, 256)), dim3(256), 0, s, tiles, N, net.w1b,
                       net.master + net.off.b[0], net.a[0]);
    int H = 64, W = 256;
    for (int l = 0; l < 4; ++l) {
        if (l > 0) {
            const int64_t nb = static_cast<int64_t>(N) * H * (W / 32);
            hipLaunchKernelGGL(conv32_mfma_kernel<0>, dim3(static_cast<unsigned>(nb)), dim3(64), 0, s,
                               net.p[l - 1], N, H, W, net.wfwd + (l - 1) * kCH * 9 * kCH,
                               net.master + net.off.b[l], static_cast<void*>(net.a[l]));
        }
        const int64_t nbp = static_cast<int64_t>(N) * (H / 2) * ((4 * (W / 2) + 255) / 256);
        hipLaunchKernelGGL(maxpool_fwd_kernel, dim3(static_cast<unsigned>(nbp)), dim3(256), 0, s, net.a[l], N, H,
                           W, net.p[l], net.idx[l]);
        H /= 2;
        W /= 2;
    }
    hipLaunchKernelGGL(gap_fc_fwd_kernel, dim3(N), dim3(64), 0, s, net.p[3], N,
                       net.master + net.off.wf, net.master + net.off.bf, net.g, net.logits);
    return hipGetLastError();
}

// Sum of per-block partials in a fixed order (two kernels; `red` holds
// kRedSlices x n floats).
static void launch_reduce(const float* part, int nparts, int stride, int n, float* red, float* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(reduce_slices_kernel, dim3(blocks(n, 64), kRedSlices), dim3(64), 0, s, part, nparts,
                       stride, n, red);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, red, n, out);
}

hipError_t launch_backward(const Net& net, const uint16_t* tiles, const float* labels, int N,
                           hipStream_t s) {
    hipLaunchKernelGGL(bce_kernel, dim3(1), dim3(256), 0, s, net.logits, labels, N, net.dlogit, net.loss);
    hipLaunchKernelGGL(fc_bwd_kernel, dim3(1), dim3(512), 0, s, net.dlogit, net.g, N, net.master + net.off.wf,
                       net.grad + net.off.wf, net.grad + net.off.bf);
    hipLaunchKernelGGL(gap_bwd_kernel, dim3(blocks(static_cast<int64_t>(N) * 64 * kCH, 256)), dim3(256), 0,
                       s, net.dlogit, net.master + net.off.wf, N, net.dp);
    const int Hs[4] = {64, 32, 16, 8}, Ws[4] = {256, 128, 64, 32};
    for (int l = 3; l >= 0; --l) {
        const int H = Hs[l], W = Ws[l];
        const int64_t nblk = static_cast<int64_t>(N) * H * ((4 * W + 255) / 256);
        hipLaunchKernelGGL(pool_relu_bwd_kernel, dim3(static_cast<unsigned>(nblk)), dim3(256), 0, s, net.dp,
                           net.idx[l], net.a[l], N, H, W, net.dz);
        const int64_t nrows = static_cast<int64_t>(N) * H;
        const int rows = kRowsPerBlock;
        const int nparts = static_cast<int>((nrows + rows - 1) / rows);
        const uint16_t* xin = l == 0 ? tiles : net.p[l - 1];
        if (l == 0) {
            hipLaunchKernelGGL(wgrad1_mfma_kernel, dim3(nparts), dim3(64), 0, s, xin, net.dz, N, H, W, rows,
                               net.part);
            launch_reduce(net.part, nparts, 320, 288, net.red, net.grad + net.off.w[0], s);
            launch_reduce(net.part + 288, nparts, 320, kCH, net.red, net.grad + net.off.b[0], s);
        } else {
            hipLaunchKernelGGL(wgrad32_mfma_kernel, dim3(nparts, 9), dim3(64), 0, s, xin, net.dz, N, H, W, rows,
                               net.part);
            launch_reduce(net.part, nparts, 9 * kCH * kCH, 9 * kCH * kCH, net.red, net.dtap, s);
            hipLaunchKernelGGL(wgrad_to_master_kernel, dim3(blocks(9 * kCH * kCH, 256)), dim3(256), 0, s,
                               net.dtap, net.grad + net.off.w[l]);
            hipLaunchKernelGGL(bias_parts_kernel, dim3(nparts), dim3(256), 0, s, net.dz, N, H, W, rows, net.part);
            launch_reduce(net.part, nparts, kCH, kCH, net.red, net.grad + net.off.b[l], s);
            // input gradient -> d p_{l-1} (float32)
            const int64_t nb = static_cast<int64_t>(N) * H * (W / 32);
            hipLaunchKernelGGL(conv32_mfma_kernel<1>, dim3(static_cast<unsigned>(nb)), dim3(64), 0, s, net.dz, N, H,
                               W, net.wdg + (l - 1) * kCH * 9 * kCH, static_cast<const float*>(nullptr),
                               static_cast<void*>(net.dp));
        }
    }
    return hipGetLastError();
}

hipError_t launch_adam(const Net& net, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, static_cast<float>(step));
    const float c2 = 1.0f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(kNumParams, 256)), dim3(256), 0, s, net.master, net.grad, net.m,
                       net.v, kNumParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_sigmoid(const float* z, int n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(sigmoid_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, z, n, out);
    return hipGetLastError();
}

hipError_t launch_finite_check(const float* a, int n, int* bad, hipStream_t s) {
    hipLaunchKernelGGL(finite_check_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, a, n, bad);
    return hipGetLastError();
}

}  // namespace tk
