// Shared declarations of the triage network kernels (triage.hip) and its
// host side (triage.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/dedisp.h"

namespace tk {

constexpr int kCH = 32;
constexpr int kRowsPerBlock = 8;
// Slices of the fixed-order reduction of per-block gradient partials.
constexpr int kRedSlices = 32;
// w1 [32][1][3][3], b1, (w, b) x 3 layers of [32][32][3][3], wf [32], bf [1]
constexpr int kNumParams = 32 * 9 + 32 + 3 * (32 * 32 * 9 + 32) + 32 + 1;

struct Offsets {
    int w[4];
    int b[4];
    int wf;
    int bf;
};

inline Offsets param_offsets() {
    Offsets o{};
    int k = 0;
    o.w[0] = k; k += 32 * 9;
    o.b[0] = k; k += 32;
    for (int l = 1; l < 4; ++l) {
        o.w[l] = k; k += 32 * 32 * 9;
        o.b[l] = k; k += 32;
    }
    o.wf = k; k += 32;
    o.bf = k; k += 1;
    return o;
}

struct TileWidths {
    int32_t w[32];
    int32_t n;
};

// Device buffers of one network instance (capacity for `cap` tiles).
struct Net {
    Offsets off;
    float* master;      // kNumParams float32
    float* grad;        // kNumParams
    float* m;           // Adam first moment
    float* v;           // Adam second moment
    uint16_t* w1b;      // [32][9] bf16
    uint16_t* wfwd;     // 3 x [32][9][32] bf16
    uint16_t* wdg;      // 3 x [32][9][32] bf16, flipped and transposed
    uint16_t* a[4];     // ReLU outputs per layer, NHWC bf16
    uint16_t* p[4];     // pooled outputs
    uint8_t* idx[4];    // pool winners
    float* g;           // [cap][32]
    float* logits;      // [cap]
    float* dlogit;      // [cap]
    float* loss;        // [1]
    float* dp;          // float32 gradient of the pooled map (largest layer)
    uint16_t* dz;       // bf16 gradient of the pre-activation (largest layer)
    float* part;        // per-block partial sums of weight / bias gradients
    float* red;         // [kRedSlices][9 * 32 * 32] slices of their reduction
    float* dtap;        // [9][32][32]
    float* scores;      // [cap]
    int* bad;           // non-finite counter
    int cap;
};

hipError_t launch_tiles(const uint16_t* series, int ndm, int64_t nout, int64_t nbx, const TileWidths& W,
                        const dedisp_event* events, int nev, const uint64_t* s1, const double* sqrt_d,
                        uint16_t* tiles, hipStream_t s);
hipError_t launch_derive(const float* master, const Offsets& off, uint16_t* w1b, uint16_t* wfwd,
                         uint16_t* wdg, hipStream_t s);
hipError_t launch_forward(const Net& net, const uint16_t* tiles, int N, hipStream_t s);
hipError_t launch_backward(const Net& net, const uint16_t* tiles, const float* labels, int N,
                           hipStream_t s);
hipError_t launch_adam(const Net& net, float lr, int step, hipStream_t s);
hipError_t launch_sigmoid(const float* z, int n, float* out, hipStream_t s);
hipError_t launch_finite_check(const float* a, int n, int* bad, hipStream_t s);

}  // namespace tk
