// Bit-sliced helpers for the dedispersion kernel.
//
// A 2-bit sample stream of one channel is stored as pairs of 32-bit
// "bit-planes" per 32-sample group: lo holds bit 0 of samples 32j..32j+31
// (sample 32j+b at bit b), hi holds bit 1.  Summing channels then works on 32
// samples per 32-bit logic operation: the carry-save trees in csa_tree.inc
// keep a per-position binary counter of NL planes.
//
// Everything here is plain integer code, usable on the host as well, so the
// CPU test suite checks it with g++.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define BS_HD __host__ __device__ __forceinline__
#else
#define BS_HD inline
#ifndef __host__
#define __host__
#define __device__
#define __forceinline__ inline
#endif
#endif

// Three-input bit operations of a full adder: on gfx950 each is one
// v_bitop3_b32 (truth tables 0x96 = odd parity, 0xE8 = majority).
#if defined(__HIP_DEVICE_COMPILE__)
#define BS_XOR3(a, b, c) __builtin_amdgcn_bitop3_b32((a), (b), (c), 0x96)
#define BS_MAJ3(a, b, c) __builtin_amdgcn_bitop3_b32((a), (b), (c), 0xE8)
#else
#define BS_XOR3(a, b, c) ((a) ^ (b) ^ (c))
#define BS_MAJ3(a, b, c) (((a) & (b)) | ((c) & ((a) ^ (b))))
#endif

#include "csa_tree.inc"

namespace bs {

// Bits [r, r+32) of the 64-bit value hi:lo, 0 <= r < 32.
BS_HD uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t r) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, r);
#else
    return static_cast<uint32_t>(((static_cast<uint64_t>(hi) << 32) | lo) >> r);
#endif
}

// Turn NL counter planes (a[L] bit b = bit L of the count at position b) into
// per-sample values: on return r[i] = V_i | (V_{i+16} << 16), i = 0..15, where
// V_b is the count at position b (must fit 16 bits).  A 16x16 bit-matrix
// transpose done in both 16-bit halves at once by 4 block-swap stages.
template <int NL>
BS_HD void planes_to_pairs(const uint32_t (&a)[NL], uint32_t (&r)[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = i < NL ? a[i] : 0u;
    // Stage s swaps the s x s off-diagonal blocks of every 2s x 2s block.
#pragma unroll
    for (int i = 0; i < 8; ++i) {  // s = 8
        const uint32_t t = ((r[i] >> 8) ^ r[i + 8]) & 0x00FF00FFu;
        r[i + 8] ^= t;
        r[i] ^= t << 8;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {  // s = 4
        if (i & 4) continue;
        const uint32_t t = ((r[i] >> 4) ^ r[i + 4]) & 0x0F0F0F0Fu;
        r[i + 4] ^= t;
        r[i] ^= t << 4;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {  // s = 2
        if (i & 2) continue;
        const uint32_t t = ((r[i] >> 2) ^ r[i + 2]) & 0x33333333u;
        r[i + 2] ^= t;
        r[i] ^= t << 2;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {  // s = 1
        if (i & 1) continue;
        const uint32_t t = ((r[i] >> 1) ^ r[i + 1]) & 0x55555555u;
        r[i + 1] ^= t;
        r[i] ^= t << 1;
    }
}

// Carry-in at level F: add the planes p and c (weight 2^F each) to the
// counter levels F..NL-1 (one full adder, then a half-adder ripple).  Sums
// never exceed 2^NL - 1, so the top level drops its (zero) carry.
// One half adder in place: a ^= k, k = old a & k.  On the device the two
// operations are kept as written (the compiler would otherwise fold pairs of
// levels into three-input operations whose results land in fresh registers,
// and a loop-carried counter then pays a copy per level).
BS_HD void half_add(uint32_t& a, uint32_t& k) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t;
    asm volatile("v_and_b32 %0, %1, %2\n\tv_xor_b32 %1, %1, %2" : "=&v"(t), "+v"(a) : "v"(k));
    k = t;
#else
    const uint32_t t = a & k;
    a ^= k;
    k = t;
#endif
}

template <int NL, int F>
BS_HD void carry_in2(uint32_t (&a)[NL], uint32_t p, uint32_t c) {
    uint32_t k = BS_MAJ3(a[F], p, c);
    a[F] = BS_XOR3(a[F], p, c);
#pragma unroll
    for (int l = F + 1; l < NL - 1; ++l) half_add(a[l], k);
    a[NL - 1] ^= k;
}

// Carry-in of one plane c at level F.
template <int NL, int F>
BS_HD void carry_in1(uint32_t (&a)[NL], uint32_t c) {
    uint32_t k = c;
#pragma unroll
    for (int l = F; l < NL - 1; ++l) {
        const uint32_t t = a[l] & k;
        a[l] ^= k;
        k = t;
    }
    a[NL - 1] ^= k;
}

}  // namespace bs
