// Exact wide-integer helpers of the sigma-cut: 128/256-bit sums, products,
// shifts, integer square root and division, and the cut level B_thr of a
// series from its exact sums.  Plain integer code for the device and the host
// alike, so the CPU test suite checks every branch with g++.
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define IM_HD __host__ __device__ __forceinline__
#define IM_HD_NOINLINE __host__ __device__
#else
#define IM_HD inline
#define IM_HD_NOINLINE inline
#endif

// Added to the double estimate of the integer square root before it is
// stepped to the exact floor; nonzero only in a host test build, to drive
// the estimate out of reach of the bounded steps (the general method then
// decides).
#ifndef INTMATH_ISQRT_NUDGE
#define INTMATH_ISQRT_NUDGE 0
#endif

namespace {

using u128 = unsigned __int128;

struct u256 {
    uint64_t w[4];
};

IM_HD u256 u256_from(u128 x) {
    return u256{{static_cast<uint64_t>(x), static_cast<uint64_t>(x >> 64), 0, 0}};
}

// a * b for a < 2^128, b < 2^64.
IM_HD u256 u256_mul_u64(u128 a, uint64_t b) {
    const uint64_t a0 = static_cast<uint64_t>(a), a1 = static_cast<uint64_t>(a >> 64);
    const u128 p0 = static_cast<u128>(a0) * b;
    const u128 p1 = static_cast<u128>(a1) * b + (p0 >> 64);
    return u256{{static_cast<uint64_t>(p0), static_cast<uint64_t>(p1), static_cast<uint64_t>(p1 >> 64), 0}};
}

IM_HD u256 u256_shr(u256 a, int s) {
    u256 r{{0, 0, 0, 0}};
    const int q = s >> 6, b = s & 63;
    for (int i = 0; i < 4; ++i) {
        const int j = i + q;
        if (j < 4) {
            uint64_t v = a.w[j] >> b;
            if (b && j + 1 < 4) v |= a.w[j + 1] << (64 - b);
            r.w[i] = v;
        }
    }
    return r;
}

IM_HD u256 u256_shl(u256 a, int s) {
    u256 r{{0, 0, 0, 0}};
    const int q = s >> 6, b = s & 63;
    for (int i = 3; i >= 0; --i) {
        const int j = i - q;
        if (j >= 0) {
            uint64_t v = a.w[j] << b;
            if (b && j - 1 >= 0) v |= a.w[j - 1] >> (64 - b);
            r.w[i] = v;
        }
    }
    return r;
}

IM_HD bool u256_ge(const u256& a, const u256& b) {
    for (int i = 3; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] > b.w[i];
    return true;
}

IM_HD u256 u256_sub(u256 a, const u256& b) {
    uint64_t borrow = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t x = a.w[i], y = b.w[i];
        const uint64_t d = x - y - borrow;
        borrow = (x < y) || (x - y < borrow) ? 1 : 0;
        a.w[i] = d;
    }
    return a;
}

IM_HD u256 u256_add(u256 a, const u256& b) {
    uint64_t carry = 0;
    for (int i = 0; i < 4; ++i) {
        const uint64_t s = a.w[i] + b.w[i];
        const uint64_t c1 = s < a.w[i];
        const uint64_t s2 = s + carry;
        const uint64_t c2 = s2 < s;
        a.w[i] = s2;
        carry = c1 | c2;
    }
    return a;
}

// floor(sqrt(x)).  Below 2^104 the root is under 2^52: a double square root
// lands within a unit or two of it, and exact 128-bit squares step it to the
// floor (at most four steps each way; if that does not bracket the root, the
// general method below decides).  Otherwise digit by digit (binary restoring
// method).
IM_HD_NOINLINE u256 u256_isqrt(u256 x) {
    if ((x.w[3] | x.w[2]) == 0 && (x.w[1] >> 40) == 0) {
        const u128 xx = static_cast<u128>(x.w[1]) << 64 | x.w[0];
        const double xd = static_cast<double>(x.w[1]) * 18446744073709551616.0 + static_cast<double>(x.w[0]);
        uint64_t r = static_cast<uint64_t>(sqrt(xd)) + INTMATH_ISQRT_NUDGE;
        if (r > (uint64_t(1) << 53)) r = uint64_t(1) << 53;
        for (int i = 0; i < 4 && r > 0 && static_cast<u128>(r) * r > xx; ++i) --r;
        for (int i = 0; i < 4 && static_cast<u128>(r + 1) * (r + 1) <= xx; ++i) ++r;
        if (static_cast<u128>(r) * r <= xx && static_cast<u128>(r + 1) * (r + 1) > xx)
            return u256{{r, 0, 0, 0}};
    }
    u256 res{{0, 0, 0, 0}};
    u256 bit{{0, 0, 0, 0}};
    // highest power of four <= x
    int top = -1;
    for (int i = 3; i >= 0 && top < 0; --i)
        if (x.w[i]) top = 64 * i + 63 - __builtin_clzll(x.w[i]);
    if (top < 0) return res;
    const int p = top & ~1;
    bit.w[p >> 6] = uint64_t(1) << (p & 63);
    while (bit.w[0] | bit.w[1] | bit.w[2] | bit.w[3]) {
        const u256 t = u256_add(res, bit);
        if (u256_ge(x, t)) {
            x = u256_sub(x, t);
            res = u256_add(u256_shr(res, 1), bit);
        } else {
            res = u256_shr(res, 1);
        }
        bit = u256_shr(bit, 2);
    }
    return res;
}

// floor(a / b), a < 2^128, b >= 1: one 64-bit division when a fits 64 bits,
// else shift-subtract.
IM_HD_NOINLINE u128 u128_div_u64(u128 a, uint64_t b) {
    if ((a >> 64) == 0) return static_cast<uint64_t>(a) / b;
    u128 q = 0, r = 0;
    for (int i = 127; i >= 0; --i) {
        r = (r << 1) | ((a >> i) & 1);
        if (r >= b) {
            r -= b;
            q |= static_cast<u128>(1) << i;
        }
    }
    return q;
}

// Round-to-nearest-even conversion of an unsigned 128-bit integer.
IM_HD_NOINLINE double u128_to_double(u128 x) {
    if ((x >> 64) == 0) return static_cast<double>(static_cast<uint64_t>(x));
    const uint64_t hi = static_cast<uint64_t>(x >> 64);
    const int lz = __builtin_clzll(hi);
    const int nbits = 128 - lz;          // 65..128
    const int drop = nbits - 53;
    u128 m = x >> drop;                  // 53 significant bits
    const u128 rem = x - (m << drop);
    const u128 half = static_cast<u128>(1) << (drop - 1);
    if (rem > half || (rem == half && (m & 1))) m += 1;
    return ldexp(static_cast<double>(static_cast<uint64_t>(m)), drop);
}

// Smallest integer value B whose S/N = (n*B - S1)/sqrt(D) exceeds k, with
// D = n*S2 - S1^2 and k = kmant * 2^kexp2 exactly:
//   B_thr = ceil((S1 + isqrt(floor(k^2 D)) + 1) / n).
// Returns -1 when D == 0 (nothing exceeds) and INT64_MAX when no value below
// 2^62 can; *d_out (may be NULL) receives D.
IM_HD_NOINLINE int64_t cut_level(uint64_t n, uint64_t s1, u128 s2, uint32_t kmant, int kexp2,
                             u128* d_out) {
    const u128 d = static_cast<u128>(n) * s2 - static_cast<u128>(s1) * s1;
    if (d_out) *d_out = d;
    if (d == 0) return -1;
    // floor(k^2 D) with k = kmant * 2^kexp2: (kmant^2 D) shifted by 2 kexp2
    const u256 kd = u256_mul_u64(d, static_cast<uint64_t>(kmant) * kmant);
    const u256 q = kexp2 >= 0 ? u256_shl(kd, 2 * kexp2) : u256_shr(kd, -2 * kexp2);
    const u256 r = u256_isqrt(q);
    // lmin = isqrt + 1 < 2^128 here; B_thr = ceil((S1 + lmin) / n)
    if (r.w[2] | r.w[3] | (r.w[1] >> 62)) return INT64_MAX;
    const u128 lmin = (static_cast<u128>(r.w[1]) << 64 | r.w[0]) + 1;
    const u128 num = static_cast<u128>(s1) + lmin;
    const u128 b = u128_div_u64(num + (n - 1), n);
    return (b >> 62) ? INT64_MAX : static_cast<int64_t>(b);
}

}  // namespace
