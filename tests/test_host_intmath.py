"""The exact wide-integer helpers of the sigma-cut (128/256-bit square root,
division, rounding to double, and the cut level B_thr), compiled for the CPU
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer, against
Python's exact integers and the oracle's threshold.  The cases cross the
2^52, 2^64 and 2^104 boundaries where the helpers change method, and one
build moves the square root's double estimate out of reach of its bounded
correction steps, so that the general digit-by-digit method runs on every
input as well."""
import math
import os
import random
import struct
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1112_0065_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cstdint>
#include "intmath.hpp"

static u128 mk(unsigned long long hi, unsigned long long lo) { return (static_cast<u128>(hi) << 64) | lo; }

int main() {
    char op[16];
    while (scanf("%15s", op) == 1) {
        if (!strcmp(op, "isqrt")) {
            u256 x;
            for (int i = 3; i >= 0; --i) { unsigned long long v; scanf("%llx", &v); x.w[i] = v; }
            const u256 r = u256_isqrt(x);
            printf("%llx %llx %llx %llx\n", (unsigned long long)r.w[3], (unsigned long long)r.w[2],
                   (unsigned long long)r.w[1], (unsigned long long)r.w[0]);
        } else if (!strcmp(op, "div")) {
            unsigned long long ah, al, b;
            scanf("%llx %llx %llx", &ah, &al, &b);
            const u128 q = u128_div_u64(mk(ah, al), b);
            printf("%llx %llx\n", (unsigned long long)(q >> 64), (unsigned long long)q);
        } else if (!strcmp(op, "dbl")) {
            unsigned long long h, l;
            scanf("%llx %llx", &h, &l);
            const double d = u128_to_double(mk(h, l));
            unsigned long long bits;
            memcpy(&bits, &d, 8);
            printf("%llx\n", bits);
        } else if (!strcmp(op, "cut")) {
            unsigned long long n, s1, s2h, s2l;
            unsigned kmant;
            int kexp2;
            scanf("%llx %llx %llx %llx %x %d", &n, &s1, &s2h, &s2l, &kmant, &kexp2);
            u128 d = 0;
            const long long t = cut_level(n, s1, mk(s2h, s2l), kmant, kexp2, &d);
            printf("%lld %llx %llx\n", t, (unsigned long long)(d >> 64), (unsigned long long)d);
        } else {
            return 2;
        }
    }
    return 0;
}
"""

M64 = (1 << 64) - 1


def _build(tmp_path, nudge):
    src = tmp_path / "im.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / f"im_{nudge}"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", f"-DINTMATH_ISQRT_NUDGE={nudge}", f"-I{CSRC}",
           str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, lines):
    r = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout.split("\n")


def _isqrt_cases():
    rnd = random.Random(104)
    xs = list(range(0, 40))
    for e in (52, 64, 104, 128, 208, 255):
        for k in range(-3, 4):
            xs.append((1 << e) + k)
    for r in [(1 << 52) - 1, 1 << 52, (1 << 52) + 1, (1 << 53) - 1, 1 << 53, (1 << 64) - 1,
              (1 << 127), (1 << 128) - 1]:
        xs += [r * r - 1, r * r, r * r + 1]
    for _ in range(300):
        r = rnd.randrange(1, 1 << rnd.choice((20, 40, 51, 52, 53, 60, 64, 100, 127)))
        xs += [r * r - 1, r * r, r * r + 1, r * r + 2 * r, r * r + 2 * r + 1]
    for bits in (30, 60, 90, 103, 104, 105, 150, 200, 254, 256):
        xs += [rnd.getrandbits(bits) for _ in range(60)]
    return [x for x in xs if 0 <= x < (1 << 256)]


@pytest.mark.parametrize("nudge", [0, 1000])
def test_isqrt_exact_on_both_methods(tmp_path, nudge):
    exe = _build(tmp_path, nudge)
    xs = _isqrt_cases()
    lines = ["isqrt " + " ".join(f"{(x >> (64 * i)) & M64:x}" for i in (3, 2, 1, 0)) for x in xs]
    out = _run(exe, lines)
    for x, line in zip(xs, out):
        w = [int(v, 16) for v in line.split()]
        got = (w[0] << 192) | (w[1] << 128) | (w[2] << 64) | w[3]
        assert got == math.isqrt(x), (nudge, x)


def test_division_both_methods(tmp_path):
    exe = _build(tmp_path, 0)
    rnd = random.Random(64)
    cases = [(0, 1), (1, 1), (M64, 1), (M64, M64), (1 << 64, 1), (1 << 64, 3), ((1 << 128) - 1, 1),
             ((1 << 128) - 1, M64), ((1 << 128) - 1, 2), ((1 << 64) + 5, (1 << 63) + 1)]
    for _ in range(400):
        a = rnd.getrandbits(rnd.choice((10, 63, 64, 65, 100, 127, 128)))
        b = rnd.randrange(1, 1 << rnd.choice((1, 20, 40, 63, 64)))
        cases.append((a, b))
    lines = [f"div {a >> 64:x} {a & M64:x} {b:x}" for a, b in cases]
    out = _run(exe, lines)
    nslow = 0
    for (a, b), line in zip(cases, out):
        h, l = (int(v, 16) for v in line.split())
        assert (h << 64) | l == a // b, (a, b)
        nslow += a >= (1 << 64)
    assert nslow > 100


def test_u128_to_double_rounds_half_even(tmp_path):
    """Python's int -> float conversion is correctly rounded, ties to even."""
    exe = _build(tmp_path, 0)
    rnd = random.Random(53)
    xs = [0, 1, M64, 1 << 64, (1 << 64) + 1, (1 << 128) - 1]
    for e in range(65, 128):
        m = (1 << 52) | rnd.getrandbits(52)
        drop = e - 52
        base = m << drop
        half = 1 << (drop - 1)
        xs += [base, base + half, base + half - 1, base + half + 1, ((m | 1) << drop) + half,
               ((m & ~1) << drop) + half]
    xs += [rnd.getrandbits(rnd.choice((50, 64, 65, 90, 127, 128))) for _ in range(300)]
    xs = [x for x in xs if 0 <= x < (1 << 128)]
    out = _run(exe, [f"dbl {x >> 64:x} {x & M64:x}" for x in xs])
    for x, line in zip(xs, out):
        got = struct.unpack("<d", struct.pack("<Q", int(line, 16)))[0]
        assert got == float(x), x


def _split(k):
    """k (float32) = kmant * 2^kexp2, kmant odd."""
    f = Fraction(float(np.float32(k)))
    num, den = f.numerator, f.denominator
    e = 0
    while num % 2 == 0:
        num //= 2
        e += 1
    while den % 2 == 0:
        den //= 2
        e -= 1
    assert den == 1
    return num, e


def test_cut_level_matches_oracle(tmp_path):
    """B_thr from (n, S1, S2, k) equals the oracle's exact threshold, on
    sums that take every method: k^2 D below and above 2^104, S1 + isqrt + 1
    below and above 2^64, D = 0, and thresholds beyond 2^62."""
    exe = _build(tmp_path, 0)
    rnd = random.Random(6)
    ks = [6.0, 3.0, 0.5, 2.75, 1e-3, 6.1, 1e6, 123456.7]
    cases = []
    for _ in range(500):
        n = rnd.randrange(1, 1 << rnd.choice((2, 17, 24, 33, 40)))
        s1 = rnd.randrange(0, 1 << rnd.choice((10, 40, 63, 64)))
        lo = (s1 * s1 + n - 1) // n          # smallest S2 with D >= 0
        extra = rnd.randrange(0, 1 << rnd.choice((1, 30, 70, 100, 120)))
        s2 = lo + extra
        if s2 >= (1 << 128) or n * s2 >= (1 << 128):
            continue
        cases.append((n, s1, s2, rnd.choice(ks)))
    # constant series (D = 0) and the survey's typical sizes
    cases += [(8, 24, 72, 6.0), (503301, 503301 * 1536, 503301 * 1536 ** 2, 6.0),
              (503301, 773070336, 1187639600000, 6.0)]
    lines = []
    for n, s1, s2, k in cases:
        km, ke = _split(k)
        lines.append(f"cut {n:x} {s1:x} {s2 >> 64:x} {s2 & M64:x} {km:x} {ke}")
    out = _run(exe, lines)
    hit = {"big_root": 0, "wide_num": 0, "none": 0, "huge": 0}
    for (n, s1, s2, k), line in zip(cases, out):
        t, dh, dl = line.split()
        d = n * s2 - s1 * s1
        assert (int(dh, 16) << 64) | int(dl, 16) == d
        ref = oracle.threshold_level(n, s1, s2, k)
        if ref is None:
            assert int(t) == -1
            hit["none"] += 1
            continue
        if ref >= (1 << 62):
            assert int(t) == (1 << 63) - 1, (n, s1, s2, k)
            hit["huge"] += 1
        else:
            assert int(t) == ref, (n, s1, s2, k)
        kk = Fraction(float(np.float32(k)))
        q = kk * kk * d
        root = math.isqrt(q.numerator // q.denominator)
        hit["big_root"] += (q.numerator // q.denominator) >= (1 << 104)
        hit["wide_num"] += s1 + root + 1 + n - 1 >= (1 << 64)
    assert min(hit.values()) >= 3, hit
