"""Host-side checks that need no GPU: the built library loads and exports
every symbol the header declares, and the bit-sliced integer helpers the
dedispersion kernel uses -- carry-save trees, the low counter with paired
carry-outs, the plane transpose -- are exact (compiled for the CPU with
g++)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1112_0065_amd", "csrc")


def test_library_exports_every_declared_symbol():
    from paper_1112_0065_amd import _lib
    L = _lib.lib()
    names = _lib.declared_symbols()
    assert "dedisp_execute" in names and "find_peaks" in names and "boxcar_filter" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.dedisp_version().decode().startswith("dedisp-gfx950")


def test_every_exported_c_symbol_is_declared():
    """The converse: no unmangled symbol leaves the library without a
    declaration in the header."""
    import shutil
    from paper_1112_0065_amd import _lib
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {f[2] for f in (line.split() for line in out.splitlines())
                if len(f) == 3 and f[1] == "T" and not f[2].startswith("_")}
    assert exported == set(_lib.declared_symbols())


def test_tile_candidates_host_only():
    from paper_1112_0065_amd import _lib
    tiles = _lib.dedisp_tile_candidates()
    assert len(tiles) == 21
    for nd, g, cs in tiles:
        assert nd in (4, 8, 16, 32) and g in (1, 2) and cs % 4 == 0


HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <random>
#include "bitslice.hpp"

// Sum channels of random 2-bit samples with the CSA trees and the plane
// transpose, and compare with plain integer sums.
template <int NL, int N>
int check(std::mt19937& rng, int reps) {
    for (int rep = 0; rep < reps; ++rep) {
        uint32_t a[NL] = {0};
        int ref[32] = {0};
        const int nch = N * (1 + rng() % ((NL == 12 ? 1364 : 21844) / N));
        for (int c0 = 0; c0 < nch; c0 += N) {
            uint32_t lo[N], hi[N];
            for (int k = 0; k < N; ++k) {
                lo[k] = rng(); hi[k] = rng();
                if (rep % 3 == 0) { lo[k] = hi[k] = 0xFFFFFFFFu; }   // all samples = 3
                for (int b = 0; b < 32; ++b) ref[b] += ((lo[k] >> b) & 1) + 2 * ((hi[k] >> b) & 1);
            }
            bs_csa<NL, N>(a, lo, hi);
        }
        uint32_t r[16];
        bs::planes_to_pairs<NL>(a, r);
        for (int b = 0; b < 32; ++b) {
            const uint32_t v = b < 16 ? (r[b] & 0xFFFF) : (r[b - 16] >> 16);
            if ((int)v != ref[b]) { printf("FAIL NL=%d N=%d rep=%d b=%d got %u want %d\n", NL, N, rep, b, v, ref[b]); return 1; }
        }
    }
    return 0;
}

// The kernel's pairing: each chunk of 8 (or 4) channels goes into the 5-level
// low counter; its carry-out waits for the next chunk's and the two enter the
// upper levels together; an odd last one enters alone.
template <int NL>
int check_pairs(std::mt19937& rng, int reps) {
    for (int rep = 0; rep < reps; ++rep) {
        uint32_t a[NL] = {0};
        uint32_t pend = 0;
        int ref[32] = {0};
        const int nchunks = 1 + rng() % ((NL == 12 ? 1364 : 21844) / 8);
        int k = 0;
        for (int ci = 0; ci < nchunks; ++ci, ++k) {
            const bool four = (rng() % 5) == 0;
            uint32_t lo[8], hi[8];
            const int n = four ? 4 : 8;
            for (int j = 0; j < n; ++j) {
                lo[j] = rng(); hi[j] = rng();
                if (rep % 3 == 0) { lo[j] = hi[j] = 0xFFFFFFFFu; }
                for (int b = 0; b < 32; ++b) ref[b] += ((lo[j] >> b) & 1) + 2 * ((hi[j] >> b) & 1);
            }
            uint32_t cy;
            if (four) {
                uint32_t l4[4] = {lo[0], lo[1], lo[2], lo[3]}, h4[4] = {hi[0], hi[1], hi[2], hi[3]};
                cy = csa5_add_4<NL>(a, l4, h4);
            } else {
                cy = csa5_add_8<NL>(a, lo, hi);
            }
            if (k & 1) bs::carry_in2<NL, 5>(a, pend, cy); else pend = cy;
        }
        if (k & 1) bs::carry_in1<NL, 5>(a, pend);
        uint32_t r[16];
        bs::planes_to_pairs<NL>(a, r);
        for (int b = 0; b < 32; ++b) {
            const uint32_t v = b < 16 ? (r[b] & 0xFFFF) : (r[b - 16] >> 16);
            if ((int)v != ref[b]) { printf("FAIL pairs NL=%d rep=%d b=%d got %u want %d\n", NL, rep, b, v, ref[b]); return 1; }
        }
    }
    return 0;
}

int funnel_check(std::mt19937& rng) {
    for (int i = 0; i < 1000; ++i) {
        uint32_t hi = rng(), lo = rng(), r = rng() % 32;
        uint64_t v = ((uint64_t)hi << 32) | lo;
        if (bs::funnel(hi, lo, r) != (uint32_t)(v >> r)) return 1;
    }
    return 0;
}

int main() {
    std::mt19937 rng(12345);
    int bad = funnel_check(rng);
    bad |= check<12, 4>(rng, 30); bad |= check<12, 8>(rng, 30); bad |= check<12, 16>(rng, 30);
    bad |= check<12, 32>(rng, 30); bad |= check<12, 64>(rng, 10);
    bad |= check<16, 4>(rng, 6); bad |= check<16, 16>(rng, 6); bad |= check<16, 32>(rng, 6);
    bad |= check_pairs<12>(rng, 60); bad |= check_pairs<16>(rng, 8);
    printf(bad ? "FAILED\n" : "ALL OK\n");
    return bad;
}
"""

DISPATCH = r"""
template <int NL, int N> void bs_csa(uint32_t (&a)[NL], const uint32_t (&lo)[N], const uint32_t (&hi)[N]);
#define S(NL_, N_) template <> void bs_csa<NL_, N_>(uint32_t (&a)[NL_], const uint32_t (&lo)[N_], const uint32_t (&hi)[N_]) { csa_add_##N_##_##NL_(a, lo, hi); }
S(12,4) S(12,8) S(12,16) S(12,32) S(12,64) S(16,4) S(16,8) S(16,16) S(16,32) S(16,64)
"""


def test_bitslice_helpers_exact(tmp_path):
    src = tmp_path / "h.cpp"
    code = HARNESS.replace('#include "bitslice.hpp"\n', '#include "bitslice.hpp"\n' + DISPATCH)
    src.write_text(code)
    exe = tmp_path / "h"
    r = subprocess.run(["g++", "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout


def test_baseline_division_by_multiply_is_exact():
    """The running-mean kernel divides the window sum n < 2^31 by the window
    w = 2R + 1 <= 16385 as (n * M) >> k, k = 31 + ceil(log2 w),
    M = ceil(2^k / w); check the identity for every w at the extreme and
    random n, and that n * M stays below 2^63."""
    import random
    rnd = random.Random(7)
    for w in range(1, 16386, 2):
        lg = (w - 1).bit_length()
        k = 31 + lg
        m = ((1 << k) + w - 1) // w
        for n in [0, 1, w - 1, w, w + 1, (1 << 31) - 1, (1 << 31) - w] + \
                [rnd.randrange(1 << 31) for _ in range(20)]:
            assert (n * m) >> k == n // w
            assert n * m < (1 << 63)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits
    before touching a device."""
    import sys
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                           capture_output=True, text=True, timeout=60,
                           env={**os.environ, **env})
        assert r.returncode == 2, (args, env, r.stderr)
        assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_handles_are_not_released_by_another_process():
    """A process forked from one that owns library handles (a multiprocessing
    pool) inherits their Python wrappers; when its garbage collector drops
    them, the destructors must not call into the library (a bogus handle
    here would crash the test if they did)."""
    import gc
    from paper_1112_0065_amd import _lib as L
    L.lib()
    objs = [L.Plan(0xDEAD0, 4, 1, 0), L.Model(0xDEAD1), L.Batch(0xDEAD2, []), L.Server(0xDEAD3, [])]
    for o in objs:
        o._pid = -1            # as if created by the parent of a fork
    del o
    objs.clear()
    gc.collect()
