"""Host-only logic of the streaming server (no GPU): admission arithmetic and
latency percentiles, through the C ABI."""
import numpy as np


def test_percentile_nearest_rank():
    from paper_1112_0065_amd import _lib as L
    v = list(range(1, 101))                      # 1..100
    assert L.dedisp_percentile_ns(v, 0.5) == 50
    assert L.dedisp_percentile_ns(v, 0.99) == 99
    assert L.dedisp_percentile_ns(v, 1.0) == 100
    assert L.dedisp_percentile_ns([7], 0.99) == 7
    assert L.dedisp_percentile_ns([], 0.5) == 0
    rng = np.random.default_rng(1)
    for _ in range(50):
        a = rng.integers(0, 10**9, size=int(rng.integers(1, 300)))
        for q in (0.5, 0.9, 0.99):
            k = int(np.ceil(q * len(a)))
            assert L.dedisp_percentile_ns(a, q) == np.sort(a)[max(k, 1) - 1]


def test_admission_arithmetic():
    from paper_1112_0065_amd import _lib as L
    gib = 1 << 30
    assert L.dedisp_serve_admission(32 * gib, 70 * (1 << 20), 450 * (1 << 20)) == \
        (32 * gib - 70 * (1 << 20)) // (450 * (1 << 20))
    assert L.dedisp_serve_admission(100, 10, 90) == 1
    assert L.dedisp_serve_admission(99, 10, 90) == 0       # not even one slot
    assert L.dedisp_serve_admission(10**15, 0, 1) == 4096  # capped
    assert L.dedisp_serve_admission(100, 10, 0) == 0
