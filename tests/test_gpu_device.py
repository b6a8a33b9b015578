"""Device description and shader-clock probe (used to relate measured rates
to the chip's peaks)."""
import pytest

from gpu_common import log, torch_dev

pytestmark = pytest.mark.gpu


def test_device_info_and_clock_probe():
    from paper_1112_0065_amd import _lib as L
    torch_dev()
    d = L.dedisp_device_info()
    log("device", d)
    assert d["arch"].startswith("gfx950") and d["compute_units"] > 0
    assert d["max_clock_khz"] > 0 and d["wall_clock_khz"] > 0
    ghz = L.dedisp_clock_probe(20000)
    log("shader clock under load (GHz)", ghz)
    assert 0.05 < ghz < 5.0
    with pytest.raises(L.DedispError):
        L.dedisp_clock_probe(10)
