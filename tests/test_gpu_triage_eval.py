"""What the trained triage network gains over the plain S/N detector.

The committed network (trained on the GPU by the library's own kernels, see
paper_1112_0065_amd/triage_train.py) scores the candidates of beams it never
saw (seeds 800..863; training used 10000.., the score cut was chosen on
600..679).  The plain detector keeps every candidate and is the yardstick:
triage must keep the recall over injected pulses within 1% of the plain
detector's while passing far fewer false candidates."""
import numpy as np
import pytest

from gpu_common import log, torch_dev

pytestmark = pytest.mark.gpu


def test_trained_triage_keeps_recall_and_cuts_false_candidates():
    torch_dev()
    from paper_1112_0065_amd import triage_train as T
    model, tau, report = T.load_default()
    tiles, labels, recs = T.build(range(800, 864), log=lambda *a: None)
    assert len(labels) > 1000 and 0 < labels.sum() < len(labels)
    sc = T.scores(model, tiles)
    assert np.isfinite(sc).all() and (sc >= 0).all() and (sc <= 1).all()
    r = T.evaluate(sc, recs, tau)
    log("triage on unseen beams", r, "trained:", report["test"])
    assert r["recall_triage"] >= r["recall_plain"] - 0.01
    assert r["false_triage"] < 0.25 * r["false_plain"]
    # the plain detector is the yardstick: with no network every candidate passes
    plain = T.evaluate(np.ones_like(sc), recs, tau)
    assert plain["recall_triage"] == plain["recall_plain"]
    assert plain["false_triage"] == plain["false_plain"]
