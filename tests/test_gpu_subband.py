"""GPU parity of subband (two-stage) dedispersion against the oracle,
through the C ABI: exact integers for every (subbands, group) shape tried,
both output types, ragged groups, the shortest input, the survey beam on
sampled trials, and the exact reduction to direct dedispersion."""
import numpy as np
import pytest

import oracle
from oracle.subband import effective_delays, subband_dedisperse
import synth
from gpu_common import log, small_case, survey_case, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _run(fb, plan, nsub, group, u16=True, packed=None, nsamps=None):
    from paper_1112_0065_amd import _lib as L
    torch = torch_dev()
    nsamps = fb.nsamps if nsamps is None else nsamps
    packed = fb.packed if packed is None else packed
    sb = L.dedisp_subband_create(plan, nsub, group)
    nout = nsamps - sb.max_delay
    ws = torch.empty(L.dedisp_subband_workspace_bytes(sb, nsamps), dtype=torch.uint8, device="cuda")
    out = torch.empty((len(fb.dm_list), nout), dtype=torch.int16 if u16 else torch.int32,
                      device="cuda")
    L.dedisp_subband_execute(sb, to_dev(packed), nsamps, out, ws)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return sb, (o.view(np.uint16).astype(np.int64) if u16 else o.astype(np.int64))


@pytest.mark.parametrize("nsub,group", [(1, 1), (4, 3), (16, 4), (64, 1), (32, 16), (8, 7), (2, 9)])
def test_small_config_matches_oracle(nsub, group):
    from paper_1112_0065_amd import _lib as L
    fb, dly, x, direct = small_case()
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    ref = subband_dedisperse(x, fb.f_top, fb.df, fb.tsamp, fb.dm_list, nsub, group)
    for u16 in (True, False):
        sb, got = _run(fb, plan, nsub, group, u16)
        assert sb.ncoarse == (100 + group - 1) // group
        assert got.shape == ref.shape and (got == ref).all(), (nsub, group, u16)
    if (nsub, group) == (1, 1):
        assert (got == direct).all()       # one subband, one trial per group: the direct sum
    log(f"nsub {nsub} group {group}: {ref.shape}, span {sb.span}")


def test_shortest_input_and_bad_arguments():
    from paper_1112_0065_amd import _lib as L
    fb, dly, x, direct = small_case()
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    sb = L.dedisp_subband_create(plan, 16, 4)
    nsamps = sb.max_delay + 1                       # one output sample
    bpt = fb.nchans // 4
    packed = fb.packed[:nsamps * bpt]
    _, got = _run(fb, plan, 16, 4, packed=packed, nsamps=nsamps)
    ref = subband_dedisperse(x[:, :nsamps], fb.f_top, fb.df, fb.tsamp, fb.dm_list, 16, 4)
    assert got.shape == (100, 1) and (got == ref).all()
    assert L.dedisp_subband_workspace_bytes(sb, sb.max_delay) == 0
    for nsub, group in ((3, 1), (128, 1), (16, 0), (16, 17)):    # 128: subbands of 2 channels
        with pytest.raises(L.DedispError) as ei:
            L.dedisp_subband_create(plan, nsub, group)
        assert ei.value.status == L.ERR_INVALID_ARG
    torch = torch_dev()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    out = torch.empty((100, 1), dtype=torch.int16, device="cuda")
    with pytest.raises(L.DedispError) as ei:
        L.dedisp_subband_execute(sb, to_dev(packed), sb.max_delay, out, ws)
    assert ei.value.status == L.ERR_TOO_FEW_SAMPLES


def test_survey_beam_sampled_trials():
    """1024 channels, 2^19 samples, 1200 trials; 32 subbands, groups of 8:
    sampled trials equal the oracle's effective-delay sum."""
    from paper_1112_0065_amd import _lib as L
    fb = survey_case()
    plan = L.dedisp_plan_create(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list)
    sb, got = _run(fb, plan, 32, 8)
    eff = effective_delays(fb.nchans, fb.f_top, fb.df, fb.tsamp, fb.dm_list, 32, 8)
    assert sb.max_delay == int(eff.max()) or sb.max_delay >= int(eff.max())
    nout = fb.nsamps - sb.max_delay
    assert got.shape == (1200, nout)
    x = oracle.unpack_2bit(fb.packed, fb.nsamps, fb.nchans)
    rows = [0, 3, 4, 599, 1195, 1199]
    ref = oracle.dedisperse(x, eff[rows], nout=nout)
    for k, d in enumerate(rows):
        assert (got[d] == ref[k]).all(), d
    log(f"survey subband: span {sb.span}, max delay {sb.max_delay}, ncoarse {sb.ncoarse}")
