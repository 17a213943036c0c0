"""The allocation-free batch entry point (rtc_process_frames_noalloc) against
rtc_process_frames, through the C ABI: two calls in a row on each of two
engines loaded alike, the second call with fewer frames; commands, slopes and
counts must be identical bit for bit (the same kernels in the same order, only
the partials and counters live in the library's static scratch), and the
commands must meet the oracle's bar."""
import numpy as np
import pytest

from rtc_cases import TOL, Case, log, mid_case, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01852_amd import rtc as mod
    mod.lib()
    return mod


def _batch(eng, case, first, n, noalloc):
    import torch
    info = eng.infos[0]
    dfr = [torch.from_numpy(np.ascontiguousarray(f[first:first + n])).cuda() for f in case.frames]
    cmds = torch.zeros((n, info["n_act"]), dtype=torch.float32, device="cuda")
    slopes = torch.zeros((n, info["n_slopes"]), dtype=torch.float32, device="cuda")
    counts = torch.zeros((n, info["n_units"]), dtype=torch.int32, device="cuda")
    eng.process_frames(0, dfr, n, cmds=cmds, slopes=slopes, counts=counts,
                       stream=torch.cuda.current_stream(), noalloc=noalloc)
    torch.cuda.synchronize()
    return cmds.cpu().numpy(), slopes.cpu().numpy(), counts.cpu().numpy()


@pytest.mark.parametrize("which,dtype", [("mid_polc", "f32"), ("scao_sh_74", "fp8")])
def test_noalloc_equals_process_frames(rtc, which, dtype):
    case = mid_case(polc=True, n_frames=8) if which == "mid_polc" else Case(which, n_frames=6)
    n1, n2 = (8, 3) if which == "mid_polc" else (6, 2)
    log(f"case {which} {dtype}: noalloc vs process_frames, {n1} then {n2} frames")
    with rtc.Engine([(case.inst, dtype)]) as a, rtc.Engine([(case.inst, dtype)]) as b:
        case.load(a)
        case.load(b)
        got = []
        for first, n in ((0, n1), (n1 - n2, n2)):
            ra = _batch(a, case, first, n, noalloc=False)
            rb = _batch(b, case, first, n, noalloc=True)
            for x, y, what in zip(ra, rb, ("commands", "slopes", "counts")):
                assert np.array_equal(x, y), f"{what} differ (call of {n} frames)"
            got.append(rb[0].astype(np.float64))
    # the oracle continues over the two calls: bank frames 0..n1-1, then n1-n2..n1-1
    ref = case.run_oracle(dtype, n=n1)["commands"]
    rel = rel_l2(got[0], ref)
    log(f"  first call max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL[dtype]
