"""GPU tests of pyramid global normalisation (one intensity sum over the pupil).

The per-launch path forms each frame's pupil sum in a fixed order, then the
slopes; the commands must match the oracle to the FP32 bar, the thresholded
pixel counts bit for bit, and the serving forms and the frame loop must give
the per-launch batch commands bit for bit.
"""
import numpy as np
import pytest

import synth
from rtc_cases import TOL, Case, log, rel_l2, run_batch, run_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01852_amd import rtc as mod
    mod.lib()
    return mod


def _global_case(n_frames: int, pupil_px: int = 92, n_act: int = 5318, index: int = 98):
    o0, o1 = (120 - pupil_px) // 2, 120 + (120 - pupil_px) // 2
    wfs = synth.PyrWfs(pupil_px=pupil_px, norm="global",
                       quad_origins=((o0, o0), (o1, o0), (o0, o1), (o1, o1)))
    inst = synth.Instance(f"pyrg{index}", (wfs,), n_act, ("f32",))
    wl = synth.Workload(index, inst.name, (inst,), n_frames=n_frames, bank=n_frames)
    synth.workloads.WORKLOADS[wl.name] = wl
    try:
        return Case(wl.name, n_frames=n_frames)
    finally:
        del synth.workloads.WORKLOADS[wl.name]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_pyramid_global_batch_vs_oracle(rtc, dtype):
    case = _global_case(6)
    log(f"case pyramid 92 px global normalisation {dtype}: per-launch batch, 6 frames")
    with rtc.Engine([(case.inst, dtype)], mode="stream") as eng:
        case.load(eng)
        cmds, slopes, counts = run_batch(eng, 0, case)
    ref = case.run_oracle(dtype)
    assert np.array_equal(counts, ref["counts"])
    ds = np.abs(slopes - ref["slopes"]).max() / np.abs(ref["slopes"]).max()
    rel = rel_l2(cmds, ref["commands"])
    log(f"  slopes max rel {ds:.3e}, commands max rel L2 {rel.max():.3e}")
    assert ds <= 1e-5
    assert rel.max() <= TOL[dtype]
    # against local normalisation the slopes differ by orders of magnitude
    loc = Case("scao_pyr_92", n_frames=1)
    assert np.abs(ref["slopes"]).max() < 0.01 * np.abs(loc.run_oracle("f32", n=1)["slopes"]).max()


def test_pyramid_global_serving_equals_batch(rtc):
    """Chunks submitted one by one (the pupil sum and slopes wait for the last
    one) give the batch commands bit for bit; a pupil sized so that the last
    chunk holds no pupil row still waits for it."""
    for px in (92, 80):
        case = _global_case(8, pupil_px=px, n_act=700, index=99 - (px == 80))
        with rtc.Engine([(case.inst, "f32")], mode="stream") as eng:
            case.load(eng)
            served, infos = run_stream(eng, 0, case)
            eng.set_state(0, None, None, 0)
            batch, _, _ = run_batch(eng, 0, case)
        assert np.array_equal(served, batch)
        ref = case.run_oracle("f32")
        assert rel_l2(served, ref["commands"]).max() <= TOL["f32"]


def test_pyramid_global_frame_loop_equals_launch_path(rtc):
    """The frame loop (each wavefront forms the pupil sum itself, in the sum
    kernel's order) gives the per-launch commands, slopes and counts bit for
    bit, in batch and in serving."""
    case = _global_case(8, pupil_px=92, n_act=700, index=97)
    with rtc.Engine([(case.inst, "f32")], mode="stream") as eng:
        case.load(eng)
        c1, s1, n1 = run_batch(eng, 0, case)
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        c2, s2, n2 = run_batch(eng, 0, case)
        eng.set_state(0, None, None, 0)
        served, _ = run_stream(eng, 0, case)
    assert np.array_equal(n1, n2)
    assert np.array_equal(s1, s2)
    assert np.array_equal(c1, c2)
    assert np.array_equal(c1, served)
