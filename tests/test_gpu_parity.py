"""GPU parity: the gfx950 path through the C ABI against the CPU oracle.

Bars: thresholded-pixel masks and counts bit-exact; stored matrix codes
bit-exact; commands within a per-frame relative L2 of 1e-5 (FP32 storage),
1e-2 (BF16), 3e-2 (FP8) of the float32-matrix oracle, and within 1e-5 of the
oracle run on the dequantised matrix.
"""
import numpy as np
import pytest

import oracle
from rtc_cases import (DEQ_TOL, SLOPE_TOL_PYR, SLOPE_TOL_SH, TOL, Case, log, mask_bits,
                       rel_l2, run_batch, run_stream)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01852_amd import rtc as mod
    mod.lib()
    return mod


def _check_slopes(case, got_slopes, got_counts, ref):
    assert np.array_equal(got_counts, ref["counts"]), "counts differ"
    kinds = np.concatenate([np.full(w.n_slopes, w.kind == "sh") for w in case.inst.wfs])
    d = np.abs(got_slopes - ref["slopes"])
    if kinds.any():
        assert d[:, kinds].max() <= SLOPE_TOL_SH, d[:, kinds].max()
    if (~kinds).any():
        assert d[:, ~kinds].max() <= SLOPE_TOL_PYR, d[:, ~kinds].max()


def test_small_sh_f32_batch(rtc):
    """16x16 SH, 8x8 px, 232 actuators: 200 frames spanning several tiles and a ragged tail."""
    case = Case("scao_sh_small", n_frames=200)
    log("case scao_sh_small f32 batch 200 frames")
    with rtc.Engine([(case.inst, "f32")]) as eng:
        case.load(eng)
        cmds, slopes, counts = run_batch(eng, 0, case)
        s_last, c_last, m_last = eng.read_slopes(0)
    ref = case.run_oracle("f32", keep_masks=True)
    _check_slopes(case, slopes, counts, ref)
    assert np.array_equal(m_last, mask_bits(ref["masks"][-1], case.inst)), "masks differ"
    assert np.array_equal(c_last, ref["counts"][-1])
    rel = rel_l2(cmds, ref["commands"])
    log(f"  max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL["f32"]


def _serve_numbered(eng, case, numbers):
    """Serving: bank frame f submitted as frame number numbers[f]."""
    out = []
    for f, no in enumerate(numbers):
        for w, bank in enumerate(case.frames):
            for c in range(case.inst.wfs[w].n_chunks):
                r0, r1 = eng.chunk_rows(0, w, c)
                eng.submit_chunk(0, w, no, c, bank[f][r0:r1])
        cmds, _ = eng.wait_commands(0, no, timeout_s=10.0)
        out.append(cmds.astype(np.float64))
    return np.stack(out)


def test_direction_follows_frame_sequence(rtc):
    """Odd frames stream every segment backwards, frames counted from the last
    state reset whatever their numbers.  The same three frames (ELT SCAO SH
    74x74, FP32) from next frame number 0 and 1, and served as frames 1, 2, 5:
    per-launch and frame-loop paths, batch and serving, agree bit for bit and
    meet the oracle's bar."""
    case = Case("scao_sh_74", n_frames=3)
    ref = case.run_oracle("f32")
    outs = []
    for mode in ("stream", "persistent"):
        with rtc.Engine([(case.inst, "f32")], mode=mode) as eng:
            case.load(eng)
            for start in (0, 1):
                log(f"case scao_sh_74 f32 {mode}: batch of 3 from frame number {start}")
                eng.set_state(0, None, None, start)
                outs.append(run_batch(eng, 0, case)[0])
            log(f"case scao_sh_74 f32 {mode}: served as frames 1, 2, 5")
            eng.set_state(0, None, None, 1)
            outs.append(_serve_numbered(eng, case, (1, 2, 5)))
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    assert rel_l2(outs[0], ref["commands"]).max() <= TOL["f32"]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_scao74_batch(rtc, dtype):
    """ELT SCAO SH (74x74, 5318 x 7944) at full size."""
    case = Case("scao_sh_74", n_frames=6)
    log(f"case scao_sh_74 {dtype} batch 6 frames")
    with rtc.Engine([(case.inst, dtype)]) as eng:
        case.load(eng)
        cmds, slopes, counts = run_batch(eng, 0, case)
        codes, scales = eng.read_matrix(0)
        s_last, c_last, m_last = eng.read_slopes(0)
    ref_codes, ref_scale = oracle.quantize(case.R, dtype)
    if dtype == "f32":
        assert np.array_equal(codes.view(np.uint32), ref_codes.view(np.uint32))
    else:
        assert np.array_equal(codes, ref_codes), "stored codes differ"
    if dtype == "fp8":
        assert np.array_equal(scales.view(np.uint32), ref_scale.view(np.uint32))
    ref = case.run_oracle(dtype, keep_masks=True)
    _check_slopes(case, slopes, counts, ref)
    assert np.array_equal(m_last, mask_bits(ref["masks"][-1], case.inst))
    rel = rel_l2(cmds, ref["commands"])
    deq = rel_l2(cmds, case.run_oracle(dtype, dequantized=True)["commands"])
    log(f"  rel L2 vs f32 oracle max {rel.max():.3e} mean {rel.mean():.3e}; "
        f"vs dequantised {deq.max():.3e}")
    assert deq.max() <= DEQ_TOL
    assert rel.max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_pyramid_batch(rtc, dtype):
    """ELT SCAO pyramid: 4 x 92 px pupils on 240x240, 5318 x 12288."""
    case = Case("scao_pyr_92", n_frames=6)
    log(f"case scao_pyr_92 {dtype} batch 6 frames")
    with rtc.Engine([(case.inst, dtype)]) as eng:
        case.load(eng)
        cmds, slopes, counts = run_batch(eng, 0, case)
        s_last, c_last, m_last = eng.read_slopes(0)
    ref = case.run_oracle(dtype, keep_masks=True)
    _check_slopes(case, slopes, counts, ref)
    assert np.array_equal(m_last, mask_bits(ref["masks"][-1], case.inst))
    rel = rel_l2(cmds, ref["commands"])
    deq = rel_l2(cmds, case.run_oracle(dtype, dequantized=True)["commands"])
    log(f"  rel L2 max {rel.max():.3e}; vs dequantised {deq.max():.3e}")
    assert deq.max() <= DEQ_TOL
    assert rel.max() <= TOL[dtype]


def test_stream_mode_equals_batch_and_oracle(rtc):
    """Chunks submitted from host memory give the batch path's commands bit for bit."""
    case = Case("scao_sh_small", n_frames=40)
    log("case scao_sh_small stream vs batch 40 frames")
    with rtc.Engine([(case.inst, "f32")]) as eng:
        case.load(eng)
        got_stream, infos = run_stream(eng, 0, case)
        eng.set_state(0, None, None, 0)
        got_batch, _, _ = run_batch(eng, 0, case)
    assert np.array_equal(got_stream, got_batch)
    ref = case.run_oracle("f32")
    assert rel_l2(got_stream, ref["commands"]).max() <= TOL["f32"]
    assert all(i["t_ready_ns"] >= i["t_last_chunk_ns"] > 0 for i in infos)


def test_polc_with_device_formed_M(rtc):
    """M = R.D formed once in FP64 on the device; POLC-on commands against the oracle."""
    import synth
    wfs = synth.ShWfs(nsub=24, px=10, obs=0.28, frame_h=240, frame_w=240, n_chunks=6)
    inst = synth.Instance("polc_mid", (wfs,), 700, ("f32",), polc=True, gain=0.4, leak=0.01)
    wl = synth.Workload(91, "polc_mid", (inst,), n_frames=30, bank=30)
    synth.workloads.WORKLOADS["polc_mid"] = wl
    try:
        case = Case("polc_mid", n_frames=30, polc_m="from_D")
    finally:
        del synth.workloads.WORKLOADS["polc_mid"]
    log("case polc_mid (D given) 30 frames")
    with rtc.Engine([(case.inst, "f32")]) as eng:
        case.load(eng)
        cmds, _, _ = run_batch(eng, 0, case)
        a, p, nf = eng.get_state(0)
    ref = case.run_oracle("f32")
    rel = rel_l2(cmds, ref["commands"])
    log(f"  max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL["f32"]
    # the stored POLC term is M a_last
    p_ref = case.oracle_M() @ ref["commands"][-1]
    assert np.linalg.norm(p - p_ref) / np.linalg.norm(p_ref) <= TOL["f32"]
    assert nf == 30


def test_abi_errors(rtc):
    case = Case("scao_sh_small", n_frames=2)
    with rtc.Engine([(case.inst, "f32")]) as eng:
        img = case.frames[0][0]
        r0, r1 = eng.chunk_rows(0, 0, 0)
        # submit before the matrices are loaded
        assert eng.submit_status(0, 0, 0, 0, img[r0:r1]) == -5
        with pytest.raises(rtc.RtcError):
            eng.process_frames(0, [], 0)
        case.load(eng)
        assert eng.submit_status(1, 0, 0, 0, img[r0:r1]) == -1     # bad instance
        assert eng.submit_status(0, 3, 0, 0, img[r0:r1]) == -1     # bad sensor
        assert eng.submit_status(0, 0, 0, 1, img[r0:r1]) == -1     # chunk out of order
        assert eng.submit_status(0, 0, 5, 0, img[r0:r1]) == 0
        assert eng.submit_status(0, 0, 4, 0, img[r0:r1]) == -7     # older frame
        assert eng.wait_status(0, 5, 0.01) == -4                   # incomplete: timeout
        assert eng.submit_status(0, 0, 6, 0, img[r0:r1]) == 0      # frame 5 dropped
        assert eng.wait_status(0, 5, 0.01) == -7
