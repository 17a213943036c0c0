"""GPU tests of the persistent frame loop (RTC_MODE_PERSISTENT).

The frame loop must give bit for bit the commands of the per-launch path (the
same partials summed in the same order), and match the oracle to the same
bars as the per-launch path.
"""
import numpy as np
import pytest

import oracle
import synth
from rtc_cases import TOL, Case, log, mid_case, rel_l2, run_batch, run_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01852_amd import rtc as mod
    mod.lib()
    return mod


def _mid_case(polc: bool, n_frames: int = 30, polc_m: str = "from_D", index: int = 92):
    return mid_case(polc, n_frames, polc_m, index)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_frame_loop_batch_equals_launch_path(rtc, dtype):
    case = Case("scao_sh_74", n_frames=6)
    log(f"case scao_sh_74 {dtype}: frame loop vs per-launch, 6 frames")
    with rtc.Engine([(case.inst, dtype)], mode="stream") as e1:
        case.load(e1)
        c1, s1, n1 = run_batch(e1, 0, case)
    with rtc.Engine([(case.inst, dtype)], mode="persistent") as e2:
        case.load(e2)
        c2, s2, n2 = run_batch(e2, 0, case)
    assert np.array_equal(n1, n2)
    assert np.array_equal(s1, s2)
    assert np.array_equal(c1, c2)


def test_frame_loop_small_sh_vs_oracle(rtc):
    case = Case("scao_sh_small", n_frames=200)
    log("case scao_sh_small frame loop 200 frames")
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        cmds, slopes, counts = run_batch(eng, 0, case)
        a, p, nf = eng.get_state(0)
    ref = case.run_oracle("f32")
    assert np.array_equal(counts, ref["counts"])
    assert np.abs(slopes - ref["slopes"]).max() <= 1e-4
    rel = rel_l2(cmds, ref["commands"])
    log(f"  max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL["f32"]
    assert np.array_equal(a, cmds[-1].astype(np.float32)) and nf == 200


def test_frame_loop_pyramid_equals_launch_path(rtc):
    case = Case("scao_pyr_92", n_frames=5)
    log("case scao_pyr_92 bf16 frame loop vs per-launch")
    outs = []
    for mode in ("stream", "persistent"):
        with rtc.Engine([(case.inst, "bf16")], mode=mode) as eng:
            case.load(eng)
            outs.append(run_batch(eng, 0, case))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_frame_loop_polc_vs_oracle_and_launch_path(rtc):
    case = _mid_case(True, n_frames=30)
    log("case mid POLC (D given) frame loop, 30 frames")
    outs = []
    for mode in ("stream", "persistent"):
        with rtc.Engine([(case.inst, "f32")], mode=mode) as eng:
            case.load(eng)
            outs.append(run_batch(eng, 0, case))
    assert np.array_equal(outs[0][0], outs[1][0])
    ref = case.run_oracle("f32")
    rel = rel_l2(outs[1][0], ref["commands"])
    log(f"  max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL["f32"]


def test_frame_loop_batches_continue_state(rtc):
    """Two back-to-back batches equal one batch of both (state carried on the device)."""
    import torch
    case = _mid_case(True, n_frames=20, index=93)
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        whole, _, _ = run_batch(eng, 0, case)
        eng.set_state(0, None, None, 0)
        dfr = [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in case.frames]
        out = torch.zeros((20, case.inst.n_act), dtype=torch.float32, device="cuda")
        st = torch.cuda.current_stream()
        eng.process_frames(0, [d[:7].contiguous() for d in dfr], 7, cmds=out[:7], stream=st)
        eng.process_frames(0, [d[7:].contiguous() for d in dfr], 13, cmds=out[7:], stream=st)
        torch.cuda.synchronize()
    assert np.array_equal(whole, out.cpu().numpy().astype(np.float64))


def test_serving_frame_loop_equals_batch(rtc):
    """Chunks through the pinned ring and doorbells give the batch commands bit for bit."""
    case = Case("scao_sh_small", n_frames=40)
    log("case scao_sh_small serving frame loop, 40 frames")
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        served, infos = run_stream(eng, 0, case)
        eng.set_state(0, None, None, 0)
        batch, _, _ = run_batch(eng, 0, case)
    assert np.array_equal(served, batch)
    assert all(i["t_ready_ns"] >= i["t_last_chunk_ns"] > 0 for i in infos)
    assert all(i["dev_ticks_cmd"] >= i["dev_ticks_start"] > 0 for i in infos)
    ref = case.run_oracle("f32")
    assert rel_l2(served, ref["commands"]).max() <= TOL["f32"]


def test_serving_two_instances_uneven_sizes(rtc):
    """Two instances of different sizes share one frame loop; each gives its solo commands."""
    big = _mid_case(True, n_frames=12, index=94)
    small = Case("scao_sh_small", n_frames=12)
    log("case two instances (mid POLC + small) in one frame loop")
    solo = []
    for case in (big, small):
        with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
            case.load(eng)
            solo.append(run_stream(eng, 0, case)[0])
    with rtc.Engine([(big.inst, "f32"), (small.inst, "f32")], mode="persistent") as eng:
        big.load(eng, 0)
        small.load(eng, 1)
        got = {0: [], 1: []}
        for f in range(12):
            # interleave the two cameras chunk by chunk
            plans = []
            for idx, case in ((0, big), (1, small)):
                img = case.frames[0][f]
                for c in range(case.inst.wfs[0].n_chunks):
                    r0, r1 = eng.chunk_rows(idx, 0, c)
                    plans.append((idx, c, img[r0:r1]))
            plans.sort(key=lambda x: x[1])
            for idx, c, rows in plans:
                eng.submit_chunk(idx, 0, f, c, rows)
            for idx in (0, 1):
                got[idx].append(eng.wait_commands(idx, f)[0].astype(np.float64))
    assert np.array_equal(np.stack(got[0]), solo[0])
    assert np.array_equal(np.stack(got[1]), solo[1])


def test_serving_gain_leak_switch(rtc):
    """rtc_set_params between frames: the oracle's switch closed form, frame for frame."""
    case = Case("scao_sh_small", n_frames=30)
    k = 12
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        first, _ = run_stream(eng, 0, case, n=k)
        f_eff = eng.set_params(0, 0.3, 0.02)
        assert f_eff == k
        rest, _ = run_stream(eng, 0, case, n=30 - k, first_frame=k)
    got = np.concatenate([first, rest])
    inst2 = synth.Instance(case.inst.name, case.inst.wfs, case.inst.n_act, ("f32",),
                           gain=case.inst.gain, leak=case.inst.leak, switch=(k, 0.3, 0.02))
    ref = oracle.run(inst2, case.frames, case.cals, case.R, 30)
    rel = rel_l2(got, ref["commands"])
    log(f"  max rel L2 {rel.max():.3e}")
    assert rel.max() <= TOL["f32"]


def test_serving_dropped_frame(rtc):
    """A frame superseded before its last chunk leaves the commands untouched."""
    case = Case("scao_sh_small", n_frames=8)
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        got = []
        for f in range(8):
            img = case.frames[0][f]
            n_ch = case.inst.wfs[0].n_chunks
            last = 1 if f == 3 else n_ch          # frame 3 delivers only its first chunk
            for c in range(last):
                r0, r1 = eng.chunk_rows(0, 0, c)
                eng.submit_chunk(0, 0, f, c, img[r0:r1])
            if f != 3:
                got.append(eng.wait_commands(0, f)[0].astype(np.float64))
        assert eng.wait_status(0, 3, 0.1) == -7
    kept = [0, 1, 2, 4, 5, 6, 7]
    frames = [case.frames[0][kept]]
    ref = oracle.run(case.inst, frames, case.cals, case.R, 7)
    assert rel_l2(np.stack(got), ref["commands"]).max() <= TOL["f32"]


def _odd_width_case(n_frames: int = 10):
    """Two sensors whose frame widths are not multiples of 8 (ring rows padded)."""
    a = synth.ShWfs(nsub=12, px=9, obs=0.3, frame_h=111, frame_w=115, origin=(2, 5), n_chunks=5)
    b = synth.ShWfs(nsub=6, px=10, obs=0.28, frame_h=60, frame_w=61, n_chunks=3)
    inst = synth.Instance("odd93", (a, b), 260, ("f32",), gain=0.5, leak=0.02)
    wl = synth.Workload(93, "odd93", (inst,), n_frames=n_frames, bank=n_frames)
    synth.workloads.WORKLOADS[wl.name] = wl
    try:
        return Case(wl.name, n_frames=n_frames)
    finally:
        del synth.workloads.WORKLOADS[wl.name]


def _run_zero_copy(eng, idx, case, n=None):
    """Serving path through rtc_acquire_chunk / rtc_commit_chunk."""
    out = []
    for f in range(case.n if n is None else n):
        for w, bank in enumerate(case.frames):
            img = bank[f % bank.shape[0]]
            for c in range(case.inst.wfs[w].n_chunks):
                r0, r1 = eng.chunk_rows(idx, w, c)
                view = eng.acquire_chunk(idx, w, f, c)
                assert view.shape == (r1 - r0, img.shape[1])
                view[...] = img[r0:r1]
                eng.commit_chunk(idx, w, f, c)
        out.append(eng.wait_commands(idx, f, timeout_s=10.0)[0].astype(np.float64))
    return np.stack(out)


@pytest.mark.parametrize("name", ["scao_sh_small", "odd"])
def test_serving_zero_copy_equals_copy_form(rtc, name):
    """Chunks written in place into the lent ring slot give the copy-form commands
    bit for bit, also where ring rows are padded past the frame width."""
    case = _odd_width_case() if name == "odd" else Case(name, n_frames=12)
    log(f"case {name} serving zero-copy chunk hand-off")
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        copied, _ = run_stream(eng, 0, case)
        eng.set_state(0, None, None, 0)
        lent = _run_zero_copy(eng, 0, case)
    assert np.array_equal(lent, copied)
    ref = case.run_oracle("f32")
    assert rel_l2(lent, ref["commands"]).max() <= TOL["f32"]


def test_zero_copy_rules(rtc):
    """One lent chunk per sensor; commits must name it; stream mode refuses; a
    newer frame started meanwhile makes the commit report the drop."""
    case = Case("scao_sh_small", n_frames=4)
    img = case.frames[0]
    with rtc.Engine([(case.inst, "f32")], mode="stream") as eng:
        case.load(eng)
        with pytest.raises(rtc.RtcError) as ei:
            eng.acquire_chunk(0, 0, 0, 0)
        assert ei.value.status == -5
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        r0, r1 = eng.chunk_rows(0, 0, 0)
        v = eng.acquire_chunk(0, 0, 0, 0)
        v[...] = img[0][r0:r1]
        assert eng.submit_status(0, 0, 0, 1, img[0][r0:r1]) == -1   # chunk 0 still lent
        assert eng.commit_status(0, 0, 0, 1) == -1                   # names another chunk
        eng.commit_chunk(0, 0, 0, 0)
        assert eng.commit_status(0, 0, 0, 0) == -1                   # nothing lent now
        for c in range(1, case.inst.wfs[0].n_chunks):
            a, b = eng.chunk_rows(0, 0, c)
            eng.submit_chunk(0, 0, 0, c, img[0][a:b])
        first = eng.wait_commands(0, 0)[0]
        # frame 1: chunk 0 lent, then frame 2 starts through the copy form
        v = eng.acquire_chunk(0, 0, 1, 0)
        assert eng.submit_status(0, 0, 2, 0, img[2][r0:r1]) == -1    # lent chunk blocks
        v[...] = img[1][r0:r1]
        eng.commit_chunk(0, 0, 1, 0)
        for c in range(case.inst.wfs[0].n_chunks):
            a, b = eng.chunk_rows(0, 0, c)
            eng.submit_chunk(0, 0, 2, c, img[2][a:b])
        assert eng.wait_status(0, 1, 0.1) == -7
        third = eng.wait_commands(0, 2)[0]
    ref = oracle.run(case.inst, [img[[0, 2]]], case.cals, case.R, 2)
    assert rel_l2(np.stack([first, third]).astype(np.float64), ref["commands"]).max() <= TOL["f32"]


def test_zero_copy_commit_after_newer_frame(rtc):
    """A chunk lent on one sensor while another sensor starts a newer frame: the
    commit reports the drop, and the newer frame's commands are the oracle's."""
    case = _odd_width_case(n_frames=3)
    with rtc.Engine([(case.inst, "f32")], mode="persistent") as eng:
        case.load(eng)
        got = []
        for f in (0, 2):
            if f == 2:
                r0, r1 = eng.chunk_rows(0, 0, 0)
                v = eng.acquire_chunk(0, 0, 1, 0)            # frame 1, sensor 0, lent
                v[...] = case.frames[0][1][r0:r1]
                a, b = eng.chunk_rows(0, 1, 0)
                eng.submit_chunk(0, 1, 1, 0, case.frames[1][1][a:b])
                eng.submit_chunk(0, 1, 2, 0, case.frames[1][2][a:b])   # supersedes frame 1
                assert eng.commit_status(0, 0, 1, 0) == -7
                assert eng.wait_status(0, 1, 0.1) == -7
            for w in (0, 1):
                for c in range(case.inst.wfs[w].n_chunks):
                    if f == 2 and w == 1 and c == 0:
                        continue
                    a, b = eng.chunk_rows(0, w, c)
                    eng.submit_chunk(0, w, f, c, case.frames[w][f][a:b])
            got.append(eng.wait_commands(0, f)[0].astype(np.float64))
    frames = [fr[[0, 2]] for fr in case.frames]
    ref = oracle.run(case.inst, frames, case.cals, case.R, 2)
    assert rel_l2(np.stack(got), ref["commands"]).max() <= TOL["f32"]
