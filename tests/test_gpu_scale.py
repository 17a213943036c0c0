"""GPU parity at the ELT scale of the MCAO and LTAO configurations.

The serving frame loop runs the full-size instances (nine or seven sensors,
the 6318 x 47688 and 5330 x 40368 matrices, implicit POLC) from the pinned
host ring, and every frame's commands are compared with the oracle: to the
storage type's tolerance against the FP32-matrix oracle, and to 1e-5 against
the oracle run on the dequantised matrix (the kernels' own exactness).
"""
import numpy as np
import pytest

import oracle
import synth
from rtc_cases import DEQ_TOL, TOL, Case, log, rel_l2, run_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rtc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_01852_amd import rtc as mod
    mod.lib()
    return mod


@pytest.fixture(scope="module")
def mcao():
    log("building MCAO 6 LGS 74x74 + 3 NGS 2x2 inputs (6318 x 47688)")
    return Case("mcao_74", n_frames=6)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_mcao_serving_vs_oracle(rtc, mcao, dtype):
    case = mcao
    log(f"case mcao_74 {dtype}: serving loop, 6 frames, POLC")
    with rtc.Engine([(case.inst, dtype)], mode="persistent") as eng:
        case.load(eng)
        got, infos = run_stream(eng, 0, case)
    ref = case.run_oracle(dtype)
    deq = case.run_oracle(dtype, dequantized=True)
    rel = rel_l2(got, ref["commands"])
    rel_d = rel_l2(got, deq["commands"])
    log(f"  max rel L2 {rel.max():.3e} (dequantised {rel_d.max():.3e})")
    assert rel.max() <= TOL[dtype]
    assert rel_d.max() <= DEQ_TOL
    assert all(i["dev_ticks_cmd"] >= i["dev_ticks_start"] > 0 for i in infos)


@pytest.fixture(scope="module")
def mcao80():
    log("building MCAO 6 LGS 80x80 + 3 NGS 2x2 inputs (6318 x 55416, the paper's LGS size)")
    return Case("mcao_80", n_frames=4)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_mcao80_serving_vs_oracle(rtc, mcao80, dtype):
    case = mcao80
    log(f"case mcao_80 {dtype}: serving loop, 4 frames, POLC")
    with rtc.Engine([(case.inst, dtype)], mode="persistent") as eng:
        case.load(eng)
        got, _ = run_stream(eng, 0, case)
    ref = case.run_oracle(dtype)
    deq = case.run_oracle(dtype, dequantized=True)
    rel = rel_l2(got, ref["commands"])
    rel_d = rel_l2(got, deq["commands"])
    log(f"  max rel L2 {rel.max():.3e} (dequantised {rel_d.max():.3e})")
    assert rel.max() <= TOL[dtype]
    assert rel_d.max() <= DEQ_TOL


def test_ltao_and_scao_in_one_launch_with_switch(rtc):
    """LTAO (POLC) beside the SCAO instance of uneven size in one persistent
    launch, the LTAO gain and leak switched through the API between frames."""
    n, k = 6, 3
    ltao = Case("ltao_68", 0, n_frames=n)
    scao = Case("ltao_68", 1, n_frames=n)
    log("case ltao_68 + scao_sh_74 in one launch, FP32, switch after frame 3")
    gain2, leak2 = ltao.inst.switch[1], ltao.inst.switch[2]
    with rtc.Engine([(ltao.inst, "f32"), (scao.inst, "f32")], mode="persistent") as eng:
        ltao.load(eng, 0)
        scao.load(eng, 1)
        got = {0: [], 1: []}
        for f in range(n):
            if f == k:
                assert eng.set_params(0, gain2, leak2) == k
            for idx, case in ((0, ltao), (1, scao)):
                for w in range(len(case.inst.wfs)):
                    img = case.frames[w][f]
                    for c in range(case.inst.wfs[w].n_chunks):
                        r0, r1 = eng.chunk_rows(idx, w, c)
                        eng.submit_chunk(idx, w, f, c, img[r0:r1])
            for idx in (0, 1):
                got[idx].append(eng.wait_commands(idx, f, timeout_s=10.0)[0].astype(np.float64))
    inst2 = synth.Instance(ltao.inst.name, ltao.inst.wfs, ltao.inst.n_act, ("f32",),
                           polc=True, gain=ltao.inst.gain, leak=ltao.inst.leak,
                           switch=(k, gain2, leak2))
    ref_l = oracle.run(inst2, ltao.frames, ltao.cals, ltao.R, n, M=ltao.oracle_M())
    ref_s = scao.run_oracle("f32")
    rl = rel_l2(np.stack(got[0]), ref_l["commands"])
    rs = rel_l2(np.stack(got[1]), ref_s["commands"])
    log(f"  LTAO max rel L2 {rl.max():.3e}, SCAO {rs.max():.3e}")
    assert rl.max() <= TOL["f32"]
    assert rs.max() <= TOL["f32"]
