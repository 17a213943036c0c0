"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a number printed in the paper,
a closed form, an exact-arithmetic recomputation, a brute-force enumeration
or an invariant.  All run on the CPU.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _facts():
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        return json.load(f)


# ------------------------------------------------------------------ geometry
def test_valid_subaps_match_paper_count():
    """4616 valid subapertures at 80x80 (section 2.3, Table 1)."""
    facts = _facts()
    for samples in (8, 16, 32, 64, 128):
        assert synth.subap_valid(80, 0.2875, samples).sum() == facts["sh80_valid_subaps"]["value"]
    wl = synth.get_workload("mcao_80")
    lgs = wl.instances[0].wfs[0]
    assert lgs.n_units == facts["sh80_valid_subaps"]["value"]
    assert lgs.n_slopes == facts["sh80_slopes"]["value"]
    assert lgs.frame_h == facts["sh80_image"]["value"]
    assert lgs.px == facts["sh80_pixels_per_subap"]["value"]


def test_actuator_totals_match_table1():
    facts = _facts()
    assert synth.get_workload("scao_sh_74").instances[0].n_act == facts["scao_actuators"]["value"]
    assert synth.get_workload("mcao_74").instances[0].n_act == facts["mcao_actuators"]["value"]
    assert synth.get_workload("ltao_68").instances[0].n_act == facts["ltao_actuators"]["value"]
    assert synth.get_workload("scao_pyr_92").instances[0].wfs[0].frame_h == facts["pyr_image"]["value"]


def test_workload_unit_counts():
    assert synth.get_workload("scao_sh_small").instances[0].wfs[0].n_units == 192
    assert synth.get_workload("scao_sh_small").instances[0].n_act == 232
    assert synth.get_workload("scao_sh_74").instances[0].wfs[0].n_units == 3972
    assert synth.get_workload("scao_pyr_92").instances[0].wfs[0].n_units == 6144
    assert synth.get_workload("ltao_68").instances[0].wfs[0].n_units == 3356
    assert synth.get_workload("ltao_68").instances[0].wfs[6].n_units == 48
    assert synth.get_workload("mcao_74").instances[0].n_slopes == 47688
    assert synth.get_workload("ltao_68").instances[0].n_slopes == 40368


# ------------------------------------------------------------------ calibration
def _f32_rne(x: Fraction) -> Fraction:
    """Exact round-to-nearest-even of a rational to IEEE binary32 (normal range)."""
    if x == 0:
        return Fraction(0)
    a = abs(x)
    e = math.floor(math.log2(a))
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    q = Fraction(2) ** (e - 23)
    k = round(a / q)               # Fraction.__round__ rounds half to even
    return (k * q) if x > 0 else -(k * q)


def test_calibration_is_binary32_per_operation():
    """Three roundings, no fused multiply-add: checked in exact rational arithmetic."""
    rng = np.random.default_rng(7)
    n = 3000
    raw = rng.integers(0, 65536, n).astype(np.uint16)
    dark = (100 + 7 * rng.standard_normal(n)).astype(np.float32)
    flat = (1 / (1 + 0.05 * rng.standard_normal(n))).astype(np.float32)
    bg = (3 * rng.standard_normal(n)).astype(np.float32)
    got = oracle.calibrate(raw, dark, flat, bg)
    fused_differs = 0
    for i in range(n):
        t = _f32_rne(Fraction(int(raw[i])) - Fraction(float(dark[i])))
        u = _f32_rne(t * Fraction(float(flat[i])))
        c = _f32_rne(u - Fraction(float(bg[i])))
        assert Fraction(float(got[i])) == c, i
        fused = _f32_rne(t * Fraction(float(flat[i])) - Fraction(float(bg[i])))
        fused_differs += fused != c
    assert fused_differs > 0   # the sample distinguishes fused from unfused


def test_threshold_tie_and_modes():
    c = np.array([9.0, 10.0, 10.5, 200.0], np.float32)
    w, m = oracle.apply_threshold(c, np.float32(10.0), "subtract")
    assert m.tolist() == [False, False, True, True]       # c == T is not above T
    assert w.tolist() == [0.0, 0.0, 0.5, 190.0]
    w, m = oracle.apply_threshold(c, np.float32(10.0), "zero")
    assert w.tolist() == [0.0, 0.0, 10.5, 200.0]
    w, m = oracle.apply_threshold(c, np.float32(10.0), "none")
    assert m.all() and w.tolist() == c.tolist()


# ------------------------------------------------------------------ SH centre of gravity
def test_uniform_subap_gives_zero_slope_exactly():
    w = np.full((5, 10, 10), 37.0)
    assert np.all(oracle.sh_cog(w) == 0.0)


def test_zero_flux_gives_zero_slope():
    w = np.zeros((3, 6, 6))
    w[1, 2, 3] = 5.0
    s = oracle.sh_cog(w, ref=np.full(6, 0.25))
    assert s[0] == 0 and s[1] == 0 and s[4] == 0 and s[5] == 0
    assert s[2] == pytest.approx(3 - 2.5 - 0.25) and s[3] == pytest.approx(2 - 2.5 - 0.25)


def test_gaussian_spot_centroid_equals_offset():
    """Pixel-integrated Gaussian on a wide window: CoG = offset up to aliasing ~1e-12."""
    from scipy.special import erf
    rng = np.random.default_rng(3)
    p, sigma = 32, 1.2
    d = rng.uniform(-2, 2, size=(20, 2))
    edges = np.arange(p + 1, dtype=np.float64)

    def prof(mu):
        z = (edges - mu) / (sigma * np.sqrt(2))
        return 0.5 * np.diff(erf(z))

    w = np.stack([np.outer(prof(p / 2 + dy), prof(p / 2 + dx)) for dx, dy in d])
    s = oracle.sh_cog(w).reshape(-1, 2)
    assert np.abs(s - d).max() < 1e-10


def test_centroid_through_uint16_within_rounding_bound():
    """Integer-rounded spot: |dCoG| <= 0.5 sum|x_i - d| / (F - 0.5 N) (rounding error bound)."""
    from scipy.special import erf
    p, sigma, peak = 16, 1.2, 6e4
    edges = np.arange(p + 1, dtype=np.float64)
    x = np.arange(p) - (p - 1) / 2
    for dx, dy in [(0.3, -0.7), (1.25, 0.5), (-1.9, 1.1)]:
        fx = 0.5 * np.diff(erf((edges - p / 2 - dx) / (sigma * np.sqrt(2))))
        fy = 0.5 * np.diff(erf((edges - p / 2 - dy) / (sigma * np.sqrt(2))))
        img = np.rint(peak * np.outer(fy, fx) / (fx.max() * fy.max()))
        s = oracle.sh_cog(img[None]).reshape(2)
        flux = img.sum()
        bx = 0.5 * p * np.abs(x - dx).sum() / (flux - 0.5 * p * p)
        by = 0.5 * p * np.abs(x - dy).sum() / (flux - 0.5 * p * p)
        assert abs(s[0] - dx) <= bx and abs(s[1] - dy) <= by


def test_centroid_brute_force_2x2():
    w = np.array([[[1.0, 3.0], [0.0, 4.0]]])
    # columns at x = -0.5, +0.5 ; rows at y = -0.5, +0.5
    F = 8.0
    sx = (1 * -0.5 + 3 * 0.5 + 0 * -0.5 + 4 * 0.5) / F
    sy = (1 * -0.5 + 3 * -0.5 + 0 * 0.5 + 4 * 0.5) / F
    assert oracle.sh_cog(w).tolist() == [sx, sy]


def test_sh_pipeline_recovers_generator_offsets():
    """End to end through the detector model: slopes track the drawn spot offsets in x and y."""
    wl = synth.get_workload("scao_sh_74")
    wfs = wl.instances[0].wfs[0]
    key = (wl.index, 0, 0)
    cal = synth.make_calibration(wl, wfs, key)
    rng = np.random.default_rng(11)
    offs = rng.uniform(-1.5, 1.5, size=(1, wfs.n_units, 2))
    frame = synth.sh_frames(wl, wfs, cal, 1, key, offsets=offs)[0]
    s, counts, masks = oracle.sh_slopes(frame, wfs, cal)
    s = s.reshape(-1, 2)
    err = s - offs[0]
    assert np.sqrt((err ** 2).mean()) < 0.15
    assert np.corrcoef(s[:, 0], offs[0, :, 0])[0, 1] > 0.98
    assert np.corrcoef(s[:, 1], offs[0, :, 1])[0, 1] > 0.98
    assert counts.min() > 0 and counts.max() <= 100
    assert np.array_equal(counts, masks.sum(axis=(1, 2)))


# ------------------------------------------------------------------ pyramid
def _pyr_cal(wfs, thr=0.0):
    h, w = wfs.frame_h, wfs.frame_w
    return synth.Calibration(dark=np.zeros((h, w), np.float32), flat=np.ones((h, w), np.float32),
                             bg=np.zeros((h, w), np.float32), thr=np.array([thr], np.float32),
                             ref=np.zeros(2 * wfs.n_units, np.float32),
                             gain_map=np.ones((h, w)), dark_true=np.zeros((h, w)))


def test_pyramid_linear_surrogate_exact():
    """I_q = (F/4)(1 + sx_q g_x + sy_q g_y) gives Sx = g_x and Sy = g_y exactly."""
    wfs = synth.PyrWfs()
    rng = np.random.default_rng(5)
    n = wfs.pupil_px
    gx = rng.integers(-32, 33, (n, n)) / 64.0
    gy = rng.integers(-32, 33, (n, n)) / 64.0
    img = np.zeros((wfs.frame_h, wfs.frame_w))
    for (r0, c0), (sx, sy) in zip(wfs.quad_origins, ((1, 1), (1, -1), (-1, 1), (-1, -1))):
        img[r0:r0 + n, c0:c0 + n] = 64.0 * (1 + sx * gx + sy * gy)
    s, counts, _ = oracle.pyr_slopes(img, wfs, _pyr_cal(wfs))
    s = s.reshape(-1, 2)
    assert np.array_equal(s[:, 0], gx[wfs.valid])
    assert np.array_equal(s[:, 1], gy[wfs.valid])
    assert np.all(counts == 4)


def test_pyramid_global_normalisation():
    """One sum over the pupil: in the linear surrogate every pixel's four images
    add to F (the gradient terms cancel), so S = N F and (Sx, Sy) = (g_x, g_y) / N
    exactly for N valid pixels; uniform images still give 0; a pupil of one
    valid pixel gives the local slopes."""
    import dataclasses
    wfs = dataclasses.replace(synth.PyrWfs(), norm="global")
    rng = np.random.default_rng(6)
    n = wfs.pupil_px
    gx = rng.integers(-32, 33, (n, n)) / 64.0
    gy = rng.integers(-32, 33, (n, n)) / 64.0
    img = np.zeros((wfs.frame_h, wfs.frame_w))
    for (r0, c0), (sx, sy) in zip(wfs.quad_origins, ((1, 1), (1, -1), (-1, 1), (-1, -1))):
        img[r0:r0 + n, c0:c0 + n] = 64.0 * (1 + sx * gx + sy * gy)
    s = oracle.pyr_slopes(img, wfs, _pyr_cal(wfs))[0].reshape(-1, 2)
    N = int(wfs.valid.sum())
    assert np.abs(s[:, 0] - gx[wfs.valid] / N).max() <= 1e-15
    assert np.abs(s[:, 1] - gy[wfs.valid] / N).max() <= 1e-15
    assert np.all(oracle.pyr_slopes(np.full_like(img, 80.0), wfs, _pyr_cal(wfs))[0] == 0)
    local = synth.PyrWfs()
    one = np.zeros_like(wfs.valid)
    one[n // 2, 3] = True
    wl_ = dataclasses.replace(local, pupil_px=n)
    g1 = type("W", (), {})()
    for k in ("pupil_px", "quad_origins", "thr_mode", "frame_h", "frame_w"):
        setattr(g1, k, getattr(wl_, k))
    g1.valid, g1.n_units, g1.norm = one, 1, "global"
    l1 = type("W", (), {})()
    for k in ("pupil_px", "quad_origins", "thr_mode", "frame_h", "frame_w"):
        setattr(l1, k, getattr(wl_, k))
    l1.valid, l1.n_units, l1.norm = one, 1, "local"
    cal = _pyr_cal(wl_)
    cal1 = synth.Calibration(dark=cal.dark, flat=cal.flat, bg=cal.bg, thr=cal.thr,
                             ref=np.zeros(2, np.float32), gain_map=cal.gain_map,
                             dark_true=cal.dark_true)
    noisy = rng.uniform(10, 200, img.shape)
    assert np.array_equal(oracle.pyr_slopes(noisy, g1, cal1)[0], oracle.pyr_slopes(noisy, l1, cal1)[0])


def test_pyramid_quadrant_signs():
    """Light in one pupil image only: (Sx, Sy) = (+,+) I1, (+,-) I2, (-,+) I3, (-,-) I4."""
    wfs = synth.PyrWfs()
    n = wfs.pupil_px
    for q, expect in enumerate([(1, 1), (1, -1), (-1, 1), (-1, -1)]):
        img = np.zeros((wfs.frame_h, wfs.frame_w))
        r0, c0 = wfs.quad_origins[q]
        img[r0:r0 + n, c0:c0 + n] = 50.0
        s = oracle.pyr_slopes(img, wfs, _pyr_cal(wfs))[0].reshape(-1, 2)
        assert np.all(s[:, 0] == expect[0]) and np.all(s[:, 1] == expect[1])
    img = np.full((wfs.frame_h, wfs.frame_w), 80.0)
    assert np.all(oracle.pyr_slopes(img, wfs, _pyr_cal(wfs))[0] == 0)
    assert np.all(oracle.pyr_slopes(np.zeros_like(img), wfs, _pyr_cal(wfs))[0] == 0)


def test_pyramid_needs_lower_half():
    """Only pupil rows whose lower-quadrant row has arrived change the slopes (section 2.2)."""
    wfs = synth.PyrWfs()
    rng = np.random.default_rng(2)
    img = rng.uniform(50, 150, (wfs.frame_h, wfs.frame_w))
    s0 = oracle.pyr_slopes(img, wfs, _pyr_cal(wfs))[0]
    img2 = img.copy()
    img2[134 + 92:, :] += 1000.0       # rows below every pupil image
    assert np.array_equal(s0, oracle.pyr_slopes(img2, wfs, _pyr_cal(wfs))[0])


# ------------------------------------------------------------------ quantisers
def test_bf16_hand_encodings():
    v = np.array([1.0, -2.0, 3.140625, 1.00390625, 1.01171875, 65504.0], np.float32)
    # 1+2^-8 is a tie between 1 (0x3F80) and 1+2^-7 (0x3F81): even -> 0x3F80;
    # 1+3*2^-8 is a tie between 0x3F81 and 0x3F82: even -> 0x3F82
    assert oracle.bf16_encode(v).tolist() == [0x3F80, 0xC000, 0x4049, 0x3F80, 0x3F82, 0x4780]


def test_bf16_is_nearest_brute_force():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-3, 3, 20000)).astype(np.float32)
    h = oracle.bf16_encode(x)
    bits = x.view(np.uint32)
    lo = (bits & 0xFFFF0000).view(np.float32).astype(np.float64)
    hi = ((bits & 0xFFFF0000) + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    got = oracle.bf16_decode(h).astype(np.float64)
    xd = x.astype(np.float64)
    best = np.minimum(np.abs(xd - lo), np.abs(xd - hi))
    assert np.all(np.abs(xd - got) == best)


def test_fp8_hand_encodings():
    v = np.array([1.0, 448.0, -0.0078125, 1.0625, 1.1875, 0.0, 2.0 ** -9, -2.0 ** -10], np.float64)
    # 1.0625 ties 1.0/1.125 -> even mantissa 0 ; 1.1875 ties 1.125/1.25 -> even mantissa 2
    # 2^-9 is the smallest subnormal; -2^-10 ties 0 / 2^-9 -> even (0) -> negative zero
    assert oracle.fp8_encode(v).tolist() == [0x38, 0x7E, 0x84, 0x38, 0x3A, 0x00, 0x01, 0x80]
    assert oracle.fp8_decode(np.array([0x7E, 0x08, 0x07, 0xB8], np.uint8)).tolist() == \
        [448.0, 2.0 ** -6, 7 * 2.0 ** -9, -1.0]


def test_fp8_is_nearest_codebook_entry():
    """Brute force over all finite e4m3fn values; ties go to the even code."""
    codes = np.arange(256, dtype=np.uint8)
    vals = oracle.fp8_decode(codes)
    fin = ~np.isnan(vals)
    book_c, book_v = codes[fin], vals[fin]
    assert book_v.max() == 448.0 and fin.sum() == 254
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-448, 448, 4000), rng.uniform(-0.05, 0.05, 4000),
                        book_v, (book_v[:-1] + book_v[1:]) / 2])
    x = np.clip(x.astype(np.float32), -448, 448)
    got = oracle.fp8_encode(x)
    for xi, gi in zip(x.astype(np.float64), got):
        d = np.abs(book_v - xi)
        cand = book_c[d == d.min()]
        vals_c = oracle.fp8_decode(cand)
        if len(set(vals_c.tolist())) == 1 and vals_c[0] != 0:
            assert gi in cand
        elif vals_c[0] == 0 and len(set(vals_c.tolist())) == 1:
            assert oracle.fp8_decode(np.array([gi], np.uint8))[0] == 0
        else:
            even = [c for c in cand if (c & 1) == 0]
            assert gi in even


def test_fp8_row_scale_uses_full_range():
    rng = np.random.default_rng(9)
    R = rng.standard_normal((50, 300)).astype(np.float32)
    R[7] = 0
    codes, scale = oracle.quantize(R, "fp8")
    assert scale.dtype == np.float32 and scale[7] == 1.0
    mags = codes & 0x7F
    assert np.all(mags[np.arange(50) != 7].max(axis=1) == 0x7E)
    deq = oracle.dequantize(codes, scale, "fp8")
    assert np.all(deq[7] == 0)
    keep = np.arange(50) != 7
    rel = np.abs(deq - R)[keep] / np.abs(R[keep]).max(axis=1, keepdims=True)
    assert rel.max() <= 16.0 / 448.0 * 1.0001     # half the top-binade quantum (32) / 448


# ------------------------------------------------------------------ reconstruction
def test_mvm_brute_force_integers():
    rng = np.random.default_rng(0)
    R = rng.integers(-5, 6, (7, 13)).astype(np.float32)
    s = rng.integers(-9, 10, 13).astype(np.float64)
    y = oracle.mvm(R, s)
    for i in range(7):
        acc = 0
        for j in range(13):
            acc += int(R[i, j]) * int(s[j])
        assert y[i] == acc


def test_mvm_linearity():
    rng = np.random.default_rng(1)
    R = rng.standard_normal((40, 90)).astype(np.float32)
    s1, s2 = rng.standard_normal(90), rng.standard_normal(90)
    lhs = oracle.mvm(R, 0.75 * s1 - 1.5 * s2)
    rhs = 0.75 * oracle.mvm(R, s1) - 1.5 * oracle.mvm(R, s2)
    assert np.abs(lhs - rhs).max() <= 1e-14 * np.abs(rhs).max()


# ------------------------------------------------------------------ integrator and POLC
def _tiny_instance(polc=False, switch=None, gain=0.4, leak=0.01, n_act=12):
    wfs = synth.ShWfs(nsub=4, px=6, obs=0.0, frame_h=24, frame_w=24, n_chunks=2)
    inst = synth.Instance("tiny", (wfs,), n_act, ("f32",), polc=polc, gain=gain, leak=leak,
                          switch=switch)
    wl = synth.Workload(90, "tiny", (inst,), n_frames=1, bank=1)
    frames, cal = synth.sensor_inputs(wl, 0, 0, n=1)
    rng = np.random.default_rng(12)
    R = (rng.standard_normal((n_act, wfs.n_slopes)) / np.sqrt(wfs.n_slopes)).astype(np.float32)
    return inst, frames, cal, R


def test_integrator_closed_form_repeated_frame():
    """POLC off, identical frames: a_n = (1 - (1-leak)^n) (gain/leak) R s."""
    inst, frames, cal, R = _tiny_instance()
    n = 1000
    out = oracle.run(inst, [frames], [cal], R, n)
    s = out["slopes"][0]
    g, lam = float(np.float32(0.4)), float(np.float32(0.01))
    for k in (1, 2, 10, 1000):
        expect = (1 - (1 - lam) ** k) * (g / lam) * (R.astype(np.float64) @ s)
        assert np.abs(out["commands"][k - 1] - expect).max() <= 1e-12 * np.abs(expect).max()


def test_integrator_gain_leak_switch_closed_form():
    k = 40
    inst, frames, cal, R = _tiny_instance(switch=(k, 0.3, 0.02))
    out = oracle.run(inst, [frames], [cal], R, 120)
    y = R.astype(np.float64) @ out["slopes"][0]
    a_k = out["commands"][k - 1]
    g2, l2 = float(np.float32(0.3)), float(np.float32(0.02))
    for n in (k + 1, k + 7, 120):
        m = n - k
        expect = (1 - l2) ** m * a_k + (1 - (1 - l2) ** m) * (g2 / l2) * y
        assert np.abs(out["commands"][n - 1] - expect).max() <= 1e-12 * np.abs(expect).max()


def test_polc_fixed_point():
    """a* = g (leak I + g I - g M)^-1 R s, from an independent float64 solve."""
    inst, frames, cal, R = _tiny_instance(polc=True, gain=0.5, leak=0.05)
    rng = np.random.default_rng(3)
    D = rng.standard_normal((R.shape[1], R.shape[0])) * 0.5 / np.sqrt(R.shape[0])
    M = oracle.polc_matrix(R, D)
    out = oracle.run(inst, [frames], [cal], R, 3000, M=M)
    y = R.astype(np.float64) @ out["slopes"][0]
    g, lam = float(np.float32(0.5)), float(np.float32(0.05))
    n = M.shape[0]
    a_star = np.linalg.solve(lam * np.eye(n) + g * np.eye(n) - g * M, g * y)
    assert np.abs(out["commands"][-1] - a_star).max() <= 1e-9 * np.abs(a_star).max()


def test_polc_with_identity_equals_plain_integrator():
    """With M = I the POLC recurrence reduces to the plain leaky integrator."""
    inst_p, frames, cal, R = _tiny_instance(polc=True)
    inst_o, _, _, _ = _tiny_instance(polc=False)
    a = oracle.run(inst_p, [frames], [cal], R, 50, M=np.eye(R.shape[0]))["commands"]
    b = oracle.run(inst_o, [frames], [cal], R, 50)["commands"]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_run_continues_another_run():
    """A run split at frame k and continued from its state (commands a_{k-1},
    POLC term M a_{k-1}, frame numbers from k) is the unsplit run."""
    k, n = 17, 45
    for polc in (False, True):
        inst, frames, cal, R = _tiny_instance(polc=polc, switch=(30, 0.3, 0.02))
        bank = np.concatenate([frames] * 3)                  # three identical frames
        rng = np.random.default_rng(5)
        M = (rng.standard_normal((R.shape[0], R.shape[0])) * 0.4 / np.sqrt(R.shape[0])
             if polc else None)
        whole = oracle.run(inst, [bank], [cal], R, n, M=M)["commands"]
        head = oracle.run(inst, [bank], [cal], R, k, M=M)["commands"]
        p0 = None if M is None else M @ head[-1]
        tail = oracle.run(inst, [bank], [cal], R, n - k, M=M, a0=head[-1], p0=p0,
                          f0=k)["commands"]
        assert np.array_equal(np.concatenate([head, tail]), whole)


def test_matrix_switch_closed_form():
    """POLC off, identical frames, reconstructor R1 for frames < k and R2 from
    k on: a_n = (1-leak)^(n-k+1) a_{k-1} + (1 - (1-leak)^(n-k+1)) (gain/leak) R2 s."""
    k, n = 25, 90
    inst, frames, cal, R1 = _tiny_instance()
    rng = np.random.default_rng(8)
    R2 = (rng.standard_normal(R1.shape) / np.sqrt(R1.shape[1])).astype(np.float32)
    head = oracle.run(inst, [frames], [cal], R1, k)
    tail = oracle.run(inst, [frames], [cal], R2, n - k, a0=head["commands"][-1], f0=k)
    y2 = R2.astype(np.float64) @ head["slopes"][0]
    g, lam = float(np.float32(0.4)), float(np.float32(0.01))
    a_prev = head["commands"][-1]
    for f in (k, k + 1, k + 9, n - 1):
        m = f - k + 1
        expect = (1 - lam) ** m * a_prev + (1 - (1 - lam) ** m) * (g / lam) * y2
        assert np.abs(tail["commands"][f - k] - expect).max() <= 1e-12 * np.abs(expect).max()


def test_polc_term_given_for_first_frame():
    """With POLC matrix I the recurrence is the plain integrator, so a first
    POLC term p0 = a0 continues the plain integrator exactly; any other p0
    enters the first frame as gain * p0 and decays through the same recurrence."""
    inst_p, frames, cal, R = _tiny_instance(polc=True)
    inst_o, _, _, _ = _tiny_instance(polc=False)
    rng = np.random.default_rng(21)
    a0 = rng.standard_normal(R.shape[0])
    eye = np.eye(R.shape[0])
    a = oracle.run(inst_p, [frames], [cal], R, 30, M=eye, a0=a0, p0=a0)["commands"]
    b = oracle.run(inst_o, [frames], [cal], R, 30, a0=a0)["commands"]
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    d = rng.standard_normal(R.shape[0])
    c = oracle.run(inst_p, [frames], [cal], R, 30, M=eye, a0=a0, p0=a0 + d)["commands"]
    g, lam = float(np.float32(0.4)), float(np.float32(0.01))
    for m in (1, 2, 30):
        expect = (1 - lam) ** (m - 1) * g * d
        assert np.abs((c - a)[m - 1] - expect).max() <= 1e-12 * np.abs(d).max()


def test_polc_matrix_brute_force_elements():
    """M = R D element by element from Python loops over small integer
    matrices (exact in float64): M[i, j] = sum_k R[i, k] D[k, j], with R
    n_act x n_s and D n_s x n_act.  The result is far from symmetric, so a
    transposed product, swapped operands or a dropped term fails."""
    rng = np.random.default_rng(31)
    n_act, n_s = 5, 7
    R = rng.integers(-9, 10, size=(n_act, n_s)).astype(np.float32)
    D = rng.integers(-9, 10, size=(n_s, n_act)).astype(np.float64)
    M = oracle.polc_matrix(R, D)
    assert M.shape == (n_act, n_act)
    for i in range(n_act):
        for j in range(n_act):
            expect = 0
            for k in range(n_s):
                expect += int(R[i, k]) * int(D[k, j])
            assert M[i, j] == expect
    assert not np.array_equal(M, M.T)


def test_polc_matrix_is_reconstruction_of_pseudo_open_loop_slopes():
    """Section 3.4: the POLC term is the reconstruction of the slopes that the
    applied commands produce: M a = R (D a) for any command vector a (two
    matrix-vector products, associativity), and a D that maps commands onto
    slopes the reconstructor inverts (R D = I on the commands) gives M = I."""
    rng = np.random.default_rng(32)
    n_act, n_s = 9, 20
    R = rng.standard_normal((n_act, n_s)).astype(np.float32)
    D = rng.standard_normal((n_s, n_act))
    M = oracle.polc_matrix(R, D)
    for _ in range(3):
        a = rng.standard_normal(n_act)
        lhs = M @ a
        rhs = oracle.mvm(R, oracle.mvm(D, a))
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    # D = right inverse of R: the pseudo-open-loop slopes of commands a
    # reconstruct to a itself
    Rd = R.astype(np.float64)
    D_inv = Rd.T @ np.linalg.inv(Rd @ Rd.T)
    assert np.abs(oracle.polc_matrix(R, D_inv) - np.eye(n_act)).max() <= 1e-12
    with pytest.raises(ValueError):
        oracle.polc_matrix(R, D.T)


def test_run_refuses_polc_without_its_matrix():
    inst, frames, cal, R = _tiny_instance(polc=True)
    with pytest.raises(ValueError):
        oracle.run(inst, [frames], [cal], R, 2)
