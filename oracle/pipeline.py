"""Plain CPU oracle of the per-frame pixel -> command path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and imports nothing from it.

Arithmetic: detector calibration is carried out in IEEE binary32 (one rounding
per operation, no fused multiply-add), because the thresholded-pixel masks are
compared bit for bit; every later step runs in float64.

Paper passages followed (Jenkins, Basden & Myers, "A many-core CPU prototype
of an MCAO and LTAO RTC for ELT-scale instruments"):

* the four per-sensor stages, calibration -> slopes -> reconstruction -> DM
  command, and the summation of per-sensor partial commands (section 1.1,
  figure of the four main AO-loop processes; section 3, master node);
* Shack-Hartmann slopes as the centre of gravity of the pixels of each
  subaperture, pyramid slopes as normalised differences of corresponding
  pixels of the four pupil images, four pixels per slope (section 2.2 and the
  figure comparing SH and pyramid pipelining);
* reconstruction as one dense control-matrix x slope-vector product
  (section 2.3, the 5318 x 9232 MVM);
* implicit pseudo-open-loop control as one extra matrix-vector product on the
  summed command, computed for the next frame (section 3.4);
* run-time parameter changes taking effect at a frame boundary (section 3.2).

Readings where the paper is silent (each is listed in the design notes):
calibration order dark -> flat -> background then threshold; ``c > T``
strict; per-subaperture thresholds; CoG coordinates centred on the
subaperture (x_i = i - (p-1)/2); zero flux gives zero slope without reference
subtraction; quadrant labels I1 top-left, I2 bottom-left, I3 top-right, I4
bottom-right with per-pixel (local) normalisation; integrator
a_f = (1-leak-gain) a_{f-1} + gain (R s_f + M a_{f-1}) with POLC and
a_f = (1-leak) a_{f-1} + gain R s_f without; BF16 round-to-nearest-even;
FP8 as OCP e4m3fn with a per-row scale max|R_r|/448.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "calibrate", "sh_blocks", "apply_threshold", "sh_cog", "sh_slopes",
    "pyr_slopes", "bf16_encode", "bf16_decode", "fp8_encode", "fp8_decode",
    "quantize", "dequantize", "mvm", "integrate", "polc_matrix", "run",
]

THR_MODES = ("subtract", "zero", "none")


# ---------------------------------------------------------------- calibration
def calibrate(raw: np.ndarray, dark: np.ndarray, flat: np.ndarray,
              bg: np.ndarray) -> np.ndarray:
    """Detector calibration in binary32: ((raw - dark) * flat) - bg.

    Section 2.3 names pixel calibration as the first per-sensor stage; the
    operation order is a reading.  numpy float32 ufuncs round once per
    operation and never fuse.
    """
    t = np.subtract(raw.astype(np.float32), dark, dtype=np.float32)
    u = np.multiply(t, flat, dtype=np.float32)
    return np.subtract(u, bg, dtype=np.float32)


def apply_threshold(c: np.ndarray, thr, mode: str):
    """Returns (w float32, mask bool).  ``mask = c > T`` (strict).

    subtract: w = c - T where masked, else 0;  zero: w = c where masked;
    none: w = c, every pixel masked.
    """
    if mode == "none":
        return c.astype(np.float32, copy=True), np.ones(c.shape, bool)
    thr = np.asarray(thr, np.float32)
    mask = c > thr
    if mode == "subtract":
        w = np.where(mask, np.subtract(c, thr, dtype=np.float32), np.float32(0))
    elif mode == "zero":
        w = np.where(mask, c, np.float32(0))
    else:
        raise ValueError(f"unknown threshold mode {mode!r}")
    return w.astype(np.float32), mask


# ---------------------------------------------------------------- Shack-Hartmann
def sh_blocks(img: np.ndarray, wfs) -> np.ndarray:
    """(n_units, p, p) pixel blocks of the valid subapertures, raster order."""
    p, ns = wfs.px, wfs.nsub
    oy, ox = wfs.origin
    sub = img[oy:oy + ns * p, ox:ox + ns * p]
    blocks = sub.reshape(ns, p, ns, p).transpose(0, 2, 1, 3)
    return blocks[wfs.valid]


def sh_cog(w: np.ndarray, ref: np.ndarray | None = None) -> np.ndarray:
    """Centre of gravity of each (p, p) block, in pixels, interleaved (x, y).

    Section 2.2: a Shack-Hartmann slope is the centre of gravity of the pixel
    values in its subaperture.  Coordinates x_i = i - (p-1)/2; a block whose
    flux is <= 0 gives (0, 0).
    """
    w = w.astype(np.float64)
    n, p, _ = w.shape
    x = np.arange(p, dtype=np.float64) - (p - 1) / 2.0
    flux = w.sum(axis=(1, 2))
    sx = (w * x[None, None, :]).sum(axis=(1, 2))
    sy = (w * x[None, :, None]).sum(axis=(1, 2))
    out = np.zeros((n, 2))
    ok = flux > 0
    out[ok, 0] = sx[ok] / flux[ok]
    out[ok, 1] = sy[ok] / flux[ok]
    if ref is not None:
        r = np.asarray(ref, np.float64).reshape(n, 2)
        out[ok] -= r[ok]
    return out.reshape(-1)


def sh_slopes(raw: np.ndarray, wfs, cal):
    """Calibrate, threshold and centroid one SH frame.

    Returns (slopes float64 (2n,), counts int32 (n,), masks bool (n, p, p)).
    """
    c = calibrate(raw, cal.dark, cal.flat, cal.bg)
    blocks = sh_blocks(c, wfs)
    thr = np.asarray(cal.thr, np.float32).reshape(-1, 1, 1)
    w, mask = apply_threshold(blocks, thr, wfs.thr_mode)
    slopes = sh_cog(w, cal.ref)
    return slopes, mask.sum(axis=(1, 2)).astype(np.int32), mask


# ---------------------------------------------------------------- pyramid
def pyr_slopes(raw: np.ndarray, wfs, cal):
    """Pyramid slopes for each valid pupil pixel, interleaved (Sx, Sy).

    Section 2.2: a pyramid slope is formed from the relative x and y
    differences of corresponding pixels of the four pupil images, four pixels
    per slope.  Sx = (I1 + I2 - I3 - I4) / S and Sy = (I1 + I3 - I2 - I4) / S
    with the local sum S = I1 + I2 + I3 + I4 (wfs.norm "local"), or with one
    sum S over every valid pupil pixel of the four images ("global"); S <= 0
    gives (0, 0).
    Returns (slopes, counts of masked quadrant pixels per pupil pixel, masks
    (n, 4)).
    """
    c = calibrate(raw, cal.dark, cal.flat, cal.bg)
    npx, valid = wfs.pupil_px, wfs.valid
    quads = []
    masks = []
    for (r0, c0) in wfs.quad_origins:
        q = c[r0:r0 + npx, c0:c0 + npx][valid]
        w, m = apply_threshold(q, np.float32(cal.thr[0]), wfs.thr_mode)
        quads.append(w.astype(np.float64))
        masks.append(m)
    i1, i2, i3, i4 = quads
    s = i1 + i2 + i3 + i4
    if getattr(wfs, "norm", "local") == "global":
        s = np.full_like(s, s.sum())
    n = s.shape[0]
    out = np.zeros((n, 2))
    ok = s > 0
    out[ok, 0] = (i1 + i2 - i3 - i4)[ok] / s[ok]
    out[ok, 1] = (i1 + i3 - i2 - i4)[ok] / s[ok]
    if cal.ref is not None:
        out[ok] -= np.asarray(cal.ref, np.float64).reshape(n, 2)[ok]
    m = np.stack(masks, axis=1)
    return out.reshape(-1), m.sum(axis=1).astype(np.int32), m


def wfs_slopes(raw, wfs, cal):
    if wfs.kind == "sh":
        return sh_slopes(raw, wfs, cal)
    return pyr_slopes(raw, wfs, cal)


# ---------------------------------------------------------------- quantisation
def bf16_encode(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest, ties to even."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_decode(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32)


def fp8_decode(code: np.ndarray) -> np.ndarray:
    """OCP e4m3fn codes -> float64 (sign, 4 exponent bits with bias 7, 3 mantissa bits)."""
    code = np.asarray(code, np.uint8).astype(np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 0xF
    m = code & 0x7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return s * val


def fp8_encode(x: np.ndarray) -> np.ndarray:
    """float32 values in [-448, 448] -> e4m3fn codes, round to nearest, ties to even.

    The quantum of a value with exponent e >= -6 is 2^(e-3); below 2^-6 it is
    2^-9 (subnormals).  Rounding |x| / quantum to the nearest integer with
    ties to even and re-assembling gives the code; a mantissa carry into the
    next binade lands on the right code because codes are ordered like values.
    """
    x = np.asarray(x, np.float64)
    if np.any(np.abs(x) > 448.0) or np.any(~np.isfinite(x)):
        raise ValueError("fp8_encode expects finite values within +-448")
    a = np.abs(x)
    e = np.where(a > 0, np.floor(np.log2(np.where(a > 0, a, 1.0))), -6.0)
    e = np.maximum(e, -6.0)
    quantum = np.exp2(e - 3.0)
    k = np.rint(a / quantum)                 # np.rint rounds half to even
    # code = (e + 7) * 8 + (k - 8) for normals; = k for the subnormal binade
    code = np.where(e > -6, (e + 7.0) * 8.0 + (k - 8.0), k)
    code = code.astype(np.int64)
    sign = np.where(np.signbit(x), 0x80, 0)
    return (code | sign).astype(np.uint8)


def quantize(R: np.ndarray, dtype: str):
    """Storage encoding of the float32 control matrix.

    f32: identity.  bf16: round-to-nearest-even bit patterns.  fp8: per-row
    scale s_r = max_j |R_rj| / 448 (float32; an all-zero row gets 1) and codes
    of R_rj / s_r (float32 division) clamped to +-448.
    Returns (codes, scale or None).
    """
    R = np.ascontiguousarray(R, np.float32)
    if dtype == "f32":
        return R, None
    if dtype == "bf16":
        return bf16_encode(R), None
    if dtype == "fp8":
        amax = np.abs(R).max(axis=1)
        scale = np.divide(amax, np.float32(448.0), dtype=np.float32)
        scale = np.where(amax > 0, scale, np.float32(1.0)).astype(np.float32)
        x = np.divide(R, scale[:, None], dtype=np.float32)
        x = np.clip(x, np.float32(-448.0), np.float32(448.0))
        return fp8_encode(x), scale
    raise ValueError(f"unknown matrix dtype {dtype!r}")


def dequantize(codes: np.ndarray, scale, dtype: str) -> np.ndarray:
    """float64 matrix represented by a storage encoding."""
    if dtype == "f32":
        return np.asarray(codes, np.float64)
    if dtype == "bf16":
        return bf16_decode(codes).astype(np.float64)
    if dtype == "fp8":
        return fp8_decode(codes) * np.asarray(scale, np.float64)[:, None]
    raise ValueError(dtype)


# ---------------------------------------------------------------- reconstruction
def mvm(R: np.ndarray, s: np.ndarray) -> np.ndarray:
    """y = R s in float64 (section 2.3: reconstruction is one dense MVM)."""
    return np.asarray(R, np.float64) @ np.asarray(s, np.float64)


def polc_matrix(R: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Implicit pseudo-open-loop operator M = R D, float64, computed once.

    Section 3.4: the pseudo-open-loop slopes add the slopes D a that the
    applied commands a produce (D: n_slopes x n_act, commands -> slopes) to
    the measured ones, and reconstructing them with R (n_act x n_slopes) adds
    R (D a) = M a to the reconstruction; M (n_act x n_act) is that composition,
    M[i, j] = sum_k R[i, k] D[k, j].
    """
    R = np.asarray(R, np.float64)
    D = np.asarray(D, np.float64)
    if R.ndim != 2 or D.ndim != 2 or R.shape[1] != D.shape[0] or R.shape[0] != D.shape[1]:
        raise ValueError(f"POLC needs R (n_act x n_s) and D (n_s x n_act), got {R.shape}, "
                         f"{D.shape}")
    return R @ D


def integrate(a_prev: np.ndarray, y: np.ndarray, gain: float, leak: float,
              p: np.ndarray | None = None) -> np.ndarray:
    """Leaky integrator, with the implicit POLC term when ``p`` is given.

    Without POLC: a_f = (1 - leak) a_{f-1} + gain y_f.
    With POLC:    a_f = (1 - leak - gain) a_{f-1} + gain (y_f + p_f),
    where p_f = M a_{f-1} (section 3.4: the POLC product is formed on the
    summed command, for the next frame).  Gain and leak are taken as float32
    parameters, widened exactly.
    """
    g = float(np.float32(gain))
    lam = float(np.float32(leak))
    if p is None:
        return (1.0 - lam) * a_prev + g * y
    return (1.0 - lam - g) * a_prev + g * (y + p)


def params_at(inst, f: int):
    if inst.switch is not None and f >= inst.switch[0]:
        return inst.switch[1], inst.switch[2]
    return inst.gain, inst.leak


def run(inst, frames, cals, R, n_frames: int, cm_dtype: str = "f32",
        M: np.ndarray | None = None, dequantized: bool = False,
        keep_masks: bool = False, a0: np.ndarray | None = None,
        p0: np.ndarray | None = None, f0: int = 0):
    """Run ``n_frames`` frames of one controller instance.

    frames[w] is a (B, H, W) uint16 bank for sensor w; frame f uses
    ``frames[w][f % B]``.  The slope vector concatenates the sensors in order.
    ``dequantized=True`` reconstructs with the dequantised storage matrix
    (checks the kernel independently of quantisation error); otherwise with
    the float32 reference matrix.
    ``a0`` is the command vector before the first frame (default zero);
    ``p0`` the POLC term of the first frame (default M a0: the product on the
    previous commands); frames are numbered from ``f0`` (bank index and
    parameter switch), so that a run can continue another one.
    Returns a dict with commands (n_frames, n_act), slopes, counts and,
    optionally, masks.
    """
    if inst.polc and M is None:
        raise ValueError("the instance has implicit POLC on: give its matrix M (n_act x n_act)")
    if dequantized:
        codes, scale = quantize(R, cm_dtype)
        Rm = dequantize(codes, scale, cm_dtype)
    else:
        Rm = np.asarray(R, np.float64)
    n_act = Rm.shape[0]
    a = np.zeros(n_act) if a0 is None else np.asarray(a0, np.float64).copy()
    cmds = np.empty((n_frames, n_act))
    slopes_all, counts_all, masks_all = [], [], []
    for f in range(f0, f0 + n_frames):
        parts_s, parts_c, parts_m = [], [], []
        for w, wfs in enumerate(inst.wfs):
            bank = frames[w]
            s, cnt, m = wfs_slopes(bank[f % bank.shape[0]], wfs, cals[w])
            parts_s.append(s)
            parts_c.append(cnt)
            parts_m.append(m)
        s = np.concatenate(parts_s)
        y = Rm @ s
        g, lam = params_at(inst, f)
        p = None
        if inst.polc:
            p = np.asarray(p0, np.float64) if (f == f0 and p0 is not None) else M @ a
        a = integrate(a, y, g, lam, p)
        cmds[f - f0] = a
        slopes_all.append(s)
        counts_all.append(np.concatenate(parts_c))
        if keep_masks:
            masks_all.append(parts_m)
    out = {"commands": cmds, "slopes": np.stack(slopes_all),
           "counts": np.stack(counts_all)}
    if keep_masks:
        out["masks"] = masks_all
    return out
