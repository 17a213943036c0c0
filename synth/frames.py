"""Seeded synthetic camera frames and detector calibration maps.

This module is a forward model of the detector only: it turns spot positions
or phase gradients into uint16 pixel values.  It performs none of the
controller's arithmetic (no calibration, centroiding or reconstruction).

Shack-Hartmann recipe (per valid subaperture, per frame): a pixel-integrated
Gaussian spot (sigma 1.2 px) displaced by U(-2, 2) px in x and y, 500 expected
photo-electrons, Poisson photon noise, a fixed per-pixel gain G ~ 1 + N(0,
0.02^2), a fixed dark map ~ N(100, 2^2) ADU, read noise N(0, 3^2), gain 1
e-/ADU, rounded and clipped to uint16.  Pixels outside valid subapertures
receive dark + read noise only.

Pyramid recipe: a random phase with a |k|^(-11/6) amplitude spectrum on the
pupil grid, its finite-difference gradients scaled so that their largest
magnitude over the pupil is 0.5, and quadrant intensities
(F/4)(1 + sx_q gx + sy_q gy) with sign patterns (+,+), (+,-), (-,+), (-,-)
for I1..I4, 100 expected photo-electrons per quadrant pixel; then the same
gain, dark, Poisson and read-noise model.

The detector calibration handed to the controller is the measured dark map
and ``flat = 1/G`` (float32), a zero background, the threshold and zero
reference slopes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import erf

from .workloads import PyrWfs, ShWfs, Workload, seed_for

__all__ = ["Calibration", "make_calibration", "sh_frames", "pyr_frames",
           "sh_spot_offsets", "sensor_inputs"]

# purposes in seed keys
_FRAMES, _CALIB, _RMAT, _DMAT, _OFFS = 0, 1, 2, 3, 4


@dataclass
class Calibration:
    dark: np.ndarray       # float32 (H, W)
    flat: np.ndarray       # float32 (H, W)
    bg: np.ndarray         # float32 (H, W)
    thr: np.ndarray        # float32 (n_units,) for SH, (1,) for pyramid
    ref: np.ndarray        # float32 (2*n_units,) reference slopes
    gain_map: np.ndarray   # float64 (H, W) the true per-pixel gain G
    dark_true: np.ndarray  # float64 (H, W)


def make_calibration(wl: Workload, wfs, key: tuple) -> Calibration:
    rng = np.random.Generator(np.random.PCG64(seed_for(*key, _CALIB)))
    h, w = wfs.frame_h, wfs.frame_w
    dark = wl.dark_mean + wl.dark_sigma * rng.standard_normal((h, w))
    gain = 1.0 + wl.flat_sigma * rng.standard_normal((h, w))
    n = wfs.n_units
    thr_len = n if wfs.kind == "sh" else 1
    return Calibration(
        dark=dark.astype(np.float32),
        flat=(1.0 / gain).astype(np.float32),
        bg=np.zeros((h, w), np.float32),
        thr=np.full(thr_len, wfs.threshold, np.float32),
        ref=np.zeros(2 * n, np.float32),
        gain_map=gain,
        dark_true=dark,
    )


def _finish(photons: np.ndarray, cal: Calibration, wl: Workload,
            rng: np.random.Generator) -> np.ndarray:
    """Detector: Poisson electrons -> gain -> dark -> read noise -> uint16."""
    e = rng.poisson(photons).astype(np.float64)
    noise = wl.read_noise * rng.standard_normal(photons.shape)
    raw = np.rint(cal.dark_true + cal.gain_map * e + noise)
    return np.clip(raw, 0, 65535).astype(np.uint16)


def sh_spot_offsets(wfs: ShWfs, n: int, rng: np.random.Generator) -> np.ndarray:
    """(n, n_units, 2) spot displacements (dx, dy) in pixels."""
    return rng.uniform(-wfs.max_offset, wfs.max_offset, size=(n, wfs.n_units, 2))


def _integrated_gaussian(p: int, centre: np.ndarray, sigma: float) -> np.ndarray:
    """Fraction of a unit Gaussian falling in pixels [i, i+1), i < p."""
    edges = np.arange(p + 1, dtype=np.float64)
    z = (edges[None, :] - centre[:, None]) / (sigma * np.sqrt(2.0))
    return 0.5 * np.diff(erf(z), axis=1)


def sh_frames(wl: Workload, wfs: ShWfs, cal: Calibration, n: int, key: tuple,
              offsets: np.ndarray | None = None) -> np.ndarray:
    """(n, H, W) uint16 Shack-Hartmann frames."""
    rng = np.random.Generator(np.random.PCG64(seed_for(*key, _FRAMES)))
    if offsets is None:
        orng = np.random.Generator(np.random.PCG64(seed_for(*key, _OFFS)))
        offsets = sh_spot_offsets(wfs, n, orng)
    p, ns = wfs.px, wfs.nsub
    oy, ox = wfs.origin
    valid = wfs.valid
    out = np.empty((n, wfs.frame_h, wfs.frame_w), np.uint16)
    for f in range(n):
        cx = p / 2.0 + offsets[f, :, 0]
        cy = p / 2.0 + offsets[f, :, 1]
        px_x = _integrated_gaussian(p, cx, wfs.spot_sigma)
        px_y = _integrated_gaussian(p, cy, wfs.spot_sigma)
        spots = wfs.photons * px_y[:, :, None] * px_x[:, None, :]
        grid = np.zeros((ns, ns, p, p))
        grid[valid] = spots
        img = np.zeros((wfs.frame_h, wfs.frame_w))
        img[oy:oy + ns * p, ox:ox + ns * p] = grid.transpose(0, 2, 1, 3).reshape(ns * p, ns * p)
        out[f] = _finish(img, cal, wl, rng)
    return out


def _phase_gradients(npx: int, valid: np.ndarray, rng: np.random.Generator):
    m = 2 * npx
    white = rng.standard_normal((m, m))
    k = np.fft.fftfreq(m)
    kk = np.hypot(k[:, None], k[None, :])
    amp = np.zeros_like(kk)
    amp[kk > 0] = kk[kk > 0] ** (-11.0 / 6.0)
    phase = np.fft.ifft2(np.fft.fft2(white) * amp).real[:npx, :npx]
    gy, gx = np.gradient(phase)
    peak = max(np.abs(gx[valid]).max(), np.abs(gy[valid]).max())
    return 0.5 * gx / peak, 0.5 * gy / peak


def pyr_frames(wl: Workload, wfs: PyrWfs, cal: Calibration, n: int, key: tuple) -> np.ndarray:
    """(n, 240, 240) uint16 pyramid frames."""
    rng = np.random.Generator(np.random.PCG64(seed_for(*key, _FRAMES)))
    prng = np.random.Generator(np.random.PCG64(seed_for(*key, _OFFS)))
    npx, valid = wfs.pupil_px, wfs.valid
    signs = ((1, 1), (1, -1), (-1, 1), (-1, -1))
    out = np.empty((n, wfs.frame_h, wfs.frame_w), np.uint16)
    for f in range(n):
        gx, gy = _phase_gradients(npx, valid, prng)
        img = np.zeros((wfs.frame_h, wfs.frame_w))
        for (r0, c0), (sx, sy) in zip(wfs.quad_origins, signs):
            inten = wfs.photons_per_px * (1.0 + sx * gx + sy * gy)
            img[r0:r0 + npx, c0:c0 + npx] = np.where(valid, inten, 0.0)
        out[f] = _finish(img, cal, wl, rng)
    return out


def sensor_inputs(wl: Workload, inst_index: int, wfs_index: int, n: int | None = None):
    """(frames, calibration) for one sensor of one instance of a workload."""
    inst = wl.instances[inst_index]
    wfs = inst.wfs[wfs_index]
    key = (wl.index, inst_index, wfs_index)
    cal = make_calibration(wl, wfs, key)
    n = wl.bank if n is None else n
    if wfs.kind == "sh":
        frames = sh_frames(wl, wfs, cal, n, key)
    else:
        frames = pyr_frames(wl, wfs, cal, n, key)
    return frames, cal
