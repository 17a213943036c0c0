"""Wavefront-sensor and deformable-mirror geometry used to configure workloads.

These masks are *inputs* to a real-time controller (in an AO system the
valid-subaperture map and the pupil-pixel map are configuration data given to
the controller), so they live here, beside the other seeded input generators,
and are handed to both the oracle and the GPU path.

Rules (the paper gives no rule, only counts; section 2.3 and Table 1 quote
4616 valid subapertures for an 80x80 Shack-Hartmann grid):

* A subaperture is valid when at least half of its area lies inside the
  annular pupil ``obs*D/2 <= r <= D/2``.  The area fraction is estimated by
  sampling an ``S x S`` grid of points inside the subaperture.  With
  ``obs = 0.2875`` an 80x80 grid gives exactly 4616 valid subapertures for
  every ``S`` from 8 to 128.
* An actuator of the ``(n+1) x (n+1)`` Fried grid is valid when it is a corner
  of at least one valid subaperture.
* A pyramid pupil pixel is valid when its centre lies in the annulus.
"""
from __future__ import annotations

import numpy as np

__all__ = ["subap_valid", "fried_actuators", "pupil_pixels"]


def subap_valid(nsub: int, obs: float, samples: int = 64) -> np.ndarray:
    """Boolean ``(nsub, nsub)`` map of valid subapertures, raster (row, col)."""
    if nsub <= 0:
        raise ValueError("nsub must be positive")
    off = (np.arange(samples) + 0.5) / samples
    c = nsub / 2.0
    r_out = nsub / 2.0
    r_in = obs * nsub / 2.0
    valid = np.zeros((nsub, nsub), dtype=bool)
    # one subaperture row at a time keeps memory at nsub*samples^2
    for i in range(nsub):
        yy = (i + off)[None, :, None] - c
        xx = (np.arange(nsub)[:, None] + off[None, :])[:, None, :] - c
        rr = np.hypot(yy, xx)
        inside = (rr <= r_out) & (rr >= r_in)
        valid[i] = inside.mean(axis=(1, 2)) >= 0.5
    return valid


def fried_actuators(valid: np.ndarray) -> np.ndarray:
    """Boolean ``(n+1, n+1)`` map of actuators that touch a valid subaperture."""
    n0, n1 = valid.shape
    a = np.zeros((n0 + 1, n1 + 1), dtype=bool)
    a[:-1, :-1] |= valid
    a[1:, :-1] |= valid
    a[:-1, 1:] |= valid
    a[1:, 1:] |= valid
    return a


def pupil_pixels(npx: int, obs: float) -> np.ndarray:
    """Boolean ``(npx, npx)`` map of pupil pixels whose centre is in the annulus."""
    c = npx / 2.0
    i = np.arange(npx) + 0.5
    rr = np.hypot(i[:, None] - c, i[None, :] - c)
    return (rr <= npx / 2.0) & (rr >= obs * npx / 2.0)
