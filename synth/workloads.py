"""Workload definitions: sensor layouts, mirror sizes, controller settings.

Sizes follow the paper's Table 1 and section 2.3 (80x80 and 74x74 SH grids
with 10x10 pixels, 5318 = 5316 + 2 actuators for M4 + M5, 2 x 500 extra
actuators for the MCAO post-focal DMs, 6 x 2 for LTAO tip-tilt, a pyramid on a
240x240 frame with four pupil images).  Every input built from these
definitions is synthetic; the AO-simulation images the paper streamed from
disk are not available.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import cached_property

import numpy as np

from .geometry import fried_actuators, pupil_pixels, subap_valid

ROOT_SEED = 190301852

__all__ = ["ShWfs", "PyrWfs", "Instance", "Workload", "WORKLOADS", "get_workload",
           "ROOT_SEED", "seed_for"]


def seed_for(*key: int) -> np.random.SeedSequence:
    """Independent, stable seed for a (workload, instance, wfs, purpose) key."""
    return np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(int(k) for k in key))


@dataclass(frozen=True)
class ShWfs:
    """Shack-Hartmann sensor: ``nsub x nsub`` subapertures of ``px x px`` pixels."""
    nsub: int
    px: int
    obs: float
    frame_h: int
    frame_w: int
    origin: tuple = (0, 0)          # (row, col) of subaperture (0,0)'s first pixel
    n_chunks: int = 16              # row chunks the camera delivers per frame
    threshold: float = 10.0         # ADU, one value per valid subaperture
    thr_mode: str = "subtract"      # "subtract" | "zero" | "none"
    photons: float = 500.0          # expected photo-electrons per spot
    spot_sigma: float = 1.2         # px
    max_offset: float = 2.0         # spot offsets ~ U(-max, max) px
    kind: str = field(default="sh", init=False)

    @cached_property
    def valid(self) -> np.ndarray:
        return subap_valid(self.nsub, self.obs)

    @property
    def n_units(self) -> int:
        return int(self.valid.sum())

    @property
    def n_slopes(self) -> int:
        return 2 * self.n_units


@dataclass(frozen=True)
class PyrWfs:
    """Pyramid sensor: four ``pupil_px`` pupil images on one frame.

    Quadrant origins are (row, col) of I1 top-left, I2 bottom-left, I3
    top-right, I4 bottom-right.
    """
    pupil_px: int = 92
    obs: float = 0.28
    frame_h: int = 240
    frame_w: int = 240
    quad_origins: tuple = ((14, 14), (134, 14), (14, 134), (134, 134))
    n_chunks: int = 16
    threshold: float = 0.0
    thr_mode: str = "none"
    photons_per_px: float = 100.0   # expected photo-electrons per quadrant pixel
    norm: str = "local"             # "local": per-pixel sum; "global": sum over the pupil
    kind: str = field(default="pyr", init=False)

    @cached_property
    def valid(self) -> np.ndarray:
        return pupil_pixels(self.pupil_px, self.obs)

    @property
    def n_units(self) -> int:
        return int(self.valid.sum())

    @property
    def n_slopes(self) -> int:
        return 2 * self.n_units


@dataclass(frozen=True)
class Instance:
    """One controller: a set of sensors driving one command vector."""
    name: str
    wfs: tuple
    n_act: int
    cm_dtypes: tuple = ("f32",)
    polc: bool = False
    gain: float = 0.4
    leak: float = 0.01
    switch: tuple | None = None     # (first frame of new params, gain, leak)

    @property
    def n_slopes(self) -> int:
        return sum(w.n_slopes for w in self.wfs)


@dataclass(frozen=True)
class Workload:
    index: int
    name: str
    instances: tuple
    n_frames: int
    bank: int                       # unique frames pre-generated per sensor
    dark_mean: float = 100.0
    dark_sigma: float = 2.0
    read_noise: float = 3.0
    flat_sigma: float = 0.02


def _lgs(nsub: int, px: int = 10, obs: float = 0.28, n_chunks: int = 16) -> ShWfs:
    return ShWfs(nsub=nsub, px=px, obs=obs, frame_h=nsub * px, frame_w=nsub * px,
                 n_chunks=n_chunks)


_SMALL = ShWfs(nsub=16, px=8, obs=0.30, frame_h=128, frame_w=128, n_chunks=4)
_NGS_2 = ShWfs(nsub=2, px=16, obs=0.28, frame_h=32, frame_w=32, n_chunks=2)
_NGS_8 = ShWfs(nsub=8, px=16, obs=0.28, frame_h=128, frame_w=128, n_chunks=4)

_small_act = int(fried_actuators(subap_valid(16, 0.30)).sum())   # 232

WORKLOADS = {
    "scao_sh_small": Workload(
        0, "scao_sh_small",
        (Instance("scao_small", (_SMALL,), _small_act, ("f32",)),),
        n_frames=1000, bank=1000),
    "scao_sh_74": Workload(
        1, "scao_sh_74",
        (Instance("scao_sh", (_lgs(74),), 5318, ("f32", "bf16", "fp8")),),
        n_frames=10000, bank=256),
    "scao_pyr_92": Workload(
        2, "scao_pyr_92",
        (Instance("scao_pyr", (PyrWfs(),), 5318, ("f32", "bf16", "fp8")),),
        n_frames=10000, bank=256),
    "mcao_74": Workload(
        3, "mcao_74",
        (Instance("mcao", tuple([_lgs(74)] * 6 + [_NGS_2] * 3), 5316 + 2 + 2 * 500,
                  ("bf16", "fp8"), polc=True),),
        n_frames=20000, bank=64),
    "ltao_68": Workload(
        4, "ltao_68",
        (Instance("ltao", tuple([_lgs(68)] * 6 + [_NGS_8]), 5316 + 2 + 6 * 2,
                  ("f32", "bf16", "fp8"), polc=True, switch=(10000, 0.3, 0.02)),
         Instance("scao_sh", (_lgs(74),), 5318, ("f32", "bf16", "fp8"))),
        n_frames=20000, bank=64),
    # the paper's own LGS size (80x80 subapertures on an 800x800 frame)
    "mcao_80": Workload(
        5, "mcao_80",
        (Instance("mcao80", tuple([_lgs(80, obs=0.2875)] * 6 + [_NGS_2] * 3),
                  5316 + 2 + 2 * 500, ("bf16", "fp8"), polc=True),),
        n_frames=20000, bank=64),
}


def get_workload(name: str) -> Workload:
    try:
        return WORKLOADS[name]
    except KeyError:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}") from None
