"""Seeded synthetic inputs (geometry, frames, calibration maps, matrices).

Shared by the oracle and by the GPU path's tests and benchmark.  Holds none of
the controller's arithmetic.
"""
from .geometry import fried_actuators, pupil_pixels, subap_valid
from .workloads import (ROOT_SEED, WORKLOADS, Instance, PyrWfs, ShWfs, Workload,
                        get_workload, seed_for)
from .frames import Calibration, make_calibration, pyr_frames, sensor_inputs, sh_frames
from .matrices import control_matrix, gaussian_matrix, interaction_matrix

__all__ = [n for n in dir() if not n.startswith("_")]
