"""Plain CPU oracle of the adaptive-optics pixel -> command path.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library or its binding.
It shares no code with the GPU path.  Every function cites the paper passage
it follows; see ``oracle.pipeline``.
"""
from .pipeline import (apply_threshold, bf16_decode, bf16_encode, calibrate, dequantize,
                       fp8_decode, fp8_encode, integrate, mvm, polc_matrix, pyr_slopes,
                       quantize, run, sh_blocks, sh_cog, sh_slopes, wfs_slopes)

__all__ = [n for n in dir() if not n.startswith("_")]
