"""MI355X-native hot path of an adaptive-optics real-time controller.

Pixels -> calibration -> Shack-Hartmann / pyramid slopes -> control-matrix
MVM -> implicit POLC + leaky integrator, in hand-written gfx950 kernels behind
the C ABI declared in ``include/rtc.h`` (library ``librtc.so`` in this
package).  ``paper_1903_01852_amd.rtc`` is the Python binding.
"""
__all__ = ["rtc", "build"]
