"""MI355X (gfx950) hot path of an adaptive-optics real-time controller.

Shack-Hartmann pixel calibration (dark, flat, threshold), centre-of-gravity
slopes, control-matrix x slope-vector reconstruction and an integrator, as hand-
written HIP kernels behind the C ABI in ``include/rtc.h``.

* :mod:`paper_1805_07254_amd.rtc`   -- ctypes binding, same names as the C ABI
* :mod:`paper_1805_07254_amd.stats` -- frame-time / latency / jitter statistics
* :mod:`paper_1805_07254_amd.build` -- builds ``librtc.so`` with hipcc
"""
