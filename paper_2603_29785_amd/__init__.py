"""MI355X-native QTAM: forward and inverse Q-transform with amplitude
demodulation (Asprea et al., arXiv 2603.29785) as hand-written HIP kernels for
gfx950 behind the C ABI of include/qtam.h.

``Plan`` builds a transform plan; ``Plan.forward`` / ``Plan.inverse`` run it on
device tensors. Importing this package loads libqtam.so and fails if it has not
been built (``python paper_2603_29785_amd/build.py``); there is no CPU fallback.
"""
from .binding import (Plan, PlanInfo, QtamError, lib, status_string, version, EXPORTED,  # noqa: F401
                      FP32, FP64, forward_sweep)

__all__ = ["Plan", "PlanInfo", "QtamError", "status_string", "version", "FP32", "FP64", "forward_sweep"]
