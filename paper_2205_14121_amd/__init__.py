"""MI355X-native (gfx950) engine for the DPD + CGMD multiple-time-stepping hot path of
"AI-aided multiscale modeling of physiologically-significant blood clots"
(arXiv 2205.14121): HIP kernels behind the C ABI of include/aimts.h, with a thin
ctypes binding in ``paper_2205_14121_amd.aimts``.
"""
__all__ = ["aimts"]
