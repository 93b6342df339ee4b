"""MI355X-native dirty imaging (grid + 2D inverse FFT per timestep x channel).

The compute lives in libblink.so (hand-written HIP for gfx950, C ABI in
include/blink.h); this package is its ctypes binding plus seeded synthetic
workloads.
"""
from .blink import (NATURAL, UNIFORM, NORM_NONE, NORM_WEIGHTS, VIS_C64, VIS_F16, VIS_BF16,  # noqa: F401
                    CALL_GRID, CALL_IMAGE, CALL_ADJOINT, EXPORTS, BlinkError, BlinkImage, Problem,
                    Inputs, blink_image, degrid_adjoint, fft2d, grid, image_batch, load_library,
                    status_string, supported_n, workspace, LIB_PATH, KCLASS, KernelTimes,
                    dynamic_spectra, REF_NONE, REF_MEAN, REF_MODEL, REF_MAX_LEN, correlate,
                    image_batch_noalloc, NOALLOC_SCRATCH_BYTES)

__all__ = ["image_batch", "grid", "fft2d", "degrid_adjoint", "BlinkImage", "blink_image",
           "dynamic_spectra", "correlate", "image_batch_noalloc", "load_library", "supported_n", "status_string"]
