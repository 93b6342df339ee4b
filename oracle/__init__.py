"""FP64 CPU oracle of the dirty-imaging path. Test infrastructure only.

Only the tests, the package smoke check and the CPU-baseline leg of the
benchmark import this package; the HIP library never does.
"""
from .blink_oracle import *  # noqa: F401,F403
from .blink_oracle import (C_LIGHT, NATURAL, UNIFORM, NORM_NONE, NORM_WEIGHTS,  # noqa: F401
                           uv_scale, cell_index, apply_gains, dequantize, grid,
                           weight, fft_last_axis, fft2, dft_matrix, dft2_matrix,
                           shift_real_cut, image_one, image_batch, direct_image,
                           adjoint_one, adjoint_batch, fft_flops_estimate)
from . import kernel_gridding  # noqa: F401,E402
from . import dynamic_spectra  # noqa: F401,E402
from . import correlator  # noqa: F401,E402
from . import phase_rotation  # noqa: F401,E402
