"""CPU FP64 oracle for frame theoretic convolutional gridding (FTCG).

TEST INFRASTRUCTURE, NOT PRODUCT CODE. Only the test suite, the smoke check of
the package entry module and the CPU-baseline leg of the benchmark may import
or call anything in this package. The GPU library never calls it, and this
package imports nothing from the GPU library.

Every routine here is a plain, slow, direct implementation of what the paper
defines, in float64/complex128, with numpy/scipy primitives (bincount, FFT,
k-d tree, lstsq) as single steps and no blocking or reordering beyond the
definition. Each function cites the passage it follows (Sec. / equation label
of arXiv:1706.08575).
"""
from .ftcg_ref import (  # noqa: F401
    kernel_beta, grid_size, pixel_coords, nudft, nudft_at, frame_weights,
    frame_weights_at, spread, spread_window, grid_to_image, deapod_factors, ftcg_image, rel_l2,
    nudft_forward, image_to_grid, interpolate, forward,
)
from .band_ref import band_columns, band_dense, band_apply  # noqa: F401,E402
from .density_ref import pipe_menon_weights  # noqa: F401,E402
from .frame_ref import window, g_integral, frame_matrix, frame_coefficients, frame_image  # noqa: F401,E402
