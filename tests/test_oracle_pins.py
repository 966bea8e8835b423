"""The FP64 oracle against the paper's closed forms, worked example and
textbook identities (CPU only)."""
import pytest

import pins
from oracle import funnel_oracle as O

CHECKS = [
    pins.check_spectrum_is_library_fft,
    pins.check_xdft_is_library_fft,
    pins.check_ydft_inverse_is_library_ifft,
    pins.check_parseval,
    pins.check_nvmt_exact_on_linear_rows,
    pins.check_nvmt_funnel_support,
    pins.check_point_to_line,
    pins.check_line_to_point,
    pins.check_fig9_worked_example,
    pins.check_fig6_intercept_wrap,
    pins.check_fig7_slope_wrap,
    pins.check_shift_equivariance,
    pins.check_linearity,
    pins.check_adjoint_dot,
    pins.check_adjoint_dense,
    pins.check_adjoint_finite_difference,
    pins.check_peaks_equal_local_maxima,
    pins.check_peak_params,
    pins.check_chirpz_slant_stack,
    pins.check_chirpz_special_rows,
    pins.check_chirpz_point_to_line,
    pins.check_chirpz_line_to_point,
    pins.check_chirpz_adjoint_dot,
    pins.check_chirpz_adjoint_dense,
    pins.check_column_samplers,
    pins.check_verify_constant_and_ramp,
    pins.check_verify_band_limits,
    pins.check_verify_ridge_and_step,
    pins.check_verify_fig9_wrap,
    pins.check_continuous_plane_cells,
    pins.check_continuous_plane_derivatives,
    pins.check_refine_line_to_point,
    pins.check_refine_stationary,
    pins.check_spectrum_z_is_library_fft,
    pins.check_dft_xy_is_library_fft2,
    pins.check_idft_z_is_library_ifft,
    pins.check_bilinear_exact_on_bilinear_slices,
    pins.check_volume_reduces_to_image,
    pins.check_volume_plane_to_point,
    pins.check_volume_point_to_plane,
    pins.check_volume_shift_equivariance,
    pins.check_volume_lines_sampler,
    pins.check_volume_peaks_equal_local_maxima,
    pins.check_plane_params_round_trip,
    pins.check_volume_spaces_focus_steep_planes,
]


@pytest.mark.parametrize("check", CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check(O)


def test_adjoint_dense_nonsquare():
    pins.check_adjoint_dense(O, N=6, M=10)


def test_peaks_literal_examples():
    import numpy as np
    B = np.array([[1, 0, 1, 0],
                  [5, 1, 1, 4],
                  [0, 1, 3, 1]], float)
    # wrap: columns 0 and 3 touch, so the 4 at (1,3) sees the 5 at (1,0)
    assert O.peaks_list(B, 5, 0.0, 1, None, True) == [4]
    # clamped border: both the 5 and the 4 are peaks, the 3 sees the 4
    assert O.peaks_list(B, 5, 0.0, 1, None, False) == [4, 7]
    # the threshold ends the list
    assert O.peaks_list(B, 5, 4.5, 1, None, False) == [4]
    # K ends the list
    assert O.peaks_list(B, 1, 0.0, 1, None, False) == [4]
    # a masked cell is visited (it still suppresses its neighbours) but never detected
    mask = np.zeros_like(B, bool)
    mask[1, 0] = True
    assert O.peaks_list(B, 5, 0.0, 1, mask, False) == [7]
