"""Each plausible mistake planted in the oracle (on the CPU) must be caught by
at least one pin, which shows the pins constrain every stage."""
import numpy as np
import pytest

import pins
from oracle import funnel_oracle as O


def _swap_lerp_weights(S, Np):
    h, M = S.shape
    xp = np.arange(M, dtype=np.int64) - M // 2
    g = np.zeros_like(S)
    for n2 in range(1, h + 1):
        f = S[n2 - 1]
        num = xp * Np + M * n2
        i0 = num // (2 * n2)
        t = (num - i0 * 2 * n2) / (2 * n2)
        f0 = np.where((i0 >= 0) & (i0 < M), f[np.clip(i0, 0, M - 1)], 0)
        f1 = np.where((i0 + 1 >= 0) & (i0 + 1 < M), f[np.clip(i0 + 1, 0, M - 1)], 0)
        g[n2 - 1] = t * f0 + (1 - t) * f1
    return g


def _omega_max_2pi(S, Np):
    # reads omega_max as 2*pi: s = n2 / Np
    h, M = S.shape
    return _REAL["nvmt"](S, 2 * Np)


def _conj_spectrum_sign(img_pad):
    return np.conj(_REAL["spectrum_y"](img_pad))


def _xdft_wrong_sign(g):
    return np.conj(_REAL["dft_x"](np.conj(g)))


def _no_conj_completion(G, Np):
    h, M = G.shape
    full = np.zeros((Np, M), complex)
    n2 = np.arange(1, h + 1)
    full[n2 + Np // 2] = G
    full[-n2 + Np // 2] = G                     # missing conjugate
    y = np.arange(Np) - Np // 2
    return ((np.exp(2j * np.pi * np.outer(y, y) / Np) @ full) / Np).real


def _no_expansion_offset(img, Np):
    N, M = img.shape
    out = np.zeros((Np, M))
    out[:N] = img                                # image placed at the top
    return out


def _adjoint_missing_two(dP, N, M, padded_len=0, kind="linear"):
    return 0.5 * _REAL["adjoint_regular"](dP, N, M, padded_len, kind)


def _peaks_only_detected_suppress(B, K, T, radius=1, mask=None, wrap=True):
    # marks only detected cells as visited (a plausible misreading)
    rows, cols = B.shape
    flat = B.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))
    det_mask = np.zeros((rows, cols), bool)
    off = np.arange(-radius, radius + 1)
    out = []
    for idx in order:
        if flat[idx] < T or len(out) == K:
            break
        r, c = divmod(int(idx), cols)
        rr, cc = r + off, c + off
        if wrap:
            rr, cc = rr % rows, cc % cols
        else:
            rr, cc = rr[(rr >= 0) & (rr < rows)], cc[(cc >= 0) & (cc < cols)]
        if not det_mask[np.ix_(rr, cc)].any() and not (mask is not None and mask[r, c]):
            det_mask[r, c] = True
            out.append(int(idx))
    return out


def _chirpz_rows(S, Np, sign=-1.0, ratio=2, scale=True, period_rows=None):
    # the fused chirp-z NVMT with one planted change; s = ratio n2 / Np
    h, M = S.shape
    x = np.arange(M, dtype=np.int64) - M // 2
    G = np.empty_like(S, dtype=complex)
    for n2 in range(1, h + 1):
        s = ratio * n2 / Np
        period = (period_rows or Np) * M
        ph = np.mod(ratio * n2 * np.outer(x, x), period)
        E = np.exp(sign * 2j * np.pi * ph / period)
        G[n2 - 1] = (s if scale else 1.0) * (E @ S[n2 - 1])
    return G


def _chirpz_wrong_sign(S, Np):
    return _chirpz_rows(S, Np, sign=+1.0)


def _chirpz_no_ratio_factor(S, Np):
    return _chirpz_rows(S, Np, scale=False)


def _chirpz_ratio_halved(S, Np):
    # reads omega_max as 2*pi: s = n2 / Np
    return _chirpz_rows(S, Np, ratio=1)


def _chirpz_phase_period_M(S, Np):
    # reduces the integer phase modulo 2 M instead of Np M
    return _chirpz_rows(S, Np, period_rows=2)


def _chirpz_transpose_no_conj(dG, Np):
    return _chirpz_rows(dG, Np)


def _band(img, space, slope, intercept, half_width=3, nearest=False, along=False, top_pad=1):
    # the band integral with one planted change
    img = np.asarray(img, dtype=np.float64)
    if space == "inverse":
        img = img.T
    if along:
        img = img.T
    rows, cols = img.shape
    D = int(half_width)
    prof, n = np.zeros(2 * D + 1), 0
    for c in range(cols):
        y = np.float32(np.float64(np.float32(slope)) * c + np.float64(np.float32(intercept)))
        r0 = int(np.floor(y))
        t = float(y) - r0
        if nearest:
            r0, t = int(np.floor(y + 0.5)), 0.0
        if r0 - D < 0 or r0 + D + top_pad > rows - 1:
            continue
        for i, d in enumerate(range(-D, D + 1)):
            nxt = img[r0 + d + 1, c] if r0 + d + 1 < rows else 0.0
            prof[i] += (1.0 - t) * img[r0 + d, c] + t * nxt
        n += 1
    return (prof / n if n else prof), n


def _band_nearest(img, space, slope, intercept, half_width=3):
    return _band(img, space, slope, intercept, half_width, nearest=True)


def _band_along(img, space, slope, intercept, half_width=3):
    return _band(img, space, slope, intercept, half_width, along=True)


def _band_limit_off_by_one(img, space, slope, intercept, half_width=3):
    return _band(img, space, slope, intercept, half_width, top_pad=0)


def _cont_plane(g, Np, m, y, msign=-1.0, ysign=1.0):
    # the plane between cells with one planted change
    h, M = g.shape
    xp = np.arange(M) - M // 2
    n2 = np.arange(1, h + 1)
    e = np.exp(msign * 2j * np.pi * m * xp / M)
    cm = msign * 2j * np.pi * xp / M
    A0, A1, A2 = g @ e, g @ (cm * e), g @ (cm * cm * e)
    w = np.exp(2j * np.pi * n2 * y / Np)
    cy = ysign * 2j * np.pi * n2 / Np
    f = 2.0 / Np
    r = lambda a: f * np.real(np.sum(a))
    return r(A0 * w), r(A1 * w), r(A0 * cy * w), r(A2 * w), r(A1 * cy * w), r(A0 * cy * cy * w)


def _cont_plane_m_conj(g, Np, m, y):
    return _cont_plane(g, Np, m, y, msign=+1.0)


def _cont_plane_dy_sign(g, Np, m, y):
    return _cont_plane(g, Np, m, y, ysign=-1.0)


def _refine_descends(g, Np, row, col, iters=4):
    # steps downhill (a sign slip in the update)
    h, M = g.shape
    m0, y0 = float(col - M // 2), float(row - Np // 2)
    m, y = m0, y0
    sg = 1.0 if O.continuous_plane(g, Np, m, y)[0] >= 0 else -1.0
    for _ in range(iters):
        P, Pm, Py = (sg * v for v in O.continuous_plane(g, Np, m, y)[:3])
        nrm = np.hypot(Pm, Py) or 1.0
        m = min(max(m - 0.25 * Pm / nrm, m0 - 1.0), m0 + 1.0)
        y = min(max(y - 0.25 * Py / nrm, y0 - 1.0), y0 + 1.0)
    return m, y, abs(O.continuous_plane(g, Np, m, y)[0])


_REAL = {name: getattr(O, name) for name in
         ("nvmt", "spectrum_y", "dft_x", "idft_y", "expand", "adjoint_regular", "peaks_list",
          "nvmt_dft_chirpz", "_nvmt_dft_chirpz_transpose",
          "nvmt_bilinear", "spectrum_z", "dft_xy", "plane_params")}

ALL_CHECKS = [
    pins.check_spectrum_is_library_fft, pins.check_xdft_is_library_fft,
    pins.check_ydft_inverse_is_library_ifft, pins.check_parseval,
    pins.check_nvmt_exact_on_linear_rows, pins.check_nvmt_funnel_support,
    pins.check_point_to_line, pins.check_line_to_point, pins.check_fig9_worked_example,
    pins.check_fig6_intercept_wrap, pins.check_fig7_slope_wrap,
    pins.check_shift_equivariance, pins.check_adjoint_dot, pins.check_adjoint_dense,
    pins.check_peaks_equal_local_maxima,
    pins.check_chirpz_slant_stack, pins.check_chirpz_special_rows,
    pins.check_chirpz_point_to_line, pins.check_chirpz_line_to_point,
    pins.check_chirpz_adjoint_dot, pins.check_chirpz_adjoint_dense,
    pins.check_verify_constant_and_ramp, pins.check_verify_band_limits,
    pins.check_verify_ridge_and_step, pins.check_verify_fig9_wrap,
    pins.check_continuous_plane_cells, pins.check_continuous_plane_derivatives,
    pins.check_refine_line_to_point, pins.check_refine_stationary,
    pins.check_spectrum_z_is_library_fft, pins.check_dft_xy_is_library_fft2,
    pins.check_idft_z_is_library_ifft, pins.check_bilinear_exact_on_bilinear_slices,
    pins.check_volume_reduces_to_image, pins.check_volume_plane_to_point,
    pins.check_volume_point_to_plane, pins.check_volume_shift_equivariance,
    pins.check_volume_peaks_equal_local_maxima, pins.check_plane_params_round_trip,
    pins.check_volume_spaces_focus_steep_planes,
]

def _bilinear_y_weights_swapped(S, Nzp, n3_first=1):
    h, Ny, Nx = S.shape
    yp = np.arange(Ny, dtype=np.int64) - Ny // 2
    xp = np.arange(Nx, dtype=np.int64) - Nx // 2
    g = np.zeros_like(S)
    for k in range(h):
        n3 = n3_first + k
        f = S[k]
        den = 2 * n3
        nu, nv = yp * Nzp + Ny * n3, xp * Nzp + Nx * n3
        i0, j0 = nu // den, nv // den
        tu = 1.0 - ((nu - i0 * den) / den)[:, None]        # weights of the two rows exchanged
        tv = ((nv - j0 * den) / den)[None, :]
        I0, J0 = i0[:, None], j0[None, :]

        def tap(ii, jj):
            inside = (ii >= 0) & (ii < Ny) & (jj >= 0) & (jj < Nx)
            return np.where(inside, f[np.clip(ii, 0, Ny - 1), np.clip(jj, 0, Nx - 1)], 0.0)

        g[k] = ((1 - tu) * (1 - tv) * tap(I0, J0) + (1 - tu) * tv * tap(I0, J0 + 1)
                + tu * (1 - tv) * tap(I0 + 1, J0) + tu * tv * tap(I0 + 1, J0 + 1))
    return g


def _bilinear_omega_max_2pi(S, Nzp, n3_first=1):
    return _REAL["nvmt_bilinear"](S, 2 * Nzp, n3_first)


def _spectrum_z_conj(vol_pad):
    return np.conj(_REAL["spectrum_z"](vol_pad))


def _dft_xy_m2_sign(g):
    Ny = g.shape[1]
    y = np.arange(Ny) - Ny // 2
    flip = np.exp(4j * np.pi * np.outer(y, y) / Ny)     # exp(-j..) -> exp(+j..) along y'
    return np.matmul(flip, _REAL["dft_xy"](g))


def _idft_z_no_conj(G, Nzp):
    h, Ny, Nx = G.shape
    full = np.zeros((Nzp, Ny, Nx), complex)
    n3 = np.arange(1, h + 1)
    full[n3 + Nzp // 2] = G
    full[-n3 + Nzp // 2] = G
    z = np.arange(Nzp) - Nzp // 2
    return np.tensordot(np.exp(2j * np.pi * np.outer(z, z) / Nzp), full, axes=(1, 0)).real / Nzp


def _expand_volume_front(vol, Nzp):
    out = np.zeros((Nzp,) + vol.shape[1:])
    out[:vol.shape[0]] = vol
    return out


def _peaks_volume_no_z(B, K, T, radius=1, mask=None, wrap=True):
    # neighbourhood taken within each slice only
    nz, ny, nx = B.shape
    flat = B.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))
    visited = np.zeros(B.shape, bool)
    off = np.arange(-radius, radius + 1)
    out = []
    for idx in order:
        if flat[idx] < T:
            break
        z, rem = divmod(int(idx), ny * nx)
        r, c = divmod(rem, nx)
        rr, cc = (r + off) % ny, (c + off) % nx
        seen = visited[z][np.ix_(rr, cc)].any()
        visited[z, r, c] = True
        if not seen and not (mask is not None and mask[z, r, c]):
            out.append(int(idx))
            if len(out) == K:
                break
    return out


def _plane_params_b_sign(z, row, col, Nz, Ny, Nx, Nzp):
    a, b, c = _REAL["plane_params"](z, row, col, Nz, Ny, Nx, Nzp)
    return a, -b, c + b * Ny


MUTANTS = {
    "lerp weights swapped": ("nvmt", _swap_lerp_weights),
    "omega_max read as 2 pi": ("nvmt", _omega_max_2pi),
    "y DFT exponent sign": ("spectrum_y", _conj_spectrum_sign),
    "x DFT exponent sign": ("dft_x", _xdft_wrong_sign),
    "Hermitian completion without conjugate": ("idft_y", _no_conj_completion),
    "expansion not centred": ("expand", _no_expansion_offset),
    "adjoint loses factor 2": ("adjoint_regular", _adjoint_missing_two),
    "peak list suppresses only by detected cells": ("peaks_list", _peaks_only_detected_suppress),
    "chirp-z exponent sign": ("nvmt_dft_chirpz", _chirpz_wrong_sign),
    "chirp-z without the ratio factor s": ("nvmt_dft_chirpz", _chirpz_no_ratio_factor),
    "chirp-z ratio read as n2 / Np": ("nvmt_dft_chirpz", _chirpz_ratio_halved),
    "chirp-z phase reduced modulo 2 M": ("nvmt_dft_chirpz", _chirpz_phase_period_M),
    "chirp-z adjoint without conjugate": ("_nvmt_dft_chirpz_transpose", _chirpz_transpose_no_conj),
    "band sampled at the nearest pixel": ("line_band_profile", _band_nearest),
    "band offsets along the line's axis": ("line_band_profile", _band_along),
    "band limit one row short": ("line_band_profile", _band_limit_off_by_one),
    "plane between cells with the slope exponent conjugated": ("continuous_plane", _cont_plane_m_conj),
    "plane between cells with the intercept derivative's sign flipped": ("continuous_plane", _cont_plane_dy_sign),
    "refinement stepping downhill": ("refine_peak", _refine_descends),
    "bilinear weights exchanged along y": ("nvmt_bilinear", _bilinear_y_weights_swapped),
    "volume NVMT with omega_max read as 2 pi": ("nvmt_bilinear", _bilinear_omega_max_2pi),
    "z DFT exponent sign": ("spectrum_z", _spectrum_z_conj),
    "m2 DFT exponent sign": ("dft_xy", _dft_xy_m2_sign),
    "z completion without conjugate": ("idft_z", _idft_z_no_conj),
    "volume expansion not centred": ("expand_volume", _expand_volume_front),
    "3D peaks without the z neighbours": ("peaks_list_volume", _peaks_volume_no_z),
    "plane parameter b with the wrong sign": ("plane_params", _plane_params_b_sign),
    "x space with rows and columns exchanged": ("VOLUME_SPACES", {"z": (0, 1, 2), "x": (2, 1, 0), "y": (1, 0, 2)}),
    "y space with rows and columns exchanged": ("VOLUME_SPACES", {"z": (0, 1, 2), "x": (2, 0, 1), "y": (1, 2, 0)}),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(O, attr, fn)
    caught = []
    for check in ALL_CHECKS:
        try:
            check(O)
        except (AssertionError, ValueError, IndexError):
            caught.append(check.__name__)
    assert caught, f"no pin catches: {name}"
