"""FP64 CPU oracle of the funnel transform (Wei, Feng, Zheng, arXiv 1904.09409).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may use it.  It shares no code with the HIP library.

Every stage is the plain definition written out in float64 with explicit DFT
matrices (a matrix product is the only library primitive used) and direct
per-row linear interpolation, in the order the paper gives the steps
(Sec. 3.1): FFT along y -> NVMT -> FFT along x' -> inverse FFT along omega_2.

Conventions (readings of the paper, each one listed with its reason in the
design notes of the repository):

* image ``I[r, c]``: N rows (height, y), M columns (width, x), both even.
* expansion (Sec. 4.2): the image is padded with zero rows to a total height
  ``Np`` (default N+M, i.e. M/2 rows above and below); the centre of the
  Cartesian frame is the frame centre, ``y = r' - Np/2`` and ``x = c - M/2``.
* omega_max = pi, so the NVMT ratio of frequency row n2 is ``s = 2 n2 / Np``
  and the slope step is 2/M (Eq. 22).
* only the top half of the spectrum, ``n2 = 1 .. Np/2-1``, is resampled; the
  bottom half follows by conjugate symmetry (Sec. 3.1); the DC and Nyquist
  rows are dropped.
* forward DFTs are unnormalised, the final inverse DFT carries 1/Np.
* two NVMT realisations: ``"linear"`` interpolation (Sec. V's O(M^2)
  option, the default) and ``"chirpz"``, the band-limited resampling the
  paper adopts (opening of Sec. IV), written out as the scaled-frequency DFT
  it equals.
* parameter plane ``P[y + Np/2, m1 + M/2]`` is real; the brightness is |P|.
  A line ``y = k x + b`` (centred) peaks at ``m1 = -k M/2``, ``y = b``
  (Eq. 19 with the sign of Eq. 13); the paper's slope index is m = -m1.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "padded_length", "expand", "spectrum_y", "nvmt", "dft_x", "idft_y",
    "nvmt_dft_chirpz", "NVMT_KINDS",
    "forward_regular", "forward_inverse", "forward",
    "adjoint_regular", "adjoint_inverse", "adjoint",
    "forward_regular_columns", "adjoint_regular_columns",
    "boundary_mask", "peaks_list", "peak_params",
    "line_band_profile", "line_verdict",
    "resampled_rows", "continuous_plane", "refine_peak",
    "padded_depth", "expand_volume", "spectrum_z", "nvmt_bilinear", "dft_xy", "idft_z",
    "forward_volume", "forward_volume_lines", "volume_boundary_mask", "peaks_list_volume",
    "plane_params", "VOLUME_SPACES", "volume_in_space", "forward_volume_space",
]


# --------------------------------------------------------------------------
# Forward transform, Sec. 3.1
# --------------------------------------------------------------------------

def padded_length(N: int, M: int, padded_len: int = 0) -> int:
    """Length of the expanded axis (Sec. 4.2): N+M by default.  An explicit
    even length >= N may be asked for; lengths below N+M give up the
    intercept-wrap protection of the expansion (Eq. 20, Fig. 6)."""
    Np = N + M if padded_len == 0 else int(padded_len)
    if Np < N or Np % 2:
        raise ValueError("padded length must be even and >= N")
    return Np


def expand(img: np.ndarray, Np: int) -> np.ndarray:
    """Sec. 4.2: place the N image rows in an Np-row zero frame with
    (Np-N)//2 zero rows above them."""
    N, M = img.shape
    top = (Np - N) // 2
    out = np.zeros((Np, M), dtype=np.float64)
    out[top:top + N] = img
    return out


def _ydft_matrix(Np: int) -> np.ndarray:
    """E[n2-1, r'] = exp(-j 2 pi n2 y / Np), y = r' - Np/2, n2 = 1..Np/2-1."""
    n2 = np.arange(1, Np // 2)
    y = np.arange(Np) - Np // 2
    return np.exp(-2j * np.pi * np.outer(n2, y) / Np)


def _xdft_matrix(M: int) -> np.ndarray:
    """W[x'+M/2, m1+M/2] = exp(-j 2 pi m1 x' / M) over centred x', m1."""
    x = np.arange(M) - M // 2
    return np.exp(-2j * np.pi * np.outer(x, x) / M)


def spectrum_y(img_pad: np.ndarray) -> np.ndarray:
    """Sec. 3.1 first step (Eq. 16): DFT of every column along y.

    Returns S[n2-1, c] = sum_y I_pad[y, c] exp(-j 2 pi n2 y / Np) for the top
    half n2 = 1 .. Np/2-1 (negative n2 follow by conjugation, Sec. 3.1)."""
    return _ydft_matrix(img_pad.shape[0]) @ img_pad


def nvmt(S: np.ndarray, Np: int) -> np.ndarray:
    """Sec. 3.1 second step, Eq. 17: the nonlinear variable-metric transform
    x' = s x with s = omega_2/omega_max = 2 n2 / Np, realised by linear
    interpolation (the O(M^2) option of Sec. V): g[x'] = f(x'/s).

    f[i] = S[n2, i - M/2] for 0 <= i < M and 0 outside.  The fractional array
    position i_p = x'/s + M/2 = (x' Np + M n2) / (2 n2) is split with an exact
    integer floor, i0 = floor(num/den), t = (num - i0 den)/den."""
    h, M = S.shape
    xp = np.arange(M, dtype=np.int64) - M // 2
    g = np.zeros_like(S)
    for n2 in range(1, h + 1):
        f = S[n2 - 1]
        num = xp * Np + M * n2
        den = 2 * n2
        i0 = num // den
        t = (num - i0 * den) / den
        ok0 = (i0 >= 0) & (i0 < M)
        ok1 = (i0 + 1 >= 0) & (i0 + 1 < M)
        f0 = np.where(ok0, f[np.clip(i0, 0, M - 1)], 0.0)
        f1 = np.where(ok1, f[np.clip(i0 + 1, 0, M - 1)], 0.0)
        g[n2 - 1] = (1.0 - t) * f0 + t * f1
    return g


def dft_x(g: np.ndarray) -> np.ndarray:
    """Sec. 3.1 third step: DFT along x' of every row,
    G[n2, m1] = sum_x' g[n2, x'] exp(-j 2 pi m1 x' / M), centred x', m1."""
    return g @ _xdft_matrix(g.shape[1])


def nvmt_dft_chirpz(S: np.ndarray, Np: int) -> np.ndarray:
    """NVMT by band-limited resampling fused with the x' DFT (Sec. 3.1's
    second and third steps, realised the way the opening of Sec. IV adopts:
    chirp-z interpolation instead of the linear one; Remark 1).

    The row f(x) = S[n2, x] is read as a band-limited function; resampling it
    as g(x') = f(x'/s) scales its spectrum, so the DFT of the resampled row is
    the row's own DTFT at the scaled frequencies s m1 / M, times s:

        G[n2, m1] = s sum_x S[n2, x] exp(-j 2 pi s m1 x / M),  s = 2 n2 / Np,

    centred x and m1 in [-M/2, M/2).  Written out as that sum with the phase
    s m1 x / M = 2 n2 m1 x / (Np M) reduced exactly in integers."""
    h, M = S.shape
    x = np.arange(M, dtype=np.int64) - M // 2
    period = Np * M
    G = np.empty_like(S, dtype=np.complex128)
    for n2 in range(1, h + 1):
        ph = np.mod(2 * n2 * np.outer(x, x), period)          # [m1, x]
        E = np.exp(-2j * np.pi * ph / period)
        G[n2 - 1] = (2.0 * n2 / Np) * (E @ S[n2 - 1])
    return G


NVMT_KINDS = ("linear", "chirpz")


def _resample_and_dft(S: np.ndarray, Np: int, kind: str) -> np.ndarray:
    if kind == "linear":
        return dft_x(nvmt(S, Np))
    if kind == "chirpz":
        return nvmt_dft_chirpz(S, Np)
    raise ValueError(f"unknown NVMT kind {kind!r}")


def idft_y(G: np.ndarray, Np: int) -> np.ndarray:
    """Sec. 3.1 fourth step (Eq. 19 / P(omega_1, y)): inverse DFT along omega_2.

    The bottom half of the spectrum is completed by G[-n2] = conj(G[n2]); the
    DC and Nyquist rows are zero.  P[y, m1] = (1/Np) sum_n2 G[n2, m1]
    exp(+j 2 pi n2 y / Np), y = -Np/2 .. Np/2-1.  The result is real; its
    imaginary part is checked to be rounding noise."""
    h, M = G.shape
    full = np.zeros((Np, M), dtype=np.complex128)   # row index n2 + Np/2
    n2 = np.arange(1, h + 1)
    full[n2 + Np // 2] = G
    full[-n2 + Np // 2] = np.conj(G)
    y = np.arange(Np) - Np // 2
    Winv = np.exp(2j * np.pi * np.outer(y, y) / Np)
    P = (Winv @ full) / Np
    scale = max(1.0, float(np.abs(P.real).max()))
    if np.abs(P.imag).max() > 1e-9 * scale:
        raise AssertionError("inverse DFT of a Hermitian spectrum is not real")
    return P.real


def forward_regular(img: np.ndarray, padded_len: int = 0, nvmt_kind: str = "linear") -> np.ndarray:
    """Funnel transform (Sec. 3.1) of one image on its expanded frame
    (Sec. 4.2): the regular parameter space, slopes in (-1, 1].
    Returns P[Np, M] in float64."""
    img = np.asarray(img, dtype=np.float64)
    N, M = img.shape
    Np = padded_length(N, M, padded_len)
    S = spectrum_y(expand(img, Np))
    return idft_y(_resample_and_dft(S, Np, nvmt_kind), Np)


def forward_inverse(img: np.ndarray, padded_len: int = 0, nvmt_kind: str = "linear") -> np.ndarray:
    """Inverse funnel transform (Sec. 3.1, dual form; Remark 1): the same four
    steps with the roles of x and y exchanged, i.e. the funnel transform of the
    transposed image.  Returns P_inv[Np, N]: rows are the x-intercept, columns
    the inverse-slope bin."""
    img = np.asarray(img, dtype=np.float64)
    return forward_regular(img.T, padded_len, nvmt_kind)


def forward(img: np.ndarray, padded_len: int = 0, nvmt_kind: str = "linear"):
    """Both parameter spaces (Sec. 4.1): (regular, inverse)."""
    return forward_regular(img, padded_len, nvmt_kind), forward_inverse(img, padded_len, nvmt_kind)


def forward_regular_columns(img: np.ndarray, cols, padded_len: int = 0,
                            nvmt_kind: str = "linear") -> np.ndarray:
    """Columns ``cols`` (array indices m1 + M/2) of ``forward_regular``, for
    checking large planes on a sample: the same four steps, with the x' DFT
    and the inverse y DFT evaluated only for the asked slope bins.
    Returns P[:, cols], shape (Np, len(cols))."""
    img = np.asarray(img, dtype=np.float64)
    N, M = img.shape
    Np = padded_length(N, M, padded_len)
    cols = np.asarray(cols, dtype=np.int64)
    S = spectrum_y(expand(img, Np))
    h = S.shape[0]
    m1 = cols - M // 2
    x = np.arange(M, dtype=np.int64) - M // 2
    if nvmt_kind == "linear":
        G = nvmt(S, Np) @ np.exp(-2j * np.pi * np.outer(x, m1) / M)
    elif nvmt_kind == "chirpz":
        G = np.empty((h, len(cols)), dtype=np.complex128)
        period = Np * M
        for n2 in range(1, h + 1):
            ph = np.mod(2 * n2 * np.outer(x, m1), period)
            G[n2 - 1] = (2.0 * n2 / Np) * (S[n2 - 1] @ np.exp(-2j * np.pi * ph / period))
    else:
        raise ValueError(f"unknown NVMT kind {nvmt_kind!r}")
    return idft_y(G, Np)


def adjoint_regular_columns(dP: np.ndarray, N: int, M: int, cols, padded_len: int = 0,
                            nvmt_kind: str = "linear") -> np.ndarray:
    """Columns ``cols`` (array indices x + M/2) of ``adjoint_regular``: the
    full C^T, then B^T and A^T evaluated only for the asked image columns.
    Returns dI[:, cols], shape (N, len(cols))."""
    dP = np.asarray(dP, dtype=np.float64)
    Np = padded_length(N, M, padded_len)
    cols = np.asarray(cols, dtype=np.int64)
    dG = (2.0 / Np) * (_ydft_matrix(Np) @ dP)
    h = dG.shape[0]
    if nvmt_kind == "linear":
        dS = _nvmt_transpose(dG @ np.conj(_xdft_matrix(M)).T, Np)[:, cols]
    elif nvmt_kind == "chirpz":
        x = cols - M // 2
        m1 = np.arange(M, dtype=np.int64) - M // 2
        period = Np * M
        dS = np.empty((h, len(cols)), dtype=np.complex128)
        for n2 in range(1, h + 1):
            ph = np.mod(2 * n2 * np.outer(m1, x), period)
            dS[n2 - 1] = (2.0 * n2 / Np) * (dG[n2 - 1] @ np.exp(2j * np.pi * ph / period))
    else:
        raise ValueError(f"unknown NVMT kind {nvmt_kind!r}")
    dI_pad = np.real(np.conj(_ydft_matrix(Np)).T @ dS)
    top = (Np - N) // 2
    return dI_pad[top:top + N]


# --------------------------------------------------------------------------
# Adjoint (transpose of the real-linear map image -> plane)
# --------------------------------------------------------------------------

def _nvmt_transpose(dg: np.ndarray, Np: int) -> np.ndarray:
    """Transpose of ``nvmt``: each interpolation weight sends dg[x'] back to
    the two samples it was read from."""
    h, M = dg.shape
    xp = np.arange(M, dtype=np.int64) - M // 2
    dS = np.zeros_like(dg)
    for n2 in range(1, h + 1):
        num = xp * Np + M * n2
        den = 2 * n2
        i0 = num // den
        t = (num - i0 * den) / den
        row = np.zeros(M, dtype=np.complex128)
        ok0 = (i0 >= 0) & (i0 < M)
        ok1 = (i0 + 1 >= 0) & (i0 + 1 < M)
        np.add.at(row, i0[ok0], (1.0 - t[ok0]) * dg[n2 - 1, ok0])
        np.add.at(row, i0[ok1] + 1, t[ok1] * dg[n2 - 1, ok1])
        dS[n2 - 1] = row
    return dS


def _nvmt_dft_chirpz_transpose(dG: np.ndarray, Np: int) -> np.ndarray:
    """Conjugate transpose of ``nvmt_dft_chirpz``: the kernel
    s exp(-j 2 pi s m1 x / M) is symmetric in (m1, x), so its adjoint is
    dS[n2, x] = s sum_m1 dG[n2, m1] exp(+j 2 pi s m1 x / M)."""
    h, M = dG.shape
    x = np.arange(M, dtype=np.int64) - M // 2
    period = Np * M
    dS = np.empty_like(dG, dtype=np.complex128)
    for n2 in range(1, h + 1):
        ph = np.mod(2 * n2 * np.outer(x, x), period)          # [x, m1]
        E = np.exp(2j * np.pi * ph / period)
        dS[n2 - 1] = (2.0 * n2 / Np) * (E @ dG[n2 - 1])
    return dS


def adjoint_regular(dP: np.ndarray, N: int, M: int, padded_len: int = 0,
                    nvmt_kind: str = "linear") -> np.ndarray:
    """Transpose of ``forward_regular`` under the real inner products of
    image and plane: dI = A^T B^T C^T dP, where C is the Hermitian inverse DFT,
    B the NVMT followed by the x' DFT and A the expansion plus y DFT."""
    dP = np.asarray(dP, dtype=np.float64)
    Np = padded_length(N, M, padded_len)
    assert dP.shape == (Np, M)
    # C^T: P = (1/Np) sum_n2 2 Re(G[n2] e^{+j theta})  =>  dG = (2/Np) sum_y dP e^{-j theta}
    dG = (2.0 / Np) * (_ydft_matrix(Np) @ dP)
    if nvmt_kind == "linear":
        # B^T: conjugate transpose of the x' DFT, then the transposed interpolation
        dg = dG @ np.conj(_xdft_matrix(M)).T
        dS = _nvmt_transpose(dg, Np)
    elif nvmt_kind == "chirpz":
        dS = _nvmt_dft_chirpz_transpose(dG, Np)
    else:
        raise ValueError(f"unknown NVMT kind {nvmt_kind!r}")
    # A^T: S = E I_pad with real I_pad  =>  dI_pad = Re(E^H dS), then crop
    dI_pad = np.real(np.conj(_ydft_matrix(Np)).T @ dS)
    top = (Np - N) // 2
    return dI_pad[top:top + N]


def adjoint_inverse(dPinv: np.ndarray, N: int, M: int, padded_len: int = 0,
                    nvmt_kind: str = "linear") -> np.ndarray:
    """Transpose of ``forward_inverse``."""
    return adjoint_regular(dPinv, M, N, padded_len, nvmt_kind).T


def adjoint(dP: np.ndarray, dPinv: np.ndarray, N: int, M: int, padded_len: int = 0,
            nvmt_kind: str = "linear") -> np.ndarray:
    """Transpose of ``forward`` (both spaces): the two image gradients add."""
    return (adjoint_regular(dP, N, M, padded_len, nvmt_kind) +
            adjoint_inverse(dPinv, N, M, padded_len, nvmt_kind))


# --------------------------------------------------------------------------
# Peak detection (Sec. 4.4) and peak -> line parameters (Eqs. 22-25)
# --------------------------------------------------------------------------

def boundary_mask(N: int, M: int, Np: int) -> np.ndarray:
    """Cells of a regular plane (Np x M) where the artificial top and bottom
    borders created by the expansion focus (Sec. 4.2, removed in Sec. VI):
    slope bins m1 in {-1, 0, 1} and rows within 2 of y = -N/2 or y = N/2.
    For the inverse plane call with (M, N, Np)."""
    mask = np.zeros((Np, M), dtype=bool)
    cols = np.array([-1, 0, 1]) + M // 2
    for edge in (-N // 2, N // 2):
        rows = np.arange(edge - 2, edge + 2) + Np // 2
        rows = rows[(rows >= 0) & (rows < Np)]
        mask[np.ix_(rows, cols)] = True
    return mask


def peaks_list(B: np.ndarray, K: int, T: float, radius: int = 1,
               mask: np.ndarray | None = None, wrap: bool = True) -> list[int]:
    """The list-based peak detection of Sec. 4.4, literally.

    Every cell goes on a candidate list sorted by brightness, descending (ties:
    lower linear index first).  Cells are visited in that order; a cell joins
    the detected list if no cell of its (2r+1)^2 neighbourhood has been
    visited before, and is marked visited either way.  The loop stops at K
    detections or at the first cell darker than T.  Cells inside ``mask`` are
    visited but never detected.  The neighbourhood wraps around the plane
    (which is periodic in both axes, Eqs. 20-21) unless ``wrap`` is False.
    Returns the linear indices of the detected cells in detection order."""
    B = np.asarray(B)
    rows, cols = B.shape
    flat = B.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))
    visited = np.zeros((rows, cols), dtype=bool)
    off = np.arange(-radius, radius + 1)
    detected: list[int] = []
    if K <= 0:
        return detected
    for idx in order:
        v = flat[idx]
        if v < T:
            break
        r, c = divmod(int(idx), cols)
        rr, cc = r + off, c + off
        if wrap:
            rr, cc = rr % rows, cc % cols
        else:
            rr, cc = rr[(rr >= 0) & (rr < rows)], cc[(cc >= 0) & (cc < cols)]
        seen = visited[np.ix_(rr, cc)].any()
        visited[r, c] = True
        if not seen and not (mask is not None and mask[r, c]):
            detected.append(int(idx))
            if len(detected) == K:
                break
    return detected


def peak_params(row: int, col: int, N: int, M: int, Np: int, space: str = "regular"):
    """Eqs. 22-25: cell -> line parameters, in pixel-index coordinates.

    Regular space (plane Np x M): m1 = col - M/2, slope k = -2 m1 / M (the
    paper's m is -m1), centred intercept y = row - Np/2; the line is
    ``row = k * col + b`` with b = y - k M/2 + N/2.
    Inverse space (plane Np x N): n1 = col - N/2, inverse slope
    k_inv = -2 n1 / N, centred x-intercept xb = row - Np/2; the line is
    ``col = k_inv * row + b_x`` with b_x = xb - k_inv N/2 + M/2.
    Returns (slope, intercept) of the respective form."""
    if space == "regular":
        k = -2.0 * (col - M // 2) / M
        y = row - Np // 2
        return k, y - k * M / 2 + N / 2
    kinv = -2.0 * (col - N // 2) / N
    xb = row - Np // 2
    return kinv, xb - kinv * N / 2 + M / 2


# --------------------------------------------------------------------------
# Line verification, Sec. 4.5
# --------------------------------------------------------------------------

def line_band_profile(img: np.ndarray, space: str, slope: float, intercept: float,
                      half_width: int = 3):
    """Sec. 4.5 steps 1-3: the band of 2D+1 pixels (D = half_width, a 3-7
    pixel band) centred on a candidate line, integrated along the line.

    Regular space: the line is ``row = slope * col + intercept``; for every
    column c the line's row is y_c, and the band holds the samples at rows
    y_c + d, d = -D..D, interpolated linearly between the two neighbouring
    pixel rows.  Inverse space: ``col = slope * row + intercept`` with the
    roles of rows and columns exchanged.  A line position enters the band
    when both interpolation pixels of every offset are inside the image.

    The line position y_c and its integer part decide which pixels are read;
    they are taken in the precision the candidate line is given in (float32),
    y_c rounded once from the exact value, so that the decision does not
    depend on the arithmetic that evaluates it.  The samples are averaged in
    float64.  Returns (profile[2D+1], length): the mean of each offset over
    the line positions in the band, and their number."""
    img = np.asarray(img, dtype=np.float64)
    if space == "inverse":
        img = img.T
    rows, cols = img.shape
    D = int(half_width)
    k = np.float32(slope)
    b = np.float32(intercept)
    prof = np.zeros(2 * D + 1)
    n = 0
    for c in range(cols):
        y = np.float32(np.float64(k) * c + np.float64(b))   # exact, then one rounding
        r0 = int(np.floor(y))
        t = float(y) - r0
        if r0 - D < 0 or r0 + D + 1 > rows - 1:
            continue
        for i, d in enumerate(range(-D, D + 1)):
            prof[i] += (1.0 - t) * img[r0 + d, c] + t * img[r0 + d + 1, c]
        n += 1
    if n:
        prof /= n
    return prof, n


def line_verdict(profile: np.ndarray, length: int, min_contrast: float, min_length: int):
    """Sec. 4.5 step 4, in this reading: a line exists when the band profile
    stands out from its edges, either as a ridge (centre against the mean of
    the two outermost offsets) or as a step (one outermost offset against
    the other), by at least ``min_contrast``, over at least ``min_length``
    line positions.  Returns (contrast, verified)."""
    p = np.asarray(profile, dtype=np.float64)
    D = (len(p) - 1) // 2
    ridge = abs(p[D] - 0.5 * (p[0] + p[2 * D]))
    step = abs(p[2 * D] - p[0])
    contrast = max(ridge, step)
    return contrast, bool(length >= min_length and contrast >= min_contrast)


# --------------------------------------------------------------------------
# Sub-cell refinement of a peak (Eqs. 19, 22-25 at non-integer cells)
# --------------------------------------------------------------------------

def resampled_rows(img: np.ndarray, padded_len: int = 0, nvmt_kind: str = "linear") -> np.ndarray:
    """The NVMT output rows g[n2, x'] (Sec. 3.1, second step) of the regular
    space: for the linear NVMT the interpolated rows themselves; for the
    chirp-z NVMT the rows whose DFT is the fused G (g = IDFT_M of G, centred
    x' and m1)."""
    img = np.asarray(img, dtype=np.float64)
    N, M = img.shape
    Np = padded_length(N, M, padded_len)
    S = spectrum_y(expand(img, Np))
    if nvmt_kind == "linear":
        return nvmt(S, Np)
    G = nvmt_dft_chirpz(S, Np)
    return G @ np.conj(_xdft_matrix(M)).T / M


def continuous_plane(g: np.ndarray, Np: int, m: float, y: float):
    """The parameter plane between cells: the last two steps of Sec. 3.1 with
    the x' DFT evaluated at a real slope bin m (the DTFT of each resampled
    row) and the inverse y DFT at a real intercept y (its trigonometric sum),
        P(m, y) = (2/Np) Re sum_n2 A(n2; m) exp(+j 2 pi n2 y / Np),
        A(n2; m) = sum_x' g[n2, x'] exp(-j 2 pi m x' / M),
    which equals the plane at integer (m, y).  Returns P and its first and
    second derivatives: (P, P_m, P_y, P_mm, P_my, P_yy)."""
    h, M = g.shape
    xp = np.arange(M) - M // 2
    n2 = np.arange(1, h + 1)
    e = np.exp(-2j * np.pi * m * xp / M)
    cm = -2j * np.pi * xp / M                 # d/dm of the exponent
    A0 = g @ e
    A1 = g @ (cm * e)
    A2 = g @ (cm * cm * e)
    w = np.exp(2j * np.pi * n2 * y / Np)
    cy = 2j * np.pi * n2 / Np                 # d/dy of the exponent
    f = 2.0 / Np
    P = f * np.real(np.sum(A0 * w))
    Pm = f * np.real(np.sum(A1 * w))
    Py = f * np.real(np.sum(A0 * cy * w))
    Pmm = f * np.real(np.sum(A2 * w))
    Pmy = f * np.real(np.sum(A1 * cy * w))
    Pyy = f * np.real(np.sum(A0 * cy * cy * w))
    return P, Pm, Py, Pmm, Pmy, Pyy


def refine_peak(g: np.ndarray, Np: int, row: int, col: int, iters: int = 4):
    """Gradient refinement of one peak to a local maximum of |P| between
    cells (the line parameters Eq. 19 focuses to are continuous; Eqs. 22-25
    read them from the maximum).  From the cell's centre, `iters` safeguarded
    Newton steps on F = sign(P) P: the Newton step when the Hessian of F is
    negative definite, otherwise a gradient step of 0.25 cell, each component
    clamped to 0.5 cell, the total displacement to 1 cell.  Returns the slope
    bin m, the intercept y (centred, real) and |P| there."""
    h, M = g.shape
    m0, y0 = float(col - M // 2), float(row - Np // 2)
    P0 = continuous_plane(g, Np, m0, y0)[0]
    sg = 1.0 if P0 >= 0 else -1.0
    m, y = m0, y0
    for _ in range(iters):
        P, Pm, Py, Pmm, Pmy, Pyy = (sg * v for v in continuous_plane(g, Np, m, y))
        det = Pmm * Pyy - Pmy * Pmy
        if Pmm < 0 and det > 0:
            dm = -(Pyy * Pm - Pmy * Py) / det
            dy = -(Pmm * Py - Pmy * Pm) / det
        else:
            nrm = np.hypot(Pm, Py)
            dm, dy = (0.25 * Pm / nrm, 0.25 * Py / nrm) if nrm > 0 else (0.0, 0.0)
        m = min(max(m + min(max(dm, -0.5), 0.5), m0 - 1.0), m0 + 1.0)
        y = min(max(y + min(max(dy, -0.5), 0.5), y0 - 1.0), y0 + 1.0)
    return m, y, abs(continuous_plane(g, Np, m, y)[0])


# --------------------------------------------------------------------------
# Funnel transform of a volume (App. A): planes <-> points
# --------------------------------------------------------------------------
#
# Volume V[r, i, c]: Nz slices (z, the depth axis), Ny rows (y), Nx columns
# (x), all even.  The App. A steps, discretised the way Sec. 3.1 is for
# images: DFT along z of the expanded volume (Eq. A.2), the NVMT x' = s x,
# y' = s y with s = omega_3 / omega_max = 2 n3 / Nzp (Eq. A.3), the 2D DFT
# along x', y' (Eq. A.4) and the inverse DFT along omega_3 (Eqs. A.5, A.9).
# A plane z = a x + b y + c (centred coordinates) focuses at
# m1 = -a Nx/2, m2 = -b Ny/2 and z = c (Eq. A.9 with omega_max = pi); the
# volume P[z + Nzp/2, m2 + Ny/2, m1 + Nx/2] is real.

def padded_depth(Nz: int, Ny: int, Nx: int, padded_len: int = 0) -> int:
    """Length of the expanded z axis: Nz + Ny + Nx by default.  Over the
    volume a plane with |a|, |b| <= 1 moves by at most (Nx + Ny)/2 along z,
    so that many zero slices on each side keep its intercept from wrapping
    (the counterpart of the expansion of Sec. 4.2).  An explicit even length
    >= Nz may be asked for."""
    Nzp = Nz + Ny + Nx if padded_len == 0 else int(padded_len)
    if Nzp < Nz or Nzp % 2:
        raise ValueError("padded depth must be even and >= Nz")
    return Nzp


def expand_volume(vol: np.ndarray, Nzp: int) -> np.ndarray:
    """The Nz slices in an Nzp-slice zero frame, (Nzp - Nz)//2 zero slices
    in front of them."""
    Nz, Ny, Nx = vol.shape
    top = (Nzp - Nz) // 2
    out = np.zeros((Nzp, Ny, Nx), dtype=np.float64)
    out[top:top + Nz] = vol
    return out


def spectrum_z(vol_pad: np.ndarray) -> np.ndarray:
    """Eq. A.2: DFT of every (y, x) line along z,
    S[n3-1, i, c] = sum_z V_pad[z, i, c] exp(-j 2 pi n3 z / Nzp), centred z,
    for n3 = 1 .. Nzp/2-1 (negative n3 follow by conjugation)."""
    Nzp = vol_pad.shape[0]
    n3 = np.arange(1, Nzp // 2)
    z = np.arange(Nzp) - Nzp // 2
    E = np.exp(-2j * np.pi * np.outer(n3, z) / Nzp)
    return np.tensordot(E, vol_pad, axes=(1, 0))


def nvmt_bilinear(S: np.ndarray, Nzp: int, n3_first: int = 1) -> np.ndarray:
    """Eq. A.3: the NVMT x' = s x, y' = s y with s = 2 n3 / Nzp, realised by
    bilinear interpolation (linear along each axis, the 2D form of the linear
    option of Sec. V): g[n3, y', x'] = f(y'/s, x'/s), f = S[n3] on its integer
    grid and zero outside it.

    The fractional grid positions u = y'/s + Ny/2 = (y' Nzp + Ny n3)/(2 n3)
    and v = (x' Nzp + Nx n3)/(2 n3) are split with exact integer floors; the
    four neighbours carry the weights (1-t_u)(1-t_v), (1-t_u) t_v,
    t_u (1-t_v) and t_u t_v.  Slice k of S is frequency n3 = n3_first + k."""
    h, Ny, Nx = S.shape
    yp = np.arange(Ny, dtype=np.int64) - Ny // 2
    xp = np.arange(Nx, dtype=np.int64) - Nx // 2
    g = np.zeros_like(S)
    for k in range(h):
        n3 = n3_first + k
        f = S[k]
        den = 2 * n3
        nu = yp * Nzp + Ny * n3
        nv = xp * Nzp + Nx * n3
        i0 = nu // den
        j0 = nv // den
        tu = ((nu - i0 * den) / den)[:, None]
        tv = ((nv - j0 * den) / den)[None, :]
        I0, J0 = i0[:, None], j0[None, :]

        def tap(ii, jj):
            inside = (ii >= 0) & (ii < Ny) & (jj >= 0) & (jj < Nx)
            return np.where(inside, f[np.clip(ii, 0, Ny - 1), np.clip(jj, 0, Nx - 1)], 0.0)

        g[k] = ((1.0 - tu) * (1.0 - tv) * tap(I0, J0) + (1.0 - tu) * tv * tap(I0, J0 + 1)
                + tu * (1.0 - tv) * tap(I0 + 1, J0) + tu * tv * tap(I0 + 1, J0 + 1))
    return g


def dft_xy(g: np.ndarray) -> np.ndarray:
    """Eq. A.4: 2D DFT over x', y' of every slice,
    G[n3, m2, m1] = sum_{y', x'} g[n3, y', x'] exp(-j 2 pi (m1 x'/Nx + m2 y'/Ny)),
    centred x', y', m1, m2."""
    h, Ny, Nx = g.shape
    return np.matmul(np.matmul(_xdft_matrix(Ny), g), _xdft_matrix(Nx))


def idft_z(G: np.ndarray, Nzp: int) -> np.ndarray:
    """Eqs. A.5 / A.9: inverse DFT along omega_3, the negative half completed
    by G[-n3] = conj(G[n3]) (DC and Nyquist zero):
    P[z, m2, m1] = (1/Nzp) sum_n3 G[n3, m2, m1] exp(+j 2 pi n3 z / Nzp),
    z = -Nzp/2 .. Nzp/2-1.  Real; the imaginary part is checked to be
    rounding noise."""
    h, Ny, Nx = G.shape
    full = np.zeros((Nzp, Ny, Nx), dtype=np.complex128)
    n3 = np.arange(1, h + 1)
    full[n3 + Nzp // 2] = G
    full[-n3 + Nzp // 2] = np.conj(G)
    z = np.arange(Nzp) - Nzp // 2
    Winv = np.exp(2j * np.pi * np.outer(z, z) / Nzp)
    P = np.tensordot(Winv, full, axes=(1, 0)) / Nzp
    scale = max(1.0, float(np.abs(P.real).max()))
    if np.abs(P.imag).max() > 1e-9 * scale:
        raise AssertionError("inverse DFT of a Hermitian spectrum is not real")
    return P.real


def forward_volume(vol: np.ndarray, padded_len: int = 0) -> np.ndarray:
    """Funnel transform of one volume (App. A) on its expanded frame.
    Returns P[Nzp, Ny, Nx] in float64."""
    vol = np.asarray(vol, dtype=np.float64)
    Nz, Ny, Nx = vol.shape
    Nzp = padded_depth(Nz, Ny, Nx, padded_len)
    S = spectrum_z(expand_volume(vol, Nzp))
    return idft_z(dft_xy(nvmt_bilinear(S, Nzp)), Nzp)


def forward_volume_lines(vol: np.ndarray, lines, padded_len: int = 0) -> np.ndarray:
    """P[:, row, col] of forward_volume for the listed (row, col) =
    (m2 + Ny/2, m1 + Nx/2) pairs only, for volumes too large for the whole
    transform: the same steps, slice by slice, with Eq. A.4 evaluated at the
    listed bins only and Eq. A.5 written as the real part of the one-sided
    sum, P = (2/Nzp) Re sum_{n3=1}^{Nzp/2-1} G[n3] exp(+j 2 pi n3 z / Nzp).
    Returns [Nzp, len(lines)]."""
    vol = np.asarray(vol, dtype=np.float64)
    Nz, Ny, Nx = vol.shape
    Nzp = padded_depth(Nz, Ny, Nx, padded_len)
    h = Nzp // 2 - 1
    rows = np.array([r for r, _ in lines])
    cols = np.array([c for _, c in lines])
    ey = _xdft_matrix(Ny)[:, rows]           # [y', line]
    ex = _xdft_matrix(Nx)[:, cols]           # [x', line]
    S = spectrum_z(expand_volume(vol, Nzp))
    G = np.empty((h, len(lines)), dtype=np.complex128)
    for k in range(h):
        g = nvmt_bilinear(S[k:k + 1], Nzp, k + 1)[0]
        G[k] = np.einsum("yl,yx,xl->l", ey, g, ex)
    z = np.arange(Nzp) - Nzp // 2
    n3 = np.arange(1, h + 1)
    return (2.0 / Nzp) * np.real(np.exp(2j * np.pi * np.outer(z, n3) / Nzp) @ G)


def volume_boundary_mask(Nz: int, Ny: int, Nx: int, Nzp: int) -> np.ndarray:
    """Cells of the parameter volume (Nzp x Ny x Nx) where the artificial
    front and back faces created by the expansion focus (planes z = -Nz/2
    and z = Nz/2 with a = b = 0): bins m1, m2 in {-1, 0, 1} and slices within
    2 of either face, the same cells as the 2D border mask of Sec. 4.2 on
    every slope bin pair next to zero."""
    mask = np.zeros((Nzp, Ny, Nx), dtype=bool)
    rows = np.array([-1, 0, 1]) + Ny // 2
    cols = np.array([-1, 0, 1]) + Nx // 2
    for edge in (-Nz // 2, Nz // 2):
        zs = np.arange(edge - 2, edge + 2) + Nzp // 2
        zs = zs[(zs >= 0) & (zs < Nzp)]
        mask[np.ix_(zs, rows, cols)] = True
    return mask


def peaks_list_volume(B: np.ndarray, K: int, T: float, radius: int = 1,
                      mask: np.ndarray | None = None, wrap: bool = True) -> list[int]:
    """The list-based peak detection of Sec. 4.4 in the 3D parameter space
    (App. A detects planes as 3D peaks): cells visited in the order
    (brightness descending, linear index ascending); a cell is detected when
    no cell of its (2r+1)^3 neighbourhood was visited before it; every cell
    is marked visited; stop at K detections or the first cell below T.  Cells
    inside ``mask`` are visited but never detected.  The neighbourhood wraps
    (all three axes are periodic) unless ``wrap`` is False.  Returns linear
    indices (z, row, col order) in detection order."""
    B = np.asarray(B)
    nz, ny, nx = B.shape
    flat = B.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))
    visited = np.zeros(B.shape, dtype=bool)
    off = np.arange(-radius, radius + 1)
    detected: list[int] = []
    if K <= 0:
        return detected
    for idx in order:
        v = flat[idx]
        if v < T:
            break
        z, rem = divmod(int(idx), ny * nx)
        r, c = divmod(rem, nx)
        zz, rr, cc = z + off, r + off, c + off
        if wrap:
            zz, rr, cc = zz % nz, rr % ny, cc % nx
        else:
            zz = zz[(zz >= 0) & (zz < nz)]
            rr = rr[(rr >= 0) & (rr < ny)]
            cc = cc[(cc >= 0) & (cc < nx)]
        seen = visited[np.ix_(zz, rr, cc)].any()
        visited[z, r, c] = True
        if not seen and not (mask is not None and mask[z, r, c]):
            detected.append(int(idx))
            if len(detected) == K:
                break
    return detected


def plane_params(z: int, row: int, col: int, Nz: int, Ny: int, Nx: int, Nzp: int):
    """Eq. A.9 read backwards: cell -> plane, in voxel-index coordinates.
    m1 = col - Nx/2, m2 = row - Ny/2, a = -2 m1 / Nx, b = -2 m2 / Ny, centred
    intercept c0 = z - Nzp/2; the plane is ``slice = a * column + b * row + c``
    with c = c0 - a Nx/2 - b Ny/2 + Nz/2.  Returns (a, b, c)."""
    a = -2.0 * (col - Nx // 2) / Nx
    b = -2.0 * (row - Ny // 2) / Ny
    c0 = z - Nzp // 2
    return a, b, c0 - a * Nx / 2 - b * Ny / 2 + Nz / 2


# Parameter spaces of a volume.  Eq. A.9 focuses planes whose depth varies
# by at most one slice per row and column (|a|, |b| <= 1).  A steeper plane is
# one whose x (or y) varies slowly along the other two axes: it is found by
# the same transform with x (or y) as the depth axis, the 3D counterpart of
# the inverse space (Sec. 3.1, Remark 1).  In each space the transform runs on
# the volume with axes (depth, rows, cols):
#   "z": (z, y, x), the volume as stored;
#   "x": (x, z, y);
#   "y": (y, z, x);
# and a plane reads depth = a * col + b * row + c in that space's voxel
# indices.
VOLUME_SPACES = {"z": (0, 1, 2), "x": (2, 0, 1), "y": (1, 0, 2)}


def volume_in_space(vol: np.ndarray, space: str) -> np.ndarray:
    """The volume with its axes in the space's (depth, rows, cols) order."""
    return np.transpose(np.asarray(vol), VOLUME_SPACES[space])


def forward_volume_space(vol: np.ndarray, space: str, padded_len: int = 0) -> np.ndarray:
    """The volume transform in one parameter space: P[Lp][rows][cols] of the
    volume with the space's axis order, Lp = Nz + Ny + Nx by default."""
    return forward_volume(volume_in_space(vol, space), padded_len)
