"""Seeded synthetic line images (inputs only; no transform arithmetic here).

The paper evaluates on normalised grayscale images in [0, 1] (Sec. VI) holding
ridge-type and step-type straight edges (Fig. 2, Remark 2), under additive
Gaussian noise (Fig. 10), occlusion (Fig. 15) and line widths of one to a few
pixels (Fig. 14).  Its benchmark and natural images are not available, so
these generators stand in for them with the same kind of content.

Geometry.  Pixel (r, c) has its centre at index coordinates (r, c).  A line
that is not transposed is ``row = k * col + b`` (|k| <= 1); a transposed line
is ``col = k * row + b`` and is rendered on the transposed image.

* ridge of width w: a pixel gains (1 - background) times the length of the
  overlap of [r - 1/2, r + 1/2] with [y0 - w/2, y0 + w/2], y0 = k c + b;
* step of contrast a: a pixel gains a times the part of [r - 1/2, r + 1/2]
  that lies below the edge (rows greater than y0);
* an occlusion gap removes the contribution over a contiguous run of the
  columns where the line is inside the image, of length U[0.1, 0.5] times
  that run.

Finally N(0, sigma^2) noise is added and the image is clipped to [0, 1] and
cast to float32.  Every image draws from its own ``numpy`` generator seeded
by ``(config_id, seed, image_index)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BACKGROUND = 0.2


@dataclass
class Line:
    kind: str            # "ridge" or "step"
    transposed: bool     # False: row = k*col + b ; True: col = k*row + b
    k: float
    b: float
    width: float = 2.0   # ridge width in pixels
    contrast: float = 0.0  # step jump
    gap: tuple | None = None  # (start, stop) along the line's free axis


@dataclass
class SynthImage:
    image: np.ndarray            # float32 [N, M]
    lines: list = field(default_factory=list)
    sigma: float = 0.0


def _render(img: np.ndarray, ln: Line, bg: float) -> None:
    """Add one line's contribution to ``img`` (float64, modified in place)."""
    work = img.T if ln.transposed else img
    rows, cols = work.shape
    c = np.arange(cols, dtype=np.float64)
    y0 = ln.k * c + ln.b
    keep = np.ones(cols, dtype=bool)
    if ln.gap is not None:
        keep[int(ln.gap[0]):int(ln.gap[1])] = False
    if ln.kind == "ridge":
        amp = 1.0 - bg
        half = 0.5 * ln.width
        base = np.floor(y0).astype(np.int64)
        for d in range(-3, 4):
            r = base + d
            ok = keep & (r >= 0) & (r < rows)
            rr = r[ok].astype(np.float64)
            lo = np.maximum(rr - 0.5, y0[ok] - half)
            hi = np.minimum(rr + 0.5, y0[ok] + half)
            cov = np.clip(hi - lo, 0.0, 1.0)
            work[r[ok], np.nonzero(ok)[0]] += amp * cov
    elif ln.kind == "step":
        r = np.arange(rows, dtype=np.float64)[:, None]
        cov = np.clip(r + 0.5 - y0[None, :], 0.0, 1.0)
        cov[:, ~keep] = 0.0
        work += ln.contrast * cov
    else:
        raise ValueError(ln.kind)


def render(N: int, M: int, lines, sigma: float, rng: np.random.Generator,
           bg: float = BACKGROUND) -> np.ndarray:
    img = np.full((N, M), bg, dtype=np.float64)
    for ln in lines:
        _render(img, ln, bg)
    if sigma > 0:
        img += rng.normal(0.0, sigma, size=(N, M))
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def _in_image_run(ln: Line, N: int, M: int):
    rows, cols = (M, N) if ln.transposed else (N, M)
    y0 = ln.k * np.arange(cols) + ln.b
    inside = np.nonzero((y0 >= -0.5) & (y0 <= rows - 0.5))[0]
    return inside


def random_line(rng: np.random.Generator, N: int, M: int, kinds=("ridge", "step"),
                p_transposed: float = 0.5, p_gap: float = 0.2,
                widths=(1, 2, 3), contrast=(0.3, 0.8)) -> Line:
    kind = kinds[int(rng.integers(len(kinds)))]
    transposed = bool(rng.random() < p_transposed)
    k = float(rng.uniform(-1.0, 1.0))
    extent = M if transposed else N
    b = float(rng.uniform(0.0, extent))
    ln = Line(kind=kind, transposed=transposed, k=k, b=b)
    if kind == "ridge":
        ln.width = float(widths[int(rng.integers(len(widths)))])
    else:
        ln.contrast = float(rng.uniform(*contrast))
    if rng.random() < p_gap:
        inside = _in_image_run(ln, N, M)
        if inside.size > 4:
            glen = int(round(rng.uniform(0.1, 0.5) * inside.size))
            start = int(inside[0] + rng.integers(0, inside.size - glen + 1))
            ln.gap = (start, start + glen)
    return ln


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def _rng(config_id: int, seed: int, index: int) -> np.random.Generator:
    return np.random.default_rng([config_id, seed, index])


def single_ridge(seed: int = 0, size: int = 128, sigma: float = 0.05) -> SynthImage:
    """One 128x128 image with one 2-px ridge of intensity 1.0, slope U[-1,1],
    intercept U[0,128], background 0.2, noise sigma 0.05."""
    rng = _rng(1, seed, 0)
    ln = Line(kind="ridge", transposed=False, k=float(rng.uniform(-1, 1)),
              b=float(rng.uniform(0, size)), width=2.0)
    return SynthImage(render(size, size, [ln], sigma, rng), [ln], sigma)


def mixed_lines(N: int, M: int, n_lines, sigma: float, rng: np.random.Generator) -> SynthImage:
    if isinstance(n_lines, tuple):
        n = int(rng.integers(n_lines[0], n_lines[1] + 1))
    else:
        n = int(n_lines)
    lines = [random_line(rng, N, M) for _ in range(n)]
    return SynthImage(render(N, M, lines, sigma, rng), lines, sigma)


SIGMAS = (0.05, 0.1, 0.2)
RAGGED_SIZES = ((240, 320), (480, 640), (720, 1280), (1080, 1920))


def batch(config: str, count: int | None = None, seed: int = 0, size: int | None = None):
    """Return a list of SynthImage for one of the workloads:

    ``"single"``  1 x 128^2, one 2-px ridge, sigma 0.05;
    ``"plain"``   64 x 512^2, 3-10 mixed lines, sigma cycling 0.05/0.1/0.2;
    ``"grad"``    32 x 1024^2, 5 mixed lines, sigma cycling;
    ``"ragged"``  256 images of 240x320 / 480x640 / 720x1280 / 1080x1920,
                  2-12 mixed lines, sigma 0.1;
    ``"precision"`` 8 x 2048^2, 10 mixed lines, sigma 0.1.
    ``count`` and ``size`` shrink a workload for tests."""
    out = []
    if config == "single":
        n = count or 1
        return [single_ridge(seed * 100003 + i, size or 128) for i in range(n)]
    if config == "plain":
        n, s, cid = count or 64, size or 512, 2
        for i in range(n):
            rng = _rng(cid, seed, i)
            out.append(mixed_lines(s, s, (3, 10), SIGMAS[i % 3], rng))
    elif config == "grad":
        n, s, cid = count or 32, size or 1024, 3
        for i in range(n):
            rng = _rng(cid, seed, i)
            out.append(mixed_lines(s, s, 5, SIGMAS[i % 3], rng))
    elif config == "ragged":
        n, cid = count or 256, 4
        for i in range(n):
            rng = _rng(cid, seed, i)
            N, M = RAGGED_SIZES[int(rng.integers(len(RAGGED_SIZES)))]
            out.append(mixed_lines(N, M, (2, 12), 0.1, rng))
    elif config == "precision":
        n, s, cid = count or 8, size or 2048, 5
        for i in range(n):
            rng = _rng(cid, seed, i)
            out.append(mixed_lines(s, s, 10, 0.1, rng))
    else:
        raise ValueError(config)
    return out


def stack(images) -> np.ndarray:
    """Stack equally sized SynthImage objects into a float32 [B, N, M] array."""
    return np.stack([im.image for im in images]).astype(np.float32)


# --------------------------------------------------------------------------
# Volumes holding planes (the 3D form, App. A)
# --------------------------------------------------------------------------
#
# Voxel (s, r, c) = (slice, row, column) has its centre at those index
# coordinates.  A sheet is the plane ``slice = a * col + b * row + c0`` with
# |a|, |b| <= 1, rendered like a ridge line along z: a voxel gains
# (1 - background) times the overlap of [s - 1/2, s + 1/2] with
# [z0 - w/2, z0 + w/2], z0 = a c + b r + c0.  Noise and clipping as for images.

@dataclass
class Sheet:
    a: float
    b: float
    c: float
    width: float = 1.0


@dataclass
class SynthVolume:
    volume: np.ndarray           # float32 [Nz, Ny, Nx]
    sheets: list = field(default_factory=list)
    sigma: float = 0.0


def render_volume(Nz: int, Ny: int, Nx: int, sheets, sigma: float, rng: np.random.Generator,
                  bg: float = BACKGROUND) -> np.ndarray:
    vol = np.full((Nz, Ny, Nx), bg, dtype=np.float64)
    r = np.arange(Ny, dtype=np.float64)[:, None]
    c = np.arange(Nx, dtype=np.float64)[None, :]
    amp = 1.0 - bg
    for sh in sheets:
        z0 = sh.a * c + sh.b * r + sh.c
        half = 0.5 * sh.width
        base = np.floor(z0).astype(np.int64)
        for d in range(-3, 4):
            s = base + d
            ok = (s >= 0) & (s < Nz)
            ss = s.astype(np.float64)
            cov = np.clip(np.minimum(ss + 0.5, z0 + half) - np.maximum(ss - 0.5, z0 - half), 0.0, 1.0)
            rr, cc = np.nonzero(ok)
            vol[s[ok], rr, cc] += amp * cov[ok]
    if sigma > 0:
        vol += rng.normal(0.0, sigma, size=vol.shape)
    return np.clip(vol, 0.0, 1.0).astype(np.float32)


def random_sheet(rng: np.random.Generator, Nz: int, Ny: int, Nx: int, widths=(1, 2)) -> Sheet:
    """A sheet with |a|, |b| < 0.9 that crosses the centre slab of the volume."""
    a = float(rng.uniform(-0.9, 0.9))
    b = float(rng.uniform(-0.9, 0.9))
    zc = float(rng.uniform(0.25 * Nz, 0.75 * Nz))        # slice at the volume's centre column
    return Sheet(a, b, zc - a * Nx / 2 - b * Ny / 2, float(widths[int(rng.integers(len(widths)))]))


def sheet_volume(Nz: int, Ny: int, Nx: int, n_sheets, sigma: float, rng: np.random.Generator) -> SynthVolume:
    if isinstance(n_sheets, tuple):
        n_sheets = int(rng.integers(n_sheets[0], n_sheets[1] + 1))
    sheets = [random_sheet(rng, Nz, Ny, Nx) for _ in range(n_sheets)]
    return SynthVolume(render_volume(Nz, Ny, Nx, sheets, sigma, rng), sheets, sigma)


def volume_batch(count: int = 4, size: int = 256, seed: int = 0, n_sheets=(2, 6), sigma: float = 0.1):
    """``count`` volumes of size^3 voxels, each with 2-6 sheets (widths 1-2
    voxels) under N(0, 0.1^2) noise; volume i draws from the generator seeded
    by (6, seed, i)."""
    return [sheet_volume(size, size, size, n_sheets, sigma, _rng(6, seed, i)) for i in range(count)]
