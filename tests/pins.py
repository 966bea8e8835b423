"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each ``check_*`` function raises AssertionError when the oracle (passed in as
a module ``O``) breaks the pin, so the same checks run against the real oracle
(tests/test_oracle_pins.py) and against deliberately broken copies of it
(tests/test_oracle_mutants.py)."""
from __future__ import annotations

import os

import numpy as np

from paper_1904_09409_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split()
            out[key] = float(val)
    return out


def expected_cell(ln: synth.Line, N: int, M: int, Np: int):
    """Line -> point (Eq. 19 with the centred frame of Sec. 4.2 and
    omega_max = pi): the plane, row and column where the line should focus.

    A line ``row = k col + b`` has centred intercept b + k M/2 - N/2 and
    peaks at m1 = -k M/2 in the regular plane; a transposed line does the same
    on the transposed image in the inverse plane."""
    if not ln.transposed:
        bc = ln.b + ln.k * M / 2 - N / 2
        return "regular", int(round(bc)) + Np // 2, (int(round(-ln.k * M / 2)) + M // 2) % M
    bc = ln.b + ln.k * N / 2 - M / 2
    return "inverse", int(round(bc)) + Np // 2, (int(round(-ln.k * N / 2)) + N // 2) % N


def torus_dist(a, b, n):
    d = abs(a - b) % n
    return min(d, n - d)


# ----------------------------------------------------------------- DFT stages

def check_spectrum_is_library_fft(O):
    """Stage a2 reduces to numpy's FFT of the expanded column: the centred
    frame only multiplies frequency n2 by (-1)^n2."""
    rng = np.random.default_rng(11)
    for (N, M, Np) in [(12, 8, 20), (6, 10, 16), (16, 16, 40)]:
        img = rng.random((N, M))
        pad = np.zeros((Np, M))
        top = (Np - N) // 2
        pad[top:top + N] = img
        ref = np.fft.fft(pad, axis=0)
        n2 = np.arange(1, Np // 2)
        ref = ref[n2] * ((-1.0) ** n2)[:, None]
        got = O.spectrum_y(O.expand(img, Np))
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def check_xdft_is_library_fft(O):
    """Stage a4 reduces to numpy's FFT with both axes centred (fftshift)."""
    rng = np.random.default_rng(12)
    g = rng.standard_normal((5, 16)) + 1j * rng.standard_normal((5, 16))
    ref = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(g, axes=1), axis=1), axes=1)
    assert np.abs(O.dft_x(g) - ref).max() <= 1e-12 * np.abs(ref).max()


def check_ydft_inverse_is_library_ifft(O):
    """Stage a5 reduces to numpy's inverse FFT of the Hermitian-completed,
    centred spectrum."""
    rng = np.random.default_rng(13)
    Np, M = 20, 6
    h = Np // 2 - 1
    G = rng.standard_normal((h, M)) + 1j * rng.standard_normal((h, M))
    full = np.zeros((Np, M), complex)          # natural FFT order
    n2 = np.arange(1, h + 1)
    full[n2] = G * ((-1.0) ** n2)[:, None]      # centred y => (-1)^n2
    full[Np - n2] = np.conj(full[n2])
    # (-1)^n2 already moves the origin: row r of the ifft is y = r - Np/2
    ref = np.fft.ifft(full, axis=0).real
    got = O.idft_y(G, Np)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def check_parseval(O):
    """Parseval per stage.  The dropped DC and Nyquist rows of stage a2 are
    the column sum and the alternating column sum (closed forms)."""
    rng = np.random.default_rng(14)
    N, M = 10, 8
    Np = N + M
    img = rng.random((N, M))
    pad = O.expand(img, Np)
    S = O.spectrum_y(pad)
    dc = pad.sum(axis=0)
    y = np.arange(Np) - Np // 2
    nyq = (pad * ((-1.0) ** y)[:, None]).sum(axis=0)
    lhs = 2 * (np.abs(S) ** 2).sum() + (dc ** 2).sum() + (nyq ** 2).sum()
    assert abs(lhs - Np * (pad ** 2).sum()) <= 1e-10 * lhs
    g = O.nvmt(S, Np)
    G = O.dft_x(g)
    assert abs((np.abs(G) ** 2).sum() - M * (np.abs(g) ** 2).sum()) <= 1e-10 * (np.abs(G) ** 2).sum()
    P = O.idft_y(G, Np)
    assert abs((P ** 2).sum() - (2.0 / Np) * (np.abs(G) ** 2).sum()) <= 1e-10 * (P ** 2).sum()


# ----------------------------------------------------------------- NVMT

def check_nvmt_exact_on_linear_rows(O):
    """Linear interpolation reproduces a row that is linear in the sample
    index exactly: g[x'] = a + b*i_p with i_p = x'/s + M/2, s = 2 n2/Np,
    wherever i_p lies in [0, M-1]; where i_p < -1 or i_p > M the row is 0."""
    M, Np = 16, 40
    h = Np // 2 - 1
    a, b = 0.7 - 0.2j, 0.3 + 0.11j
    i = np.arange(M)
    S = np.tile(a + b * i, (h, 1))
    g = O.nvmt(S, Np)
    xp = np.arange(M) - M // 2
    for n2 in range(1, h + 1):
        s = 2.0 * n2 / Np
        ip = xp / s + M / 2
        inside = (ip >= 0) & (ip <= M - 1)
        assert np.abs(g[n2 - 1, inside] - (a + b * ip[inside])).max() < 1e-12
        outside = (ip < -1) | (ip > M)
        assert np.abs(g[n2 - 1, outside]).max(initial=0.0) == 0.0


def check_nvmt_funnel_support(O):
    """Fig. 1: the rectangular support of a row is compressed to width s*M
    (the double triangle), i.e. about 2 n2 M / Np nonzero samples."""
    M, Np = 64, 128
    h = Np // 2 - 1
    S = np.ones((h, M), complex)
    g = O.nvmt(S, Np)
    for n2 in range(1, h + 1):
        width = np.count_nonzero(np.abs(g[n2 - 1]) > 0)
        assert abs(width - 2.0 * n2 * M / Np) <= 2.0, (n2, width)


# ----------------------------------------------------------------- whole forward

def check_point_to_line(O):
    """Eq. 13 with omega_max = pi: a single bright pixel at centred (u, v)
    becomes the line y = v + 2 u m1 / M.  Linear interpolation of a one-sample
    delta aliases column by column (the paper's relation assumes exact
    resampling), so the pin is a |P|^2-weighted least-squares line through
    the cells within +-6 rows of the prediction over the central half of the
    slope bins: intercept within half a cell, slope within 15 %."""
    N = M = 128
    Np = N + M
    for (u, v) in [(10, 5), (-13, -7), (20, 0), (-25, 11), (7, -20)]:
        img = np.zeros((N, M))
        img[v + N // 2, u + M // 2] = 1.0
        B2 = O.forward_regular(img) ** 2
        xs, ys, ws = [], [], []
        for col in range(M):
            m1 = col - M // 2
            if abs(m1) > M // 4:
                continue
            pred = v + 2.0 * u * m1 / M
            y = np.arange(int(np.floor(pred)) - 6, int(np.floor(pred)) + 8)
            xs += [m1] * len(y)
            ys += list(y)
            ws += list(B2[(y + Np // 2) % Np, col])
        xs, ys, ws = (np.asarray(a, dtype=np.float64) for a in (xs, ys, ws))
        A = np.stack([np.ones_like(xs), xs], axis=1) * np.sqrt(ws)[:, None]
        icpt, slope = np.linalg.lstsq(A, ys * np.sqrt(ws), rcond=None)[0]
        assert abs(icpt - v) <= 0.5, (u, v, icpt)
        assert abs(slope - 2.0 * u / M) <= 0.15 * abs(2.0 * u / M), (u, v, slope)


def check_line_to_point(O):
    """Eq. 19: an ideal long ridge line y = k x + b focuses within one cell of
    (m1 = -k M/2, y = b); lines with |slope| > 1 focus the same way in the
    inverse plane."""
    rng = np.random.default_rng(21)
    N = M = 96
    Np = N + M
    hits = 0
    for trial in range(8):
        transposed = bool(trial % 2)
        k = float(rng.uniform(-0.9, 0.9))
        extent = M if transposed else N
        # keep the whole line inside the frame so it is long
        b = float(rng.uniform(0.3 * extent, 0.7 * extent)) - k * extent / 2
        ln = synth.Line("ridge", transposed, k, b, width=1.0)
        img = synth.render(N, M, [ln], 0.0, rng, bg=0.0)
        space, er, ec = expected_cell(ln, N, M, Np)
        P = O.forward_regular(img) if space == "regular" else O.forward_inverse(img)
        B = np.abs(P)
        r, c = np.unravel_index(np.argmax(B), B.shape)
        assert torus_dist(r, er, B.shape[0]) <= 1 and torus_dist(c, ec, B.shape[1]) <= 1, \
            (trial, space, (r, c), (er, ec))
        hits += 1
    assert hits == 8


def check_fig9_worked_example(O):
    """Sec. 4.5, Fig. 9: a 170x428 (width x height) image holding one line of
    slope 3.27.  The paper reads its inverse-space peak at (m, n) = (18, 65)
    and a wrapped regular-space peak at (-61, -58).  A ridge of that slope
    through the centred point (18, 0) reproduces the inverse peak exactly;
    the wrapped regular peak lands within one cell of the printed one (the
    printed slope has two decimals, and the printed cells are mutually
    consistent only to about one cell: m = -61 alone means slope 3.282)."""
    gold = read_golden("fig9_wrap_example.txt")
    M, N = int(gold["width_M"]), int(gold["height_N"])
    Np = N + M
    kinv = 1.0 / gold["slope"]
    bx = gold["inverse_peak_m"] - kinv * N / 2 + M / 2
    ln = synth.Line("ridge", True, kinv, bx, width=1.0)
    img = synth.render(N, M, [ln], 0.0, np.random.default_rng(0), bg=0.2)
    P, Pinv = O.forward(img)
    # inverse space: global maximum outside the border cells
    Bi = np.where(O.boundary_mask(M, N, Np), 0.0, np.abs(Pinv))
    r, c = np.unravel_index(np.argmax(Bi), Bi.shape)
    assert r - Np // 2 == gold["inverse_peak_m"]
    assert -(c - N // 2) == gold["inverse_peak_n"]           # paper n = -n1
    # the x-intercept and inverse slope read back by Eqs. 24-25
    kinv_read = 2.0 * gold["inverse_peak_n"] / N
    assert abs(1.0 / kinv_read - gold["slope"]) < 0.03
    # regular space: the strongest peak is the wrapped one
    B = np.abs(P)
    det = O.peaks_list(B, 1, 0.0, 1, O.boundary_mask(N, M, Np))
    rr, cc = divmod(det[0], M)
    m_paper = -(cc - M // 2)
    n_paper = rr - Np // 2
    assert abs(m_paper - gold["regular_peak_m"]) <= 1
    assert abs(n_paper - gold["regular_peak_n"]) <= 1
    k_read = 2.0 * m_paper / M                                # Eq. 22
    assert abs(k_read - gold["regular_slope_read"]) <= 2.0 / M + 0.01
    # Eq. 21: the wrapped slope is the true one minus 2q
    assert abs((gold["slope"] - 4.0) - k_read) <= 2.0 / M + 0.01


def check_fig6_intercept_wrap(O):
    """Eq. 20 / Fig. 6: with no expansion (Np = N) a line whose intercept
    exceeds N/2 shows up wrapped at b - N; on the expanded frame (Np = N+M)
    it shows up at b.  The slope cell is the same in both."""
    N, M = 64, 256
    k, bc = 0.5, 40.0
    b = bc - k * M / 2 + N / 2
    ln = synth.Line("ridge", False, k, b, width=2.0)
    img = synth.render(N, M, [ln], 0.0, np.random.default_rng(0), bg=0.0)
    for Np, want in [(N, bc - N), (N + M, bc)]:
        B = np.abs(O.forward_regular(img, Np))
        r, c = np.unravel_index(np.argmax(B), B.shape)
        assert abs((r - Np // 2) - want) <= 1, (Np, r - Np // 2, want)
        assert c - M // 2 == int(round(-k * M / 2))


def check_fig7_slope_wrap(O):
    """Eq. 21 / Fig. 7: a line of slope sqrt(3) (second group) appears in the
    regular plane wrapped to slope sqrt(3) - 2: a local maximum within one
    slope cell of m1 = -(sqrt(3)-2) M/2 and y = its intercept."""
    N = M = 128
    Np = N + M
    k = np.sqrt(3.0)
    x0 = 10.0                                   # line through centred (10, 0)
    kinv = 1.0 / k
    bx = x0 - kinv * N / 2 + M / 2
    ln = synth.Line("ridge", True, kinv, bx, width=1.0)
    img = synth.render(N, M, [ln], 0.0, np.random.default_rng(0), bg=0.0)
    B = np.abs(O.forward_regular(img))
    er = int(round(-k * x0)) + Np // 2
    ec = int(round(-(k - 2.0) * M / 2)) + M // 2
    win = B[er - 2:er + 3, ec - 2:ec + 3]
    r, c = np.unravel_index(np.argmax(win), win.shape)
    r, c = r + er - 2, c + ec - 2
    assert abs(r - er) <= 1 and abs(c - ec) <= 1
    nb = B[r - 1:r + 2, c - 1:c + 2].copy()
    nb[1, 1] = -1
    assert B[r, c] > nb.max()


def check_shift_equivariance(O):
    """Moving the content d rows down inside the frame rolls the plane by d
    rows exactly (the y DFT and the inverse y DFT use opposite phases)."""
    rng = np.random.default_rng(31)
    N, M, d = 32, 24, 5
    img = np.zeros((N, M))
    img[4:N - 8] = rng.random((N - 12, M))
    sh = np.roll(img, d, axis=0)
    P0 = O.forward_regular(img)
    P1 = O.forward_regular(sh)
    assert np.abs(P1 - np.roll(P0, d, axis=0)).max() <= 1e-12 * np.abs(P0).max()


def check_linearity(O):
    rng = np.random.default_rng(32)
    a, b = rng.random((12, 8)), rng.random((12, 8))
    Pa, Pb = O.forward(a)[0], O.forward(b)[0]
    Pab = O.forward(2.0 * a - 3.0 * b)[0]
    assert np.abs(Pab - (2.0 * Pa - 3.0 * Pb)).max() <= 1e-12 * np.abs(Pab).max()


# ----------------------------------------------------------------- adjoint

def check_adjoint_dot(O, kind="linear"):
    """<F x, y> = <x, F^T y> for both spaces together."""
    rng = np.random.default_rng(41)
    for (N, M) in [(8, 8), (10, 6), (16, 12)]:
        Np = N + M
        x = rng.standard_normal((N, M))
        y0 = rng.standard_normal((Np, M))
        y1 = rng.standard_normal((Np, N))
        P, Pi = O.forward(x, 0, kind)
        lhs = (P * y0).sum() + (Pi * y1).sum()
        rhs = (x * O.adjoint(y0, y1, N, M, 0, kind)).sum()
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def dense_forward(O, N, M, space, kind="linear"):
    f = O.forward_regular if space == "regular" else O.forward_inverse
    cols = []
    for i in range(N * M):
        e = np.zeros(N * M)
        e[i] = 1.0
        cols.append(f(e.reshape(N, M), 0, kind).ravel())
    return np.stack(cols, axis=1)


def dense_adjoint(O, N, M, space, kind="linear"):
    Np = N + M
    shape = (Np, M) if space == "regular" else (Np, N)
    f = O.adjoint_regular if space == "regular" else O.adjoint_inverse
    rows = []
    for j in range(shape[0] * shape[1]):
        e = np.zeros(shape[0] * shape[1])
        e[j] = 1.0
        rows.append(f(e.reshape(shape), N, M, 0, kind).ravel())
    return np.stack(rows, axis=1)


def check_adjoint_dense(O, N=8, M=8, kind="linear"):
    """The adjoint applied to every unit plane equals the transpose of the
    forward applied to every unit image."""
    for space in ("regular", "inverse"):
        F = dense_forward(O, N, M, space, kind)
        Ft = dense_adjoint(O, N, M, space, kind)
        assert np.abs(Ft - F.T).max() <= 1e-12 * np.abs(F).max()


def check_adjoint_finite_difference(O):
    """Central finite differences (h = 1e-4, FP64) of the loss
    L = sum over chosen cells of |P| agree with the adjoint applied to
    sign(P) on those cells.  L is piecewise linear, so the difference is
    exact up to rounding wherever no chosen cell crosses zero within h."""
    rng = np.random.default_rng(42)
    N = M = 16
    Np = N + M
    img = rng.random((N, M))
    P, Pi = O.forward(img)
    sel = np.argsort(-np.abs(P).ravel())[:6]
    seli = np.argsort(-np.abs(Pi).ravel())[:6]

    def loss(x):
        a, b = O.forward(x)
        return np.abs(a.ravel()[sel]).sum() + np.abs(b.ravel()[seli]).sum()

    dP = np.zeros(Np * M)
    dP[sel] = np.sign(P.ravel()[sel])
    dPi = np.zeros(Np * N)
    dPi[seli] = np.sign(Pi.ravel()[seli])
    grad = O.adjoint(dP.reshape(Np, M), dPi.reshape(Np, N), N, M)
    h = 1e-4
    fd = np.zeros_like(img)
    for i in range(N):
        for j in range(M):
            e = np.zeros_like(img)
            e[i, j] = h
            fd[i, j] = (loss(img + e) - loss(img - e)) / (2 * h)
    assert np.abs(fd - grad).max() <= 1e-7 * np.abs(grad).max()


# ----------------------------------------------------------------- peaks

def local_max_peaks(B, K, T, radius=1, mask=None, wrap=True):
    """Brute force: a cell precedes another if it is brighter, or equally
    bright with a lower linear index.  The first K cells (in that order) that
    precede every other cell of their neighbourhood, are >= T and not masked."""
    rows, cols = B.shape
    out = []
    for r in range(rows):
        for c in range(cols):
            if B[r, c] < T or (mask is not None and mask[r, c]):
                continue
            me = r * cols + c
            ok = True
            for dr in range(-radius, radius + 1):
                for dc in range(-radius, radius + 1):
                    rr, cc = r + dr, c + dc
                    if wrap:
                        rr, cc = rr % rows, cc % cols
                    elif not (0 <= rr < rows and 0 <= cc < cols):
                        continue
                    q = rr * cols + cc
                    if q == me:
                        continue
                    if B[rr, cc] > B[r, c] or (B[rr, cc] == B[r, c] and q < me):
                        ok = False
            if ok:
                out.append(me)
    out.sort(key=lambda i: (-B.flat[i], i))
    return out[:K]


def check_peaks_equal_local_maxima(O, trials=150):
    """The literal list algorithm of Sec. 4.4 equals 'first K local maxima
    under the total order' (every cell is marked visited when reached, so a
    visited neighbour is exactly a preceding neighbour).  Tie-heavy planes."""
    rng = np.random.default_rng(51)
    for t in range(trials):
        rows, cols = int(rng.integers(3, 9)), int(rng.integers(3, 9))
        B = rng.integers(0, 4, size=(rows, cols)).astype(np.float64)
        K = int(rng.integers(1, 8))
        T = float(rng.integers(0, 3))
        radius = int(rng.integers(1, 3))
        wrap = bool(rng.integers(2))
        mask = rng.random((rows, cols)) < 0.15
        got = O.peaks_list(B, K, T, radius, mask, wrap)
        want = local_max_peaks(B, K, T, radius, mask, wrap)
        assert got == want, (t, got, want)


def check_peak_params(O):
    """Eqs. 22-25: reading the focus cell of a line back gives its slope to
    within one slope step and its intercept to within a pixel plus half a
    slope step times the half width."""
    rng = np.random.default_rng(61)
    N, M = 48, 64
    Np = N + M
    for transposed in (False, True):
        for _ in range(10):
            k = float(rng.uniform(-1, 1))
            ln = synth.Line("ridge", transposed, k, float(rng.uniform(0, M if transposed else N)))
            space, r, c = expected_cell(ln, N, M, Np)
            kk, bb = O.peak_params(r, c, N, M, Np, space)
            width = N if transposed else M
            kd = (kk - k + 1.0) % 2.0 - 1.0          # slope is periodic (Eq. 21)
            assert abs(kd) <= 1.0 / width + 1e-12
            if abs(kk - k) < 0.5:
                assert abs(bb - ln.b) <= 0.5 + (1.0 / width) * width / 2 + 1e-9


# ----------------------------------------------------------------- chirp-z (band-limited) NVMT

def ramp_kernel(t, Np):
    """h(t) = (1/Np) sum over n2 != 0, Np/2 of |2 n2 / Np| exp(j 2 pi n2 t / Np):
    the ramp filter of the y DFT's rows, as a real cosine sum."""
    n = np.arange(1, Np // 2)
    t = np.asarray(t, dtype=np.float64)
    return (2.0 / Np) * (np.cos(2 * np.pi * np.multiply.outer(t, n) / Np) * (2.0 * n / Np)).sum(axis=-1)


def slant_stack(img, Np):
    """Band-limited funnel transform evaluated in the image domain: every
    pixel (x, y0) spreads the ramp kernel along its line y = y0 + 2 m1 x / M
    of the parameter plane (point-to-line mapping, Eq. 13 with omega_max = pi,
    under the ramp weighting |s| of the NVMT):
        P(m1, y) = sum_{x, y0} I(x, y0) h(y - y0 - 2 m1 x / M).
    This is the chirp-z funnel transform composed in closed form; it shares
    no step with the oracle's DFT route."""
    N, M = img.shape
    top = (Np - N) // 2
    m1 = np.arange(M) - M // 2
    y = np.arange(Np) - Np // 2
    P = np.zeros((Np, M))
    for r in range(N):
        for c in range(M):
            if img[r, c] == 0.0:
                continue
            x, y0 = c - M // 2, r + top - Np // 2
            P += img[r, c] * ramp_kernel(y[:, None] - y0 - 2.0 * m1[None, :] * x / M, Np)
    return P


def check_chirpz_slant_stack(O):
    """The chirp-z oracle equals the slant-stack closed form in both spaces,
    for the default and an enlarged padded length, square and not."""
    rng = np.random.default_rng(51)
    for (N, M, pl) in [(8, 8, 0), (16, 12, 0), (10, 14, 30), (12, 6, 0)]:
        img = rng.random((N, M))
        Np = O.padded_length(N, M, pl)
        P, Pi = O.forward(img, pl, "chirpz")
        for got, want in ((P, slant_stack(img, Np)), (Pi, slant_stack(img.T, Np))):
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), (N, M, pl)


def check_chirpz_special_rows(O):
    """Rows whose ratio s is 1/2 or 1/4 are zero-padded DFTs: with K = 1/s,
    G[m1] = s * FFT_{K M}(row placed at x mod K M)[m1 mod K M]."""
    rng = np.random.default_rng(52)
    M, Np = 24, 48
    h = Np // 2 - 1
    S = rng.standard_normal((h, M)) + 1j * rng.standard_normal((h, M))
    G = O.nvmt_dft_chirpz(S, Np)
    x = np.arange(M) - M // 2
    for K in (2, 4):
        n2 = Np // (2 * K)
        a = np.zeros(K * M, dtype=np.complex128)
        a[x % (K * M)] = S[n2 - 1]
        want = np.fft.fft(a)[x % (K * M)] / K
        assert np.abs(G[n2 - 1] - want).max() <= 1e-12 * np.abs(want).max(), K


def check_chirpz_point_to_line(O):
    """A one-pixel image at centred (u, v) maps to the ramp kernel centred on
    the line y = v + 2 u m1 / M: in every slope column where that offset is a
    whole number of rows, the column's maximum sits exactly on the line."""
    N = M = 64
    Np = N + M
    for (u, v) in [(16, 5), (-16, -9), (8, 0), (-24, 13)]:
        img = np.zeros((N, M))
        img[v + N // 2, u + M // 2] = 1.0
        P = O.forward_regular(img, 0, "chirpz")
        checked = 0
        for col in range(M):
            m1 = col - M // 2
            if (2 * u * m1) % M:
                continue
            y = v + 2 * u * m1 // M
            assert int(np.argmax(P[:, col])) == (y + Np // 2) % Np, (u, v, m1)
            checked += 1
        assert checked >= M // 4


def check_chirpz_line_to_point(O):
    """Eq. 19 holds for the band-limited NVMT as for the linear one: a long
    ridge line focuses within one cell of (m1 = -k M/2, y = b)."""
    rng = np.random.default_rng(23)
    N = M = 64
    Np = N + M
    for trial in range(6):
        transposed = bool(trial % 2)
        k = float(rng.uniform(-0.9, 0.9))
        extent = M if transposed else N
        b = float(rng.uniform(0.3 * extent, 0.7 * extent)) - k * extent / 2
        ln = synth.Line("ridge", transposed, k, b, width=1.0)
        img = synth.render(N, M, [ln], 0.0, rng, bg=0.0)
        space, er, ec = expected_cell(ln, N, M, Np)
        P = O.forward_regular(img, 0, "chirpz") if space == "regular" else O.forward_inverse(img, 0, "chirpz")
        B = np.abs(P)
        r, c = np.unravel_index(np.argmax(B), B.shape)
        assert torus_dist(r, er, B.shape[0]) <= 1 and torus_dist(c, ec, B.shape[1]) <= 1, \
            (trial, space, (r, c), (er, ec))


def check_chirpz_adjoint_dot(O):
    check_adjoint_dot(O, "chirpz")


def check_chirpz_adjoint_dense(O):
    check_adjoint_dense(O, 8, 8, "chirpz")


def check_column_samplers(O):
    """The column samplers used on large planes return exactly the columns of
    the whole-plane oracle (both NVMT kinds, non-default padding)."""
    rng = np.random.default_rng(53)
    for kind in O.NVMT_KINDS:
        for (N, M, pl) in [(12, 16, 0), (10, 8, 24)]:
            img = rng.random((N, M))
            Np = O.padded_length(N, M, pl)
            cols = np.array([0, 3, M // 2, M - 1])
            P = O.forward_regular(img, pl, kind)
            assert np.abs(O.forward_regular_columns(img, cols, pl, kind) - P[:, cols]).max() <= 1e-12 * np.abs(P).max()
            dP = rng.standard_normal((Np, M))
            dI = O.adjoint_regular(dP, N, M, pl, kind)
            got = O.adjoint_regular_columns(dP, N, M, cols, pl, kind)
            assert np.abs(got - dI[:, cols]).max() <= 1e-12 * np.abs(dI).max()


# ----------------------------------------------------------------- line verification (Sec. 4.5)

def check_verify_constant_and_ramp(O):
    """On a constant image every offset of the band averages to the constant;
    on a linear ramp I = a r + b c + g linear interpolation is exact, so the
    profile is a (mean y_c + d) + b mean(c) + g over the positions in the
    band, which for a line inside the image is every column."""
    N, M = 48, 64
    for D in (1, 2, 3):
        prof, n = O.line_band_profile(np.full((N, M), 0.37), "regular", 0.25, 10.3, D)
        assert n == M and np.allclose(prof, 0.37, rtol=0, atol=1e-12)
    a, b, g = 0.013, -0.004, 0.5
    r, c = np.mgrid[0:N, 0:M]
    img = a * r + b * c + g
    k, icpt = 0.25, 10.3
    cols = np.arange(M)
    ys = (np.float64(np.float32(k)) * cols + np.float64(np.float32(icpt))).astype(np.float32).astype(np.float64)
    for D in (1, 3):
        prof, n = O.line_band_profile(img, "regular", k, icpt, D)
        want = a * (ys.mean() + np.arange(-D, D + 1)) + b * cols.mean() + g
        assert n == M and np.abs(prof - want).max() <= 1e-12
    # inverse space: col = k row + icpt over the rows, same ramp read across columns
    prof, n = O.line_band_profile(img, "inverse", -0.3, 40.2, 2)
    rows = np.arange(N)
    xs = (np.float64(np.float32(-0.3)) * rows + np.float64(np.float32(40.2))).astype(np.float32).astype(np.float64)
    want = a * rows.mean() + b * (xs.mean() + np.arange(-2, 3)) + g
    assert n == N and np.abs(prof - want).max() <= 1e-12


def check_verify_band_limits(O):
    """A line position y enters the band only when the rows it reads,
    floor(y) - D .. floor(y) + D + 1, are all inside the image (the last one
    even when its weight is zero): a horizontal line at row 1.5 has no
    position with D = 3 and every column with D = 1 (rows 0..3)."""
    img = np.ones((16, 20))
    assert O.line_band_profile(img, "regular", 0.0, 1.5, 3)[1] == 0
    assert O.line_band_profile(img, "regular", 0.0, 1.5, 1)[1] == 20
    assert O.line_band_profile(img, "regular", 0.0, 12.5, 2)[1] == 20     # rows 10..15
    assert O.line_band_profile(img, "regular", 0.0, 13.0, 2)[1] == 0      # rows 11..16
    # a slope of 1 from row 3 with D = 3: columns 0 .. 8 (rows 0..7 up to 8..15)
    assert O.line_band_profile(img, "regular", 1.0, 3.0, 3)[1] == 9
    # the inverse space counts rows: col = 0.5 row + 2 with D = 2 on 20 columns
    # needs floor(x) >= 2 and floor(x) <= 16: every row of 16
    assert O.line_band_profile(img, "inverse", 0.5, 2.0, 2)[1] == 16


def check_verify_ridge_and_step(O):
    """Step 4 on exact patterns: a one-pixel ridge of height H on the line is a
    profile B, .., B + H, .., B (ridge contrast H), half of it on each of two
    offsets when the line lies half-way between pixel rows; a step edge half
    a pixel from the line is a profile a, .., a, (a+b)/2 ... b (step contrast
    |b - a|); a line elsewhere on a flat background is rejected."""
    N, M, B, H = 40, 50, 0.2, 0.6
    img = np.full((N, M), B)
    img[17, :] += H
    prof, n = O.line_band_profile(img, "regular", 0.0, 17.0, 3)
    assert n == M and np.allclose(prof, [B, B, B, B + H, B, B, B], atol=1e-12)
    c, ok = O.line_verdict(prof, n, 0.3, 20)
    assert abs(c - H) < 1e-12 and ok
    prof, n = O.line_band_profile(img, "regular", 0.0, 16.5, 3)
    assert np.allclose(prof, [B, B, B, B + H / 2, B + H / 2, B, B], atol=1e-12)
    step = np.where(np.arange(N)[:, None] < 20, 0.1, 0.7) * np.ones((1, M))
    prof, n = O.line_band_profile(step, "regular", 0.0, 19.5, 3)
    assert np.allclose(prof, [0.1, 0.1, 0.1, 0.4, 0.7, 0.7, 0.7], atol=1e-12)
    c, ok = O.line_verdict(prof, n, 0.3, 20)
    assert abs(c - 0.6) < 1e-12 and ok
    prof, n = O.line_band_profile(img, "regular", 0.0, 30.0, 3)
    c, ok = O.line_verdict(prof, n, 0.05, 20)
    assert c < 1e-12 and not ok
    # too short: the contrast is there but the band holds fewer positions than asked
    assert not O.line_verdict(*O.line_band_profile(img, "regular", 0.0, 17.0, 3), 0.3, M + 1)[1]


def check_verify_fig9_wrap(O):
    """Sec. 4.5, Fig. 9: the wrapped regular-space peak names a line that is
    not in the image (flat band, rejected), while the same line's inverse-space
    peak names the real line (ridge, verified)."""
    gold = read_golden("fig9_wrap_example.txt")
    M, N = int(gold["width_M"]), int(gold["height_N"])
    Np = N + M
    kinv = 1.0 / gold["slope"]
    bx = gold["inverse_peak_m"] - kinv * N / 2 + M / 2
    ln = synth.Line("ridge", True, kinv, bx, width=1.0)
    img = synth.render(N, M, [ln], 0.0, np.random.default_rng(0), bg=0.2)
    P, Pinv = O.forward(img)
    det = O.peaks_list(np.abs(P), 1, 0.0, 1, O.boundary_mask(N, M, Np))
    k, b = O.peak_params(*divmod(det[0], M), N, M, Np, "regular")
    prof, n = O.line_band_profile(img, "regular", k, b, 3)
    c_wrap, ok_wrap = O.line_verdict(prof, n, 0.2, 32)
    Bi = np.where(O.boundary_mask(M, N, Np), 0.0, np.abs(Pinv))
    ki, bi = O.peak_params(*np.unravel_index(np.argmax(Bi), Bi.shape), N, M, Np, "inverse")
    prof_i, n_i = O.line_band_profile(img, "inverse", ki, bi, 3)
    c_true, ok_true = O.line_verdict(prof_i, n_i, 0.2, 32)
    assert not ok_wrap and ok_true, (c_wrap, c_true)
    assert c_true > 0.3 and c_wrap < 0.05


# ----------------------------------------------------------------- sub-cell refinement

def check_continuous_plane_cells(O):
    """The plane between cells equals the plane at every integer cell, for
    both NVMT kinds, square, non-square and with enlarged padding."""
    rng = np.random.default_rng(61)
    for kind in O.NVMT_KINDS:
        for (N, M, pl) in [(16, 12, 0), (10, 14, 30)]:
            img = rng.random((N, M))
            Np = O.padded_length(N, M, pl)
            g = O.resampled_rows(img, pl, kind)
            P = O.forward_regular(img, pl, kind)
            for r in range(0, Np, 3):
                for c in range(M):
                    v = O.continuous_plane(g, Np, c - M // 2, r - Np // 2)[0]
                    assert abs(v - P[r, c]) <= 1e-12 * np.abs(P).max(), (kind, N, M, r, c)


def check_continuous_plane_derivatives(O):
    """First and second derivatives against central finite differences
    (h = 1e-5) at points between cells."""
    rng = np.random.default_rng(62)
    img = rng.random((16, 12))
    Np = 28
    g = O.resampled_rows(img, 0, "linear")
    h = 1e-5
    for (m, y) in [(0.3, 1.7), (-2.4, -5.1), (4.9, 9.3)]:
        v = O.continuous_plane(g, Np, m, y)
        f = lambda mm, yy, i: O.continuous_plane(g, Np, mm, yy)[i]
        fd = [(f(m + h, y, 0) - f(m - h, y, 0)) / (2 * h), (f(m, y + h, 0) - f(m, y - h, 0)) / (2 * h),
              (f(m + h, y, 1) - f(m - h, y, 1)) / (2 * h), (f(m, y + h, 1) - f(m, y - h, 1)) / (2 * h),
              (f(m, y + h, 2) - f(m, y - h, 2)) / (2 * h)]
        scale = max(abs(x) for x in v)
        for a, b in zip(v[1:], fd):
            assert abs(a - b) <= 1e-6 * scale, (m, y, a, b)


def check_refine_line_to_point(O):
    """Eq. 19 with real-valued parameters: a long ridge focuses at the
    continuous cell (m = -k M/2, y = b_centre).  For both NVMT kinds the
    refined maximum is within 0.1 cell of it in every trial and 0.02 cell on
    average (the rendered, anti-aliased ridge is not an ideal line), where
    the integer cell is off by 0.3 cell or more on average."""
    rng = np.random.default_rng(63)
    N = M = 128
    Np = N + M
    for kind in O.NVMT_KINDS:
        cell_err, ref_err = [], []
        for t in range(8):
            k = float(rng.uniform(-0.8, 0.8))
            b = float(rng.uniform(40, 88)) - k * M / 2
            ln = synth.Line("ridge", False, k, b, width=1.0)
            img = synth.render(N, M, [ln], 0.0, rng, bg=0.0)
            P = O.forward_regular(img, 0, kind)
            r, c = np.unravel_index(np.argmax(np.abs(P)), P.shape)
            g = O.resampled_rows(img, 0, kind)
            mt, yt = -k * M / 2, b + k * M / 2 - N / 2
            m, y, v = O.refine_peak(g, Np, r, c, 5)
            ref_err.append(np.hypot(m - mt, y - yt))
            assert ref_err[-1] <= 0.1, (kind, t, m, mt, y, yt)
            assert v >= abs(P[r, c])
            cell_err.append(np.hypot(c - M // 2 - mt, r - Np // 2 - yt))
        assert np.mean(ref_err) <= 0.02 and np.mean(cell_err) > 0.3


def check_refine_stationary(O):
    """After the refinement the gradient of |P| vanishes (to 1e-6 of |P| per
    cell) and the Hessian is negative definite: a local maximum."""
    rng = np.random.default_rng(64)
    N, M = 64, 48
    img = synth.mixed_lines(N, M, (2, 4), 0.05, rng).image
    Np = N + M
    g = O.resampled_rows(img, 0, "linear")
    P = O.forward_regular(img, 0, "linear")
    for idx in O.peaks_list(np.abs(P), 3, 0.0, 1, O.boundary_mask(N, M, Np), True):
        r, c = divmod(idx, M)
        m, y, v = O.refine_peak(g, Np, r, c, 6)
        Pv, Pm, Py, Pmm, Pmy, Pyy = O.continuous_plane(g, Np, m, y)
        sg = 1.0 if Pv >= 0 else -1.0
        if abs(m - (c - M // 2)) < 0.999 and abs(y - (r - Np // 2)) < 0.999:   # not stopped at the trust bound
            assert np.hypot(Pm, Py) <= 1e-6 * abs(Pv), (idx, Pm, Py)
            assert sg * Pmm < 0 and Pmm * Pyy - Pmy * Pmy > 0


# ----------------------------------------------------------------- volumes (App. A)

def expected_cell_volume(sh: synth.Sheet, Nz: int, Ny: int, Nx: int, Nzp: int):
    """Plane -> point (Eq. A.9 with omega_max = pi): the sheet
    slice = a col + b row + c has the centred intercept c + a Nx/2 + b Ny/2
    - Nz/2 and focuses at m1 = -a Nx/2, m2 = -b Ny/2.  Returns (z, row, col)."""
    cc = sh.c + sh.a * Nx / 2 + sh.b * Ny / 2 - Nz / 2
    return (int(round(cc)) + Nzp // 2, (int(round(-sh.b * Ny / 2)) + Ny // 2) % Ny,
            (int(round(-sh.a * Nx / 2)) + Nx // 2) % Nx)


def check_spectrum_z_is_library_fft(O):
    """Eq. A.2 on the centred frame: S[n3] = (-1)^n3 FFT_z(V_pad)[n3]."""
    rng = np.random.default_rng(101)
    vol = O.expand_volume(rng.random((6, 4, 6)), 20)
    S = O.spectrum_z(vol)
    n3 = np.arange(1, 10)
    want = np.fft.fft(vol, axis=0)[1:10] * ((-1.0) ** n3)[:, None, None]
    assert S.shape == (9, 4, 6) and np.abs(S - want).max() <= 1e-12 * np.abs(want).max()


def check_dft_xy_is_library_fft2(O):
    """Eq. A.4 with centred indices is the shifted 2D FFT of every slice."""
    rng = np.random.default_rng(102)
    g = rng.standard_normal((3, 6, 10)) + 1j * rng.standard_normal((3, 6, 10))
    want = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(g, axes=(1, 2))), axes=(1, 2))
    assert np.abs(O.dft_xy(g) - want).max() <= 1e-12 * np.abs(want).max()


def check_idft_z_is_library_ifft(O):
    """Eq. A.5: the inverse z DFT of the Hermitian-completed half spectrum
    equals numpy's inverse FFT of the full spectrum (natural order, the
    centred n3 carried as (-1)^n3)."""
    rng = np.random.default_rng(103)
    Nzp = 14
    G = rng.standard_normal((6, 3, 4)) + 1j * rng.standard_normal((6, 3, 4))
    full = np.zeros((Nzp, 3, 4), complex)
    for n3 in range(1, 7):
        full[n3] = G[n3 - 1] * (-1.0) ** n3
        full[Nzp - n3] = np.conj(G[n3 - 1]) * (-1.0) ** n3
    # (-1)^n3 moves the origin: slice r of the inverse FFT is z = r - Nzp/2
    want = np.fft.ifft(full, axis=0).real
    assert np.abs(O.idft_z(G, Nzp) - want).max() <= 1e-12 * np.abs(want).max()


def check_bilinear_exact_on_bilinear_slices(O):
    """Bilinear interpolation reproduces a slice of the form
    alpha + beta i + gamma j + delta i j exactly wherever the position
    (u, v) = (y'/s + Ny/2, x'/s + Nx/2) lies on the grid's hull, and gives 0
    where u or v is more than one cell outside it."""
    Ny, Nx, Nzp = 8, 12, 40
    h = Nzp // 2 - 1
    al, be, ga, de = 0.3 + 0.1j, -0.2 + 0.05j, 0.15 - 0.3j, 0.02 + 0.01j
    i = np.arange(Ny)[:, None]
    j = np.arange(Nx)[None, :]
    S = np.tile(al + be * i + ga * j + de * i * j, (h, 1, 1))
    g = O.nvmt_bilinear(S, Nzp)
    yp = (np.arange(Ny) - Ny // 2)[:, None]
    xp = (np.arange(Nx) - Nx // 2)[None, :]
    for n3 in range(1, h + 1):
        s = 2.0 * n3 / Nzp
        u, v = yp / s + Ny / 2, xp / s + Nx / 2
        inside = (u >= 0) & (u <= Ny - 1) & (v >= 0) & (v <= Nx - 1)
        want = al + be * u + ga * v + de * u * v
        assert np.abs(g[n3 - 1][inside] - np.broadcast_to(want, g[n3 - 1].shape)[inside]).max(initial=0.0) < 1e-12
        outside = (u < -1) | (u > Ny) | (v < -1) | (v > Nx)
        assert np.abs(g[n3 - 1][np.broadcast_to(outside, g[n3 - 1].shape)]).max(initial=0.0) == 0.0


def check_volume_reduces_to_image(O):
    """A volume that is nonzero only in its centre row (y = 0) holds one
    image I[z, x]; its transform is the 2D funnel transform of I on the same
    padded length, the same for every m2 (the y' resampling of a delta at
    y = 0 is a delta at y' = 0).  Likewise the centre column (x = 0) with
    the 2D transform of I[z, y] for every m1.  Ties the x and y axes each to
    the pinned 2D transform."""
    rng = np.random.default_rng(104)
    Nz, Ny, Nx = 10, 8, 12
    Nzp = O.padded_depth(Nz, Ny, Nx)
    I = rng.random((Nz, Nx))
    vol = np.zeros((Nz, Ny, Nx))
    vol[:, Ny // 2, :] = I
    P3 = O.forward_volume(vol)
    P2 = O.forward_regular(I, Nzp)
    assert np.abs(P3 - P2[:, None, :]).max() <= 1e-11 * np.abs(P2).max()
    J = rng.random((Nz, Ny))
    vol = np.zeros((Nz, Ny, Nx))
    vol[:, :, Nx // 2] = J
    P3 = O.forward_volume(vol)
    P2 = O.forward_regular(J, Nzp)
    assert np.abs(P3 - P2[:, :, None]).max() <= 1e-11 * np.abs(P2).max()


def check_volume_plane_to_point(O):
    """Eq. A.9: a thin sheet slice = a col + b row + c focuses within one cell
    of (z = c_centred, m2 = -b Ny/2, m1 = -a Nx/2), in a volume whose three
    sides differ."""
    rng = np.random.default_rng(105)
    Nz, Ny, Nx = 24, 16, 20
    Nzp = O.padded_depth(Nz, Ny, Nx)
    for trial in range(6):
        a, b = float(rng.uniform(-0.85, 0.85)), float(rng.uniform(-0.85, 0.85))
        zc = float(rng.uniform(0.35 * Nz, 0.65 * Nz))
        sh = synth.Sheet(a, b, zc - a * Nx / 2 - b * Ny / 2, 1.0)
        vol = synth.render_volume(Nz, Ny, Nx, [sh], 0.0, rng, bg=0.0).astype(np.float64)
        B = np.abs(O.forward_volume(vol))
        got = np.unravel_index(np.argmax(B), B.shape)
        want = expected_cell_volume(sh, Nz, Ny, Nx, Nzp)
        for g, w, n in zip(got, want, B.shape):
            assert torus_dist(int(g), w, n) <= 1, (trial, got, want)


def check_volume_point_to_plane(O):
    """Eq. A.5 with omega_max = pi: one bright voxel at centred (x0, y0, z0)
    becomes the plane z = z0 + 2 x0 m1 / Nx + 2 y0 m2 / Ny.  As for the 2D
    point -> line pin, linear resampling of a delta aliases, so the pin is a
    |P|^2-weighted least-squares plane through the cells within +-6 slices of
    the prediction over the central half of both bin ranges: intercept within
    half a cell, both slopes within 15 %."""
    Nz, Ny, Nx = 32, 32, 40
    Nzp = O.padded_depth(Nz, Ny, Nx)
    for (x0, y0, z0) in [(8, 5, 3), (-10, 6, -4), (12, -7, 0), (-6, -9, 5)]:
        vol = np.zeros((Nz, Ny, Nx))
        vol[z0 + Nz // 2, y0 + Ny // 2, x0 + Nx // 2] = 1.0
        B2 = O.forward_volume(vol) ** 2
        rows, w = [], []
        for r in range(Ny):
            m2 = r - Ny // 2
            if abs(m2) > Ny // 4:
                continue
            for c in range(Nx):
                m1 = c - Nx // 2
                if abs(m1) > Nx // 4:
                    continue
                pred = z0 + 2.0 * x0 * m1 / Nx + 2.0 * y0 * m2 / Ny
                for z in range(int(np.floor(pred)) - 6, int(np.floor(pred)) + 8):
                    rows.append((1.0, m1, m2, z))
                    w.append(B2[(z + Nzp // 2) % Nzp, r, c])
        X = np.asarray(rows)
        sw = np.sqrt(np.asarray(w))
        coef = np.linalg.lstsq(X[:, :3] * sw[:, None], X[:, 3] * sw, rcond=None)[0]
        assert abs(coef[0] - z0) <= 0.5, (x0, y0, z0, coef)
        assert abs(coef[1] - 2.0 * x0 / Nx) <= 0.15 * abs(2.0 * x0 / Nx), (x0, y0, z0, coef)
        assert abs(coef[2] - 2.0 * y0 / Ny) <= 0.15 * abs(2.0 * y0 / Ny), (x0, y0, z0, coef)


def check_volume_shift_equivariance(O):
    """Moving the content d slices along z inside the frame rolls the
    parameter volume by d slices exactly."""
    rng = np.random.default_rng(106)
    Nz, Ny, Nx, d = 16, 6, 8, 3
    vol = np.zeros((Nz, Ny, Nx))
    vol[2:Nz - 6] = rng.random((Nz - 8, Ny, Nx))
    P0 = O.forward_volume(vol)
    P1 = O.forward_volume(np.roll(vol, d, axis=0))
    assert np.abs(P1 - np.roll(P0, d, axis=0)).max() <= 1e-12 * np.abs(P0).max()


def check_volume_lines_sampler(O):
    """The per-line evaluation equals the whole transform on its lines."""
    rng = np.random.default_rng(107)
    vol = rng.random((10, 6, 8))
    lines = [(0, 0), (3, 5), (5, 7), (2, 1)]
    P = O.forward_volume(vol, 30)
    L = O.forward_volume_lines(vol, lines, 30)
    for k, (r, c) in enumerate(lines):
        assert np.abs(L[:, k] - P[:, r, c]).max() <= 1e-12 * np.abs(P).max()


def local_max_peaks_volume(B, K, T, radius=1, mask=None, wrap=True):
    """Brute force in 3D, as local_max_peaks."""
    nz, ny, nx = B.shape
    out = []
    for z in range(nz):
        for r in range(ny):
            for c in range(nx):
                if B[z, r, c] < T or (mask is not None and mask[z, r, c]):
                    continue
                me = (z * ny + r) * nx + c
                ok = True
                for dz in range(-radius, radius + 1):
                    for dr in range(-radius, radius + 1):
                        for dc in range(-radius, radius + 1):
                            zz, rr, cc = z + dz, r + dr, c + dc
                            if wrap:
                                zz, rr, cc = zz % nz, rr % ny, cc % nx
                            elif not (0 <= zz < nz and 0 <= rr < ny and 0 <= cc < nx):
                                continue
                            q = (zz * ny + rr) * nx + cc
                            if q == me:
                                continue
                            if B[zz, rr, cc] > B[z, r, c] or (B[zz, rr, cc] == B[z, r, c] and q < me):
                                ok = False
                if ok:
                    out.append(me)
    out.sort(key=lambda i: (-B.flat[i], i))
    return out[:K]


def check_volume_peaks_equal_local_maxima(O, trials=80):
    """The list algorithm in 3D equals 'first K local maxima under the total
    order', on tie-heavy volumes, with and without wrapping."""
    rng = np.random.default_rng(108)
    for t in range(trials):
        shape = tuple(int(rng.integers(3, 7)) for _ in range(3))
        B = rng.integers(0, 4, size=shape).astype(np.float64)
        K = int(rng.integers(1, 8))
        T = float(rng.integers(0, 3))
        radius = int(rng.integers(1, 3))
        wrap = bool(rng.integers(2))
        mask = rng.random(shape) < 0.15
        got = O.peaks_list_volume(B, K, T, radius, mask, wrap)
        want = local_max_peaks_volume(B, K, T, radius, mask, wrap)
        assert got == want, (t, got, want)


def check_plane_params_round_trip(O):
    """A cell's plane (Eq. A.9 read backwards), rendered as a thin sheet and
    transformed, focuses back on that cell."""
    rng = np.random.default_rng(109)
    Nz, Ny, Nx = 20, 16, 24
    Nzp = O.padded_depth(Nz, Ny, Nx)
    for _ in range(5):
        cell = (int(rng.integers(Nzp // 2 - 4, Nzp // 2 + 5)), int(rng.integers(Ny // 2 - 6, Ny // 2 + 7)),
                int(rng.integers(Nx // 2 - 9, Nx // 2 + 10)))
        a, b, c = O.plane_params(*cell, Nz, Ny, Nx, Nzp)
        vol = synth.render_volume(Nz, Ny, Nx, [synth.Sheet(a, b, c, 1.0)], 0.0, rng, bg=0.0).astype(np.float64)
        B = np.abs(O.forward_volume(vol))
        got = tuple(int(v) for v in np.unravel_index(np.argmax(B), B.shape))
        assert got == cell, (cell, got, (a, b, c))


def check_volume_spaces_focus_steep_planes(O):
    """Planes steeper than 45 degrees from the z axis focus in the x and y
    spaces: a sheet x = a*y + b*z + c (or y = a*x + b*z + c), |a|, |b| < 0.85,
    rendered in the world volume, focuses within one cell of Eq. A.9's cell of
    that space (depth x or y, rows z, columns y or x)."""
    rng = np.random.default_rng(110)
    Nz, Ny, Nx = 20, 16, 24
    Lp = Nz + Ny + Nx
    frames = {"x": ((Nx, Nz, Ny), (1, 2, 0)), "y": ((Ny, Nz, Nx), (1, 0, 2))}
    for space, ((D, R, C), back) in frames.items():
        for trial in range(3):
            a, b = float(rng.uniform(-0.85, 0.85)), float(rng.uniform(-0.85, 0.85))
            dc = float(rng.uniform(0.35 * D, 0.65 * D))
            sh = synth.Sheet(a, b, dc - a * C / 2 - b * R / 2, 1.0)
            W = synth.render_volume(D, R, C, [sh], 0.0, rng, bg=0.0).astype(np.float64)
            vol = np.transpose(W, back)                      # world axes (z, y, x)
            assert vol.shape == (Nz, Ny, Nx)
            B = np.abs(O.forward_volume_space(vol, space))
            got = np.unravel_index(np.argmax(B), B.shape)
            want = expected_cell_volume(sh, D, R, C, Lp)
            for g, w, n in zip(got, want, B.shape):
                assert torus_dist(int(g), w, n) <= 1, (space, trial, got, want)
