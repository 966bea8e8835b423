"""The FFT-based CPU reference that bench.py times for context, against the
FP64 oracle (same transform, dense DFTs): forward planes of both spaces and
the image gradient agree to FP64 rounding at small shapes, including a
non-square image, enlarged padding and odd half-widths (W/2 odd)."""
import numpy as np
import pytest

import bench
from oracle import funnel_oracle as O


@pytest.mark.parametrize("N,M,pad", [(16, 16, 0), (24, 40, 0), (12, 20, 40), (18, 10, 0)])
def test_fft_reference_matches_oracle(N, M, pad):
    rng = np.random.default_rng([5, N, M, pad])
    img = rng.random((N, M))
    Np = O.padded_length(N, M, pad)
    pr, pi = bench.fft_reference_forward(img, Np)
    qr, qi = O.forward(img, Np)
    for got, want in ((pr, qr), (pi, qi)):
        assert got.shape == want.shape
        assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
    dr, di = rng.standard_normal((Np, M)), rng.standard_normal((Np, N))
    got = bench.fft_reference_adjoint(dr, di, N, M, Np)
    want = O.adjoint(dr, di, N, M, Np)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
