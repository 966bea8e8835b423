"""CPU emulation of the split-precision DFT passes (the matrix-core engine of
FT_PREC_BF16X3 / FT_PREC_FP16X3), written from their arithmetic, not from the
HIP code: Stockham passes of radix 16 then 8 (power-of-two lengths), each
input multiplied by its twiddle power read from an FP32 table (FP32 complex
product), then every R-point DFT evaluated as the real product
[Y_re; Y_im] = [[C, +-S], [-+S, C]] [X_re; X_im] with both operands split
into a high and a low half-precision part, X = X_hi + X_lo (rounded to
nearest each) and A = A_hi + A_lo, keeping A_lo X_hi + A_hi X_lo + A_hi X_hi
summed in FP32 in that order; FP16 operands are first scaled per butterfly by
the power of two that puts the largest input magnitude in [2^14, 2^15).
Also the FP32 passes (radix 16/8/4/2, each butterfly's twiddle powers built
from one table value by balanced products) for comparison.  Used to derive
the error each precision's transforms add, and from it the bound the GPU
tests hold the split paths to."""
from __future__ import annotations

import numpy as np

F32 = np.float32


def round_bf16(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), as FP32."""
    u = np.ascontiguousarray(x, dtype=F32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(F32)


def round_fp16(x):
    return np.asarray(x, dtype=F32).astype(np.float16).astype(F32)


ROUND = {"bf16": round_bf16, "fp16": round_fp16}


def split(x, prec):
    r = ROUND[prec]
    hi = r(x)
    lo = r((x - hi).astype(F32))
    return hi, lo


def mfma_radices(L):
    """Radix-16 passes, then radix-8 ones (3 y = a mod 4 for L = 2^a)."""
    a = int(np.log2(L))
    assert 1 << a == L and 6 <= a <= 12
    y = (3 * a) % 4
    x = (a - 3 * y) // 4
    return [16] * x + [8] * y


def fp32_radices(L):
    a = int(np.log2(L))
    out = [16] * (a // 4)
    if a % 4:
        out.append(1 << (a % 4))
    return out


def twiddle_table(L):
    m = np.arange(L)
    return np.exp(-2j * np.pi * m / L).astype(np.complex64)


def cmul32(a, b):
    """FP32 complex product as two FP32 products and a sum per part."""
    ar, ai = a.real.astype(F32), a.imag.astype(F32)
    br, bi = b.real.astype(F32), b.imag.astype(F32)
    re = (ar * br).astype(F32) - (ai * bi).astype(F32)
    im = (ar * bi).astype(F32) + (ai * br).astype(F32)
    return (re.astype(F32) + 1j * im.astype(F32)).astype(np.complex64)


def dft_matrix_parts(R, inv):
    """The R-point DFT as real 2R x 2R blocks, coefficients rounded to FP32."""
    q = np.arange(R)[:, None]
    r = np.arange(R)[None, :]
    ang = 2 * np.pi * ((q * r) % R) / R
    c = np.cos(ang).astype(F32)
    s = np.sin(ang).astype(F32)
    if inv:
        s = -s
    # forward e^{-i t}: Y_re = C X_re + S X_im, Y_im = -S X_re + C X_im
    top = np.concatenate([c, s], axis=1)
    bot = np.concatenate([-s, c], axis=1)
    return np.concatenate([top, bot], axis=0).astype(F32)     # (2R, 2R): rows (re outs, im outs)


def _dot32(A, B):
    """A (2R, 2R) times B (2R, n) with an FP32 result (products of
    half-precision values are exact in FP32; the sum is rounded once)."""
    return (A.astype(np.float64) @ B.astype(np.float64)).astype(F32)


def split_butterflies(X, R, inv, prec):
    """R-point DFTs of the columns of X (complex64, shape (R, n)) by the
    three split products."""
    A = dft_matrix_parts(R, inv)
    A_hi, A_lo = split(A, prec)
    B = np.concatenate([X.real, X.imag], axis=0).astype(F32)      # (2R, n)
    sc = np.ones(B.shape[1], dtype=F32)
    if prec == "fp16":
        m = np.abs(B).max(axis=0)
        e = np.floor(np.log2(np.maximum(m, np.finfo(F32).tiny)))
        sc = np.exp2(14 - e).astype(F32)                          # m * sc in [2^14, 2^15)
    Bs = (B * sc).astype(F32)
    B_hi, B_lo = split(Bs, prec)
    y = _dot32(A_lo, B_hi)
    y = (y + _dot32(A_hi, B_lo)).astype(F32)
    y = (y + _dot32(A_hi, B_hi)).astype(F32)
    y = (y / sc).astype(F32)
    return (y[:R] + 1j * y[R:]).astype(np.complex64)


def exact_butterflies(X, R, inv):
    q = np.arange(R)[:, None]
    r = np.arange(R)[None, :]
    W = np.exp((2j if inv else -2j) * np.pi * q * r / R)
    return (W @ X.astype(np.complex128)).astype(np.complex64)


def fp32_butterflies(X, R, inv):
    """R-point DFT in FP32 arithmetic (rounded after the exact small DFT; the
    radix-16/8/4 kernels are a few FP32 additions and rotations deep)."""
    return exact_butterflies(X, R, inv)


def stockham(x, inv, prec):
    """Transform of the complex vector x (length L) by the passes of
    precision prec ('fp32', 'bf16', 'fp16'), forward e^{-i} or inverse e^{+i},
    unnormalised."""
    L = x.size
    radices = fp32_radices(L) if prec == "fp32" else mfma_radices(L)
    tw = twiddle_table(L)
    if inv:
        tw = np.conj(tw)
    cur = x.astype(np.complex64)
    NS = 1
    for R in radices:
        NB = L // R
        j = np.arange(NB)
        X = cur[j[None, :] + np.arange(R)[:, None] * NB]          # (R, NB): input r of butterfly j
        if NS > 1:
            k = j % NS
            st = k * (L // (NS * R))
            if prec == "fp32":
                # one table power per butterfly, the rest by balanced products
                w = [None] * R
                w[1] = tw[st]
                for r in range(2, R):
                    w[r] = cmul32(w[r // 2], w[r - r // 2])
                for r in range(1, R):
                    X[r] = cmul32(X[r], w[r])
            else:
                for r in range(1, R):
                    X[r] = cmul32(X[r], tw[r * st])
        if prec == "fp32":
            Y = fp32_butterflies(X, R, inv)
        else:
            Y = split_butterflies(X, R, inv, prec)
        out = np.empty(L, dtype=np.complex64)
        base = (j // NS) * NS * R + (j % NS)
        for q in range(R):
            out[base + q * NS] = Y[q]
        cur = out
        NS *= R
    return cur


def transform_error(L, prec, inv=False, trials=4, seed=0):
    """Relative L2 error of the emulated transform against the FP64 DFT of
    the same (FP32) input, over `trials` random vectors."""
    rng = np.random.default_rng([seed, L])
    errs = []
    for _ in range(trials):
        x = (rng.standard_normal(L) + 1j * rng.standard_normal(L)).astype(np.complex64)
        want = np.fft.ifft(x.astype(np.complex128)) * L if inv else np.fft.fft(x.astype(np.complex128))
        got = stockham(x, inv, prec).astype(np.complex128)
        errs.append(np.linalg.norm(got - want) / np.linalg.norm(want))
    return float(np.sqrt(np.mean(np.square(errs))))


def nvmt_gain(S, Np):
    """How much the NVMT raises the relative weight of an error spread
    evenly over the spectrum S (rows n2 = 1 .. h, the y-DFT of the expanded
    image) against the signal: row n2 is resampled at ratio s = 2 n2 / Np,
    keeping about s M of its M samples, so a white error keeps about half its
    energy while the signal keeps sum_n2 s |S_n2|^2, mostly in the low rows.
    Returns sqrt((|S|^2 / 2) / sum_n2 s |S_n2|^2)."""
    h = S.shape[0]
    s = 2.0 * np.arange(1, h + 1) / Np
    rows = np.sum(np.abs(S) ** 2, axis=1)
    return float(np.sqrt(0.5 * rows.sum() / np.sum(s * rows)))


def predicted_path_error(S, Np, W, prec):
    """Expected relative L2 error of a parameter plane computed with the
    transforms of precision prec: the first y-DFT's error (length Np) raised
    by the NVMT gain, the x' DFT's (length W) and the inverse y-DFT's (length
    Np) added in quadrature.  Rounding of the linear interpolation itself
    (FP32 in every precision) is below these."""
    eN = transform_error(Np, prec)
    eW = transform_error(W, prec)
    k = nvmt_gain(S, Np)
    return float(np.sqrt((k * eN) ** 2 + eW ** 2 + eN ** 2))


def predicted_adjoint_error(Np, W, prec):
    """Expected relative L2 error of an image gradient: the three transforms
    of the adjoint in quadrature (a plane gradient spread over all cells
    passes the transposed NVMT with no such gain), with FP32's transform
    error as the floor (the interpolation, twiddle products and the
    separation of the real lines stay FP32 in every precision)."""
    e = [max(transform_error(n, prec), transform_error(n, "fp32")) for n in (Np, W, Np)]
    return float(np.sqrt(sum(x * x for x in e)))
