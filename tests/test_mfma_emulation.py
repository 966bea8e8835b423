"""The CPU emulation of the split-precision DFT passes (tests/mfma_emulation.py)
against what fixes it independently: numpy's FFT for the pass structure, and
the size of the representation error of a hi + lo split."""
import numpy as np
import pytest

import mfma_emulation as E


@pytest.mark.parametrize("L", [64, 128, 512, 2048, 4096])
@pytest.mark.parametrize("inv", [False, True])
def test_pass_structure_matches_numpy(L, inv):
    """With FP32 operands (no split) the emulated Stockham passes -- radix
    order, butterfly indices, twiddle powers, output placement -- reproduce
    numpy's FFT to FP32 rounding; a misplaced index or power would give O(1)."""
    assert E.transform_error(L, "fp32", inv) < 1e-6


@pytest.mark.parametrize("L", [2048, 4096])
def test_split_error_is_second_order(L):
    """hi + lo leaves |x - hi - lo| <= u^2 |x| and the dropped lo * lo
    product is of the same order, u = 2^-8 (BF16) or 2^-11 (FP16), so a
    transform's relative error is a small multiple of u^2 times its depth,
    and far below the first-order u of a single half-precision product."""
    u_bf, u_fp = 2.0 ** -8, 2.0 ** -11
    e_bf = E.transform_error(L, "bf16")
    e_fp = E.transform_error(L, "fp16")
    assert u_bf ** 2 / 20 < e_bf < u_bf ** 2, e_bf
    assert e_fp < 2 * u_fp ** 2, e_fp
    assert e_bf < 1e-2 * u_bf


def test_dropping_the_low_parts_is_caught():
    """A planted mistake: keeping only hi * hi (one half-precision product)
    gives a first-order error, hundreds of times the three-product form."""
    x = (np.random.default_rng(3).standard_normal((16, 64)) + 0j).astype(np.complex64)
    A = E.dft_matrix_parts(16, False)
    B = np.concatenate([x.real, x.imag]).astype(np.float32)
    one = E._dot32(E.round_bf16(A), E.round_bf16(B))
    three = E.split_butterflies(x, 16, False, "bf16")
    exact = E.exact_butterflies(x, 16, False).astype(np.complex128)
    e1 = np.linalg.norm((one[:16] + 1j * one[16:]) - exact) / np.linalg.norm(exact)
    e3 = np.linalg.norm(three - exact) / np.linalg.norm(exact)
    assert e1 > 100 * e3, (e1, e3)


def test_nvmt_gain_of_a_flat_spectrum():
    """A spectrum of equal row energies gains sqrt(1/2 / mean(s)) = 1."""
    Np = 256
    S = np.ones((Np // 2 - 1, 64))
    assert abs(E.nvmt_gain(S, Np) - 1.0) < 0.02
