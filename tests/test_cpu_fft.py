"""The CPU FFT-based baseline (oracle/cpu_fft.py) against the direct sums.

The baseline regroups the same quadrature sum (Section 4), so it must agree
with the direct-sum oracle to rounding; it also inherits the exactness of the
quadrature (round trip on bandlimited coefficients)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.cpu_fft import CpuFFTPlan


def _rel(a, r):
    return np.linalg.norm(np.asarray(a) - np.asarray(r)) / np.linalg.norm(r)


@pytest.mark.parametrize("B", [1, 2, 3, 4, 6, 8])
def test_cpu_fft_equals_direct_sums(B):
    pl = CpuFFTPlan(B, workers=2)
    x = synth.samples_uniform(B, 2, seed=40 + B)
    c = synth.coeffs(B, 2, seed=50 + B)
    assert _rel(pl.forward(x), np.stack([oracle.forward(B, v) for v in x])) < 1e-13
    N = 2 * B
    ri = np.stack([oracle.inverse(B, v) for v in c]).reshape(2, N, N, N)
    ra = np.stack([oracle.adjoint(B, v) for v in c]).reshape(2, N, N, N)
    assert _rel(pl.inverse(c), ri) < 1e-13
    assert _rel(pl.adjoint(c), ra) < 1e-13


@pytest.mark.parametrize("B", [12, 16])
def test_cpu_fft_round_trip(B):
    pl = CpuFFTPlan(B, workers=2)
    c = synth.coeffs(B, 2, seed=60 + B)
    assert _rel(pl.forward(pl.inverse(c)), c) < 1e-12


@pytest.mark.parametrize("B", [4, 12])
def test_cpu_fft_single_precision_baseline(B):
    """The single-precision variant (the second CPU baseline) computes the
    same sums in float32 / complex64: within single-precision rounding of the
    double-precision plan, in every direction, and in complex64."""
    x = synth.samples_uniform(B, 2, seed=60 + B)
    c = synth.coeffs(B, 2, seed=70 + B)
    p64 = CpuFFTPlan(B, workers=2)
    p32 = CpuFFTPlan(B, workers=2, dtype=np.complex64)
    for got, ref in ((p32.forward(x), p64.forward(x)), (p32.inverse(c), p64.inverse(c)),
                     (p32.adjoint(c), p64.adjoint(c))):
        assert got.dtype == np.complex64
        assert _rel(got, ref) < 1e-5
