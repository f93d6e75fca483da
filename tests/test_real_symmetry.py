"""The Hermitian relation that real-signal plans rely on, fixed by the oracle's
direct sums (CPU): for real f, fhat(l)_{-m,-n} = (-1)^{m-n} conj(fhat(l)_{mn});
and the real part of a synthesis is the synthesis of the Hermitian part of
the coefficients, (c_{mn} + (-1)^{m-n} conj(c_{-m,-n})) / 2."""
import numpy as np
import pytest

import oracle
import synth


def _mirror(B, c):
    """c'_{l,m,n} = (-1)^{m-n} conj(c_{l,-m,-n}) over the flat coefficient layout."""
    out = np.empty_like(c)
    for tl in range(B):
        for tm in range(-tl, tl + 1, 2):
            for tn in range(-tl, tl + 1, 2):
                sg = -1.0 if ((tm - tn) // 2) & 1 else 1.0
                out[..., oracle.coeff_index(tl, tm, tn)] = sg * np.conj(c[..., oracle.coeff_index(tl, -tm, -tn)])
    return out


@pytest.mark.parametrize("B", [1, 2, 3, 4, 6])
def test_forward_of_real_signal_is_hermitian(B):
    x = synth.samples_uniform(B, 1, seed=60 + B)[0].real.astype(np.complex128)
    c = oracle.forward(B, x)
    assert np.allclose(_mirror(B, c), c, rtol=0, atol=1e-14 * np.abs(c).max())
    # and a complex signal is not (the relation is not an identity)
    xc = synth.samples_uniform(B, 1, seed=70 + B)[0]
    cc = oracle.forward(B, xc)
    if B > 1:
        assert not np.allclose(_mirror(B, cc), cc, atol=1e-6)


@pytest.mark.parametrize("B", [2, 3, 4])
def test_real_part_of_synthesis_is_synthesis_of_hermitian_part(B):
    c = synth.coeffs(B, 1, seed=80 + B)[0]
    h = 0.5 * (c + _mirror(B, c))
    for fn in (oracle.inverse, oracle.adjoint):
        full = fn(B, c)
        herm = fn(B, h)
        assert np.allclose(full.real, herm.real, rtol=0, atol=1e-13 * np.abs(full).max())
        assert np.abs(herm.imag).max() < 1e-13 * np.abs(full).max()
