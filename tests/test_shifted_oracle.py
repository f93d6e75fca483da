"""Pins of the shifted-recurrence oracle (oracle/shifted.py) against what the
paper and mathematics fix independently of it:

* at m = n = 0 the one-step matrix is the Legendre recurrence of the lemma,
  A_r^0 = P_r and B_r^0 = 0 (the initial conditions stated with the
  composition rule), checked against scipy's Legendre polynomials;
* d^{L+r} = A_r^L d^L + B_r^L d^{L-1} with d from the oracle's Jacobi-form
  Wigner-d (a different route: no l-recurrence there);
* the composition rule (matrix product of shifts);
* the divide-and-conquer projections (k = 1, the four-term worked example
  k = 2, and k = 3, 4 splits) equal the direct inner product <s, d^{L+r}>."""
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle
from oracle import shifted


def _dvec(tl, tm, tn, beta):
    """d^l_{nm}(beta_k) over the nodes from the Jacobi-form oracle."""
    return np.array([oracle.wigner_d(tl, tn, tm, b) for b in beta])


def _nodes(N=24):
    beta = np.pi * np.arange(N) / (N - 1)
    return beta, np.cos(beta)


def test_legendre_case_step_is_the_lemma():
    for l in range(0, 12):
        a, b, c = shifted.step_coeffs(2 * l, 0, 0)
        assert a == pytest.approx((2 * l + 1) / (l + 1), rel=1e-15)
        assert b == 0.0
        assert c == pytest.approx(l / (l + 1), rel=1e-15, abs=0)


def test_level_zero_shifts_are_legendre():
    beta, x = _nodes()
    for r in range(0, 10):
        A, _, B, _ = shifted.shifted_AB(0, r, 0, 0, x)
        assert np.allclose(A, eval_legendre(r, x), rtol=0, atol=1e-14)
        assert np.all(B == 0.0)


@pytest.mark.parametrize("tm,tn", [(0, 0), (1, 1), (1, -1), (2, 4), (-3, 5), (6, -6), (3, 7)])
def test_shift_reproduces_wigner_d(tm, tn):
    beta, x = _nodes()
    l0 = max(abs(tm), abs(tn))
    for tL in (l0 + 2, l0 + 4):
        dL, dLm1 = _dvec(tL, tm, tn, beta), _dvec(tL - 2, tm, tn, beta)
        for r in (0, 1, 2, 5, 8):
            A, _, B, _ = shifted.shifted_AB(tL, r, tm, tn, x)
            ref = _dvec(tL + 2 * r, tm, tn, beta)
            assert np.allclose(A * dL + B * dLm1, ref, rtol=0, atol=1e-12), (tm, tn, tL, r)


def test_composition_rule():
    beta, x = _nodes(11)
    tm, tn, tL = 3, -1, 5
    for r, s in ((1, 1), (2, 3), (4, 2), (0, 5), (3, 0)):
        left = shifted.shift_matrix(tL, r + s, tm, tn, x)
        Mr = shifted.shift_matrix(tL, r, tm, tn, x)
        Ms = shifted.shift_matrix(tL + 2 * r, s, tm, tn, x)
        right = np.einsum("ijk,jlk->ilk", Ms, Mr)
        assert np.allclose(left, right, rtol=0, atol=1e-12), (r, s)


@pytest.mark.parametrize("tm,tn", [(0, 0), (2, -2), (1, 3), (-5, 1)])
def test_projections_equal_direct_inner_product(tm, tn):
    beta, x = _nodes(32)
    rng = np.random.default_rng(7)
    s = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    l0 = max(abs(tm), abs(tn))
    tL = l0 + 2
    dL, dLm1 = _dvec(tL, tm, tn, beta), _dvec(tL - 2, tm, tn, beta)
    for r in (1, 3, 6, 9):
        direct = np.dot(s, _dvec(tL + 2 * r, tm, tn, beta))
        scale = np.linalg.norm(s)
        assert abs(shifted.projection_k1(s, dL, dLm1, tL, r, tm, tn, x) - direct) < 1e-12 * scale
        for n1 in range(0, r + 1):
            got = shifted.projection_k2(s, dL, dLm1, tL, n1, r - n1, tm, tn, x)
            assert abs(got - direct) < 1e-12 * scale, (r, n1)
        for parts in ((r,), (1, r - 1), (r - 1, 1)) + (((1, 1, r - 2), (2, 1, r - 3)) if r >= 3 else ()):
            got = shifted.projection_general(s, dL, dLm1, tL, parts, tm, tn, x)
            assert abs(got - direct) < 1e-12 * scale, parts


def test_worked_example_terms_individually():
    """The four terms of the k = 2 example, each formed as printed, sum to the k = 1 form."""
    beta, x = _nodes(20)
    rng = np.random.default_rng(3)
    s = rng.standard_normal(20)
    tm, tn, tL, n1, n2 = 1, 1, 3, 2, 3
    dL, dLm1 = _dvec(tL, tm, tn, beta), _dvec(tL - 2, tm, tn, beta)
    A1, A1p, B1, B1p = shifted.shifted_AB(tL, n1, tm, tn, x)
    A2, _, B2, _ = shifted.shifted_AB(tL + 2 * n1, n2, tm, tn, x)
    terms = [np.dot(s * dL, A2 * A1), np.dot(s * dL, B2 * A1p), np.dot(s * dLm1, A2 * B1), np.dot(s * dLm1, B2 * B1p)]
    k1 = shifted.projection_k1(s, dL, dLm1, tL, n1 + n2, tm, tn, x)
    assert abs(sum(terms) - k1) < 1e-12 * np.linalg.norm(s)
