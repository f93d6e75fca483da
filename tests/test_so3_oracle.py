"""Pins of the SO(3) oracle (oracle/so3.py): orthonormality of its grid,
exact round trip and Plancherel on bandlimited coefficients, the adjoint
identity, and agreement with the independently pinned SU(2) oracle at the
grid points the two grids share (both have N = 2B nodes per angle and the
same alpha and beta nodes; the SO(3) node gamma_l = -pi + 2 pi l / N is the
SU(2) node gamma_{(l + N/2) / 2} for even l)."""
import numpy as np
import pytest

import oracle
from oracle import so3
import synth


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2)


@pytest.mark.parametrize("B", [2, 4, 6])
def test_grid_orthonormality(B):
    alpha, beta, gamma, W = so3.grid(B)
    N = 2 * B
    assert abs(N * N * W.sum() - 1.0) < 1e-14       # the weights of all N^3 points sum to 1
    C = so3.num_coeffs(B)
    basis = np.zeros((C, N, N, N), dtype=np.complex128)
    for l, m, n in so3.triples(B):
        e = np.zeros(C, dtype=np.complex128)
        e[so3.coeff_index(l, m, n)] = 1.0
        basis[so3.coeff_index(l, m, n)] = so3.inverse(B, e) / (2 * l + 1)
    G = np.einsum("ak,bk->ab", basis.reshape(C, -1) * np.repeat(W, N * N)[None, :], np.conj(basis.reshape(C, -1)))
    d = np.array([1.0 / (2 * l + 1) for l, m, n in so3.triples(B)])
    assert np.allclose(G, np.diag(d), rtol=0, atol=1e-13)


@pytest.mark.parametrize("B", [2, 4, 8])
def test_round_trip_plancherel_adjoint(B):
    C = so3.num_coeffs(B)
    c = _rand(C, B)
    x = so3.inverse(B, c)
    assert np.allclose(so3.forward(B, x), c, rtol=0, atol=1e-12)
    _, _, _, W = so3.grid(B)
    lhs = np.sum(W[:, None, None] * np.abs(x) ** 2)
    rhs = sum((2 * l + 1) * abs(c[so3.coeff_index(l, m, n)]) ** 2 for l, m, n in so3.triples(B))
    assert abs(lhs - rhs) < 1e-12 * rhs
    y = _rand((2 * B) ** 3, B + 1)
    assert abs(np.vdot(so3.forward(B, y), c) - np.vdot(y, so3.adjoint(B, c).reshape(-1))) < 1e-12 * np.linalg.norm(c)


@pytest.mark.parametrize("B", [4, 8])
def test_agrees_with_su2_oracle_on_shared_points(B):
    """Integer-l coefficients synthesised by both oracles agree at the points
    both grids contain (beta = 0 and beta = pi)."""
    C = so3.num_coeffs(B)
    c = _rand(C, 7 * B)
    x3 = so3.inverse(B, c)
    c2 = np.zeros(oracle.num_coeffs(B), dtype=np.complex128)
    for l, m, n in so3.triples(B):
        c2[oracle.coeff_index(2 * l, 2 * m, 2 * n)] = c[so3.coeff_index(l, m, n)]
    N = 2 * B
    pts, ref = [], []
    for k in range(N):
        for j in range(N):
            for l in range(0, N, 2):
                pts.append((k * N + j) * N + (l + N // 2) // 2)
                ref.append(x3[k, j, l])
    got = oracle.inverse(B, c2, np.array(pts))
    assert np.allclose(got, np.array(ref), rtol=0, atol=1e-12)
