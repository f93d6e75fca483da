"""Direct-sum transform on SO(3) (integer degrees only) -- TEST INFRASTRUCTURE ONLY
(same import restriction as the rest of ``oracle/``).

The paper's grid (Definition 4.1) puts both phi and psi on [-pi, pi]; that is
the group SO(3) = SU(2)/{+-1}, on which only integer l occur.  This module is
the transform of Definition 3.4 restricted to that case, on the paper's
domain with periodic nodes and N = 2B nodes per angle (B bounds 2l, as
everywhere in this package; the same N as the SU(2) grid):

    alpha_j = -pi + 2 pi j / N,  gamma_l = -pi + 2 pi l / N,  beta_k = pi k / (N - 1),
    W_k = w_k / (2 N^2)   (Clenshaw-Curtis w_k on cos beta_k; (2pi/N)^2 w_k / (8 pi^2)),

    forward  fhat(l)_{mn} = sum_{j,k,l'} W_k f(alpha_j, beta_k, gamma_l') conj(t^l_{nm}),
    inverse  f = sum_{l integer, 2l < B} (2l+1) sum_{m,n} fhat(l)_{mn} t^l_{nm},
    adjoint  W_k sum c_{lmn} t^l_{nm},

with the basis values P^l_{nm}(cos beta) taken from the SU(2) oracle
(``oracle.basis``: i^{m-n} d^l_{nm}, Jacobi form).  The sum is exact for
bandlimited input: |n - n'| <= B - 1 < N, and d^l d^{l'} has degree
l + l' <= B - 1 <= N - 1 in cos beta, which Clenshaw-Curtis on N nodes integrates.

Coefficient layout (integer degrees l = 0 .. (B-1)//2): the block of l starts at
l (2l-1)(2l+1) / 3 and is row-major over m = -l..l (rows), n = -l..l (columns).
Plain numpy, float64; the sums are direct (no FFT, no reuse across coefficients
beyond per-axis exponential tables).
"""
from __future__ import annotations

import numpy as np

from . import basis, cc_weight


def num_coeffs(B: int) -> int:
    L = (B - 1) // 2 + 1           # integer degrees 0 .. L-1
    return L * (2 * L - 1) * (2 * L + 1) // 3


def coeff_index(l: int, m: int, n: int) -> int:
    if l < 0 or abs(m) > l or abs(n) > l:
        return -1
    return l * (2 * l - 1) * (2 * l + 1) // 3 + (m + l) * (2 * l + 1) + (n + l)


def triples(B: int):
    for l in range((B - 1) // 2 + 1):
        for m in range(-l, l + 1):
            for n in range(-l, l + 1):
                yield l, m, n


def grid(B: int):
    """(alpha, beta, gamma, W), N = 2B nodes per angle."""
    N = 2 * B
    j = np.arange(N)
    alpha = -np.pi + 2 * np.pi * j / N
    gamma = -np.pi + 2 * np.pi * j / N
    beta = np.pi * j / (N - 1)
    W = np.array([cc_weight(N - 1, k) for k in range(N)]) / (2.0 * N * N)
    return alpha, beta, gamma, W


def _P(B, l, m, n, beta):
    return np.array([basis(2 * l, 2 * m, 2 * n, b) for b in beta])


def forward(B: int, f: np.ndarray, sel=None) -> np.ndarray:
    """Coefficients of samples f ([k][j][l'], N^3 complex values): all of them,
    or those at the flat indices `sel`."""
    N = 2 * B
    alpha, beta, gamma, W = grid(B)
    f = np.asarray(f, dtype=np.complex128).reshape(N, N, N)
    trip = list(triples(B))
    if sel is not None:
        by_index = {coeff_index(*t): t for t in trip}
        trip = [by_index[int(i)] for i in sel]
    out = np.zeros(len(trip), dtype=np.complex128)
    for i, (l, m, n) in enumerate(trip):
        Ea = np.exp(1j * n * alpha)          # conj(e^{-i n alpha})
        Eg = np.exp(1j * m * gamma)
        Pc = np.conj(_P(B, l, m, n, beta))
        out[i] = np.sum(W[:, None, None] * Pc[:, None, None] * f * Ea[None, :, None] * Eg[None, None, :])
    return out


def _synth(B: int, c: np.ndarray, weights: np.ndarray, scale_2l1: bool) -> np.ndarray:
    N = 2 * B
    alpha, beta, gamma, _ = grid(B)
    c = np.asarray(c, dtype=np.complex128).reshape(-1)
    out = np.zeros((N, N, N), dtype=np.complex128)
    for l, m, n in triples(B):
        s = (2 * l + 1) if scale_2l1 else 1.0
        Ea = np.exp(-1j * n * alpha)
        Eg = np.exp(-1j * m * gamma)
        P = _P(B, l, m, n, beta) * weights
        out += s * c[coeff_index(l, m, n)] * P[:, None, None] * Ea[None, :, None] * Eg[None, None, :]
    return out


def inverse(B: int, c: np.ndarray) -> np.ndarray:
    return _synth(B, c, np.ones(2 * B), True)


def inverse_at(B: int, c: np.ndarray, pts) -> np.ndarray:
    """The inverse at the flat sample indices `pts` only (direct sum per point)."""
    N = 2 * B
    alpha, beta, gamma, _ = grid(B)
    pts = np.asarray(pts)
    k, j, l = pts // (N * N), (pts // N) % N, pts % N
    c = np.asarray(c, dtype=np.complex128).reshape(-1)
    out = np.zeros(pts.size, dtype=np.complex128)
    for lv, m, n in triples(B):
        P = np.array([basis(2 * lv, 2 * m, 2 * n, b) for b in beta[k]])
        out += (2 * lv + 1) * c[coeff_index(lv, m, n)] * P * np.exp(-1j * (n * alpha[j] + m * gamma[l]))
    return out


def adjoint(B: int, c: np.ndarray) -> np.ndarray:
    return _synth(B, c, grid(B)[3], False)
