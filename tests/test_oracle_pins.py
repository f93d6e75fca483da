"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: every expected value comes from
a different route -- the paper's Theorem 3.2 matrix coefficients, its
Rodrigues-type Euler-angle formula (both in high precision, tests/_exact.py),
closed forms, library routines for special cases (Legendre), quadrature
moments solved independently, or invariants (unitarity, homomorphism,
orthonormality, Plancherel, exact round trip, translation covariance, the
adjoint identity).
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle
from _exact import D_group, P_rodrigues, t_euler, t_group, to_complex, u_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 40


def _rng(seed):
    return np.random.default_rng(seed)


def _triples(tl):
    return [(tm, tn) for tm in range(-tl, tl + 1, 2) for tn in range(-tl, tl + 1, 2)]


def _coeff_list(B):
    out = []
    for tl in range(B):
        for tm in range(-tl, tl + 1, 2):
            for tn in range(-tl, tl + 1, 2):
                out.append((tl, tm, tn))
    return out


def _grid_independent(B):
    """Grid nodes and weights rebuilt here from their definitions; the beta
    weights solve the moment equations sum_k w_k x_k^p = int_{-1}^{1} x^p dx,
    p = 0..N-1, at x_k = cos(beta_k) (the quadrature that integrates products
    of bandlimited basis functions exactly)."""
    N = 2 * B
    alpha = -np.pi + 2 * np.pi * np.arange(N) / N
    beta = np.pi * np.arange(N) / (N - 1)
    gamma = -2 * np.pi + 4 * np.pi * np.arange(N) / N
    x = np.cos(beta)
    V = np.vander(x, N, increasing=True).T        # V[p, k] = x_k^p
    mom = np.array([2.0 / (p + 1) if p % 2 == 0 else 0.0 for p in range(N)])
    w = np.linalg.solve(V, mom)
    W = w / (2.0 * N * N)                          # (2pi/N)(4pi/N) / (16 pi^2) = 1/(2N^2)
    return alpha, beta, gamma, W


# ---------------------------------------------------------------- basis pins

def test_theorem32_equals_euler_form():
    """Theorem 3.2 (polynomial derivative at u) == its Euler-angle form, 2l <= 5."""
    rng = _rng(1)
    worst = 0.0
    for tl in range(6):
        for tm, tn in _triples(tl):
            ph, th, ps = rng.uniform(-3, 3), rng.uniform(0.05, 3.1), rng.uniform(-6, 6)
            worst = max(worst, abs(t_group(tl, tm, tn, u_matrix(ph, th, ps)) - t_euler(tl, tm, tn, ph, th, ps)))
    assert worst < 1e-30


def test_representation_unitary_and_homomorphism():
    """D^l(u) = [t^l_{mn}(u)] is unitary and D(uv) = D(u) D(v) (Peter-Weyl, Section 2-3)."""
    u = u_matrix(0.3, 1.1, -2.0)
    v = u_matrix(-1.0, 0.4, 0.7)
    for tl in range(1, 5):
        Du, Dv, Duv = D_group(tl, u), D_group(tl, v), D_group(tl, u * v)
        assert mp.mnorm(Duv - Du * Dv) < 1e-30
        assert mp.mnorm(Du * Du.H - mp.eye(tl + 1)) < 1e-30


def test_spin_half_is_u():
    """For l = 1/2, [t^{1/2}_{mn}(u)] with m, n in (-1/2, +1/2) order is u itself."""
    for ang in [(0.3, 1.1, -2.0), (2.5, 0.2, 3.7)]:
        u = u_matrix(*ang)
        assert mp.mnorm(D_group(1, u) - u) < 1e-35


def test_closed_forms_golden():
    """P^{1/2} and P^1 closed forms (golden, hand-specialised from the paper's formula)
    against the paper's formula in high precision and against the oracle's basis."""
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        g = json.load(fh)
    env = {"cos": np.cos, "sin": np.sin, "sqrt": np.sqrt}
    for key, tl in (("P_half", 1), ("P_one", 2)):
        order = list(range(tl, -tl - 1, -2))        # descending
        for b in (0.1, 0.7, 1.9, 2.8):
            env["b"] = b
            for r, tm in enumerate(order):
                for c, tn in enumerate(order):
                    want = complex(eval(g[key][r][c], env))
                    assert abs(complex(P_rodrigues(tl, tm, tn, mp.cos(b))) - want) < 1e-14
                    # the oracle's basis returns P^l_{nm}: swap the indices
                    assert abs(oracle.basis(tl, tn, tm, b) - want) < 1e-14


def test_oracle_basis_equals_paper_P_small_l():
    """Every (l, m, n) with 2l <= 10: oracle basis == paper's P^l_{nm} (Rodrigues form)."""
    rng = _rng(2)
    worst = 0.0
    for tl in range(11):
        for tm, tn in _triples(tl):
            b = rng.uniform(0.02, np.pi - 0.02)
            want = complex(P_rodrigues(tl, tn, tm, mp.cos(b)))
            worst = max(worst, abs(oracle.basis(tl, tm, tn, b) - want))
    assert worst < 1e-14


def test_oracle_wigner_large_l_against_paper_formula():
    """Sampled triples up to 2l = 127 (B = 128): oracle basis vs the paper's formula
    evaluated exactly (integer polynomial derivative, high-precision evaluation)."""
    rng = _rng(3)
    worst = 0.0
    for _ in range(40):
        tl = int(rng.integers(60, 128))
        tm = int(rng.integers(0, tl + 1)) * 2 - tl
        tn = int(rng.integers(0, tl + 1)) * 2 - tl
        b = float(rng.uniform(0.02, np.pi - 0.02))
        want = complex(P_rodrigues(tl, tn, tm, mp.cos(mp.mpf(b))))
        worst = max(worst, abs(oracle.basis(tl, tm, tn, b) - want))
    assert worst < 1e-12


def test_legendre_column():
    """m = n = 0 reduces to the Legendre polynomials (Lemma 4.3's P_l), checked
    against scipy's Legendre routine, and P_0 = 1, P_1 = x."""
    for l in range(0, 64):
        for b in (0.0, 0.3, 1.2, 2.9, np.pi):
            assert abs(oracle.wigner_d(2 * l, 0, 0, b) - eval_legendre(l, np.cos(b))) < 1e-13
    assert oracle.wigner_d(0, 0, 0, 0.4) == 1.0
    assert abs(oracle.wigner_d(2, 0, 0, 0.4) - np.cos(0.4)) < 1e-16


def test_identity_at_beta_zero():
    """u(0, 0, 0) = I, so D^l = I: d^l_{ab}(0) = delta_ab."""
    for tl in range(0, 20):
        for tm, tn in _triples(tl):
            want = 1.0 if tm == tn else 0.0
            assert abs(oracle.wigner_d(tl, tm, tn, 0.0) - want) < 1e-15


def test_beta_pi_against_group_element():
    """At beta = pi the basis must match Theorem 3.2 at u(0, pi, 0) = [[0, i], [i, 0]]."""
    u = u_matrix(0, mp.pi, 0)
    for tl in range(0, 8):
        D = to_complex(D_group(tl, u))
        idx = list(range(-tl, tl + 1, 2))
        for r, ta in enumerate(idx):
            for c, tb in enumerate(idx):
                # t^l_{ab}(u) = P^l_{ab}; the oracle's basis(tl, tm, tn) is P^l_{nm}
                assert abs(oracle.basis(tl, tb, ta, np.pi) - D[r, c]) < 1e-14


# ---------------------------------------------------------- quadrature pins

@pytest.mark.parametrize("N", [2, 4, 6, 8, 12, 16, 32, 48, 64, 96, 128, 256])
def test_clenshaw_curtis_moments(N):
    """sum_k w_k x_k^p = int_{-1}^{1} x^p dx for p = 0..N-1 (exactness of the beta rule)."""
    n = N - 1
    x = np.cos(np.pi * np.arange(N) / n)
    w = np.array([oracle.cc_weight(n, k) for k in range(N)])
    for p in range(N):
        want = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** p) - want) < 1e-13


@pytest.mark.parametrize("B", [1, 2, 3, 4, 6, 8])
def test_grid_matches_independent_construction(B):
    a, b, g, W = oracle.grid(B)
    a2, b2, g2, W2 = _grid_independent(B)
    assert np.allclose(a, a2, atol=1e-15) and np.allclose(b, b2, atol=1e-15)
    assert np.allclose(g, g2, atol=1e-15)
    assert np.allclose(W, W2, atol=1e-14 / (4 * B * B))
    assert abs(np.sum(W) * (2 * B) ** 2 - 1.0) < 1e-14          # total volume normalised to 1


# ---------------------------------------------------- transform-level pins

def _samples_from_group(B, fn):
    """Evaluate fn(u) (u from Theorem 3.2) on the grid, layout [k][j][l]."""
    alpha, beta, gamma, _ = _grid_independent(B)
    N = 2 * B
    out = np.zeros((N, N, N), dtype=np.complex128)
    for k in range(N):
        for j in range(N):
            for l in range(N):
                out[k, j, l] = fn(u_matrix(alpha[j], beta[k], gamma[l]))
    return out


@pytest.mark.parametrize("B", [1, 2, 3])
def test_forward_brute_force_theorem32(B):
    """Forward = sum_grid W_k f conj(t^l_{nm}(u(alpha_j, beta_k, gamma_l))) with t
    from Theorem 3.2 (no Euler-angle formula involved)."""
    rng = _rng(10 + B)
    N = 2 * B
    f = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    alpha, beta, gamma, W = _grid_independent(B)
    want = np.zeros(oracle.num_coeffs(B), dtype=np.complex128)
    for k in range(N):
        for j in range(N):
            for l in range(N):
                u = u_matrix(alpha[j], beta[k], gamma[l])
                for tl in range(B):
                    D = to_complex(D_group(tl, u))          # D[a, b] = t^l_{ab}
                    for (tm, tn) in _triples(tl):
                        i = oracle.coeff_index(tl, tm, tn)
                        t_nm = D[(tn + tl) // 2, (tm + tl) // 2]
                        want[i] += W[k] * f[k, j, l] * np.conj(t_nm)
    got = oracle.forward(B, f)
    assert np.max(np.abs(got - want)) < 1e-14 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("B", [1, 2, 3])
def test_inverse_brute_force_theorem32(B):
    """Inverse = sum (2l+1) fhat(l)_{mn} t^l_{nm}(u) with t from Theorem 3.2."""
    rng = _rng(20 + B)
    C = oracle.num_coeffs(B)
    c = rng.standard_normal(C) + 1j * rng.standard_normal(C)

    def fn(u):
        s = 0j
        for tl in range(B):
            D = to_complex(D_group(tl, u))
            for (tm, tn) in _triples(tl):
                s += (tl + 1) * c[oracle.coeff_index(tl, tm, tn)] * D[(tn + tl) // 2, (tm + tl) // 2]
        return s

    want = _samples_from_group(B, fn)
    got = oracle.inverse(B, c)
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("B", [2, 3, 4])
def test_orthonormality_on_grid(B):
    """<t^l_{nm}, t^l'_{n'm'}> on the grid = delta/(2l+1): the forward transform of
    samples of one basis function (Theorem 3.2 values) is delta/(2l+1)."""
    rng = _rng(30 + B)
    C = oracle.num_coeffs(B)
    triples = _coeff_list(B)
    picks = rng.choice(len(triples), size=min(C, 4), replace=False)
    for pick in picks:
        tl, tm, tn = triples[pick]
        q = oracle.coeff_index(tl, tm, tn)
        samples = _samples_from_group(B, lambda u: complex(t_group(tl, tn, tm, u)))   # t^l_{nm}
        got = oracle.forward(B, samples)
        want = np.zeros(C, dtype=np.complex128)
        want[q] = 1.0 / (tl + 1)
        assert np.max(np.abs(got - want)) < 1e-14


@pytest.mark.parametrize("B", [1, 2, 3, 4, 6, 8])
def test_round_trip_and_plancherel(B):
    """Exact quadrature: forward(inverse(c)) = c and sum W|f|^2 = sum (2l+1)|fhat|^2."""
    rng = _rng(40 + B)
    C = oracle.num_coeffs(B)
    c = (rng.standard_normal(C) + 1j * rng.standard_normal(C)) / np.sqrt(2)
    f = oracle.inverse(B, c)
    c2 = oracle.forward(B, f)
    assert np.max(np.abs(c2 - c)) < 1e-13
    _, _, _, W = _grid_independent(B)
    lhs = np.sum(W[:, None, None] * np.abs(f) ** 2)
    tls = np.array([t for t in range(B) for _ in range((t + 1) ** 2)])
    rhs = np.sum((tls + 1) * np.abs(c) ** 2)
    assert abs(lhs - rhs) < 1e-12 * rhs


def test_bandlimit_one_is_the_mean():
    """B = 1: the only coefficient is fhat(0) = sum_grid W_k f (t^0 = 1)."""
    rng = _rng(50)
    f = rng.standard_normal((2, 2, 2)) + 1j * rng.standard_normal((2, 2, 2))
    _, _, _, W = _grid_independent(1)
    assert abs(oracle.forward(1, f)[0] - np.sum(W[:, None, None] * f)) < 1e-15


def test_translation_covariance():
    """g(x) = f(y^{-1} x)  =>  ghat(l) = fhat(l) D^l(y)^H (D a unitary homomorphism)."""
    B = 3
    rng = _rng(60)
    C = oracle.num_coeffs(B)
    c = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    y = u_matrix(0.7, 1.3, -0.4)
    yinv = y.H

    def blocks(vec):
        out = []
        for tl in range(B):
            base = oracle.coeff_index(tl, -tl, -tl)
            out.append(np.array(vec[base:base + (tl + 1) ** 2]).reshape(tl + 1, tl + 1))
        return out

    fb = blocks(c)

    def g_of(u):
        x = yinv * u
        s = 0j
        for tl in range(B):
            D = to_complex(D_group(tl, x))
            s += (tl + 1) * np.trace(fb[tl] @ D)
        return s

    g = _samples_from_group(B, g_of)
    gb = blocks(oracle.forward(B, g))
    for tl in range(B):
        Dy = to_complex(D_group(tl, y))
        assert np.max(np.abs(gb[tl] - fb[tl] @ Dy.conj().T)) < 1e-13


@pytest.mark.parametrize("B", [2, 4, 6])
def test_adjoint_identity(B):
    """<F x, y> = <x, F^H y> for random (not bandlimited) x and random y."""
    rng = _rng(70 + B)
    N = 2 * B
    C = oracle.num_coeffs(B)
    x = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    y = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    lhs = np.vdot(y, oracle.forward(B, x))
    rhs = np.vdot(oracle.adjoint(B, y), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_adjoint_is_weighted_synthesis():
    """F^H c = W_k * synthesis(c / (2l+1)) (the adjoint differs from the inverse
    only by the weights)."""
    B = 4
    rng = _rng(80)
    C = oracle.num_coeffs(B)
    c = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    tls = np.array([t for t in range(B) for _ in range((t + 1) ** 2)])
    _, _, _, W = _grid_independent(B)
    want = W[:, None, None] * oracle.inverse(B, c / (tls + 1))
    assert np.max(np.abs(oracle.adjoint(B, c) - want)) < 1e-15


def test_selected_outputs_match_full():
    B = 4
    N = 2 * B
    rng = _rng(90)
    C = oracle.num_coeffs(B)
    f = rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))
    c = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    full_f, full_c = oracle.forward(B, f), oracle.inverse(B, c)
    sel = rng.choice(C, 17, replace=False)
    assert np.array_equal(oracle.forward(B, f, sel), full_f[sel])
    pts = rng.choice(N ** 3, 23, replace=False)
    assert np.array_equal(oracle.inverse(B, c, pts), full_c.reshape(-1)[pts])


def test_coefficient_layout_is_a_bijection():
    for B in (1, 2, 5, 8):
        seen = sorted(oracle.coeff_index(*t) for t in _coeff_list(B))
        assert seen == list(range(oracle.num_coeffs(B)))
        assert oracle.num_coeffs(B) == B * (B + 1) * (2 * B + 1) // 6
    assert oracle.coeff_index(2, 1, 0) == -1 and oracle.coeff_index(1, 3, 1) == -1


def test_thread_count_does_not_change_results():
    """The CPU baselines time the oracle on one core and on all of them; its
    sums are per-coefficient and per-sample, so the thread count changes no
    bit of a result."""
    B = 4
    rng = np.random.default_rng(81)
    N = 2 * B
    x = rng.standard_normal(N ** 3) + 1j * rng.standard_normal(N ** 3)
    C = oracle.num_coeffs(B)
    c = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    full = oracle.num_threads()
    try:
        oracle.set_num_threads(1)
        f1, i1 = oracle.forward(B, x), oracle.inverse(B, c)
    finally:
        oracle.set_num_threads(max(full, 1))
    assert np.array_equal(f1, oracle.forward(B, x))
    assert np.array_equal(i1, oracle.inverse(B, c))
