"""Shifted three-term recurrence and the divide-and-conquer projection of
Section 4 -- TEST INFRASTRUCTURE ONLY (same import restriction as the rest of
``oracle/``).

The paper derives, for the Legendre case m = n = 0 and "analogously" for
general (m, n), that a polynomial L + r steps up the recurrence is a
combination of the two at levels L and L - 1,

    d^{L+r} = A_r^L d^L + B_r^L d^{L-1},      A_0 = 1, B_0 = 0, A_{-1} = 0, B_{-1} = 1,

where (A_r^L, B_r^L) follow the same one-step transfer matrix as d itself
(the matrix recurrence proposition), compose by matrix products (the
composition-rule proposition), and turn a projection <s, d^{L+r}> into
<s^L, A_r^L> + <s^{L-1}, B_r^L> with the stored pointwise products
s^j = s * d^j (the divide-and-conquer theorem); splitting r = n1 + ... + nk
gives 2^k terms of Hadamard products of lower-order shifted polynomials (the
worked example is k = 2 with four terms).

For general (m, n) the one-step matrix is the Wigner-d recurrence in l
(degree l -> l + 1, integer or half-integer l, fixed m, n):

    d^{l+1} = a_l (x - b_l) d^l - c_l d^{l-1},  x = cos(beta),
    a_l = (l+1)(2l+1) / sqrt(((l+1)^2 - m^2)((l+1)^2 - n^2)),
    b_l = m n / (l (l+1)),  c_l = a_l sqrt((l^2 - m^2)(l^2 - n^2)) / (l (2l+1)),
    (b_0 = c_0 = 0),

which at m = n = 0 is the Legendre recurrence of the lemma ((2l+1)/(l+1) and
l/(l+1)).  Degrees use doubled integers (tl = 2l) like the rest of the oracle.
Everything here is plain numpy in float64.
"""
from __future__ import annotations

import itertools

import numpy as np


def step_coeffs(tl: int, tm: int, tn: int):
    """(a_l, b_l, c_l) of the step that produces degree l + 1 from l and l - 1."""
    l, m, n = tl / 2.0, tm / 2.0, tn / 2.0
    a = (l + 1) * (2 * l + 1) / np.sqrt(((l + 1) ** 2 - m * m) * ((l + 1) ** 2 - n * n))
    if l == 0:
        return a, 0.0, 0.0
    b = m * n / (l * (l + 1))
    c = a * np.sqrt((l * l - m * m) * (l * l - n * n)) / (l * (2 * l + 1))
    return a, b, c


def transfer(tl: int, tm: int, tn: int, x):
    """One-step matrix [[a (x - b), -c], [1, 0]] at degree l (maps (d^l, d^{l-1}) to (d^{l+1}, d^l))."""
    a, b, c = step_coeffs(tl, tm, tn)
    x = np.asarray(x, dtype=np.float64)
    return np.array([[a * (x - b), np.full_like(x, -c)], [np.ones_like(x), np.zeros_like(x)]])


def shifted_AB(tL: int, r: int, tm: int, tn: int, x):
    """(A_r^L, A_{r-1}^L, B_r^L, B_{r-1}^L) at the points x, from the matrix
    recurrence started at A_0 = 1, B_0 = 0, A_{-1} = 0, B_{-1} = 1 (level L = tL / 2)."""
    x = np.asarray(x, dtype=np.float64)
    A, Ap = np.ones_like(x), np.zeros_like(x)     # A_0, A_{-1}
    Bv, Bp = np.zeros_like(x), np.ones_like(x)    # B_0, B_{-1}
    if r < 0:
        return Ap, None, Bp, None
    for j in range(r):
        a, b, c = step_coeffs(tL + 2 * j, tm, tn)
        t = a * (x - b)
        A, Ap = t * A - c * Ap, A
        Bv, Bp = t * Bv - c * Bp, Bv
    return A, Ap, Bv, Bp


def shift_matrix(tL: int, r: int, tm: int, tn: int, x):
    """[[A_r, B_r], [A_{r-1}, B_{r-1}]] of level L (r >= 0)."""
    A, Ap, Bv, Bp = shifted_AB(tL, r, tm, tn, x)
    return np.array([[A, Bv], [Ap, Bp]])


def projection_k1(s, dL, dLm1, tL: int, r: int, tm: int, tn: int, x):
    """<s, d^{L+r}> = <s^L, A_r^L> + <s^{L-1}, B_r^L> with s^j = s * d^j (k = 1)."""
    A, _, Bv, _ = shifted_AB(tL, r, tm, tn, x)
    return np.dot(s * dL, A) + np.dot(s * dLm1, Bv)


def projection_k2(s, dL, dLm1, tL: int, n1: int, n2: int, tm: int, tn: int, x):
    """The four-term form of the worked example (k = 2, r = n1 + n2):
    <s^L, A_{n2}^{L+n1} A_{n1}^L> + <s^L, B_{n2}^{L+n1} A_{n1-1}^L>
    + <s^{L-1}, A_{n2}^{L+n1} B_{n1}^L> + <s^{L-1}, B_{n2}^{L+n1} B_{n1-1}^L>."""
    A1, A1p, B1, B1p = shifted_AB(tL, n1, tm, tn, x)
    A2, _, B2, _ = shifted_AB(tL + 2 * n1, n2, tm, tn, x)
    if n1 == 0:   # A_{-1} = 0, B_{-1} = 1
        A1p, B1p = np.zeros_like(A1), np.ones_like(A1)
    sL, sLm1 = s * dL, s * dLm1
    return (np.dot(sL, A2 * A1) + np.dot(sL, B2 * A1p) + np.dot(sLm1, A2 * B1) + np.dot(sLm1, B2 * B1p))


def projection_general(s, dL, dLm1, tL: int, parts, tm: int, tn: int, x):
    """The divide-and-conquer expansion for r = n_1 + ... + n_k: a sum over
    tau_1 in {A, B} and eps_1..eps_{k-1} in {0, 1} of
    <s^{L*(tau_1)}, tau_1{}_{n_1 - eps_1}^{L} * prod_{i >= 2} tau_i(eps_{i-1})_{n_i - eps_i}^{L_{i-1}}>,
    with tau_i(0) = A, tau_i(1) = B and L_{i-1} = L + n_1 + ... + n_{i-1}.

    (The index n_i - eps_i with eps_k = 0 on the last factor reads the
    theorem's product so that it reproduces the composition rule; the worked
    k = 2 example is the case parts = (n1, n2).)"""
    parts = list(parts)
    k = len(parts)
    levels = [tL]
    for n in parts[:-1]:
        levels.append(levels[-1] + 2 * n)
    # per factor i: (A_{n_i}, A_{n_i - 1}, B_{n_i}, B_{n_i - 1}) at level levels[i]
    facs = []
    for i, n in enumerate(parts):
        A, Ap, Bv, Bp = shifted_AB(levels[i], n, tm, tn, x)
        if n == 0:
            Ap, Bp = np.zeros_like(A), np.ones_like(A)
        facs.append({("A", 0): A, ("A", 1): Ap, ("B", 0): Bv, ("B", 1): Bp})
    sL, sLm1 = s * dL, s * dLm1
    total = 0.0
    for tau1 in ("A", "B"):
        for eps in itertools.product((0, 1), repeat=k - 1):
            e = list(eps) + [0]
            v = facs[0][(tau1, e[0])].copy()
            for i in range(1, k):
                tau_i = "A" if e[i - 1] == 0 else "B"
                v = v * facs[i][(tau_i, e[i])]
            total = total + np.dot(sL if tau1 == "A" else sLm1, v)
    return total
