"""Exact, paper-definition routes used to pin the oracle (tests only).

Everything here is evaluated in high precision (mpmath) straight from the
paper's formulas, by routes that share nothing with the oracle's Jacobi-form
evaluation or with the GPU library:

* ``u_matrix`` / ``t_group``: Theorem 3.2 -- the SU(2) element u(phi, theta, psi)
  and the matrix coefficients t^l_{mn}(u) as the mixed derivative
  d^{l-m}/dz1^{l-m} d^{l+m}/dz2^{l+m} of (z1 a + z2 c)^{l-n} (z1 b + z2 d)^{l+n},
  divided by sqrt((l-m)!(l+m)!(l-n)!(l+n)!).  The polynomial is homogeneous of
  degree 2l, so the derivative is (l-m)!(l+m)! times one monomial coefficient.
* ``P_rodrigues``: the Euler-angle form that follows Theorem 3.2,
  P^l_{mn}(x) = c^l_{mn} (1-x)^{(n-m)/2} (1+x)^{-(m+n)/2} (d/dx)^{l-m}[(1-x)^{l-n}(1+x)^{l+n}],
  c^l_{mn} = 2^{-l} (-1)^{l-n} i^{n-m} sqrt((l+m)!/(l-m)!) / sqrt((l-n)!(l+n)!),
  with the polynomial differentiated exactly in integers.

All indices are doubled (tl = 2l, tm = 2m, tn = 2n) so half-integers stay exact.
"""
from __future__ import annotations

from math import comb, factorial

import mpmath as mp
import numpy as np


def _half(t2: int) -> int:
    assert t2 % 2 == 0
    return t2 // 2


def u_matrix(phi, theta, psi):
    """u(phi, theta, psi) of Theorem 3.2 as a 2x2 mpmath matrix."""
    phi, theta, psi = mp.mpf(phi), mp.mpf(theta), mp.mpf(psi)
    I = mp.mpc(0, 1)
    c, s = mp.cos(theta / 2), mp.sin(theta / 2)
    a = mp.exp(I * (phi + psi) / 2) * c
    b = mp.exp(I * (phi - psi) / 2) * I * s
    cc = mp.exp(-I * (phi - psi) / 2) * I * s
    d = mp.exp(-I * (phi + psi) / 2) * c
    return mp.matrix([[a, b], [cc, d]])


def t_group(tl: int, tm: int, tn: int, u) -> mp.mpc:
    """t^l_{mn}(u) by Theorem 3.2 (doubled indices), u a 2x2 matrix [[a, b], [c, d]]."""
    a, b, c, d = u[0, 0], u[0, 1], u[1, 0], u[1, 1]
    lmm, lpm = _half(tl - tm), _half(tl + tm)
    lmn, lpn = _half(tl - tn), _half(tl + tn)
    # coefficient of z1^{l-m} z2^{l+m} in (z1 a + z2 c)^{l-n} (z1 b + z2 d)^{l+n}
    coef = mp.mpc(0)
    for i in range(0, lmn + 1):          # power of z1 taken from the first factor
        k = lmm - i                       # power of z1 taken from the second factor
        if k < 0 or k > lpn:
            continue
        coef += comb(lmn, i) * a ** i * c ** (lmn - i) * comb(lpn, k) * b ** k * d ** (lpn - k)
    deriv = factorial(lmm) * factorial(lpm) * coef
    return deriv / mp.sqrt(factorial(lmm) * factorial(lpm) * factorial(lmn) * factorial(lpn))


def D_group(tl: int, u) -> mp.matrix:
    """The (2l+1)x(2l+1) matrix [t^l_{mn}(u)], rows m and columns n ascending (-l..l)."""
    idx = list(range(-tl, tl + 1, 2))
    M = mp.matrix(tl + 1, tl + 1)
    for r, tm in enumerate(idx):
        for s_, tn in enumerate(idx):
            M[r, s_] = t_group(tl, tm, tn, u)
    return M


def _poly_mul(p, q):
    out = [0] * (len(p) + len(q) - 1)
    for i, x in enumerate(p):
        if x:
            for j, y in enumerate(q):
                out[i + j] += x * y
    return out


def _poly_pow_linear(c0, c1, e):
    """(c0 + c1 x)^e as an integer coefficient list (ascending powers)."""
    return [comb(e, i) * c0 ** (e - i) * c1 ** i for i in range(e + 1)]


def _poly_deriv(p, times):
    for _ in range(times):
        p = [i * p[i] for i in range(1, len(p))] or [0]
    return p


def P_rodrigues(tl: int, tm: int, tn: int, x) -> mp.mpc:
    """The paper's P^l_{mn}(x) (Euler-angle form after Theorem 3.2), doubled indices."""
    x = mp.mpf(x)
    lmn, lpn = _half(tl - tn), _half(tl + tn)
    lmm, lpm = _half(tl - tm), _half(tl + tm)
    poly = _poly_mul(_poly_pow_linear(1, -1, lmn), _poly_pow_linear(1, 1, lpn))
    poly = _poly_deriv(poly, lmm)
    big = max(abs(v) for v in poly) if poly else 1
    with mp.workdps(mp.mp.dps + len(str(big)) + 10):
        val = mp.mpf(0)
        for i in reversed(range(len(poly))):
            val = val * x + poly[i]
        I = mp.mpc(0, 1)
        # i^{n-m} with n-m integer
        ipow = [1, I, -1, -I][_half(tn - tm) % 4]
        sign = -1 if (lmn % 2) else 1
        c = (mp.mpf(2) ** (-mp.mpf(tl) / 2) * sign * ipow
             * mp.sqrt(mp.mpf(factorial(lpm)) / factorial(lmm))
             / mp.sqrt(mp.mpf(factorial(lmn)) * factorial(lpn)))
        pref = (1 - x) ** (mp.mpf(tn - tm) / 4) * (1 + x) ** (-mp.mpf(tm + tn) / 4)
        res = c * pref * val
    return +res


def t_euler(tl: int, tm: int, tn: int, phi, theta, psi) -> mp.mpc:
    """t^l_{mn}(phi, theta, psi) = P^l_{mn}(cos theta) exp(-i(m phi + n psi))."""
    I = mp.mpc(0, 1)
    return P_rodrigues(tl, tm, tn, mp.cos(theta)) * mp.exp(
        -I * (mp.mpf(tm) / 2 * mp.mpf(phi) + mp.mpf(tn) / 2 * mp.mpf(psi)))


def to_complex(M) -> np.ndarray:
    return np.array([[complex(M[i, j]) for j in range(M.cols)] for i in range(M.rows)])
