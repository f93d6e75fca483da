"""Plain CPU separated transform -- TEST INFRASTRUCTURE / CPU BASELINE ONLY.

The same restriction as the rest of ``oracle/`` applies: only ``tests/``, the
smoke check and the CPU-baseline leg of ``bench.py`` use it.

It evaluates the regrouped quadrature sum of Section 4 (the core equation
that turns the inner sums over alpha and gamma into a 2D DFT on every beta
ring and leaves one projection over the beta nodes per (m, n)), with library
FFTs (``scipy.fft``) and matrix products (``numpy.matmul``) in double
precision (or, as a second CPU baseline, in single precision: the tables
rounded to float32 and every array complex64), on the grid and basis of the
direct-sum oracle:

  forward:  G_k[j, q] = sum_l f[k, j, l] e^{+2 pi i q l / N},            q = 2m mod N
            H_k[p, q] = sum_j G_k[j, q] e^{i pi j / N} e^{+2 pi i p j / N}  (half-integer n; no
                        e^{i pi j / N} for integer n), p = n mod N resp. (n - 1/2) mod N
            S_k(m, n) = W_k (-1)^{2m} e^{-i pi n} H_k[p, q]
            fhat(l)_{mn} = i^{n-m} sum_k d^l_{nm}(beta_k) S_k(m, n)
  inverse:  the same chain transposed and conjugated, with (2l + 1) in place
            of W_k; adjoint: W_k instead of (2l + 1).

The Wigner-d tables come from the oracle's Jacobi-form evaluation and are
built once per plan (not part of a timed transform).  Tests pin this module to
the direct sums of ``oracle.forward`` / ``oracle.inverse`` / ``oracle.adjoint``.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from . import coeff_index, grid, num_coeffs, wigner_d_many


class CpuFFTPlan:
    def __init__(self, B: int, workers: int | None = None, dtype=np.complex128):
        self.B, self.N = B, 2 * B
        self.workers = workers or os.cpu_count() or 1
        self.cdt = np.dtype(dtype)
        self.rdt = np.float32 if self.cdt == np.complex64 else np.float64
        N = self.N
        _, beta, _, W = grid(B)
        self.W = W.astype(self.rdt)
        self.twist = np.exp(1j * np.pi * np.arange(N) / N).astype(self.cdt)
        # retained pairs, grouped by their number of degrees L for batched products
        groups = {}
        for tm in range(-(B - 1), B):
            for tn in range(-(B - 1), B):
                if (tn - tm) & 1:
                    continue
                tl0 = max(abs(tm), abs(tn))
                L = (B - 1 - tl0) // 2 + 1
                groups.setdefault(L, []).append((tm, tn, tl0))
        self.groups = []
        for L, prs in sorted(groups.items()):
            tm = np.array([x[0] for x in prs])
            tn = np.array([x[1] for x in prs])
            tl0 = np.array([x[2] for x in prs])
            tls = tl0[:, None] + 2 * np.arange(L)[None, :]                       # (G, L)
            # d^l_{nm}(beta_k), shape (G, L, N)
            args = [np.broadcast_to(v, (len(prs), L, N)).ravel() for v in
                    (tls[:, :, None], tn[:, None, None], tm[:, None, None], beta[None, None, :])]
            d = wigner_d_many(*args).reshape(len(prs), L, N)
            cidx = np.array([[coeff_index(int(a), int(m), int(n)) for a in row]
                             for row, m, n in zip(tls, tm, tn)])
            q = np.mod(tm, N)
            odd = (tm & 1).astype(bool)
            p = np.where(odd, np.mod((tn - 1) // 2, N), np.mod(tn // 2, N))
            ring_phase = (-1.0) ** tm * np.exp(-1j * np.pi * tn / 2)            # (-1)^{2m} e^{-i pi n}
            beta_phase = 1j ** np.mod((tn - tm) // 2, 4)                        # i^{n-m}
            self.groups.append(dict(L=L, d=d.astype(self.rdt), cidx=cidx, q=q, p=p, odd=odd,
                                    scale=(tls + 1).astype(self.rdt), ring_phase=ring_phase.astype(self.cdt),
                                    beta_phase=beta_phase.astype(self.cdt)))

    # ---- forward ----
    def forward(self, f: np.ndarray) -> np.ndarray:
        """f: (batch, N, N, N) samples [b][k][j][l] -> (batch, C) coefficients."""
        N, w = self.N, self.workers
        f = np.asarray(f, dtype=self.cdt).reshape(-1, N, N, N)
        G = sfft.ifft(f, axis=3, workers=w) * N                       # sum_l e^{+2 pi i q l / N}
        A0 = sfft.ifft(G, axis=2, workers=w) * N                      # integer n
        A1 = sfft.ifft(G * self.twist[None, None, :, None], axis=2, workers=w) * N   # half-integer n
        out = np.zeros((f.shape[0], num_coeffs(self.B)), dtype=self.cdt)
        for g in self.groups:
            H = np.where(g["odd"][None, None, :], A1[:, :, g["p"], g["q"]], A0[:, :, g["p"], g["q"]])  # (b, k, G)
            S = H * self.W[None, :, None] * g["ring_phase"][None, None, :]
            # (G, L, N) @ (G, N, b) -> (G, L, b)
            c = np.matmul(g["d"], np.transpose(S, (2, 1, 0)))
            c *= g["beta_phase"][:, None, None]
            out[:, g["cidx"].ravel()] = np.transpose(c, (2, 0, 1)).reshape(f.shape[0], -1)
        return out

    # ---- inverse / adjoint ----
    def _synth(self, c: np.ndarray, adjoint: bool) -> np.ndarray:
        N, w = self.N, self.workers
        c = np.asarray(c, dtype=self.cdt).reshape(-1, num_coeffs(self.B))
        nb = c.shape[0]
        H0 = np.zeros((nb, N, N, N), dtype=self.cdt)        # [b][k][p][q], integer n
        H1 = np.zeros_like(H0)                               # half-integer n
        for g in self.groups:
            cc = c[:, g["cidx"]]                                         # (b, G, L)
            if not adjoint:
                cc = cc * g["scale"][None, :, :]
            cc = cc * np.conj(g["beta_phase"])[None, :, None]
            S = np.matmul(np.transpose(g["d"], (0, 2, 1)), np.transpose(cc, (1, 2, 0)))  # (G, N, b)
            S = np.transpose(S, (2, 1, 0)) * np.conj(g["ring_phase"])[None, None, :]       # (b, k, G)
            if adjoint:
                S = S * self.W[None, :, None]
            odd = g["odd"]
            H0[:, :, g["p"][~odd], g["q"][~odd]] = S[:, :, ~odd]
            H1[:, :, g["p"][odd], g["q"][odd]] = S[:, :, odd]
        X = sfft.fft(H0, axis=2, workers=w) + sfft.fft(H1, axis=2, workers=w) * np.conj(self.twist)[None, None, :, None]
        return sfft.fft(X, axis=3, workers=w)                           # sum_q e^{-2 pi i q l / N}

    def inverse(self, c: np.ndarray) -> np.ndarray:
        return self._synth(c, False).reshape(-1, self.N, self.N, self.N)

    def adjoint(self, c: np.ndarray) -> np.ndarray:
        return self._synth(c, True).reshape(-1, self.N, self.N, self.N)
