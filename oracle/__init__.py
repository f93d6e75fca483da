"""Reference oracle for the SU(2) Fourier transform -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_2605_23923_amd``) never imports it and shares no code with it.

The arithmetic lives in ``su2_oracle.c`` (plain C, double precision, direct
quadrature sums of Definition 3.4 / Theorem 5.1); this module only marshals
arrays through ctypes.  See the header of ``su2_oracle.c`` for the grid,
basis and layout conventions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "su2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, IEEE semantics) into ``liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    i64 = ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_int64)
    lib.orc_num_coeffs.restype = i64
    lib.orc_num_coeffs.argtypes = [ctypes.c_int]
    lib.orc_coeff_index.restype = i64
    lib.orc_coeff_index.argtypes = [ctypes.c_int] * 3
    lib.orc_cc_weight.restype = ctypes.c_double
    lib.orc_cc_weight.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.orc_grid.restype = None
    lib.orc_grid.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    lib.orc_jacobi.restype = ctypes.c_double
    lib.orc_jacobi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.orc_wigner_d.restype = ctypes.c_double
    lib.orc_wigner_d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_wigner_d_many.restype = None
    lib.orc_wigner_d_many.argtypes = [i64, ip, ip, ip, dp, dp]
    lib.orc_basis.restype = None
    lib.orc_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
    lib.orc_forward.restype = None
    lib.orc_forward.argtypes = [ctypes.c_int, dp, i64, lp, dp]
    lib.orc_synth.restype = None
    lib.orc_synth.argtypes = [ctypes.c_int, dp, ctypes.c_int, i64, lp, dp]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def num_coeffs(B: int) -> int:
    return int(_load().orc_num_coeffs(B))


def coeff_index(tl: int, tm: int, tn: int) -> int:
    """Flat index of fhat(l)_{mn} from doubled indices (2l, 2m, 2n); -1 if invalid."""
    return int(_load().orc_coeff_index(tl, tm, tn))


def cc_weight(n: int, k: int) -> float:
    return float(_load().orc_cc_weight(n, k))


def grid(B: int):
    """(alpha, beta, gamma, W) node arrays of length N = 2B."""
    N = 2 * B
    a, b, g, w = (np.zeros(N) for _ in range(4))
    _load().orc_grid(B, _dptr(a), _dptr(b), _dptr(g), _dptr(w))
    return a, b, g, w


def jacobi(s: int, a: int, b: int, x: float) -> float:
    return float(_load().orc_jacobi(s, a, b, x))


def wigner_d(tl: int, ta: int, tb: int, beta: float) -> float:
    """Wigner small-d d^l_{a b}(beta) with doubled indices."""
    return float(_load().orc_wigner_d(tl, ta, tb, float(beta)))


def wigner_d_many(tl, ta, tb, beta) -> np.ndarray:
    """Vectorised ``wigner_d`` over equally long argument arrays."""
    tl, ta, tb = (np.ascontiguousarray(np.asarray(v, dtype=np.int32)) for v in (tl, ta, tb))
    be = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
    out = np.zeros(be.size)
    ip = ctypes.POINTER(ctypes.c_int)
    _load().orc_wigner_d_many(be.size, tl.ctypes.data_as(ip), ta.ctypes.data_as(ip), tb.ctypes.data_as(ip),
                              _dptr(be), _dptr(out))
    return out


def basis(tl: int, tm: int, tn: int, beta: float) -> complex:
    """P^l_{nm}(cos beta) as the oracle's sums use it (doubled indices)."""
    out = np.zeros(2)
    _load().orc_basis(tl, tm, tn, float(beta), _dptr(out))
    return complex(out[0], out[1])


def forward(B: int, f: np.ndarray, sel=None) -> np.ndarray:
    """Direct-sum forward transform of samples f (complex, shape (N, N, N) or
    flat N^3, layout [k][j][l]).  Returns all C(B) coefficients, or those at
    the flat indices ``sel``."""
    N = 2 * B
    fa = np.ascontiguousarray(np.asarray(f, dtype=np.complex128).reshape(N * N * N))
    if sel is None:
        out = np.zeros(num_coeffs(B), dtype=np.complex128)
        _load().orc_forward(B, _dptr(fa.view(np.float64)), 0, None, _dptr(out.view(np.float64)))
    else:
        s = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
        out = np.zeros(s.size, dtype=np.complex128)
        _load().orc_forward(B, _dptr(fa.view(np.float64)), s.size, _lptr(s), _dptr(out.view(np.float64)))
    return out


def _synth(B: int, c: np.ndarray, mode: int, sel) -> np.ndarray:
    N = 2 * B
    ca = np.ascontiguousarray(np.asarray(c, dtype=np.complex128).reshape(num_coeffs(B)))
    if sel is None:
        out = np.zeros(N * N * N, dtype=np.complex128)
        _load().orc_synth(B, _dptr(ca.view(np.float64)), mode, 0, None, _dptr(out.view(np.float64)))
        return out.reshape(N, N, N)
    s = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    out = np.zeros(s.size, dtype=np.complex128)
    _load().orc_synth(B, _dptr(ca.view(np.float64)), mode, s.size, _lptr(s), _dptr(out.view(np.float64)))
    return out


def inverse(B: int, c: np.ndarray, sel=None) -> np.ndarray:
    """Synthesis f = sum (2l+1) fhat(l)_{mn} t^l_{nm} at all grid points
    (shape (N, N, N)) or at the flat sample indices ``sel``."""
    return _synth(B, c, 0, sel)


def adjoint(B: int, c: np.ndarray, sel=None) -> np.ndarray:
    """Conjugate transpose of ``forward``: W_k sum c_{lmn} t^l_{nm}."""
    return _synth(B, c, 1, sel)
