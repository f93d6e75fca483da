"""Seeded synthetic inputs shared by the tests and the benchmark.

Random numbers only: no step of the transform is computed here.  Both the
oracle side (tests) and the GPU side (tests, bench) draw their inputs from
these generators so that the two compare the same data.

Recipes (numpy PCG64 via ``default_rng(seed)``):
* coefficients: complex Gaussian, E|c|^2 = var(l), re and im i.i.d. N(0, var/2);
  var(l) = 1 ("flat") or (2l+1)^-2 ("decay"); optional blocks 2l in
  ``spike_tl`` scaled by ``spike_scale`` (small-l spikes);
* samples: re and im i.i.d. uniform on [-1, 1] (not bandlimited).
Coefficient layout: 2l-major blocks of (2l+1)^2 values (rows m, columns n);
for the integer-degree (SO(3)) generator, l-major blocks of (2l+1)^2.
"""
from __future__ import annotations

import numpy as np


def num_coeffs(B: int) -> int:
    return B * (B + 1) * (2 * B + 1) // 6


def two_l_of_index(B: int) -> np.ndarray:
    """2l of every coefficient position (block tl has (tl+1)^2 entries)."""
    return np.repeat(np.arange(B), (np.arange(B) + 1) ** 2)


def coeffs(B: int, batch: int = 1, seed: int = 0, spectrum: str = "flat", spike_tl=(), spike_scale: float = 1.0,
           dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    C = num_coeffs(B)
    z = (rng.standard_normal((batch, C)) + 1j * rng.standard_normal((batch, C))) / np.sqrt(2.0)
    tl = two_l_of_index(B)
    if spectrum == "decay":
        z = z / (tl + 1.0)
    elif spectrum != "flat":
        raise ValueError(spectrum)
    if len(spike_tl):
        mask = np.isin(tl, np.asarray(spike_tl))
        z[:, mask] *= spike_scale
    return z.astype(dtype)


def num_coeffs_so3(B: int) -> int:
    """Integer degrees l with 2l < B: sum of (2l+1)^2."""
    L = (B - 1) // 2 + 1
    return L * (2 * L - 1) * (2 * L + 1) // 3


def coeffs_so3(B: int, batch: int = 1, seed: int = 0, spectrum: str = "flat", dtype=np.complex128) -> np.ndarray:
    """Coefficients of integer degrees only (l-major blocks of (2l+1)^2 values)."""
    rng = np.random.default_rng(seed)
    C = num_coeffs_so3(B)
    z = (rng.standard_normal((batch, C)) + 1j * rng.standard_normal((batch, C))) / np.sqrt(2.0)
    L = (B - 1) // 2 + 1
    l = np.repeat(np.arange(L), (2 * np.arange(L) + 1) ** 2)
    if spectrum == "decay":
        z = z / (2.0 * l + 1.0)
    elif spectrum != "flat":
        raise ValueError(spectrum)
    return z.astype(dtype)


def samples_uniform(B: int, batch: int = 1, seed: int = 0, dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    N = 2 * B
    z = rng.uniform(-1.0, 1.0, (batch, N, N, N)) + 1j * rng.uniform(-1.0, 1.0, (batch, N, N, N))
    return z.astype(dtype)


def bandlimits_mixed(count: int, choices=(16, 24, 32, 48, 64), seed: int = 33) -> list:
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.asarray(choices), size=count)]
