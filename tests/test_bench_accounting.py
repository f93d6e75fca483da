"""The measurement bookkeeping of bench.py, checked on the host: the sizes
behind its roofline figures (retained pairs, coefficients, algorithmic bytes
and useful flops per launch) against counts made independently here by
enumerating the bandlimited index sets, and the one-GPU contract of its
command line."""
import os
import subprocess
import sys

import pytest

import bench
import oracle
import oracle.so3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pairs(B):
    """(2m, 2n) with |2m|, |2n| <= B - 1 and 2m = 2n mod 2: the (m, n) that some
    degree 2l < B carries (l - m and l - n integers)."""
    return [(tm, tn) for tm in range(-(B - 1), B) for tn in range(-(B - 1), B) if (tm - tn) % 2 == 0]


def _degrees(B):
    """All (2l, 2m, 2n) of the SU(2) bandlimit 2l < B."""
    return [(tl, tm, tn) for tl in range(B) for tm in range(-tl, tl + 1, 2) for tn in range(-tl, tl + 1, 2)]


@pytest.mark.parametrize("B", [1, 2, 3, 8, 17, 64])
def test_pair_and_coefficient_counts(B):
    assert bench.retained_pairs(B) == len(_pairs(B))
    assert bench.num_coeffs(B, "c64") == len(_degrees(B)) == oracle.num_coeffs(B)
    # SO(3): integer degrees l <= (B - 1) / 2 and integer m, n
    so3 = [(tl, tm, tn) for tl, tm, tn in _degrees(B) if tl % 2 == 0]
    assert bench.num_coeffs(B, "c64_so3") == len(so3) == oracle.so3.num_coeffs(B)


def _table_columns(B):
    """Distinct Wigner-d columns up to sign: d^l_{-n,-m} = (-1)^{m-n} d^l_{nm}
    pairs (m, n) with (-m, -n), so one column per degree of every pair with
    (2m, 2n) >= (0, 0) in lexicographic order."""
    return len([1 for tl, tm, tn in _degrees(B) if (tm, tn) >= (0, 0)])


def test_algorithmic_bytes_at_the_bench_workload():
    B, batch, N = 64, 32, 128
    samples = N ** 3 * 8                      # 16.78 MB per signal (complex float)
    spectra = len(_pairs(B)) * N * 8          # 8.26 MB per signal
    coeffs = len(_degrees(B)) * 8             # 0.72 MB per signal
    table = _table_columns(B) * N * 4         # symmetry-reduced FP32 table, read once per launch
    assert _table_columns(B) == (len(_degrees(B)) + 32) // 2
    assert bench.algorithmic_bytes("ring_forward", B, batch, "c64") == batch * (samples + spectra) == 801144832
    assert bench.algorithmic_bytes("ring_inverse", B, batch, "c64") == batch * (samples + spectra)
    assert bench.algorithmic_bytes("beta_forward", B, batch, "c64") == batch * (spectra + coeffs) + table
    assert bench.algorithmic_bytes("beta_inverse", B, batch, "c128") == \
        batch * 2 * (spectra + coeffs) + _table_columns(B) * N * 8
    # real signals: real samples, half of the pairs (2m >= 0 without mirrors), the reduced table
    half = len([1 for tm, tn in _pairs(B) if tm > 0 or (tm == 0 and tn >= 0)])
    assert bench.algorithmic_bytes("ring_forward", B, batch, "c64_real") == batch * (samples // 2 + half * N * 8)
    assert bench.algorithmic_bytes("beta_forward", B, batch, "c64_real") == \
        batch * (half * N * 8 + coeffs) + table
    # SO(3): integer (m, n), |m|, |n| <= 31
    so3_pairs = len([1 for tm, tn in _pairs(B) if tm % 2 == 0])
    assert bench.algorithmic_bytes("ring_inverse", B, batch, "c64_so3") == batch * (samples + so3_pairs * N * 8)


def test_useful_flops_per_contraction():
    # one real multiply-add per (coefficient, node) on the real and imaginary
    # parts: 4 flops; 45.8 MFLOP per signal at B = 64
    assert bench.useful_flops("beta_forward", 64, 1) == 4 * 128 * 89440 == 45793280
    assert bench.useful_flops("ring_forward", 64, 1) == 0.0


@pytest.mark.parametrize("extra", [[], ["--shifted-forms"], ["--copy-calibration", "1"]])
def test_more_than_one_gpu_is_refused(extra):
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *extra], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_shifted_depth1_flops():
    # A_{rho-1} s^{Lb} + B_{rho-1} s^{Lb-1}: two real x complex multiply-adds
    # per (coefficient, node, signal), twice the table form's count
    assert bench.shifted_depth1_flops(64, 1) == 2 * bench.useful_flops("beta_forward", 64, 1) == 8 * 128 * 89440
    assert bench.shifted_depth1_flops(64, 32) == 32 * bench.shifted_depth1_flops(64, 1)


def test_step_bytes_adds_the_stages_of_every_bandlimit():
    """A step is forward + inverse + adjoint: three ring stages and three
    contraction stages per bandlimit, each at the bandlimit's own sizes."""
    one = {64: 32}
    per_dir = bench.algorithmic_bytes("ring_forward", 64, 32, "c64") + bench.algorithmic_bytes("beta_forward", 64, 32, "c64")
    assert bench.step_bytes(one, "c64") == 3 * per_dir
    mixed = {16: 3, 32: 5, 64: 2}
    assert bench.step_bytes(mixed, "c64") == sum(bench.step_bytes({b: n}, "c64") for b, n in mixed.items())
    # 1 ms per step at exactly the peak's bytes is a fraction of 1
    ms = bench.step_bytes(one, "c64") / bench.HBM_PEAK * 1e3
    assert abs(bench.step_hbm_frac(one, "c64", ms) - 1.0) < 1e-3
