"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, validates arguments before touching
the device, and its host helpers (sizes, indices, grid) agree with the
oracle's independent implementations."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2605_23923_amd as su2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(su2_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(su2.library_path())
    names = _header_functions()
    assert "su2_forward" in names and "su2_plan_create" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/ but not exported"


def test_sizes_and_indices_match_oracle():
    for B in (1, 2, 3, 8, 64, 128):
        assert su2.num_coeffs(B) == oracle.num_coeffs(B)
        assert su2.num_samples(B) == (2 * B) ** 3
    for tl in range(0, 12):
        for tm in range(-tl - 1, tl + 2):
            for tn in range(-tl - 1, tl + 2):
                assert su2.coeff_index(tl, tm, tn) == oracle.coeff_index(tl, tm, tn)
    assert su2.num_coeffs(0) == -1 and su2.num_samples(-3) == -1


@pytest.mark.parametrize("B", [1, 2, 3, 4, 8, 24, 64, 128])
def test_grid_matches_oracle(B):
    a, b, g, w = (np.array(v) for v in su2.grid(B))
    A, Bt, G, W = oracle.grid(B)
    # the library builds the grid in long double and rounds once; the oracle in
    # double: agreement to a few units in the last place
    assert np.max(np.abs(a - A)) < 4e-15 and np.max(np.abs(b - Bt)) < 4e-15
    assert np.max(np.abs(g - G)) < 8e-15
    assert np.max(np.abs(w - W)) < 4e-15 * np.max(np.abs(W))


def _lib():
    su2._load()
    return su2._lib


def _create(B, batch, dtype):
    h = ctypes.c_void_p()
    st = _lib().su2_plan_create(B, batch, dtype, ctypes.byref(h))
    return st, h


def test_argument_validation_before_any_device_call():
    lib = _lib()
    assert _create(0, 1, 0)[0] == 1           # B < 1
    assert _create(8, 0, 0)[0] == 1           # batch < 1
    assert _create(8, 1, 7)[0] == 1           # unknown dtype
    assert _create(5, 1, 0)[0] == 2           # N = 10 is not 2^a 3^b
    assert _create(129, 1, 0)[0] == 2         # beyond the largest bandlimit
    assert _create(64, 131073, 1)[0] == 2     # one pair tile's spectra beyond 32-bit offsets
    assert _create(8, 524289, 0)[0] == 2
    assert lib.su2_plan_create(8, 1, 0, None) == 1
    assert lib.su2_forward(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 1
    assert lib.su2_inverse(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 1
    assert lib.su2_adjoint(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 1
    assert lib.su2_forward_noalloc(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 1
    assert lib.su2_plan_destroy(None) == 0
    bs = (ctypes.c_int32 * 2)(8, 5)
    h = ctypes.c_void_p()
    assert lib.su2_plan_create_mixed(bs, 2, 1, ctypes.byref(h)) == 2
    bs = (ctypes.c_int32 * 2)(8, 0)
    assert lib.su2_plan_create_mixed(bs, 2, 1, ctypes.byref(h)) == 1
    assert lib.su2_grid(0, None, None, None, None) == 1
    assert lib.su2_status_string(2).startswith(b"SU2_ERR_UNSUPPORTED")
    # plan options: unknown bits, and on-the-fly tables with the split-BF16 mode
    lib.su2_plan_create_ex.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_void_p)]
    assert lib.su2_plan_create_ex(8, 1, 1, 8, ctypes.byref(h)) == 1
    assert lib.su2_plan_create_ex(8, 1, 1, 0x80000000, ctypes.byref(h)) == 1
    assert lib.su2_plan_create_ex(8, 1, 2, 1, ctypes.byref(h)) == 2
    assert lib.su2_plan_create_ex(0, 1, 1, 1, ctypes.byref(h)) == 1
    # real signals and SO(3): every mode and bandlimit, not with generated
    # tables and not together (accepted combinations need a device: not here)
    for dt in (0, 1, 2):
        for B in (8, 24, 128):
            assert lib.su2_plan_create_ex(B, 1, dt, 3, ctypes.byref(h)) == 2   # real + on the fly
            assert lib.su2_plan_create_ex(B, 1, dt, 5, ctypes.byref(h)) == 2   # SO(3) + on the fly
            assert lib.su2_plan_create_ex(B, 1, dt, 6, ctypes.byref(h)) == 2   # real + SO(3)
    # mixed plans with options: the same rules, unknown bits rejected first
    bs2 = (ctypes.c_int32 * 2)(8, 24)
    assert lib.su2_plan_create_mixed_ex(bs2, 2, 1, 8, ctypes.byref(h)) == 1
    assert lib.su2_plan_create_mixed_ex(bs2, 2, 1, 1, ctypes.byref(h)) == 2
    assert lib.su2_plan_create_mixed_ex(bs2, 2, 1, 6, ctypes.byref(h)) == 2
    assert lib.su2_plan_create_mixed_ex(None, 2, 1, 2, ctypes.byref(h)) == 1
    assert lib.su2_plan_create_ex(8, 0, 0, 4, ctypes.byref(h)) == 1


def test_so3_layout_helpers_match_the_oracle():
    """The SO(3) coefficient layout the library exports is the oracle's: the
    same count for every B and the same flat index for every (l, m, n)."""
    from oracle import so3 as oso3
    lib = _lib()
    lib.su2_so3_num_coeffs.argtypes = [ctypes.c_int32]
    lib.su2_so3_num_coeffs.restype = ctypes.c_int64
    lib.su2_so3_coeff_index.argtypes = [ctypes.c_int32] * 3
    lib.su2_so3_coeff_index.restype = ctypes.c_int64
    for B in range(1, 70):
        assert lib.su2_so3_num_coeffs(B) == oso3.num_coeffs(B)
    for l in range(0, 32):
        for m in range(-l, l + 1):
            for n in (-l, 0, l):
                assert lib.su2_so3_coeff_index(l, m, n) == oso3.coeff_index(l, m, n)
    assert lib.su2_so3_coeff_index(2, 3, 0) == -1
    assert lib.su2_so3_coeff_index(-1, 0, 0) == -1
    assert lib.su2_so3_num_coeffs(0) == -1


def test_valid_plan_without_device_reports_no_device():
    st, h = _create(8, 1, 1)
    if st == 0:                                # a GPU is visible: the plan is real
        assert _lib().su2_plan_destroy(h) == 0
    else:
        assert st == 5, f"expected SU2_ERR_NO_DEVICE, got {st}"
        assert not h.value


def test_calibration_arguments_validated_before_any_device_call():
    lib = _lib()
    vp = ctypes.c_void_p
    p16, p32, p8 = vp(1 << 20), vp((1 << 20) + (1 << 16)), vp((1 << 20) + 8)
    assert lib.su2_calib_copy(None, p16, 4096, None) == 1
    assert lib.su2_calib_copy(p16, p32, 0, None) == 1                 # empty
    assert lib.su2_calib_copy(p16, p32, 4100, None) == 1              # not a multiple of 16
    assert lib.su2_calib_copy(p8, p32, 4096, None) == 1               # misaligned
    assert lib.su2_calib_copy(p16, vp((1 << 20) + 4096), 8192, None) == 1   # overlapping ranges
    assert lib.su2_calib_fill(None, 4096, ctypes.c_float(1.0), None) == 1
    assert lib.su2_calib_fill(p16, -16, ctypes.c_float(1.0), None) == 1
    flops = ctypes.c_double()
    assert lib.su2_calib_mfma(3, 1, 1, p16, ctypes.byref(flops), None) == 1      # unknown kind
    assert lib.su2_calib_mfma(1, 0, 1, p16, ctypes.byref(flops), None) == 1      # no workgroups
    assert lib.su2_calib_mfma(1, 1, 0, p16, ctypes.byref(flops), None) == 1      # no iterations
    assert lib.su2_calib_mfma(1, 1, 1, None, ctypes.byref(flops), None) == 1
