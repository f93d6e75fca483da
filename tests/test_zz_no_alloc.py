"""su2_forward_noalloc through the C ABI: the forward transform with the ring
spectra in the library's static device scratch.  Its output equals
su2_forward's on the same plan and input bitwise (the same kernels run on the
same values; only the buffer between the two stages differs), on two calls in
a row, each with a smaller input than the one before, so that a call reads
only what it wrote over the previous call's leftovers.  Plans whose ring
spectra do not fit the scratch, and plans with a second workspace (B = 128 in
FP64), are refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2605_23923_amd as su2
import synth

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _spectra_bytes(B, batch, cb):
    P = 2 * B * B - 2 * B + 1
    return cb * 2 * B * batch * ((P + 15) // 16 * 16)


def _noalloc(plan, x, out):
    lib = su2._load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.su2_forward_noalloc(plan._handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   stream)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_forward_equals_forward_two_calls(dtype):
    npdt = np.complex64 if dtype == "c64" else np.complex128
    cb = 8 if dtype == "c64" else 16
    # calls in a row, each with a smaller input than the one before (over the
    # previous call's leftovers): c64 B = 128 batch 1 (66.6 MB of spectra),
    # then B = 64 (c64: batch 3, 24.8 MB; c128: batch 1), then B = 16 batch 2
    shapes = ([(128, 1)] if dtype == "c64" else []) + [(64, 3 if dtype == "c64" else 1), (16, 2)]
    for B, batch in shapes:
        assert _spectra_bytes(B, batch, cb) <= SCRATCH_BYTES
        print(f"noalloc forward {dtype} B={B} batch {batch}", flush=True)
        plan = su2.Plan(B, batch, dtype)
        x = torch.from_numpy(synth.samples_uniform(B, batch, seed=70 + B, dtype=npdt)).to("cuda")
        ref = plan.forward(x)
        out = torch.full(plan.coeff_shape, float("nan"), dtype=plan.torch_dtype, device="cuda")
        assert _noalloc(plan, x, out) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"B={B} {dtype}: noalloc forward differs from su2_forward"
        plan.close()


def test_noalloc_refuses_what_does_not_fit():
    # buffers of the plans' full sizes, so that nothing could be out of bounds
    # even if a refusal failed
    plan = su2.Plan(64, 9, "c64")                  # 74.5 MB of ring spectra
    assert _spectra_bytes(64, 9, 8) > SCRATCH_BYTES
    x = torch.zeros(plan.sample_shape, dtype=torch.complex64, device="cuda")
    out = torch.zeros(plan.coeff_shape, dtype=torch.complex64, device="cuda")
    assert _noalloc(plan, x, out) == 2
    plan.close()
    del x, out
    # B = 128 in FP64: 133 MB of spectra, and two-pass rings with a second
    # plan-owned buffer
    assert _spectra_bytes(128, 1, 16) > SCRATCH_BYTES
    plan = su2.Plan(128, 1, "c128")
    x = torch.zeros(plan.sample_shape, dtype=torch.complex128, device="cuda")
    out = torch.zeros(plan.coeff_shape, dtype=torch.complex128, device="cuda")
    assert _noalloc(plan, x, out) == 2
    plan.close()
    del x, out
    mixed = su2.MixedPlan([8, 16], "c64")
    x = torch.zeros(mixed.sample_shape, dtype=torch.complex64, device="cuda")
    out = torch.zeros(mixed.coeff_shape, dtype=torch.complex64, device="cuda")
    assert _noalloc(mixed, x, out) == 1
    mixed.close()
    lib = su2._load()
    assert lib.su2_forward_noalloc(None, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), None) == 1
    torch.cuda.synchronize()
