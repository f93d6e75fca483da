"""su2fft: the separated Fourier transform on SU(2) on MI355X (gfx950).

Thin Python binding of the C ABI in ``include/su2fft.h`` (ctypes).  It only
marshals arguments: every step of the transform runs in the HIP library
``libsu2fft.so`` built next to this file.  PyTorch provides device memory and
the current stream; there is no CPU or PyTorch fallback -- a missing or
unloadable library raises.

    plan = Plan(B=64, batch=32, dtype="c64")
    coeffs = plan.forward(samples)        # (batch, C(B)) complex, 2l-major blocks
    samples = plan.inverse(coeffs)        # (batch, N, N, N) complex, [k][j][l]
    grad = plan.adjoint(coeffs)           # conjugate transpose of forward
    coeffs = SU2Transform.apply(samples, plan)   # differentiable forward
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["Plan", "MixedPlan", "SU2Transform", "SU2Error", "num_coeffs", "num_samples", "coeff_index",
           "so3_num_coeffs", "so3_coeff_index", "grid", "library_path", "C128", "C64", "C64_BF16X3"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsu2fft.so")

C128, C64, C64_BF16X3 = 0, 1, 2
_DTYPES = {"c128": C128, "c64": C64, "c64_bf16x3": C64_BF16X3, C128: C128, C64: C64, C64_BF16X3: C64_BF16X3}
_TORCH_DTYPE = {C128: torch.complex128, C64: torch.complex64, C64_BF16X3: torch.complex64}

_STATUS = {0: "SU2_OK", 1: "SU2_ERR_INVALID_VALUE", 2: "SU2_ERR_UNSUPPORTED", 3: "SU2_ERR_OUT_OF_MEMORY",
           4: "SU2_ERR_HIP", 5: "SU2_ERR_NO_DEVICE"}

_lib = None


class SU2Error(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = f"{where}: {_STATUS.get(status, status)}"
        if status == 4 and _lib is not None:
            msg += f" (hip error {_lib.su2_last_hip_error()})"
        super().__init__(msg)


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"su2fft HIP library not built: {_LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python -m paper_2605_23923_amd._build)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    dp = ctypes.POINTER(ctypes.c_double)
    lib.su2_plan_create.argtypes = [i32, i32, i32, ctypes.POINTER(vp)]
    lib.su2_plan_create.restype = i32
    lib.su2_plan_create_ex.argtypes = [i32, i32, i32, ctypes.c_uint32, ctypes.POINTER(vp)]
    lib.su2_plan_create_ex.restype = i32
    lib.su2_plan_create_mixed.argtypes = [ctypes.POINTER(i32), i32, i32, ctypes.POINTER(vp)]
    lib.su2_plan_create_mixed.restype = i32
    lib.su2_plan_create_mixed_ex.argtypes = [ctypes.POINTER(i32), i32, i32, ctypes.c_uint32, ctypes.POINTER(vp)]
    lib.su2_plan_create_mixed_ex.restype = i32
    lib.su2_plan_destroy.argtypes = [vp]
    lib.su2_plan_destroy.restype = i32
    for name in ("su2_forward", "su2_inverse", "su2_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp]
        f.restype = i32
    lib.su2_forward_noalloc.argtypes = [vp, vp, vp, vp]
    lib.su2_forward_noalloc.restype = i32
    lib.su2_run_stage.argtypes = [vp, i32, vp, vp, vp]
    lib.su2_beta_forward_shifted.argtypes = [vp, i32, i32, vp, vp]
    lib.su2_beta_forward_shifted.restype = i32
    lib.su2_run_stage.restype = i32
    lib.su2_num_samples.argtypes = [i32]
    lib.su2_num_samples.restype = i64
    lib.su2_num_coeffs.argtypes = [i32]
    lib.su2_num_coeffs.restype = i64
    lib.su2_coeff_index.argtypes = [i32, i32, i32]
    lib.su2_coeff_index.restype = i64
    lib.su2_so3_num_coeffs.argtypes = [i32]
    lib.su2_so3_num_coeffs.restype = i64
    lib.su2_so3_coeff_index.argtypes = [i32, i32, i32]
    lib.su2_so3_coeff_index.restype = i64
    lib.su2_grid.argtypes = [i32, dp, dp, dp, dp]
    lib.su2_grid.restype = i32
    lib.su2_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i64)]
    lib.su2_plan_info.restype = i32
    lib.su2_plan_dtable.argtypes = [vp, i32, i32, dp, ctypes.POINTER(i32)]
    lib.su2_plan_dtable.restype = i32
    lib.su2_plan_tuning.argtypes = [vp, ctypes.POINTER(i32)]
    lib.su2_plan_tuning.restype = i32
    lib.su2_plan_tile_shapes.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    lib.su2_plan_tile_shapes.restype = i32
    lib.su2_status_string.argtypes = [i32]
    lib.su2_status_string.restype = ctypes.c_char_p
    lib.su2_last_hip_error.argtypes = []
    lib.su2_last_hip_error.restype = i32
    lib.su2_calib_copy.argtypes = [vp, vp, i64, vp]
    lib.su2_calib_copy.restype = i32
    lib.su2_calib_fill.argtypes = [vp, i64, ctypes.c_float, vp]
    lib.su2_calib_fill.restype = i32
    lib.su2_calib_mfma.argtypes = [i32, i32, i32, vp, dp, vp]
    lib.su2_calib_mfma.restype = i32
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise SU2Error(status, where)


def num_samples(B: int) -> int:
    return int(_load().su2_num_samples(B))


def num_coeffs(B: int) -> int:
    return int(_load().su2_num_coeffs(B))


def coeff_index(two_l: int, two_m: int, two_n: int) -> int:
    return int(_load().su2_coeff_index(two_l, two_m, two_n))


def so3_num_coeffs(B: int) -> int:
    """Coefficients per signal of an SO(3) plan: integer l with 2l < B."""
    return int(_load().su2_so3_num_coeffs(B))


def so3_coeff_index(l: int, m: int, n: int) -> int:
    """Flat index of fhat(l)_{mn} in an SO(3) plan's coefficient vector (plain integers)."""
    return int(_load().su2_so3_coeff_index(l, m, n))


def grid(B: int):
    """(alpha, beta, gamma, W) as lists of 2B floats (host computation)."""
    N = 2 * B
    arrs = [(ctypes.c_double * N)() for _ in range(4)]
    _check(_load().su2_grid(B, *[ctypes.cast(a, ctypes.POINTER(ctypes.c_double)) for a in arrs]), "su2_grid")
    return tuple(list(a) for a in arrs)


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _device_buffer(t, what: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{what}: a contiguous device tensor is required")
    return ctypes.c_void_p(t.data_ptr())


def calib_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Streaming copy of src's bytes into dst on the current stream (calibration
    kernel: 2 x nbytes of HBM traffic)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("calib_copy: dst is smaller than src")
    _check(_load().su2_calib_copy(_device_buffer(src, "calib_copy"), _device_buffer(dst, "calib_copy"), n,
                                  _stream_handle(src.device)), "su2_calib_copy")


def calib_fill(dst: torch.Tensor, value: float) -> None:
    """Streaming write of `value` to every float of dst on the current stream."""
    _check(_load().su2_calib_fill(_device_buffer(dst, "calib_fill"), dst.numel() * dst.element_size(),
                                  float(value), _stream_handle(dst.device)), "su2_calib_fill")


CALIB_MFMA_KINDS = {"fp64": 0, "fp32": 1, "bf16": 2}


def calib_mfma(kind: str, workgroups: int, iters: int, out: torch.Tensor) -> float:
    """Back-to-back matrix-core products (kind 'fp64', 'fp32' or 'bf16') on the
    current stream; out holds workgroups x 256 float32.  Returns the flops the
    launch executes."""
    if out.dtype != torch.float32 or out.numel() < workgroups * 256:
        raise ValueError("calib_mfma: out must hold workgroups x 256 float32 values")
    flops = ctypes.c_double(0.0)
    _check(_load().su2_calib_mfma(CALIB_MFMA_KINDS[kind], int(workgroups), int(iters), _device_buffer(out, "calib_mfma"),
                                  ctypes.byref(flops), _stream_handle(out.device)), "su2_calib_mfma")
    return flops.value


class _PlanBase:
    _handle = None

    def _check_tensor(self, t: torch.Tensor, numel: int, what: str, dtype=None):
        dtype = self.torch_dtype if dtype is None else dtype
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{what} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")
        if t.device != self.device:
            raise ValueError(f"{what} is on {t.device}, plan is on {self.device}")

    def _call(self, fn: str, src: torch.Tensor, dst: torch.Tensor):
        status = getattr(_load(), fn)(self._handle, ctypes.c_void_p(src.data_ptr()),
                                      ctypes.c_void_p(dst.data_ptr()), _stream_handle(self.device))
        _check(status, fn)

    @property
    def sample_dtype(self):
        """torch dtype of the samples: complex, or real for real-signal plans."""
        return getattr(self, "_sample_dtype", self.torch_dtype)

    def forward(self, samples: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(samples, self.total_samples, "samples", self.sample_dtype)
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.torch_dtype, device=self.device)
        self._check_tensor(out, self.total_coeffs, "out")
        self._call("su2_forward", samples, out)
        return out

    def forward_noalloc(self, samples: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """su2_forward_noalloc: the forward transform with the ring spectra in
        the library's static device scratch; `out` must be given (the call
        allocates nothing)."""
        self._check_tensor(samples, self.total_samples, "samples", self.sample_dtype)
        self._check_tensor(out, self.total_coeffs, "out")
        self._call("su2_forward_noalloc", samples, out)
        return out

    def inverse(self, coeffs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(coeffs, self.total_coeffs, "coeffs")
        if out is None:
            out = torch.empty(self.sample_shape, dtype=self.sample_dtype, device=self.device)
        self._check_tensor(out, self.total_samples, "out", self.sample_dtype)
        self._call("su2_inverse", coeffs, out)
        return out

    def adjoint(self, coeffs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(coeffs, self.total_coeffs, "coeffs")
        if out is None:
            out = torch.empty(self.sample_shape, dtype=self.sample_dtype, device=self.device)
        self._check_tensor(out, self.total_samples, "out", self.sample_dtype)
        self._call("su2_adjoint", coeffs, out)
        return out

    STAGES = {"ring_forward": 0, "beta_forward": 1, "beta_inverse": 2, "ring_inverse": 3,
              "beta_adjoint": 4, "ring_adjoint": 5}

    def run_stage(self, stage: str, inp: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """Launch one kernel stage (see su2_run_stage); the ring spectra stay in
        the plan workspace between stages."""
        code = self.STAGES[stage]
        # the tensor each stage reads or writes is checked like forward/inverse's
        # arguments: a wrong size or dtype would otherwise reach the kernels
        needs = {"ring_forward": ("inp", self.total_samples, self.sample_dtype),
                 "beta_forward": ("out", self.total_coeffs, self.torch_dtype),
                 "beta_inverse": ("inp", self.total_coeffs, self.torch_dtype),
                 "beta_adjoint": ("inp", self.total_coeffs, self.torch_dtype),
                 "ring_inverse": ("out", self.total_samples, self.sample_dtype),
                 "ring_adjoint": ("out", self.total_samples, self.sample_dtype)}[stage]
        t = inp if needs[0] == "inp" else out
        if t is None:
            raise ValueError(f"run_stage({stage!r}) needs the {needs[0]} tensor")
        self._check_tensor(t, needs[1], f"run_stage({stage!r}) {needs[0]}", needs[2])
        pin = ctypes.c_void_p(inp.data_ptr()) if inp is not None else ctypes.c_void_p()
        pout = ctypes.c_void_p(out.data_ptr()) if out is not None else ctypes.c_void_p()
        _check(_load().su2_run_stage(self._handle, code, pin, pout, _stream_handle(self.device)), "su2_run_stage")

    def beta_forward_shifted(self, out: torch.Tensor | None = None, depth: int = 1, block: int = 4) -> torch.Tensor:
        """The forward contraction stage in the shifted-recurrence
        (divide-and-conquer) form, from the ring spectra a preceding
        run_stage("ring_forward") left in the plan (see su2_beta_forward_shifted)."""
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.torch_dtype, device=self.device)
        self._check_tensor(out, self.total_coeffs, "out")
        _check(_load().su2_beta_forward_shifted(self._handle, int(depth), int(block), ctypes.c_void_p(out.data_ptr()),
                                                _stream_handle(self.device)), "su2_beta_forward_shifted")
        return out

    def dtable(self, two_m: int, two_n: int):
        """The plan's FP64 Wigner-d table of pair (m, n) as a list of rows
        [k][i] = d^{l0+i}_{nm}(beta_k) (diagnostic, synchronous)."""
        lib = _load()
        L = ctypes.c_int32(0)
        _check(lib.su2_plan_dtable(self._handle, two_m, two_n, None, ctypes.byref(L)), "su2_plan_dtable")
        n = self.N * L.value
        buf = (ctypes.c_double * max(n, 1))()
        with torch.cuda.device(self.device):
            _check(lib.su2_plan_dtable(self._handle, two_m, two_n,
                                       ctypes.cast(buf, ctypes.POINTER(ctypes.c_double)), None), "su2_plan_dtable")
        return [list(buf[k * L.value:(k + 1) * L.value]) for k in range(self.N)]

    def device_bytes(self) -> int:
        n = ctypes.c_int64(0)
        _check(_load().su2_plan_info(self._handle, None, None, None, ctypes.byref(n)), "su2_plan_info")
        return int(n.value)

    def close(self):
        if self._handle is not None and _lib is not None:
            with torch.cuda.device(self.device):
                _lib.su2_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PLAN_TABLES_ON_THE_FLY = 1  # SU2_PLAN_TABLES_ON_THE_FLY
PLAN_REAL_SIGNALS = 2       # SU2_PLAN_REAL_SIGNALS
PLAN_SO3 = 4                # SU2_PLAN_SO3


class Plan(_PlanBase):
    """Transform plan for `batch` signals of bandlimit B (2l < B).

    tables: "stored" keeps the Wigner-d table in device memory (generated once
    at plan creation); "on_the_fly" generates the values inside the
    contraction kernels on every call (c128 and c64 only).

    real: real-signal plan (any mode and bandlimit, stored tables): samples
    are float64 / float32 tensors; forward returns every coefficient, inverse
    and adjoint return the real part of the complex result (see
    SU2_PLAN_REAL_SIGNALS).

    group: "su2" (default), or "so3" for the transform on SO(3) (any mode and
    bandlimit, stored tables, complex samples): integer l with 2l < B on the
    same N = 2B grid with gamma over [-pi, pi) (see SU2_PLAN_SO3);
    coefficients indexed by so3_coeff_index."""

    def __init__(self, B: int, batch: int = 1, dtype="c128", device=None, tables="stored", real=False,
                 group="su2"):
        if tables not in ("stored", "on_the_fly"):
            raise ValueError(f"tables must be 'stored' or 'on_the_fly', got {tables!r}")
        if group not in ("su2", "so3"):
            raise ValueError(f"group must be 'su2' or 'so3', got {group!r}")
        flags = ((PLAN_TABLES_ON_THE_FLY if tables == "on_the_fly" else 0) | (PLAN_REAL_SIGNALS if real else 0) |
                 (PLAN_SO3 if group == "so3" else 0))
        self.tables = tables
        self.real = bool(real)
        self.group = group
        lib = _load()
        self.B, self.batch = int(B), int(batch)
        self.dtype = _DTYPES[dtype]
        self.torch_dtype = _TORCH_DTYPE[self.dtype]
        if self.real:
            self._sample_dtype = torch.float64 if self.torch_dtype == torch.complex128 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.N = 2 * self.B
        if self.B < 1:
            self.ncoef = 0
        else:
            self.ncoef = so3_num_coeffs(self.B) if group == "so3" else num_coeffs(self.B)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.su2_plan_create_ex(self.B, self.batch, self.dtype, flags, ctypes.byref(h)),
                   "su2_plan_create_ex")
        self._handle = h
        self.sample_shape = (self.batch, self.N, self.N, self.N)
        self.coeff_shape = (self.batch, self.ncoef)
        self.total_samples = self.batch * self.N ** 3
        self.total_coeffs = self.batch * self.ncoef


class MixedPlan(_PlanBase):
    """Plan for a batch of signals with individual bandlimits, concatenated
    in order (flat sample and coefficient buffers).  real and group as for
    Plan (see su2_plan_create_mixed_ex)."""

    def __init__(self, Bs, dtype="c64", device=None, real=False, group="su2"):
        if group not in ("su2", "so3"):
            raise ValueError(f"group must be 'su2' or 'so3', got {group!r}")
        lib = _load()
        self.Bs = [int(b) for b in Bs]
        self.batch = len(self.Bs)
        self.dtype = _DTYPES[dtype]
        self.torch_dtype = _TORCH_DTYPE[self.dtype]
        self.real = bool(real)
        self.group = group
        if self.real:
            self._sample_dtype = torch.float64 if self.torch_dtype == torch.complex128 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        flags = (PLAN_REAL_SIGNALS if real else 0) | (PLAN_SO3 if group == "so3" else 0)
        arr = (ctypes.c_int32 * self.batch)(*self.Bs)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.su2_plan_create_mixed_ex(arr, self.batch, self.dtype, flags, ctypes.byref(h)),
                   "su2_plan_create_mixed_ex")
        self._handle = h
        self.sample_offsets = [0]
        self.coeff_offsets = [0]
        ncoef = so3_num_coeffs if group == "so3" else num_coeffs
        for b in self.Bs:
            self.sample_offsets.append(self.sample_offsets[-1] + num_samples(b))
            self.coeff_offsets.append(self.coeff_offsets[-1] + ncoef(b))
        self.total_samples = self.sample_offsets[-1]
        self.total_coeffs = self.coeff_offsets[-1]
        self.sample_shape = (self.total_samples,)
        self.coeff_shape = (self.total_coeffs,)

    def tuning(self):
        """Workgroups per CU the autotuner chose for the four work-list kernels
        (0: one workgroup per task)."""
        arr = (ctypes.c_int32 * 4)()
        _check(_load().su2_plan_tuning(self._handle, arr), "su2_plan_tuning")
        return list(arr)

    def tile_shapes(self):
        """Contraction tile shapes the autotuner chose, per bandlimit group in
        increasing B: (B, forward signals per tile, inverse signals per tile,
        forward nodes per chunk)."""
        lib = _load()
        n = ctypes.c_int32()
        _check(lib.su2_plan_tile_shapes(self._handle, None, 0, ctypes.byref(n)), "su2_plan_tile_shapes")
        arr = (ctypes.c_int32 * (4 * n.value))()
        _check(lib.su2_plan_tile_shapes(self._handle, arr, 4 * n.value, ctypes.byref(n)), "su2_plan_tile_shapes")
        return [tuple(arr[4 * g:4 * g + 4]) for g in range(n.value)]


class SU2Transform(torch.autograd.Function):
    """Differentiable forward transform.  The backward pass is the adjoint
    kernel chain (PyTorch's complex convention: grad_in = F^H grad_out)."""

    @staticmethod
    def forward(ctx, samples: torch.Tensor, plan: _PlanBase):
        ctx.plan = plan
        return plan.forward(samples.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = ctx.plan.adjoint(grad_out.contiguous())
        return g, None
