// Calibration kernels: what the device actually sustains, measured beside the
// transform so that its roofline fractions can be read against both the
// published and the achievable peaks.
//   copy  - streaming device-to-device copy, 16-byte non-temporal loads and stores
//   fill  - streaming write of a constant (HBM write rate alone)
//   mfma  - back-to-back matrix-core products with no memory traffic, in the
//           three precisions the contraction uses (FP64 16x16x4, FP32 16x16x4,
//           BF16 16x16x32 with FP32 accumulation)
#include "su2fft_plan.h"
#include "../../include/su2fft_calib.h"

namespace su2 {
namespace {

typedef float calib_f32x4 __attribute__((ext_vector_type(4)));
typedef double calib_f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 calib_bf16x8 __attribute__((ext_vector_type(8)));

constexpr int CALIB_NT = 256;      // threads per workgroup (4 waves)
constexpr int CALIB_UNROLL = 4;    // 16-byte elements in flight per thread and sweep
constexpr int CALIB_CHAINS = 4;    // independent accumulators per wave
constexpr int CALIB_STEPS = 16;    // products per chain and loop trip (amortises the loop's register moves)
constexpr int CALIB_MAX_BLOCKS = 8192;

// element i of the sweep starting at `base` is base + CALIB_NT * u; the sweep
// covers CALIB_NT * CALIB_UNROLL consecutive elements, the grid strides over sweeps
__global__ __launch_bounds__(CALIB_NT) void calib_copy_kernel(const calib_f32x4* __restrict__ src,
                                                              calib_f32x4* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * CALIB_NT * CALIB_UNROLL;
  for (long long base = (long long)blockIdx.x * CALIB_NT * CALIB_UNROLL + threadIdx.x; base < n; base += stride) {
    calib_f32x4 v[CALIB_UNROLL];
#pragma unroll
    for (int u = 0; u < CALIB_UNROLL; u++) {
      const long long i = base + (long long)CALIB_NT * u;
      if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < CALIB_UNROLL; u++) {
      const long long i = base + (long long)CALIB_NT * u;
      if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

__global__ __launch_bounds__(CALIB_NT) void calib_fill_kernel(calib_f32x4* __restrict__ dst, long long n, float value) {
  const calib_f32x4 v = {value, value, value, value};
  const long long stride = (long long)gridDim.x * CALIB_NT * CALIB_UNROLL;
  for (long long base = (long long)blockIdx.x * CALIB_NT * CALIB_UNROLL + threadIdx.x; base < n; base += stride) {
#pragma unroll
    for (int u = 0; u < CALIB_UNROLL; u++) {
      const long long i = base + (long long)CALIB_NT * u;
      if (i < n) __builtin_nontemporal_store(v, dst + i);
    }
  }
}

// Every lane feeds small integers (a = lane mod 3 + 1, b = lane mod 5 + 1) to
// every product, so short runs have exact results a test can check; each
// thread writes the sum of its accumulator elements to out[thread].
template <int KIND>
__global__ __launch_bounds__(CALIB_NT) void calib_mfma_kernel(int iters, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const float a = (float)(lane % 3 + 1), b = (float)(lane % 5 + 1);
  float r = 0.f;
  if constexpr (KIND == 0) {
    calib_f64x4 acc[CALIB_CHAINS];
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) acc[u] = calib_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; it++)
#pragma unroll
      for (int st = 0; st < CALIB_STEPS; st++)
#pragma unroll
        for (int u = 0; u < CALIB_CHAINS; u++)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) r += (float)(acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3]);
  } else if constexpr (KIND == 1) {
    calib_f32x4 acc[CALIB_CHAINS];
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) acc[u] = calib_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; it++)
#pragma unroll
      for (int st = 0; st < CALIB_STEPS; st++)
#pragma unroll
        for (int u = 0; u < CALIB_CHAINS; u++) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) r += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  } else {
    calib_bf16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; e++) {
      av[e] = (__bf16)a;
      bv[e] = (__bf16)b;
    }
    calib_f32x4 acc[CALIB_CHAINS];
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) acc[u] = calib_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; it++)
#pragma unroll
      for (int st = 0; st < CALIB_STEPS; st++)
#pragma unroll
        for (int u = 0; u < CALIB_CHAINS; u++)
          acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < CALIB_CHAINS; u++) r += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  }
  out[(size_t)blockIdx.x * CALIB_NT + threadIdx.x] = r;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int stream_blocks(long long n) {
  const long long per_block = (long long)CALIB_NT * CALIB_UNROLL;
  const long long need = (n + per_block - 1) / per_block;
  return (int)(need < CALIB_MAX_BLOCKS ? need : CALIB_MAX_BLOCKS);
}

su2_status_t launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SU2_OK : hip_fail(e);
}

}  // namespace
}  // namespace su2

using namespace su2;

extern "C" {

su2_status_t su2_calib_copy(const void* d_src, void* d_dst, int64_t bytes, hipStream_t stream) {
  if (!d_src || !d_dst || bytes <= 0 || bytes % 16 || !aligned16(d_src) || !aligned16(d_dst))
    return SU2_ERR_INVALID_VALUE;
  const uintptr_t s = (uintptr_t)d_src, d = (uintptr_t)d_dst;
  if (s < d + (uintptr_t)bytes && d < s + (uintptr_t)bytes) return SU2_ERR_INVALID_VALUE;  // overlap
  const long long n = bytes / 16;
  calib_copy_kernel<<<stream_blocks(n), CALIB_NT, 0, stream>>>(
      static_cast<const calib_f32x4*>(d_src), static_cast<calib_f32x4*>(d_dst), n);
  return launch_status();
}

su2_status_t su2_calib_fill(void* d_dst, int64_t bytes, float value, hipStream_t stream) {
  if (!d_dst || bytes <= 0 || bytes % 16 || !aligned16(d_dst)) return SU2_ERR_INVALID_VALUE;
  const long long n = bytes / 16;
  calib_fill_kernel<<<stream_blocks(n), CALIB_NT, 0, stream>>>(static_cast<calib_f32x4*>(d_dst), n, value);
  return launch_status();
}

su2_status_t su2_calib_mfma(int32_t kind, int32_t workgroups, int32_t iters, float* d_out, double* flops,
                            hipStream_t stream) {
  if (kind < 0 || kind > 2 || workgroups < 1 || workgroups > (1 << 20) || iters < 1 || iters > (1 << 24) ||
      !d_out || !aligned16(d_out))
    return SU2_ERR_INVALID_VALUE;
  const hipStream_t st = stream;
  if (kind == 0) calib_mfma_kernel<0><<<workgroups, CALIB_NT, 0, st>>>(iters, d_out);
  else if (kind == 1) calib_mfma_kernel<1><<<workgroups, CALIB_NT, 0, st>>>(iters, d_out);
  else calib_mfma_kernel<2><<<workgroups, CALIB_NT, 0, st>>>(iters, d_out);
  if (flops) {
    // 16 x 16 x K products: 2 * 16 * 16 * K flops per wave instruction
    const double per_inst = 2.0 * 16 * 16 * (kind == 2 ? 32 : 4);
    *flops = (double)workgroups * (CALIB_NT / 64) * (double)iters * CALIB_STEPS * CALIB_CHAINS * per_inst;
  }
  return launch_status();
}

}  // extern "C"
