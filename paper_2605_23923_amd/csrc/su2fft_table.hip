// Wigner-d tables for the beta contraction, generated on the GPU in FP64.
//
// For every retained pair (m, n) and node beta_k the table holds
// d^l_{nm}(beta_k) for l = l0 .. l0 + L - 1, l0 = max(|m|, |n|), from the
// three-term recurrence in l (Section 4: Lemma 4.3 is its m = n = 0 case; the
// section closes by extending the recurrence to the Jacobi / general (m, n)
// case, which is this one):
//
//   d^{l+1} = (l+1)(2l+1) / sqrt(((l+1)^2 - a^2)((l+1)^2 - b^2))
//             * [ (cos beta - a b / (l(l+1))) d^l - sqrt((l^2 - a^2)(l^2 - b^2)) / (l(2l+1)) d^{l-1} ]
//
// with (a, b) = (n, m), d^{l0 - 1} = 0, and the seed d^{l0} the single term of
// Wigner's sum that survives at l0 = max(|a|, |b|):
//   l0 =  a:  (-1)^{l0-b} sqrt(C(2 l0, l0+b)) cos^{l0+b}(beta/2) sin^{l0-b}(beta/2)
//   l0 = -a:              sqrt(C(2 l0, l0+b)) cos^{l0-b}(beta/2) sin^{l0+b}(beta/2)
//   l0 =  b:              sqrt(C(2 l0, l0+a)) cos^{l0+a}(beta/2) sin^{l0-a}(beta/2)
//   l0 = -b:  (-1)^{l0+a} sqrt(C(2 l0, l0+a)) cos^{l0-a}(beta/2) sin^{l0+a}(beta/2)
// The recurrence runs in FP64: seeds reach 1e-281 at B = 128 and the FP32
// recurrence loses about 10 digits there; reduced-precision tables are
// rounded from the FP64 values afterwards.
#include "su2fft_internal.h"

namespace su2 {

__device__ double binom_d(int n, int k) {
  if (k > n - k) k = n - k;
  double r = 1.0;
  for (int i = 1; i <= k; i++) r = r * (double)(n - k + i) / (double)i;
  return r;
}

// table layout: tile-major, d^{l0+i}(beta_k) at pairs[p].tab + k * lsum + coff + i
__global__ void dtable_kernel(int B, int N, int npairs, const PairInfo* __restrict__ pairs,
                              const double* __restrict__ beta, double* __restrict__ tab) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)npairs * N) return;
  const int pidx = (int)(gid / N), k = (int)(gid - (long long)pidx * N);
  const PairInfo pi = pairs[pidx];
  if (pi.L == 0) return;
  const int ta = pi.tn, tb = pi.tm;  // d^l_{a b} with a = n, b = m
  const int t0 = pi.tl0;
  const double bk = beta[k];
  const double ch = cos(0.5 * bk), sh = sin(0.5 * bk), x = cos(bk);
  // seed (all exponents are integers: t0 +- ta, t0 +- tb are even)
  int pc, ps, top, neg;
  wigner_seed_form(t0, ta, tb, &top, &pc, &ps, &neg);
  double dl = (neg ? -1.0 : 1.0) * sqrt(binom_d(t0, top)) * pow(ch, (double)pc) * pow(sh, (double)ps);
  double dlm1 = 0.0;
  double* out = tab + pi.tab + (long long)k * pi.lsum + pi.coff;
  out[0] = dl;
  const double a = 0.5 * ta, b = 0.5 * tb;
  for (int i = 1; i < pi.L; i++) {
    const double l = 0.5 * (t0 + 2 * (i - 1));  // current degree; produce l + 1
    const double lp1 = l + 1.0;
    const double pre = lp1 * (2.0 * l + 1.0) / sqrt((lp1 * lp1 - a * a) * (lp1 * lp1 - b * b));
    double term1, term2;
    if (l == 0.0) {
      term1 = x * dl;
      term2 = 0.0;
    } else {
      term1 = (x - a * b / (l * lp1)) * dl;
      term2 = sqrt((l * l - a * a) * (l * l - b * b)) / (l * (2.0 * l + 1.0)) * dlm1;
    }
    const double dn = pre * (term1 - term2);
    dlm1 = dl;
    dl = dn;
    out[i] = dl;
  }
}

__global__ void round_f32_kernel(long long n, const double* __restrict__ src, float* __restrict__ dst) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// round-to-nearest-even of a float to bfloat16 (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__global__ void split_bf16_kernel(long long n, const double* __restrict__ src, bf16x2_t* __restrict__ dst) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = src[i];
    const unsigned short hi = bf16_rne((float)v);
    const unsigned short lo = bf16_rne((float)(v - (double)bf16_to_f32(hi)));
    dst[i] = {hi, lo};
  }
}

hipError_t launch_dtable(int B, int N, int npairs, const PairInfo* pairs, const double* beta, double* tab64,
                         hipStream_t s) {
  const long long total = (long long)npairs * N;
  const int threads = 256;
  const long long blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(dtable_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, B, N, npairs, pairs, beta, tab64);
  return hipGetLastError();
}

hipError_t launch_round_table_f32(long long n, const double* src, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(round_f32_kernel, dim3(1024), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

// inverse layout (see PairInfo::itab): one workgroup per pair, values
// rounded from the FP64 table as the tile-major copies are
template <class T>
__global__ void inverse_table_kernel(int N, const PairInfo* __restrict__ pairs, const double* __restrict__ tab,
                                     T* __restrict__ dst) {
  const PairInfo pi = pairs[blockIdx.x];
  const int S = (pi.L + 3) / 4;
  const long long n = inverse_table_elems(pi.L, N);
  for (long long e = threadIdx.x; e < n; e += blockDim.x) {
    const int lane = (int)(e & 63);
    const long long g = e >> 6;
    const int kb = (int)(g / S), s = (int)(g - (long long)kb * S);
    const int k = 16 * kb + (lane & 15), l = 4 * s + (lane >> 4);
    const double v = (k < N && l < pi.L) ? tab[pi.tab + (long long)k * pi.lsum + pi.coff + l] : 0.0;
    dst[pi.itab + e] = (T)v;
  }
}

template <class T>
hipError_t launch_inverse_table(int N, int npairs, const PairInfo* pairs, const double* tab64, T* dst, hipStream_t s) {
  hipLaunchKernelGGL(inverse_table_kernel<T>, dim3(npairs), dim3(256), 0, s, N, pairs, tab64, dst);
  return hipGetLastError();
}
template hipError_t launch_inverse_table<float>(int, int, const PairInfo*, const double*, float*, hipStream_t);
template hipError_t launch_inverse_table<double>(int, int, const PairInfo*, const double*, double*, hipStream_t);

hipError_t launch_split_table_bf16(long long n, const double* src, bf16x2_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(split_bf16_kernel, dim3(1024), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

}  // namespace su2
