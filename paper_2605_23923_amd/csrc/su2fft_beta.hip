// Stage 2 of the separated transform: the contraction over the beta nodes
// (Section 4, the inner product <s, P^l_{nm}> of the core equation, taken for
// every (m, n) pair; cost model of Proposition 6.2 at depth k = 1, which
// Theorem 6.3 shows to be the optimum: one precomputed vector per (l, m, n)).
//
// For a pair (m, n) with L degrees l = l0 .. l0 + L - 1 and the batch as
// columns (re and im of every signal are separate real columns, the table is
// real):
//   forward:  fhat(l)_{mn}[b] = sum_k d^l_{nm}(beta_k) S_k(m, n)[b]          (M = L, K = N)
//   inverse:  S'_k(m, n)[b]   = sum_l s_l d^l_{nm}(beta_k) fhat(l)_{mn}[b]    (M = N, K = L)
// with s_l = 2l + 1 (synthesis) or 1 (adjoint, whose W_k is applied on the
// ring side).  The phases were applied on the ring side.
//
// Both are small dense GEMMs per pair, run on the matrix cores
// (V_MFMA_F32_16X16X4_F32 / V_MFMA_F64_16X16X4_F64; 16x4 by 4x16 blocks).
// Operand layout per 64-lane wave: A[i][kk] in lane i + 16 kk, B[kk][j] in
// lane j + 16 kk.  Accumulator element r of lane (j + 16 g) is D[4 g + r][j]
// for the FP32 instruction and D[g + 4 r][j] for the FP64 one (both measured).
#include "su2fft_internal.h"

namespace su2 {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T>
struct acc4;
template <>
struct acc4<float> {
  typedef floatx4 type;
};
template <>
struct acc4<double> {
  typedef doublex4 type;
};

__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16x16x4(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class T>
__device__ __forceinline__ int acc_row(int lane, int r);
template <>
__device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <>
__device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

__device__ __forceinline__ long long coeff_index(int tl, int tm, int tn) {
  return (long long)tl * (tl + 1) * (2 * tl + 1) / 6 + (long long)((tm + tl) / 2) * (tl + 1) + (tn + tl) / 2;
}

constexpr int BT = 16;        // signals per workgroup (32 real columns)
constexpr int KC = 16;        // beta nodes per LDS chunk (forward)
constexpr int CPITCH = 2 * BT + 4;

// Forward contraction.  Grid: (pair tiles, signal tiles).  Wave w owns pairs
// w, w+4, w+8, w+12 of the tile; the tile's S slab streams through LDS in
// chunks of KC nodes.
template <class T, int RTMAX>
__global__ __launch_bounds__(GEMM_THREADS) void beta_forward_kernel(const cpx<T>* __restrict__ S,
                                                                    cpx<T>* __restrict__ coeffs, BetaParams<T> p) {
  typedef typename acc4<T>::type accT;
  __shared__ T lds[PT][KC][CPITCH];
  const int tile = blockIdx.x;
  const int b0 = blockIdx.y * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int N = p.N;

  PairInfo pi[4];
#pragma unroll
  for (int i = 0; i < 4; i++) pi[i] = p.pairs[tile * PT + wave + 4 * i];

  accT acc[4][RTMAX][2];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++)
#pragma unroll
      for (int ct = 0; ct < 2; ct++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[i][rt][ct][r] = T(0);

  const int lrow = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < N; k0 += KC) {
    __syncthreads();
    for (int e = threadIdx.x; e < KC * BT * PT; e += GEMM_THREADS) {
      const int pp = e % PT, bb = (e / PT) % BT, kk = e / (PT * BT);
      const int k = k0 + kk;
      cpx<T> v = {T(0), T(0)};
      if (k < N && bb < nb) v = S[(((size_t)tile * N + k) * p.batch + b0 + bb) * PT + pp];
      lds[pp][kk][2 * bb] = v.re;
      lds[pp][kk][2 * bb + 1] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int L = pi[i].L;
      if (L == 0) continue;
      const int pp = wave + 4 * i;
      const T* tab = p.tab + pi[i].tab;
      for (int ks = 0; ks < KC; ks += 4) {
        const int k = k0 + ks + lk;
        T bop0 = lds[pp][ks + lk][lrow];
        T bop1 = lds[pp][ks + lk][16 + lrow];
#pragma unroll
        for (int rt = 0; rt < RTMAX; rt++) {
          if (rt * 16 < L) {
            const int l = rt * 16 + lrow;
            T a = (l < L && k < N) ? tab[(size_t)k * L + l] : T(0);
            acc[i][rt][0] = mfma16x16x4(a, bop0, acc[i][rt][0]);
            acc[i][rt][1] = mfma16x16x4(a, bop1, acc[i][rt][1]);
          }
        }
      }
    }
  }
  // epilogue: scatter into the 2l-major coefficient layout
  T* out = reinterpret_cast<T*>(coeffs);
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int L = pi[i].L;
    if (L == 0) continue;
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++) {
      if (rt * 16 >= L) continue;
#pragma unroll
      for (int ct = 0; ct < 2; ct++) {
        const int c = ct * 16 + lrow;
        const int bb = c >> 1, reim = c & 1;
        if (bb >= nb) continue;
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int l = rt * 16 + acc_row<T>(lane, r);
          if (l < L) {
            const long long idx = coeff_index(pi[i].tl0 + 2 * l, pi[i].tm, pi[i].tn);
            out[(((size_t)(b0 + bb)) * p.ncoef + idx) * 2 + reim] = acc[i][rt][ct][r];
          }
        }
      }
    }
  }
}

// Inverse contraction.  Wave w handles pairs w, w+4, ... of the tile one at a
// time; the N output rows are produced in groups of 4 row blocks (64 nodes).
template <class T>
__global__ __launch_bounds__(GEMM_THREADS) void beta_inverse_kernel(const cpx<T>* __restrict__ coeffs,
                                                                    cpx<T>* __restrict__ S, BetaParams<T> p) {
  typedef typename acc4<T>::type accT;
  const int tile = blockIdx.x;
  const int b0 = blockIdx.y * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lrow = lane & 15, lk = lane >> 4;
  const int N = p.N;
  const T* cin = reinterpret_cast<const T*>(coeffs);
  T* sout = reinterpret_cast<T*>(S);
  for (int i = 0; i < 4; i++) {
    const int pp = wave + 4 * i;
    const PairInfo pi = p.pairs[tile * PT + pp];
    const int L = pi.L;
    if (L == 0) continue;
    const T* tab = p.tab + pi.tab;
    // B operand column of this lane: signal bb, re/im
    const int c0 = lrow;  // columns c0 and 16 + c0
    for (int kt0 = 0; kt0 < N; kt0 += 64) {
      accT acc[4][2];
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int ct = 0; ct < 2; ct++)
#pragma unroll
          for (int r = 0; r < 4; r++) acc[t][ct][r] = T(0);
      for (int l0 = 0; l0 < L; l0 += 4) {
        const int l = l0 + lk;
        T bop[2];
#pragma unroll
        for (int ct = 0; ct < 2; ct++) {
          const int c = ct * 16 + c0;
          const int bb = c >> 1, reim = c & 1;
          T v = T(0);
          if (l < L && bb < nb) {
            const int tl = pi.tl0 + 2 * l;
            const long long idx = coeff_index(tl, pi.tm, pi.tn);
            const T s = p.scale_mode == 0 ? T(tl + 1) : T(1);
            v = s * cin[(((size_t)(b0 + bb)) * p.ncoef + idx) * 2 + reim];
          }
          bop[ct] = v;
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const int k = kt0 + t * 16 + lrow;
          T a = (l < L && k < N) ? tab[(size_t)k * L + l] : T(0);
          acc[t][0] = mfma16x16x4(a, bop[0], acc[t][0]);
          acc[t][1] = mfma16x16x4(a, bop[1], acc[t][1]);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; t++)
#pragma unroll
        for (int ct = 0; ct < 2; ct++) {
          const int c = ct * 16 + lrow;
          const int bb = c >> 1, reim = c & 1;
          if (bb >= nb) continue;
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int k = kt0 + t * 16 + acc_row<T>(lane, r);
            if (k < N) sout[((((size_t)tile * N + k) * p.batch + b0 + bb) * PT + pp) * 2 + reim] = acc[t][ct][r];
          }
        }
    }
  }
}

template <class T>
hipError_t launch_beta_forward(const BetaParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, hipStream_t s) {
  dim3 grid(p.ntiles, (p.batch + BT - 1) / BT);
  const int lmax = (p.B + 1) / 2;
  if (lmax <= 16)
    hipLaunchKernelGGL((beta_forward_kernel<T, 1>), grid, dim3(GEMM_THREADS), 0, s, S, coeffs, p);
  else if (lmax <= 32)
    hipLaunchKernelGGL((beta_forward_kernel<T, 2>), grid, dim3(GEMM_THREADS), 0, s, S, coeffs, p);
  else
    hipLaunchKernelGGL((beta_forward_kernel<T, 4>), grid, dim3(GEMM_THREADS), 0, s, S, coeffs, p);
  return hipGetLastError();
}

template <class T>
hipError_t launch_beta_inverse(const BetaParams<T>& p, const cpx<T>* coeffs, cpx<T>* S, hipStream_t s) {
  dim3 grid(p.ntiles, (p.batch + BT - 1) / BT);
  hipLaunchKernelGGL(beta_inverse_kernel<T>, grid, dim3(GEMM_THREADS), 0, s, coeffs, S, p);
  return hipGetLastError();
}

template hipError_t launch_beta_forward<float>(const BetaParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_beta_forward<double>(const BetaParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);
template hipError_t launch_beta_inverse<float>(const BetaParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_beta_inverse<double>(const BetaParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);

}  // namespace su2
