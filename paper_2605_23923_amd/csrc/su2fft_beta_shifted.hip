// Forward beta contraction in the divide-and-conquer form of Section 4
// (the shifted three-term recurrence: the matrix-recurrence and
// composition-rule propositions and the divide-and-conquer theorem, with the
// four-term worked example as depth 2), generalised from the Legendre case to
// the Wigner-d recurrence of every (m, n) pair.
//
// For a pair with degrees l0 .. l0 + L - 1 and base level Lb = l0 + 1, the
// stored pointwise products of the method are s^{Lb} = S d^{l0+1} and
// s^{Lb-1} = S d^{l0} (S the ring spectrum of the pair over the nodes), and
//   fhat(l0)          = <s^{Lb-1}, 1>
//   fhat(l0 + 1 + r)  = <s^{Lb}, A_r^{Lb}> + <s^{Lb-1}, B_r^{Lb}>                       (depth 1)
//                     = <u, A_{n2}^{Lb+n1}> + <v, B_{n2}^{Lb+n1}>,  r = n1 + n2,          (depth 2)
//                       u = A_{n1}^{Lb} s^{Lb} + B_{n1}^{Lb} s^{Lb-1},
//                       v = A_{n1-1}^{Lb} s^{Lb} + B_{n1-1}^{Lb} s^{Lb-1},
// the depth-2 line being the worked example's four terms grouped by bilinearity
// (n1 runs over multiples of BLK, n2 over 0 .. BLK-1).  A and B follow the
// one-step matrix [[a (x - b), -c], [1, 0]] of the recurrence from A_0 = 1,
// B_0 = 0, A_{-1} = 0, B_{-1} = 1.
//
// Everything here is evaluated in FP64, whatever the plan's type: near the
// poles s^{Lb} can be far below the FP32 range while A_r^{Lb} is large, so the
// method's stored products need the FP64 exponent range.  One thread per
// (pair, signal) walks the nodes and keeps its L accumulators in registers;
// the shifted polynomials are generated per node from the plan's per-pair
// recurrence coefficients (the same scalars as the on-the-fly tables).
#include "su2fft_internal.h"

namespace su2 {

constexpr int SH_THREADS = 512;  // 16 pairs x 32 signals
constexpr int SH_BT = SH_THREADS / PT;

template <class T, int LMAX, int DEPTH, int BLK>
__global__ __launch_bounds__(SH_THREADS) void beta_forward_shifted_kernel(const cpx<T>* __restrict__ S,
                                                                          cpx<T>* __restrict__ coeffs,
                                                                          OtfParams<T> op) {
  const BetaParams<T>& p = op.b;
  const int tile = blockIdx.x;
  const int t = threadIdx.x;
  const int i = t / SH_BT, b = blockIdx.y * SH_BT + (t % SH_BT);
  const int pidx = tile * PT + i;
  const PairInfo q = p.pairs[pidx];
  const int N = p.N, L = q.L;
  if (L == 0 || b >= p.batch) return;  // no barriers below
  const double* rc = op.rcoef + 3 * (q.tab / N + q.coff);  // step producing degree index j: rc[3j .. 3j+2]
  double accr[LMAX], acci[LMAX];
#pragma unroll
  for (int l = 0; l < LMAX; l++) accr[l] = acci[l] = 0.0;

  for (int k = 0; k < N; k++) {
    const cpx<T> sv = S[(((size_t)tile * N + k) * p.batch + b) * PT + i];
    const double sr = (double)sv.re, si = (double)sv.im;
    const double x = op.xk[k];
    const double d0 = otf_seed(op, q, pidx, k);
    accr[0] += d0 * sr;
    acci[0] += d0 * si;
    if (L == 1) continue;
    const double d1 = (rc[3] * x - rc[4]) * d0;
    // stored products s^{Lb} = S d^{l0+1}, s^{Lb-1} = S d^{l0}
    const double sLr = d1 * sr, sLi = d1 * si, sMr = d0 * sr, sMi = d0 * si;
    if constexpr (DEPTH == 1) {
      double A = 1.0, Ap = 0.0, Bv = 0.0, Bp = 1.0;
#pragma unroll
      for (int r = 0; r + 1 < LMAX; r++) {
        if (r + 1 < L) {
          accr[r + 1] += A * sLr + Bv * sMr;
          acci[r + 1] += A * sLi + Bv * sMi;
          const double tt = rc[3 * (r + 2)] * x - rc[3 * (r + 2) + 1], c = rc[3 * (r + 2) + 2];
          const double An = tt * A - c * Ap, Bn = tt * Bv - c * Bp;
          Ap = A; A = An;
          Bp = Bv; Bv = Bn;
        }
      }
    } else {
      double Ac = 1.0, Acp = 0.0, Bc = 0.0, Bcp = 1.0;  // coarse shift n1 from level Lb
#pragma unroll
      for (int n1 = 0; n1 + 1 < LMAX; n1 += BLK) {
        if (n1 + 1 < L) {
          const double ur = Ac * sLr + Bc * sMr, ui = Ac * sLi + Bc * sMi;
          const double vr = Acp * sLr + Bcp * sMr, vi = Acp * sLi + Bcp * sMi;
          double Af = 1.0, Afp = 0.0, Bf = 0.0, Bfp = 1.0;  // fine shift n2 from level Lb + n1
#pragma unroll
          for (int n2 = 0; n2 < BLK; n2++) {
            const int r = n1 + n2;
            if (r + 1 < LMAX && r + 1 < L) {
              accr[r + 1] += Af * ur + Bf * vr;
              acci[r + 1] += Af * ui + Bf * vi;
              const double tt = rc[3 * (r + 2)] * x - rc[3 * (r + 2) + 1], c = rc[3 * (r + 2) + 2];
              const double An = tt * Af - c * Afp, Bn = tt * Bf - c * Bfp;
              Afp = Af; Af = An;
              Bfp = Bf; Bf = Bn;
            }
          }
          // advance the coarse shift by BLK steps
#pragma unroll
          for (int j = 0; j < BLK; j++) {
            const int r = n1 + j;
            if (r + 1 < LMAX && r + 1 < L) {
              const double tt = rc[3 * (r + 2)] * x - rc[3 * (r + 2) + 1], c = rc[3 * (r + 2) + 2];
              const double An = tt * Ac - c * Acp, Bn = tt * Bc - c * Bcp;
              Acp = Ac; Ac = An;
              Bcp = Bc; Bc = Bn;
            }
          }
        }
      }
    }
  }
  T* out = reinterpret_cast<T*>(coeffs);
  const size_t base = coef_offset(p.coff, b, p.ncoef);
#pragma unroll
  for (int l = 0; l < LMAX; l++) {
    if (l < L) {
      const long long idx = coef_index_of(0, q.tl0 + 2 * l, q.tm, q.tn);
      out[(base + idx) * 2] = (T)accr[l];
      out[(base + idx) * 2 + 1] = (T)acci[l];
    }
  }
}

template <class T, int LMAX>
static hipError_t launch_shifted_l(const OtfParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, int depth, int blk,
                                   hipStream_t s) {
  const dim3 grid(p.b.ntiles, (p.b.batch + SH_BT - 1) / SH_BT);
  if (depth == 1)
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 1, 1>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  else if (blk == 2)
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 2, 2>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  else if (blk == 4)
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 2, 4>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  else
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 2, 8>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  return hipGetLastError();
}

bool shifted_supported(int B) { return (B + 1) / 2 <= 32; }

template <class T>
hipError_t launch_beta_forward_shifted(const OtfParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, int depth, int blk,
                                       hipStream_t s) {
  const int lmax = (p.b.B + 1) / 2;
  if ((depth != 1 && depth != 2) || (depth == 2 && blk != 2 && blk != 4 && blk != 8) || lmax > 32)
    return hipErrorInvalidValue;
  if (lmax <= 8) return launch_shifted_l<T, 8>(p, S, coeffs, depth, blk, s);
  if (lmax <= 16) return launch_shifted_l<T, 16>(p, S, coeffs, depth, blk, s);
  return launch_shifted_l<T, 32>(p, S, coeffs, depth, blk, s);
}

template hipError_t launch_beta_forward_shifted<float>(const OtfParams<float>&, const cpx<float>*, cpx<float>*, int,
                                                       int, hipStream_t);
template hipError_t launch_beta_forward_shifted<double>(const OtfParams<double>&, const cpx<double>*, cpx<double>*,
                                                        int, int, hipStream_t);

}  // namespace su2
