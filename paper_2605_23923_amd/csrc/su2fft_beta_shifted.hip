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
// method's stored products need the FP64 exponent range.  The shifted
// polynomials are generated per node from the plan's per-pair recurrence
// coefficients (the same scalars as the on-the-fly tables).
//
// Depth 1 runs on the matrix cores.  With A_{-1} = 0 and B_{-1} = 1 the
// depth-1 line also gives fhat(l0) (as <s^{Lb-1}, 1>), so row rho = 0 .. L-1
// of a pair is
//   fhat(l0 + rho) = sum_k A_{rho-1}(x_k) s^{Lb}_k + B_{rho-1}(x_k) s^{Lb-1}_k,
// the product of an L x 2N matrix (A and B at the nodes) with the 2N x batch
// matrix of stored products: FP64 16x16x4 products whose K index runs over
// (node, polynomial).  Depth 2 keeps one thread per (pair, signal), which
// walks the nodes with its L accumulators in registers.
#include "su2fft_internal.h"

namespace su2 {

// ---- depth 1: matrix cores ----
//
// Workgroup: 16 pairs (one tile) x 32 signals, 8 waves; wave w owns pairs w
// and w + 8.  Per chunk of SK nodes the workgroup stages the ring spectra of
// its pairs and signals in LDS, and generates into LDS the rows A_{rho-1},
// B_{rho-1} (one FP64 chain per (pair, node, polynomial) and thread) and
// d^{l0}, d^{l0+1} of every (pair, node).  The generation is the serial part
// (L dependent steps between barriers), so a workgroup takes as many signals
// as its accumulators allow and reads nothing but LDS while generating.  The B operand of a product is the
// spectrum value times d^{l0+1} (K index of an A row) or d^{l0} (of a B row):
// the method's stored products, formed as they are loaded.
template <class T, int RTMAX>
struct ShMfma {
  static constexpr int BT = 32;  // signals per workgroup (64 real columns)
  static constexpr int SK = 8;   // nodes per chunk
  static constexpr int PB = 2 * PT + 2;
  static constexpr int PK = BT * PB + 16;
  static constexpr int TMAX = PT * 16 * RTMAX;  // longest tile row (sum of L)
  static constexpr size_t OFF_G = (size_t)SK * PK * sizeof(T);                    // [node][A | B][lsum]
  static constexpr size_t OFF_D = OFF_G + (size_t)SK * 2 * TMAX * sizeof(double);  // [node][pair][d1 | d0]
  static constexpr size_t OFF_C = OFF_D + (size_t)SK * PT * 2 * sizeof(double);    // recurrence coefficients
  static constexpr size_t OFF_X = OFF_C + (size_t)TMAX * 3 * sizeof(double);     // x, cos, sin of the nodes
  static constexpr int NX = 128;                                                   // nodes (B <= 64)
  static constexpr size_t END = OFF_X + (size_t)3 * NX * sizeof(double);
  static constexpr size_t ROUND = CoefRound<T, BT, FWD_THREADS>::ELEMS * sizeof(T);  // epilogue, reusing the LDS
  static constexpr size_t SMEM = END > ROUND ? END : ROUND;
  static_assert(OFF_G % 8 == 0, "FP64 rows aligned");
};

template <class T, int RTMAX>
__device__ __forceinline__ void beta_forward_shifted_mfma_body(const cpx<T>* __restrict__ S,
                                                               cpx<T>* __restrict__ coeffs, const OtfParams<T>& op,
                                                               int tile, int bt, unsigned char* smem, int tid) {
  typedef ShMfma<T, RTMAX> G;
  const BetaParams<T>& p = op.b;
  constexpr int BT = G::BT, CT = 2 * BT / 16, SK = G::SK, PB = G::PB, PK = G::PK;
  constexpr int VC = 16 / (int)sizeof(cpx<T>);
  constexpr int SV = SK * BT * PT / VC;
  constexpr int SPT = SV / FWD_THREADS;
  static_assert(SV % FWD_THREADS == 0 && 2 * PT * SK <= FWD_THREADS && SK % 2 == 0, "chunk geometry");
  T* sS = reinterpret_cast<T*>(smem);
  double* sG = reinterpret_cast<double*>(smem + G::OFF_G);
  double* sD = reinterpret_cast<double*>(smem + G::OFF_D);
  double* sC = reinterpret_cast<double*>(smem + G::OFF_C);
  double* sX = reinterpret_cast<double*>(smem + G::OFF_X);

  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = tid >> 6, lane = tid & 63;
  const int lrow = lane & 15, lk = lane >> 4;
  const int N = p.N;
  const PairInfo p0 = p.pairs[tile * PT];
  const int lsum = p0.lsum;
  const long long row0 = p0.tab / N;  // first recurrence-coefficient row of the tile

  PairInfo pi[2];
#pragma unroll
  for (int i = 0; i < 2; i++) pi[i] = p.pairs[tile * PT + wave + 8 * i];

  doublex4 acc[2][RTMAX][CT];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++) acc[i][rt][ct] = doublex4{0.0, 0.0, 0.0, 0.0};

  // rows of nodes g0 .. g0 + SK - 1: thread (pair gi, node g0 + gk,
  // polynomial h) runs X_{-1}, X_0, X_1, .. with X = A (h = 0) or B (h = 1);
  // past the last node the stored products are zero.  The pair, its seed's
  // constant and exponents are the thread's for the whole launch.
  const int gh = tid & 1, ggk = (tid >> 1) % SK, ggi = (tid >> 1) / SK;
  const bool gthr = tid < 2 * PT * SK;
  PairInfo gq = p.pairs[tile * PT + (gthr ? ggi : 0)];
  if (!gthr) gq.L = 0;
  int gtop = 0, gpc = 0, gps = 0, gneg = 0;
  double gseed = 0.0;
  if (gq.L > 0) {
    wigner_seed_form(gq.tl0, gq.tn, gq.tm, &gtop, &gpc, &gps, &gneg);
    gseed = op.seedc[tile * PT + ggi];
  }
  auto generate = [&](int g0) {
    if (gq.L > 0) {
      const int k = g0 + ggk;
      const bool kin = k < N;
      const int kc = kin ? k : N - 1;
      const double x = sX[kc];
      const double* rc = sC + 3 * gq.coff;
      const double d0 = kin ? gseed * powi_d(sX[G::NX + kc], gpc) * powi_d(sX[2 * G::NX + kc], gps) : 0.0;
      const double d1 = gq.L > 1 ? (rc[3] * x - rc[4]) * d0 : 0.0;
      sD[(ggk * PT + ggi) * 2 + gh] = gh ? d0 : d1;
      double* out = sG + (ggk * 2 + gh) * lsum + gq.coff;
      double xm = gh ? 1.0 : 0.0, xc = gh ? 0.0 : 1.0;
      out[0] = xm;
      if (gq.L > 1) out[1] = xc;
      if (gq.L > 2) {
        // coefficients of step r + 1 are read while step r computes
        double c0 = rc[6], c1 = rc[7], c2 = rc[8];
        for (int r = 2; r < gq.L; r++) {
          const int rn = r + 1 < gq.L ? r + 1 : r;
          const double n0 = rc[3 * rn], n1 = rc[3 * rn + 1], n2 = rc[3 * rn + 2];
          const double xn = (c0 * x - c1) * xc - c2 * xm;
          xm = xc;
          xc = xn;
          out[r] = xn;
          c0 = n0;
          c1 = n1;
          c2 = n2;
        }
      }
    }
  };

  typedef T vec16 __attribute__((ext_vector_type(16 / sizeof(T))));
  vec16 sreg[SPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < SPT; i++) {
      const int v = tid + FWD_THREADS * i;
      const int kk = v / (BT * PT / VC), rem = v - kk * (BT * PT / VC);
      const int bb = rem / (PT / VC), pv = rem - bb * (PT / VC);
      const int k = k0 + kk;
      if (k < N && bb < nb)
        sreg[i] = *reinterpret_cast<const vec16*>(S + (((size_t)tile * N + k) * p.batch + b0 + bb) * PT + pv * VC);
      else
        sreg[i] = vec16(T(0));
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int i = 0; i < SPT; i++) {
      const int v = tid + FWD_THREADS * i;
      const int kk = v / (BT * PT / VC), rem = v - kk * (BT * PT / VC);
      const int bb = rem / (PT / VC), pv = rem - bb * (PT / VC);
#pragma unroll
      for (int q = 0; q < 2 * VC; q++) sS[kk * PK + bb * PB + 2 * pv * VC + q] = sreg[i][q];
    }
  };

  const int nchunk = (N + SK - 1) / SK;
  otf_load_coeffs(sC, op.rcoef, row0, lsum, tid, FWD_THREADS);
  for (int j = tid; j < N; j += FWD_THREADS) {
    sX[j] = op.xk[j];
    sX[G::NX + j] = op.ck[j];
    sX[2 * G::NX + j] = op.sk[j];
  }
  fetch(0);
  commit();
  __syncthreads();  // recurrence coefficients and nodes
  generate(0);
  for (int c = 0; c < nchunk; c++) {
    __syncthreads();  // chunk c: spectra, rows and seeds in LDS
    if (c + 1 < nchunk) fetch((c + 1) * SK);
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const int L = pi[i].L;
      if (L == 0) continue;
      const int pp = wave + 8 * i;
      const int coff = pi[i].coff;
#pragma unroll
      for (int ks = 0; ks < SK; ks += 2) {
        // K index lk: node ks + lk / 2, polynomial lk % 2
        const int kk = ks + (lk >> 1), h = lk & 1;
        const bool kin = c * SK + kk < N;
        const double ds = sD[(kk * PT + pp) * 2 + h];
        double bop[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
          const int cc = ct * 16 + lrow;
          bop[ct] = (double)sS[kk * PK + (cc >> 1) * PB + 2 * pp + (cc & 1)] * ds;
        }
#pragma unroll
        for (int rt = 0; rt < RTMAX; rt++) {
          if (rt * 16 < L) {
            const int rho = rt * 16 + lrow;
            const double a = (rho < L && kin) ? sG[(kk * 2 + h) * lsum + coff + rho] : 0.0;
#pragma unroll
            for (int ct = 0; ct < CT; ct++) acc[i][rt][ct] = mfma16x16x4(a, bop[ct], acc[i][rt][ct]);
          }
        }
      }
    }
    __syncthreads();  // chunk c consumed
    if (c + 1 < nchunk) {
      commit();
      generate((c + 1) * SK);
    }
  }

  // epilogue: the coefficients leave through LDS (CoefRound), 8 degrees of
  // all 16 pairs per round, rounded to the plan's type
  typedef CoefRound<T, BT, FWD_THREADS> CR;
  static_assert(CR::ELEMS * sizeof(T) <= G::SMEM, "coefficient rounds fit");
  T* cst = reinterpret_cast<T*>(smem);
#pragma unroll
  for (int j0 = 0; j0 < 16 * RTMAX; j0 += CR::JC) {
    const int rt = j0 / 16, r0 = j0 % 16;
    __syncthreads();  // LDS free (main loop, or the previous round's reads)
#pragma unroll
    for (int h = 0; h < 2; h++) {
      if (rt * 16 < pi[h].L) {
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int row = acc_row<double>(lane, r) - r0;
            if (row >= 0 && row < CR::JC)
              cst[(wave + 8 * h) * CR::PS + row * CR::CWP + ct * 16 + lrow] = (T)acc[h][rt][ct][r];
          }
      }
    }
    __syncthreads();
    CR::store(coeffs, p, tile, j0, b0, nb, cst, tid);
  }
}

template <class T, int RTMAX>
__global__ __launch_bounds__(FWD_THREADS) void beta_forward_shifted_mfma_kernel(const cpx<T>* __restrict__ S,
                                                                                cpx<T>* __restrict__ coeffs,
                                                                                OtfParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  beta_forward_shifted_mfma_body<T, RTMAX>(S, coeffs, p, blockIdx.x, blockIdx.y, smem_raw, threadIdx.x);
}

// ---- depth 2: one thread per (pair, signal) ----

constexpr int SH_THREADS = 512;  // 16 pairs x 32 signals
constexpr int SH_BT = SH_THREADS / PT;

template <class T, int LMAX, int BLK>
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
    {
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
  if (depth == 1) {
    constexpr int RT = (LMAX + 15) / 16;
    typedef ShMfma<T, RT> G;
    if (p.b.N > G::NX) return hipErrorInvalidValue;
    hipError_t e = set_smem(beta_forward_shifted_mfma_kernel<T, RT>, G::SMEM);
    if (e != hipSuccess) return e;
    const dim3 grid(p.b.ntiles, (p.b.batch + G::BT - 1) / G::BT);
    hipLaunchKernelGGL((beta_forward_shifted_mfma_kernel<T, RT>), grid, dim3(FWD_THREADS), G::SMEM, s, S, coeffs, p);
    return hipGetLastError();
  }
  const dim3 grid(p.b.ntiles, (p.b.batch + SH_BT - 1) / SH_BT);
  if (blk == 2)
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 2>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  else if (blk == 4)
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 4>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
  else
    hipLaunchKernelGGL((beta_forward_shifted_kernel<T, LMAX, 8>), grid, dim3(SH_THREADS), 0, s, S, coeffs, p);
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
