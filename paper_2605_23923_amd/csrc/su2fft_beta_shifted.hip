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
// (node, polynomial).  Depth 2 with a coarse step of 16 (one matrix-core row
// tile) runs on the same kernel: rows rho = 16 + n2 + 1 contract the fine
// polynomials A_{n2}, B_{n2} of level Lb + 16 against the shifted stored
// products u = A_16 s^{Lb} + B_16 s^{Lb-1} and v = A_15 s^{Lb} + B_15 s^{Lb-1},
// so the fine chains of the two row tiles are independent and run side by
// side (16-18 dependent steps instead of L).  Depth 2 with coarse steps 2, 4
// or 8 keeps one thread per (pair, signal), which walks the nodes with its L
// accumulators in registers.
#include "su2fft_internal.h"

namespace su2 {

// ---- depth 1, and depth 2 with coarse step 16: matrix cores ----
//
// Workgroup: 16 pairs (one tile) x 32 signals, 8 waves; wave w owns pairs w
// and w + 8.  Per chunk of SK nodes the workgroup stages the ring spectra of
// its pairs and signals in LDS, and generates into LDS the rows A_{rho-1},
// B_{rho-1} (FP64 chains per (pair, node, polynomial)) and d^{l0}, d^{l0+1}
// of every (pair, node).  The generation runs between barriers and does not
// depend on the signals, so a workgroup takes as many signals as its
// accumulators allow, and reads nothing but LDS while generating.  The B
// operand of a product is the spectrum value times d^{l0+1} (K index of an
// A row) or d^{l0} (of a B row): the method's stored products, formed as
// they are loaded.
template <class T, int RTMAX>
struct ShMfma {
  static constexpr int BT = 32;  // signals per workgroup (64 real columns)
  static constexpr int SK = 8;   // nodes per chunk
  static constexpr int PB = 2 * PT + 2;
  static constexpr int PK = BT * PB + 16;
  static constexpr int TMAX = PT * 16 * RTMAX;  // longest tile row (sum of L)
  // generated rows: element (degree row j of the tile, node kk, polynomial h)
  // at j * GS + 2 kk + h; the odd stride GS spreads a step's writes (16
  // (node, polynomial) of a pair side by side) and the operand reads (16
  // consecutive degrees) over distinct banks
  static constexpr int GS = 2 * SK + 1;
  static constexpr size_t OFF_G = (size_t)SK * PK * sizeof(T);
  // per (node, pair): d^{l0+1}, d^{l0}, then (depth 2) A_16, B_16, A_15, B_15 of level Lb
  static constexpr int DS = 6;
  static constexpr size_t OFF_D = OFF_G + (size_t)TMAX * GS * sizeof(double);
  static constexpr size_t OFF_C = OFF_D + (size_t)SK * PT * DS * sizeof(double);  // recurrence coefficients
  static constexpr size_t OFF_X = OFF_C + (size_t)TMAX * 3 * sizeof(double);     // x, cos, sin of the nodes
  static constexpr int NX = 128;                                                   // nodes (B <= 64)
  static constexpr size_t END = OFF_X + (size_t)3 * NX * sizeof(double);
  static constexpr size_t ROUND = CoefRound<T, BT, FWD_THREADS>::ELEMS * sizeof(T);  // epilogue, reusing the LDS
  static constexpr size_t SMEM = END > ROUND ? END : ROUND;
  static_assert(OFF_G % 8 == 0, "FP64 rows aligned");
};

template <class T, int RTMAX, bool SPLIT>
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

  // rows of nodes g0 .. g0 + SK - 1: thread (pair gi, node g0 + gk, row
  // tile gt, polynomial h) runs X_{-1}, X_0, X_1, .. with X = A (h = 0) or
  // B (h = 1) of level Lb + 16 gt, from the recurrence coefficients of the
  // degrees it stands for.  At depth 1 one chain (gt = 0) covers all L rows;
  // at depth 2 the chain of tile 0 runs on to A_15, A_16 (B_15, B_16), the
  // coarse polynomials of the shifted stored products.  Past the last node
  // the stored products are zero.  The pair, its seed's constant and
  // exponents are the thread's for the whole launch.
  constexpr int GT = SPLIT ? RTMAX : 1;
  constexpr int DS = G::DS;
  static_assert(2 * GT * PT * SK <= FWD_THREADS, "one generation thread per chain");
  const int gh = tid & 1, gt = (tid >> 1) % GT, ggk = (tid / (2 * GT)) % SK, ggi = tid / (2 * GT * SK);
  const bool gthr = tid < 2 * GT * PT * SK;
  int gL, gcoff, gpc = 0, gps = 0;
  double gseed = 0.0;
  {
    const PairInfo q = p.pairs[tile * PT + (gthr ? ggi : 0)];
    gL = gthr && q.L > 16 * gt ? q.L : 0;
    gcoff = q.coff;
    if (gL > 0) {
      int top, neg;
      wigner_seed_form(q.tl0, q.tn, q.tm, &top, &gpc, &gps, &neg);
      gseed = op.seedc[tile * PT + ggi];
    }
  }
  const int gs = 16 * gt;                               // level shift of the chain
  const int nrow = SPLIT ? min(gL - gs, 16) : gL;        // rows it writes
  const int jend = SPLIT && gt == 0 ? min(gL, 18) : nrow;  // steps it runs
  auto generate = [&](int g0) {
    if (gL > 0) {
      const int k = g0 + ggk;
      const bool kin = k < N;
      const int kc = kin ? k : N - 1;
      const double x = sX[kc];
      const double* rc = sC + 3 * (gcoff + gs);
      double* dd = sD + (ggk * PT + ggi) * DS;
      if (gt == 0) {
        const double d0 = kin ? gseed * powi_d(sX[G::NX + kc], gpc) * powi_d(sX[2 * G::NX + kc], gps) : 0.0;
        const double d1 = gL > 1 ? (rc[3] * x - rc[4]) * d0 : 0.0;
        dd[gh] = gh ? d0 : d1;
        if (SPLIT) dd[2 + gh] = dd[4 + gh] = 0.0;  // A_16, A_15 (B_16, B_15) where the chain stops short
      }
      double* out = sG + (gcoff + gs) * G::GS + 2 * ggk + gh;
      double xm = gh ? 1.0 : 0.0, xc = gh ? 0.0 : 1.0;
      out[0] = xm;
      if (nrow > 1) out[G::GS] = xc;
      if (jend > 2) {
        // coefficients of step j + 1 are read while step j computes
        double c0 = rc[6], c1 = rc[7], c2 = rc[8];
        for (int j = 2; j < jend; j++) {
          const int jn = j + 1 < jend ? j + 1 : j;
          const double n0 = rc[3 * jn], n1 = rc[3 * jn + 1], n2 = rc[3 * jn + 2];
          const double xn = (c0 * x - c1) * xc - c2 * xm;
          xm = xc;
          xc = xn;
          if (j < nrow) out[j * G::GS] = xn;
          if (SPLIT && j >= 16) dd[(j == 16 ? 4 : 2) + gh] = xn;  // X_15, X_16
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
        const double* dd = sD + (kk * PT + pp) * DS;
        const double d1 = dd[0], d0 = dd[1];
#pragma unroll
        for (int rt = 0; rt < RTMAX; rt++) {
          if (rt * 16 < L) {
            // B operand: the stored products s^{Lb} (A rows) or s^{Lb-1} (B
            // rows); for the second tile at depth 2 the shifted ones,
            // u = A_16 s^{Lb} + B_16 s^{Lb-1} (A rows) and
            // v = A_15 s^{Lb} + B_15 s^{Lb-1} (B rows), formed with the
            // spectrum factored out: S (A d^{l0+1} + B d^{l0})
            const double sc = (SPLIT && rt == 1) ? dd[2 + 2 * h] * d1 + dd[3 + 2 * h] * d0 : (h ? d0 : d1);
            double bop[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
              const int cc = ct * 16 + lrow;
              bop[ct] = (double)sS[kk * PK + (cc >> 1) * PB + 2 * pp + (cc & 1)] * sc;
            }
            const int rho = rt * 16 + lrow;
            const double a = (rho < L && kin) ? sG[(coff + rho) * G::GS + 2 * kk + h] : 0.0;
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

template <class T, int RTMAX, bool SPLIT>
__global__ __launch_bounds__(FWD_THREADS) void beta_forward_shifted_mfma_kernel(const cpx<T>* __restrict__ S,
                                                                                cpx<T>* __restrict__ coeffs,
                                                                                OtfParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  beta_forward_shifted_mfma_body<T, RTMAX, SPLIT>(S, coeffs, p, blockIdx.x, blockIdx.y, smem_raw, threadIdx.x);
}

// ---- depth 2, coarse steps 2, 4, 8: one thread per (pair, signal) ----

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
  if (depth == 1 || blk == 16) {
    constexpr int RT = (LMAX + 15) / 16;
    typedef ShMfma<T, RT> G;
    if (p.b.N > G::NX) return hipErrorInvalidValue;
    const dim3 grid(p.b.ntiles, (p.b.batch + G::BT - 1) / G::BT);
    hipError_t e;
    if (depth == 1) {
      if ((e = set_smem(beta_forward_shifted_mfma_kernel<T, RT, false>, G::SMEM)) != hipSuccess) return e;
      hipLaunchKernelGGL((beta_forward_shifted_mfma_kernel<T, RT, false>), grid, dim3(FWD_THREADS), G::SMEM, s, S,
                         coeffs, p);
    } else {
      if ((e = set_smem(beta_forward_shifted_mfma_kernel<T, RT, true>, G::SMEM)) != hipSuccess) return e;
      hipLaunchKernelGGL((beta_forward_shifted_mfma_kernel<T, RT, true>), grid, dim3(FWD_THREADS), G::SMEM, s, S,
                         coeffs, p);
    }
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
  if ((depth != 1 && depth != 2) || (depth == 2 && blk != 2 && blk != 4 && blk != 8 && blk != 16) || lmax > 32)
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
