// Beta contraction with the Wigner-d values generated inside the kernels
// (no stored table): the same products as the table kernels of
// su2fft_beta.hip, with d^l_{nm}(beta_k) produced by the FP64 three-term
// recurrence in l (Section 4: Lemma 4.3 is its m = n = 0 case, extended at the
// end of the section to general (m, n)) from its single-term seed, and
// rounded to the contraction's type where it is consumed.  Only per-pair and
// per-node scalars are read (OtfParams), so the table bytes of a launch
// (C(B) N values) drop to about 3 C(B) + P doubles.
//
// Forward: a workgroup generates the table rows of its 16 pairs for GK nodes
// at a time into LDS (one recurrence chain per (pair, node) and thread), then
// runs the KC-node chunks of S through the matrix cores as the table kernel
// does.  Inverse: every lane generates the A operands it needs for its node
// (one chain per pair and lane, keeping the degrees l = lk mod 4 it feeds to
// the matrix cores), so no LDS is needed for the table.
#include "su2fft_internal.h"

namespace su2 {

// x^n for an integer n >= 0 by repeated squaring (n <= 128 here)
__device__ __forceinline__ double powi_d(double x, int n) {
  double r = 1.0;
  while (n) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

// seed d^{l0}_{nm}(beta_k) of a pair (a = n, b = m, doubled indices)
template <class T>
__device__ __forceinline__ double otf_seed(const OtfParams<T>& p, const PairInfo& q, int pidx, int k) {
  int top, pc, ps, neg;
  wigner_seed_form(q.tl0, q.tn, q.tm, &top, &pc, &ps, &neg);
  return p.seedc[pidx] * powi_d(p.ck[k], pc) * powi_d(p.sk[k], ps);
}

template <class T, int RTMAX, int BT_ = BetaCfg<T>::BT>
struct OtfFwd {
  static constexpr int BT = BT_;  // signals per workgroup (16 for FP32 batches of at most 16)
  static constexpr int KC = 8;                 // nodes per S chunk
  static constexpr int PB = 2 * PT + 2;
  static constexpr int PK = BT * PB + 16;
  static constexpr int TMAX = PT * 16 * RTMAX;  // longest tile row (sum of L)
  static constexpr int GK0 = (65536 / (int)sizeof(T)) / TMAX;
  static constexpr int GK = GK0 >= 32 ? 32 : GK0;   // nodes generated at a time (64 KB of rows)
  static_assert(GK % KC == 0 && PT * GK <= FWD_THREADS, "generation geometry");
  // generated values: (degree row j of the tile, node gk) at j * GS + gk; the
  // odd stride spreads a chain step's writes (GK nodes side by side) and the
  // operand reads (16 consecutive degrees) over distinct banks
  static constexpr int GS = GK + 1;
  // S chunk, the generated values, then the tile's recurrence coefficients (3 doubles per row element)
  static constexpr size_t SMEM_C = (size_t)KC * PK * sizeof(T) + (size_t)TMAX * GS * sizeof(T);
  static constexpr size_t SMEM = SMEM_C + (size_t)TMAX * 3 * sizeof(double);
};

// the tile's recurrence coefficients (rows row0 .. row0 + lsum - 1) into LDS
__device__ __forceinline__ void otf_load_coeffs(double* sC, const double* rcoef, long long row0, int lsum, int tid,
                                                int nthreads) {
  for (int j = tid; j < 3 * lsum; j += nthreads) sC[j] = rcoef[3 * row0 + j];
}

template <class T, int RTMAX, int BT_ = BetaCfg<T>::BT>
__device__ __forceinline__ void beta_forward_otf_body(const cpx<T>* __restrict__ S, cpx<T>* __restrict__ coeffs,
                                                      const OtfParams<T>& op, int tile, int bt, unsigned char* smem,
                                                      int tid) {
  typedef OtfFwd<T, RTMAX, BT_> G;
  typedef typename acc4<T>::type accT;
  const BetaParams<T>& p = op.b;
  constexpr int BT = G::BT, CT = 2 * BT / 16, KC = G::KC, PB = G::PB, PK = G::PK, GK = G::GK;
  constexpr int VC = 16 / (int)sizeof(cpx<T>);
  constexpr int SV = KC * BT * PT / VC;
  constexpr int SPT = SV / FWD_THREADS;
  static_assert(SV % FWD_THREADS == 0, "chunk split");
  T* sS = reinterpret_cast<T*>(smem);
  T* sT = sS + KC * PK;  // GK nodes of the tile's lsum degree rows
  double* sC = reinterpret_cast<double*>(smem + G::SMEM_C);

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

  accT acc[2][RTMAX][CT];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[i][rt][ct][r] = T(0);

  // table rows of nodes g0 .. g0 + GK - 1: thread (pair gi, node gk) runs one chain
  // the generating thread's pair (gi) and seed, fixed for the launch
  const int gi = tid / GK, gk = tid - gi * GK;
  int gL = 0, gcoff = 0, gpc = 0, gps = 0;
  double gseed = 0.0;
  if (gi < PT) {
    const PairInfo q = p.pairs[tile * PT + gi];
    gL = q.L;
    gcoff = q.coff;
    if (gL > 0) {
      int top, neg;
      wigner_seed_form(q.tl0, q.tn, q.tm, &top, &gpc, &gps, &neg);
      gseed = op.seedc[tile * PT + gi];
    }
  }
  auto generate = [&](int g0) {
    const int k = g0 + gk;
    if (gL > 0 && k < N) {
      T* out = sT + gcoff * G::GS + gk;
      double d = gseed * powi_d(op.ck[k], gpc) * powi_d(op.sk[k], gps), dm1 = 0.0;
      const double x = op.xk[k];
      const double* rc = sC + 3 * gcoff;
      out[0] = (T)d;
      for (int i = 1; i < gL; i++) {
        const double dn = (rc[3 * i] * x - rc[3 * i + 1]) * d - rc[3 * i + 2] * dm1;
        dm1 = d;
        d = dn;
        out[i * G::GS] = (T)d;
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

  const int nchunk = (N + KC - 1) / KC;
  otf_load_coeffs(sC, op.rcoef, row0, lsum, tid, FWD_THREADS);
  fetch(0);
  commit();
  int g0 = 0;
  for (int c = 0; c < nchunk; c++) {
    __syncthreads();
    if (c + 1 < nchunk) fetch((c + 1) * KC);
    if ((c * KC) % GK == 0) {  // the next GK nodes' table rows
      g0 = c * KC;
      generate(g0);
      __syncthreads();
    }
    const int toff = c * KC - g0;  // first node of the chunk in the generated block
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const int L = pi[i].L;
      if (L == 0) continue;
      const int pp = wave + 8 * i;
      const int coff = pi[i].coff;
#pragma unroll
      for (int ks = 0; ks < KC; ks += 4) {
        const int kk = ks + lk;
        const bool kin = c * KC + kk < N;
        T bop[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
          const int cc = ct * 16 + lrow;
          bop[ct] = sS[kk * PK + (cc >> 1) * PB + 2 * pp + (cc & 1)];
        }
#pragma unroll
        for (int rt = 0; rt < RTMAX; rt++) {
          if (rt * 16 < L) {
            const int l = rt * 16 + lrow;
            const T a = (l < L && kin) ? sT[(coff + l) * G::GS + toff + kk] : T(0);
#pragma unroll
            for (int ct = 0; ct < CT; ct++) acc[i][rt][ct] = mfma16x16x4(a, bop[ct], acc[i][rt][ct]);
          }
        }
      }
    }
    __syncthreads();
    if (c + 1 < nchunk) commit();
  }

  // epilogue: the coefficients leave through LDS (CoefRound), 8 degrees of
  // all 16 pairs per round
  typedef CoefRound<T, BT, FWD_THREADS> CR;
  static_assert(CR::ELEMS * sizeof(T) <= G::SMEM_C, "coefficient rounds fit");
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
            const int row = acc_row<T>(lane, r) - r0;
            if (row >= 0 && row < CR::JC)
              cst[(wave + 8 * h) * CR::PS + row * CR::CWP + ct * 16 + lrow] = acc[h][rt][ct][r];
          }
      }
    }
    __syncthreads();
    CR::store(coeffs, p, tile, j0, b0, nb, cst, tid);
  }
}

template <class T, int RTMAX, int BT>
__global__ __launch_bounds__(FWD_THREADS) void beta_forward_otf_kernel(const cpx<T>* __restrict__ S,
                                                                       cpx<T>* __restrict__ coeffs, OtfParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileSlot sl = contraction_slot(blockIdx.x, p.b.ntiles, (p.b.batch + BT - 1) / BT, p.b.paired);
  if (!sl.valid) return;
  beta_forward_otf_body<T, RTMAX, BT>(S, coeffs, p, sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// generated values of the inverse (GEN_LDS): (degree row j of the tile, node
// k0 + gk) at j * INV_GS + gk, so that a chain step's writes (16 nodes of a
// pair) and an operand read (16 nodes of one degree) are contiguous; no
// padding, which would push the largest tiles past the LDS limit
constexpr int INV_GS = 16;

// Inverse: as beta_inverse_body, with the A operands (node k = k0 + lrow,
// degree l = 4 s + lk) generated per lane.
template <class T, int LQ, bool GEN_LDS, int BT_ = BetaCfg<T>::BT>
__device__ __forceinline__ void beta_inverse_otf_body(const cpx<T>* __restrict__ coeffs, cpx<T>* __restrict__ S,
                                                      const OtfParams<T>& op, int tile, int bt, unsigned char* smem,
                                                      int tid) {
  typedef typename acc4<T>::type accT;
  const BetaParams<T>& p = op.b;
  constexpr int BT = BT_, CT = 2 * BT / 16;  // BT_: 16 for FP32 batches of at most 16
  constexpr int PB = InvStage<T>::PB, NRS = InvStage<T>::NRS;
  T* stage = reinterpret_cast<T*>(smem);
  double* sC = reinterpret_cast<double*>(smem + inverse_smem<T>());  // the tile's recurrence coefficients
  T* sT = reinterpret_cast<T*>(sC + (size_t)PT * 4 * LQ * 3);          // GEN_LDS: 16 nodes of lsum degree rows
  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = tid >> 6, lane = tid & 63;
  const int lrow = lane & 15, lk = lane >> 4;
  const int N = p.N;
  const PairInfo p0 = p.pairs[tile * PT];
  const long long row0 = p0.tab / N;
  otf_load_coeffs(sC, op.rcoef, row0, p0.lsum, tid, INV_THREADS);

  PairInfo pi[2];
#pragma unroll
  for (int q = 0; q < 2; q++) pi[q] = p.pairs[tile * PT + wave + 8 * q];
  // B operands: the scaled coefficients gathered through LDS (CoefRound)
  constexpr int J = 4 * LQ;
  typedef CoefRound<T, BT, INV_THREADS> CR;
  static_assert(CR::ELEMS <= (size_t)16 * NRS && J % CR::JC == 0, "coefficient rounds fit in the stage buffer");
  T bop[2][LQ][CT];
#pragma unroll
  for (int j0 = 0; j0 < J; j0 += CR::JC) {
    CR::gather(coeffs, p, tile, j0, b0, nb, stage, tid);
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
      for (int s = j0 / 4; s < (j0 + CR::JC) / 4; s++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          bop[h][s][ct] = stage[(wave + 8 * h) * CR::PS + (4 * s - j0 + lk) * CR::CWP + ct * 16 + lrow];
    __syncthreads();
  }

  // GEN_LDS: thread (pair gi, node k0 + gk) of each block runs one chain;
  // its pair and seed are fixed for the launch
  const int gi = tid / 16, gk = tid - gi * 16;
  int gL = 0, gcoff = 0, gpc = 0, gps = 0;
  double gseed = 0.0;
  if (GEN_LDS && tid < 16 * PT) {
    const PairInfo q = p.pairs[tile * PT + gi];
    gL = q.L;
    gcoff = q.coff;
    if (gL > 0) {
      int top, neg;
      wigner_seed_form(q.tl0, q.tn, q.tm, &top, &gpc, &gps, &neg);
      gseed = op.seedc[tile * PT + gi];
    }
  }

  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += 16) {
    const int k = k0 + lrow;
    const int kc = k < N ? k : N - 1;  // lanes past the last node compute a valid chain and are zeroed
    T av[2][LQ];
    if constexpr (GEN_LDS) {
      // one chain per (pair, node) of the block: threads tid < 16 * PT, then
      // every lane reads its operands (node kc, degrees l = 4 s + lk)
      if (gL > 0) {
        const int kg = k0 + gk < N ? k0 + gk : N - 1;
        T* out = sT + gcoff * INV_GS + gk;
        double dd = gseed * powi_d(op.ck[kg], gpc) * powi_d(op.sk[kg], gps), ddm1 = 0.0;
        const double xg = op.xk[kg];
        const double* rc = sC + 3 * gcoff;
        out[0] = (T)dd;
        for (int i = 1; i < gL; i++) {
          const double dn = (rc[3 * i] * xg - rc[3 * i + 1]) * dd - rc[3 * i + 2] * ddm1;
          ddm1 = dd;
          dd = dn;
          out[i * INV_GS] = (T)dd;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; q++)
#pragma unroll
        for (int s = 0; s < LQ; s++) {
          const int l = 4 * s + lk;
          av[q][s] = (l < pi[q].L && k < N) ? sT[(pi[q].coff + l) * INV_GS + lrow] : T(0);
        }
    } else {
      // this lane's chains for both pairs, advanced together (independent FP64
      // chains interleave): degrees l0 .. l0 + L - 1 at node kc; keep l = 4 s + lk
      double d[2], dm1[2];
      const double x = op.xk[kc];
#pragma unroll
      for (int q = 0; q < 2; q++) {
        d[q] = pi[q].L > 0 ? otf_seed(op, pi[q], tile * PT + wave + 8 * q, kc) : 0.0;
        dm1[q] = 0.0;
      }
#pragma unroll
      for (int s = 0; s < LQ; s++) {
#pragma unroll
        for (int q = 0; q < 2; q++) av[q][s] = T(0);
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int l = 4 * s + j;
#pragma unroll
          for (int q = 0; q < 2; q++) {
            if (l < pi[q].L) {
              if (l > 0) {
                const double* rc = sC + 3 * (pi[q].coff + l);
                const double dn = (rc[0] * x - rc[1]) * d[q] - rc[2] * dm1[q];
                dm1[q] = d[q];
                d[q] = dn;
              }
              if (j == lk) av[q][s] = (T)d[q];
            }
          }
        }
        if (k >= N) {
#pragma unroll
          for (int q = 0; q < 2; q++) av[q][s] = T(0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int L = pi[q].L;
      const int pp = wave + 8 * q;
      accT acc[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[ct][r] = T(0);
#pragma unroll
      for (int s = 0; s < LQ; s++) {
        if (4 * s < L) {
#pragma unroll
          for (int ct = 0; ct < CT; ct++) acc[ct] = mfma16x16x4(av[q][s], bop[q][s][ct], acc[ct]);
        }
      }
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int cc = ct * 16 + lrow;
        const int bb = cc >> 1, reim = cc & 1;
#pragma unroll
        for (int r = 0; r < 4; r++) stage[acc_row<T>(lane, r) * NRS + bb * PB + 2 * pp + reim] = acc[ct][r];
      }
    }
    __syncthreads();
    constexpr int VC = 16 / (int)sizeof(cpx<T>);
    for (int v = tid; v < 16 * BT * (PT / VC); v += INV_THREADS) {
      const int row = v / (PT / VC), pv = v - row * (PT / VC);
      const int kk = row / BT, bb = row - kk * BT;
      const int kn = k0 + kk;
      if (kn < N && bb < nb) {
        const T* src = stage + kk * NRS + bb * PB + 2 * pv * VC;
        float4 w;
        T* wd = reinterpret_cast<T*>(&w);
#pragma unroll
        for (int e = 0; e < 2 * VC; e++) wd[e] = src[e];
        *reinterpret_cast<float4*>(S + (((size_t)tile * N + kn) * p.batch + b0 + bb) * PT + pv * VC) = w;
      }
    }
    __syncthreads();
  }
}

template <class T, int LQ, bool GEN_LDS, int BT>
__global__ __launch_bounds__(INV_THREADS) void beta_inverse_otf_kernel(const cpx<T>* __restrict__ coeffs,
                                                                       cpx<T>* __restrict__ S, OtfParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileSlot sl = contraction_slot(blockIdx.x, p.b.ntiles, (p.b.batch + BT - 1) / BT, p.b.paired);
  if (!sl.valid) return;
  beta_inverse_otf_body<T, LQ, GEN_LDS, BT>(coeffs, S, p, sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// LDS of the inverse: staging, recurrence coefficients and (GEN_LDS) the
// generated rows of one block of 16 nodes
template <class T, int LQ, bool GEN_LDS>
constexpr size_t inverse_otf_smem() {
  return inverse_smem<T>() + (size_t)PT * 4 * LQ * 3 * sizeof(double) +
         (GEN_LDS ? (size_t)INV_GS * PT * 4 * LQ * sizeof(T) : 0);
}
// generated rows in LDS where they fit next to the staging buffer (all but
// FP64 at B = 128, which generates per lane)
template <class T, int LQ>
constexpr bool inverse_gen_lds() { return inverse_otf_smem<T, LQ, true>() <= 160 * 1024; }

template <class T>
hipError_t launch_beta_forward_otf(const OtfParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, hipStream_t s) {
  constexpr int BTW = BetaCfg<T>::BT, BTN = BTW > 16 ? 16 : BTW;  // widest tile; batches of at most 16
  const int bt = p.b.batch <= BTN ? BTN : BTW;
  const dim3 grid(contraction_grid(p.b.ntiles, (p.b.batch + bt - 1) / bt, p.b.paired));
  const int rt = beta_rtmax(p.b.B);
  hipError_t e;
#define SU2_OTF_FWD(R, BTC)                                                                                     \
  if (rt == R && bt == BTC) {                                                                                   \
    if ((e = set_smem(beta_forward_otf_kernel<T, R, BTC>, OtfFwd<T, R, BTC>::SMEM)) != hipSuccess) return e;      \
    hipLaunchKernelGGL((beta_forward_otf_kernel<T, R, BTC>), grid, dim3(FWD_THREADS), (OtfFwd<T, R, BTC>::SMEM), s, \
                       S, coeffs, p);                                                                           \
    return hipGetLastError();                                                                                   \
  }
  SU2_OTF_FWD(1, BTW)
  SU2_OTF_FWD(2, BTW)
  SU2_OTF_FWD(4, BTW)
  if constexpr (BTN != BTW) {
    SU2_OTF_FWD(1, BTN)
    SU2_OTF_FWD(2, BTN)
    SU2_OTF_FWD(4, BTN)
  }
#undef SU2_OTF_FWD
  return hipErrorInvalidValue;
}

template <class T>
hipError_t launch_beta_inverse_otf(const OtfParams<T>& p, const cpx<T>* coeffs, cpx<T>* S, hipStream_t s) {
  constexpr int BTW = BetaCfg<T>::BT, BTN = BTW > 16 ? 16 : BTW;  // widest tile; batches of at most 16
  const int bt = p.b.batch <= BTN ? BTN : BTW;
  const dim3 grid(contraction_grid(p.b.ntiles, (p.b.batch + bt - 1) / bt, p.b.paired));
  const int lq = beta_lq(p.b.B);
  hipError_t e;
#define SU2_OTF_INV(Q, BTC)                                                                                   \
  if (lq == Q && bt == BTC) {                                                                                 \
    constexpr bool GL = inverse_gen_lds<T, Q>();                                                              \
    constexpr size_t smem = inverse_otf_smem<T, Q, GL>();                                                     \
    if ((e = set_smem(beta_inverse_otf_kernel<T, Q, GL, BTC>, smem)) != hipSuccess) return e;                 \
    hipLaunchKernelGGL((beta_inverse_otf_kernel<T, Q, GL, BTC>), grid, dim3(INV_THREADS), smem, s, coeffs, S, \
                       p);                                                                                    \
    return hipGetLastError();                                                                                 \
  }
  SU2_OTF_INV(2, BTW)
  SU2_OTF_INV(4, BTW)
  SU2_OTF_INV(8, BTW)
  SU2_OTF_INV(16, BTW)
  if constexpr (BTN != BTW) {
    SU2_OTF_INV(2, BTN)
    SU2_OTF_INV(4, BTN)
    SU2_OTF_INV(8, BTN)
    SU2_OTF_INV(16, BTN)
  }
#undef SU2_OTF_INV
  return hipErrorInvalidValue;
}

template hipError_t launch_beta_forward_otf<float>(const OtfParams<float>&, const cpx<float>*, cpx<float>*,
                                                   hipStream_t);
template hipError_t launch_beta_forward_otf<double>(const OtfParams<double>&, const cpx<double>*, cpx<double>*,
                                                    hipStream_t);
template hipError_t launch_beta_inverse_otf<float>(const OtfParams<float>&, const cpx<float>*, cpx<float>*,
                                                   hipStream_t);
template hipError_t launch_beta_inverse_otf<double>(const OtfParams<double>&, const cpx<double>*, cpx<double>*,
                                                    hipStream_t);

}  // namespace su2
