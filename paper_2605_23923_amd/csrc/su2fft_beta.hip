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
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// word 3 of a raw buffer resource on CDNA (gfx9 family): 32-bit data format,
// no swizzle; range checking against word 2 (bytes) with stride 0
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;

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

template <class T>
struct BetaCfg;
template <>
struct BetaCfg<float> {
  static constexpr int BT = 32;  // signals per workgroup (64 real columns)
};
template <>
struct BetaCfg<double> {
  static constexpr int BT = 16;  // 32 real columns
};

// compute units of the current device (read once per process)
inline int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
              ? n
              : 256;
  }
  return cus;
}

// ---- coefficients through LDS ----
//
// A wave's matrix-core operands (inverse) or results (forward) belong to two
// pairs and all the workgroup's signals; read or written straight from the
// coefficient vectors, every lane would touch its own 4- or 8-byte piece of a
// different cache line.  Instead the workgroup moves them through LDS in
// rounds of all 16 pairs of the tile x 8 degree indices j, with thread
// (i, j) = (tid % 16, (tid / 16) % 8) handling coefficient (l_j, m_i, n_i) of
// its signals: 16 neighbouring lanes cover the 16 pairs' values of one degree
// and signal, which lie side by side in the coefficient vector (a whole
// 128-byte line for FP32) when the pairs share m.  LDS layout of a round:
// cst[i * PS + (j - j0) * CWP + 2 * signal + (re, im)].
template <class T, int BT, int NTHR>
struct CoefRound {
  static constexpr int JC = 8;                  // degree indices per round
  static constexpr int CW = 2 * BT, CWP = CW + 16, PS = JC * CWP + 4;
  static constexpr int STEP = NTHR / (PT * JC);  // signals between a thread's coefficients
  static constexpr int RPT = BT / STEP;          // coefficients per thread and round
  static constexpr size_t ELEMS = (size_t)PT * PS;
  static_assert(NTHR % (PT * JC) == 0 && BT % STEP == 0, "coefficient round split");

  // inverse: the scaled coefficients (2l+1 or 1) of the tile's pairs, degree
  // indices j0..j0+7, into LDS (zero past L or the batch; the Hermitian part
  // for real plans).  Ends with a barrier: the round is readable.
  __device__ static void gather(const cpx<T>* __restrict__ coeffs, const BetaParams<T>& p, int tile, int j0, int b0,
                                int nb, T* cst, int tid) {
    const int ci = tid % PT, cj = (tid / PT) % JC, cb0 = tid / (PT * JC);
    PairInfo pc = p.pairs[tile * PT + ci];
    if (p.real && mirrored_pair(pc.tm, pc.tn)) pc.L = 0;
    const T sg = (((pc.tm - pc.tn) / 2) & 1) ? T(-1) : T(1);
    const int j = j0 + cj;
    const bool jok = j < pc.L;
    const int tl = pc.tl0 + 2 * j;
    const int idx = jok ? coef_index_of(p.so3, tl, pc.tm, pc.tn) : 0;
    const int mdx = jok ? coef_index_of(p.so3, tl, -pc.tm, -pc.tn) : 0;
    // (2l+1) or 1, times the sign of a mirror column of a stored table
    const T sc = (p.scale_mode == 0 ? T(tl + 1) : T(1)) * ((p.table_signs && pc.tsign < 0) ? T(-1) : T(1));
    cpx<T> v[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) {  // every load issued unconditionally, masked afterwards
      const int bb = cb0 + r * STEP;
      const bool ok = jok && bb < nb;
      const cpx<T>* c = coeffs + coef_offset(p.coff, b0 + (bb < nb ? bb : 0), p.ncoef);
      v[r] = c[ok ? idx : 0];
      if (p.real) {
        // Hermitian part: (c_{mn} + (-1)^{m-n} conj(c_{-m,-n})) / 2
        const cpx<T> w = c[ok ? mdx : 0];
        v[r].re = T(0.5) * (v[r].re + sg * w.re);
        v[r].im = T(0.5) * (v[r].im - sg * w.im);
      }
      v[r].re = ok ? v[r].re * sc : T(0);
      v[r].im = ok ? v[r].im * sc : T(0);
    }
#pragma unroll
    for (int r = 0; r < RPT; r++) {
      T* d = cst + ci * PS + cj * CWP + 2 * (cb0 + r * STEP);
      d[0] = v[r].re;
      d[1] = v[r].im;
    }
    __syncthreads();
  }

  // forward: the sums parked in LDS for the tile's pairs, degree indices
  // j0..j0+7, out to the coefficient vectors (with the mirror
  // (-1)^{m-n} conj(fhat) at (-m, -n) for real plans).
  __device__ static void store(cpx<T>* __restrict__ coeffs, const BetaParams<T>& p, int tile, int j0, int b0, int nb,
                               const T* cst, int tid) {
    const int ci = tid % PT, cj = (tid / PT) % JC, cb0 = tid / (PT * JC);
    PairInfo pc = p.pairs[tile * PT + ci];
    if (p.real && mirrored_pair(pc.tm, pc.tn)) pc.L = 0;
    const int j = j0 + cj;
    if (j >= pc.L) return;
    const bool mirror = p.real && (pc.tm != 0 || pc.tn != 0);
    const T sg = (((pc.tm - pc.tn) / 2) & 1) ? T(-1) : T(1);
    const T ts = (p.table_signs && pc.tsign < 0) ? T(-1) : T(1);  // mirror column of a stored table
    const int tl = pc.tl0 + 2 * j;
    const int idx = coef_index_of(p.so3, tl, pc.tm, pc.tn);
    const int mdx = coef_index_of(p.so3, tl, -pc.tm, -pc.tn);
#pragma unroll
    for (int r = 0; r < RPT; r++) {
      const int bb = cb0 + r * STEP;
      if (bb < nb) {
        const T* src = cst + ci * PS + cj * CWP + 2 * bb;
        cpx<T> v;
        v.re = ts * src[0];
        v.im = ts * src[1];
        cpx<T>* c = coeffs + coef_offset(p.coff, b0 + bb, p.ncoef);
        c[idx] = v;
        if (mirror) {
          cpx<T> w;
          w.re = sg * v.re;
          w.im = -sg * v.im;
          c[mdx] = w;
        }
      }
    }
  }
};

// Forward contraction.  One workgroup per (pair tile, signal tile), in the
// order of contraction_slot; 8 waves; wave w owns pairs w and w + 8 of the
// tile.  The workgroup streams the tile's S slab and table rows through LDS
// in chunks of KC nodes, fetching chunk c+1 into registers (16-byte loads)
// while the matrix cores work on chunk c.
constexpr int FWD_THREADS = 512;

// KC: beta nodes per streamed chunk.  4 when the grid has at least 1.5
// workgroups per CU (fewer prefetch registers, two resident workgroups: FP32
// measured 14 % faster than 8 at B = 64 batch 32, FP64 19 % once its pair
// descriptors sit in scalar registers: 114 instead of 144 VGPRs), otherwise
// 8 (more bytes in flight per workgroup: measured better for grids of one
// workgroup per CU).  fwd_kc_default is the mixed plans' default.
template <class T>
constexpr int fwd_kc_default() { return sizeof(T) == 4 ? 4 : 8; }

template <class T, int RTMAX, int KC_ = fwd_kc_default<T>(), int BT_ = BetaCfg<T>::BT>
struct FwdGeom {
  static constexpr int KC = KC_;
  static constexpr int BT = BT_;
  static constexpr int PB = 2 * PT + 2;
  static constexpr int PK = BT * PB + 16;
  static constexpr int TMAX = PT * 16 * RTMAX;
  static constexpr int VE = 16 / (int)sizeof(T);
  static constexpr int TV = (KC * TMAX) / VE + 2;
  static constexpr int TVT = (TV + FWD_THREADS - 1) / FWD_THREADS;
  static constexpr size_t SMEM_LOOP = (size_t)(KC * PK + TVT * FWD_THREADS * VE) * sizeof(T);
  // the epilogue's coefficient rounds reuse the same LDS: 16 pairs x 8 degrees
  static constexpr size_t SMEM_EPI = (size_t)PT * ((2 * BT + 16) * 8 + 4) * sizeof(T);
  static constexpr size_t SMEM = SMEM_LOOP > SMEM_EPI ? SMEM_LOOP : SMEM_EPI;
};

// BT_ signals per workgroup: BetaCfg<T>::BT, or 16 for FP32 batches of at
// most 16, which would leave half of a 32-signal tile's columns empty.
template <class T, int RTMAX, int KC_ = fwd_kc_default<T>(), int BT_ = BetaCfg<T>::BT>
__device__ __forceinline__ void beta_forward_body(const cpx<T>* __restrict__ S, cpx<T>* __restrict__ coeffs,
                                                  const BetaParams<T>& p, int tile, int bt, unsigned char* smem, int tid) {
  typedef typename acc4<T>::type accT;
  constexpr int BT = BT_, CT = 2 * BT / 16;
  constexpr int KC = KC_;
  constexpr int PB = 2 * PT + 2;            // reals per (node, signal) row: 16 pairs x (re, im) + pad
  constexpr int PK = BT * PB + 16;          // reals per node
  constexpr int TMAX = PT * 16 * RTMAX;     // longest tile row
  constexpr int VE = 16 / (int)sizeof(T);   // table elements per 16-byte load
  constexpr int TV = (KC * TMAX) / VE + 2;  // 16-byte loads covering one table chunk
  constexpr int TVT = (TV + FWD_THREADS - 1) / FWD_THREADS;
  constexpr int VC = 16 / (int)sizeof(cpx<T>);            // complex values per 16-byte load
  constexpr int SV = KC * BT * PT / VC;                     // 16-byte loads per S chunk
  constexpr int SPT = SV / FWD_THREADS;
  static_assert(SV % FWD_THREADS == 0, "chunk split");
  T* sS = reinterpret_cast<T*>(smem);      // KC * PK reals (a multiple of 16 bytes)
  T* sT = sS + KC * PK;

  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  // the wave index is uniform: the pairs' descriptors load into scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lrow = lane & 15, lk = lane >> 4;
  const int N = p.N;
  const PairInfo p0 = p.pairs[tile * PT];
  const int lsum = p0.lsum;
  const long long tbase = p0.tab;                         // element offset of the tile block
  const long long vlast = (tbase + (long long)N * lsum + VE - 1) / VE;   // one past the block's last vector

  PairInfo pi[2];
#pragma unroll
  for (int i = 0; i < 2; i++) {
    pi[i] = p.pairs[tile * PT + wave + 8 * i];
    if (p.real && mirrored_pair(pi[i].tm, pi[i].tn)) pi[i].L = 0;
  }

  accT acc[2][RTMAX][CT];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[i][rt][ct][r] = T(0);

  typedef T vec16 __attribute__((ext_vector_type(16 / sizeof(T))));   // one 16-byte load of S, kept in T lanes
  vec16 sreg[SPT];
  float4 treg[TVT];
  const float4* tabv = reinterpret_cast<const float4*>(p.tab);
  long long tv0 = 0;  // first table vector of the chunk held in sT
  auto fetch = [&](int k0, long long& vstart) {
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
    // the chunk's table rows only: [k0 lsum, (k0 + KC) lsum) of the tile block
    vstart = (tbase + (long long)k0 * lsum) / VE;
    const long long vend = min(vlast, (tbase + (long long)(k0 + KC) * lsum + VE - 1) / VE);
#pragma unroll
    for (int i = 0; i < TVT; i++) {
      const long long v = vstart + tid + FWD_THREADS * i;
      if (tid + FWD_THREADS * i < TV && v < vend) treg[i] = tabv[v];
      else treg[i] = make_float4(0.f, 0.f, 0.f, 0.f);
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
#pragma unroll
    for (int i = 0; i < TVT; i++)
      reinterpret_cast<float4*>(sT)[tid + FWD_THREADS * i] = treg[i];
  };

  const int nchunk = (N + KC - 1) / KC;
  long long vnext = 0;
  fetch(0, tv0);
  commit();
  for (int c = 0; c < nchunk; c++) {
    __syncthreads();
    if (c + 1 < nchunk) fetch((c + 1) * KC, vnext);
    // position of this chunk's first table element inside sT
    const int toff = (int)(tbase + (long long)c * KC * lsum - tv0 * VE);
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
          const int cc = ct * 16 + lrow;  // column: signal cc / 2, re/im cc % 2
          bop[ct] = sS[kk * PK + (cc >> 1) * PB + 2 * pp + (cc & 1)];
        }
#pragma unroll
        for (int rt = 0; rt < RTMAX; rt++) {
          if (rt * 16 < L) {
            const int l = rt * 16 + lrow;
            const T a = (l < L && kin) ? sT[toff + kk * lsum + coff + l] : T(0);
#pragma unroll
            for (int ct = 0; ct < CT; ct++) acc[i][rt][ct] = mfma16x16x4(a, bop[ct], acc[i][rt][ct]);
          }
        }
      }
    }
    __syncthreads();
    if (c + 1 < nchunk) {
      commit();
      tv0 = vnext;
    }
  }

  // epilogue: the coefficients leave through LDS (CoefRound), 8 degrees of
  // all 16 pairs per round; each wave parks the rows of its two pairs that
  // fall in the round
  typedef CoefRound<T, BT, FWD_THREADS> CR;
  static_assert(CR::ELEMS * sizeof(T) <= FwdGeom<T, RTMAX, KC, BT>::SMEM, "coefficient rounds fit");
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

template <class T, int RTMAX, int KC, int BT>
__global__ __launch_bounds__(FWD_THREADS) void beta_forward_kernel(const cpx<T>* __restrict__ S,
                                                                   cpx<T>* __restrict__ coeffs, BetaParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileSlot sl = contraction_slot(blockIdx.x, p.ntiles - p.tile0, (p.batch + BT - 1) / BT, p.paired);
  if (!sl.valid) return;
  beta_forward_body<T, RTMAX, KC, BT>(S, coeffs, p, p.tile0 + sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// Inverse contraction.  One workgroup per (pair tile, signal tile), in the
// order of contraction_slot; 8 waves; wave w owns pairs w and w + 8.  Each
// wave keeps its pairs' scaled coefficients as matrix-core B operands in
// registers, then sweeps the N nodes in blocks of 16; a block's outputs for
// all 16 pairs are gathered in LDS and written as full PT-pair rows of S.
// The table values of the next block are requested before the current
// block's products (see fetch_a), and the stores of S stay in flight while
// the next block's products run.
constexpr int INV_THREADS = 512;

// staging buffer: 16 node rows of BT (signal) rows of PB reals, each node row
// padded by 4 reals so that the four accumulator row groups of a wave's
// stores fall into different LDS banks
template <class T>
struct InvStage {
  static constexpr int PB = 2 * PT + 2;
  static constexpr int NRS = BetaCfg<T>::BT * PB + 4;  // sized for the widest signal tile
};

template <class T>
constexpr size_t inverse_smem() { return (size_t)16 * InvStage<T>::NRS * sizeof(T); }

// BT signals per workgroup: BetaCfg<T>::BT, or 16 for FP32 batches of at
// most 16, which would leave half of a 32-signal tile's columns empty.
// WPP pairs per wave: 2 (8 waves, INV_THREADS threads) or 1 (16 waves):
// one pair per wave halves the coefficient operands each lane holds, which
// lets FP64 with 17-32 degrees keep 16 waves per CU instead of 8.
template <int WPP>
constexpr int inverse_threads() { return 64 * PT / WPP; }
// pairs per wave of the inverse for a type and degree-group count: one for
// FP64 with 17-32 degrees (B = 33-64: 110 instead of 176 VGPRs, 16 waves per
// CU instead of 8, B = 64 batch 32 0.187 -> 0.167 ms; with fewer degrees the
// 8-wave form is as fast or faster), else two
template <class T>
constexpr int inverse_wpp(int lq) { return sizeof(T) == 8 && lq == 8 ? 1 : 2; }

template <class T, int LQ, int BT = BetaCfg<T>::BT, int WPP = 2>
__device__ __forceinline__ void beta_inverse_body(const cpx<T>* __restrict__ coeffs, cpx<T>* __restrict__ S,
                                                  const BetaParams<T>& p, int tile, int bt, unsigned char* smem, int tid) {
  constexpr int NTH = inverse_threads<WPP>(), PW = PT / WPP;  // threads; pair stride between a wave's pairs
  typedef typename acc4<T>::type accT;
  constexpr int CT = 2 * BT / 16;
  static_assert(BT <= BetaCfg<T>::BT && BT % 8 == 0, "signal tile");
  constexpr int PB = InvStage<T>::PB, NRS = InvStage<T>::NRS;
  T* stage = reinterpret_cast<T*>(smem);
  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lrow = lane & 15, lk = lane >> 4;
  const int N = p.N;

  PairInfo pi[WPP];
#pragma unroll
  for (int q = 0; q < WPP; q++) {
    pi[q] = p.pairs[tile * PT + wave + PW * q];
    if (p.real && mirrored_pair(pi[q].tm, pi[q].tn)) pi[q].L = 0;
  }

  // table values of a block of 16 nodes: A operands (row = node, col =
  // degree), from the inverse-layout table: one load of 64 consecutive
  // values per group of 4 degrees (zeros past N and L are stored there).
  // The next block's values are requested before this block's products, so
  // they have the whole block (products, staging, stores) to arrive; where
  // two register sets do not fit (FP64 with 64 degrees), after the products.
  // FP32 with 64 degrees in 16-signal tiles (B = 128, batches of at most 16)
  // also fetches late: without the second set the kernel fits 128 VGPRs and
  // two workgroups share a CU (B = 128 batch 16: 0.502 -> 0.474 ms).
  constexpr bool EARLY = sizeof(T) * LQ <= 64 && !(LQ == 16 && BT == 16);
  T av[WPP][LQ], avn[WPP][LQ];
  auto fetch_a = [&](T (&dst)[WPP][LQ], int kb) {
#pragma unroll
    for (int q = 0; q < WPP; q++) {
      const T* src = p.tabi + pi[q].itab + (long long)kb * ((pi[q].L + 3) / 4) * 64 + lane;
#pragma unroll
      for (int s = 0; s < LQ; s++) {
        dst[q][s] = T(0);
        if (4 * s < pi[q].L) dst[q][s] = src[64 * s];  // wave-uniform branch
      }
    }
  };
  fetch_a(av, 0);  // in flight while the coefficients are gathered

  // B operands: the scaled coefficients of the wave's WPP pairs, gathered
  // through LDS (CoefRound) in rounds of 8 degrees of all 16 pairs
  constexpr int J = 4 * LQ;  // degrees held per pair
  typedef CoefRound<T, BT, NTH> CR;
  static_assert(CR::ELEMS <= (size_t)16 * NRS && J % CR::JC == 0, "coefficient rounds fit in the stage buffer");
  T bop[WPP][LQ][CT];
#pragma unroll
  for (int j0 = 0; j0 < J; j0 += CR::JC) {
    CR::gather(coeffs, p, tile, j0, b0, nb, stage, tid);
#pragma unroll
    for (int h = 0; h < WPP; h++)
#pragma unroll
      for (int s = j0 / 4; s < (j0 + CR::JC) / 4; s++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          bop[h][s][ct] = stage[(wave + PW * h) * CR::PS + (4 * s - j0 + lk) * CR::CWP + ct * 16 + lrow];
    __syncthreads();
  }

  // the tile's slab of S as a buffer resource: stores of rows whose node or
  // signal does not exist get an offset past the slab, and the hardware range
  // check drops them; every lane issues the same unconditional stores
  constexpr int VC = 16 / (int)sizeof(cpx<T>);
  constexpr int NV = 16 * BT * (PT / VC);  // 16-byte stores per block of 16 nodes
  static_assert(NV % NTH == 0, "store split");
  const long long slab = (long long)N * p.batch * PT;
  const __amdgpu_buffer_rsrc_t srsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(S + (size_t)tile * slab), (short)0, (int)(slab * (long long)sizeof(cpx<T>)), BUFFER_RSRC_WORD3);
  for (int k0 = 0; k0 < N; k0 += 16) {
    if constexpr (EARLY)
      if (k0 + 16 < N) fetch_a(avn, k0 / 16 + 1);
#pragma unroll
    for (int q = 0; q < WPP; q++) {
      const int L = pi[q].L;
      const int pp = wave + PW * q;
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
    if constexpr (!EARLY)
      if (k0 + 16 < N) fetch_a(av, k0 / 16 + 1);
    __syncthreads();
    // write the block: rows (node, signal) of PT pairs, 16 bytes per store.
    // The thread index passes through an empty asm statement so that the
    // store addresses are formed here rather than hoisted out of the node
    // loop, where they would hold registers throughout.
    int tq = tid;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int i = 0; i < NV / NTH; i++) {
      const int v = tq + NTH * i;
      const int row = v / (PT / VC), pv = v - row * (PT / VC);
      const int kk = row / BT, bb = row - kk * BT;
      const int k = k0 + kk;
      const T* src = stage + kk * NRS + bb * PB + 2 * pv * VC;
      u32x4 w;
      T* wd = reinterpret_cast<T*>(&w);
#pragma unroll
      for (int e = 0; e < 2 * VC; e++) wd[e] = src[e];
      const unsigned off = (k < N && bb < nb)
                               ? (unsigned)((((long long)k * p.batch + b0 + bb) * PT + pv * VC) * (long long)sizeof(cpx<T>))
                               : 0x80000000u;
      __builtin_amdgcn_raw_buffer_store_b128(w, srsrc, off, 0, 0);
    }
    __syncthreads();
    if constexpr (EARLY) {
#pragma unroll
      for (int q = 0; q < WPP; q++)
#pragma unroll
        for (int s = 0; s < LQ; s++) av[q][s] = avn[q][s];
    }
  }
}

template <class T, int LQ, int BT, int WPP>
__global__ __launch_bounds__(inverse_threads<WPP>()) void beta_inverse_kernel(const cpx<T>* __restrict__ coeffs,
                                                                              cpx<T>* __restrict__ S, BetaParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the inverse keeps the natural order (tiles with a shared block far apart
  // in time): measured 2-3 % faster than pairing them, unlike the forward
  const TileSlot sl = contraction_slot(blockIdx.x, p.ntiles - p.tile0, (p.batch + BT - 1) / BT);
  if (!sl.valid) return;
  beta_inverse_body<T, LQ, BT, WPP>(coeffs, S, p, p.tile0 + sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// allow the kernel `smem` bytes of dynamic LDS (beyond the 64 KB default)
template <class K>
static hipError_t set_smem(K kern, size_t smem) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
}

template <class T, int RTMAX, int KC, int BT>
static hipError_t launch_forward_shape(const BetaParams<T>& p, dim3 grid, const cpx<T>* S, cpx<T>* coeffs,
                                       hipStream_t s) {
  constexpr size_t smem = FwdGeom<T, RTMAX, KC, BT>::SMEM;
  hipError_t e;
  if ((e = set_smem(beta_forward_kernel<T, RTMAX, KC, BT>, smem)) != hipSuccess) return e;
  hipLaunchKernelGGL((beta_forward_kernel<T, RTMAX, KC, BT>), grid, dim3(FWD_THREADS), smem, s, S, coeffs, p);
  return hipGetLastError();
}

template <class T, int RTMAX, int BT>
static hipError_t launch_forward_rt(const BetaParams<T>& p, dim3 grid, const cpx<T>* S, cpx<T>* coeffs,
                                    hipStream_t s) {
  // two resident workgroups per CU pay off once most CUs get two (grids of
  // at least 1.5 workgroups per CU)
  if (2LL * grid.x >= 3LL * device_cus()) return launch_forward_shape<T, RTMAX, 4, BT>(p, grid, S, coeffs, s);
  return launch_forward_shape<T, RTMAX, 8, BT>(p, grid, S, coeffs, s);
}

// 16-signal tiles instead of the widest (FP32): for batches of at most 16,
// and where the widest tiles would leave fewer than 1.5 workgroups per CU
// (real-signal and SO(3) plans at B = 64 batch 32 contract about 250 pair
// tiles), so that most CUs hold two workgroups
template <class T>
bool narrow_tiles(const BetaParams<T>& p, int units) {
  constexpr int BTW = BetaCfg<T>::BT;
  if (BTW <= 16) return false;
  return p.batch <= 16 || 2LL * units * ((p.batch + BTW - 1) / BTW) < 3LL * device_cus();
}

template <class T>
hipError_t launch_beta_forward(const BetaParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, hipStream_t s) {
  constexpr int BTW = BetaCfg<T>::BT;      // widest signal tile
  constexpr int BTN = BTW > 16 ? 16 : BTW;  // narrow tiles (narrow_tiles)
  const int rt = beta_rtmax(p.B);
  if (BTN != BTW && narrow_tiles(p, p.ntiles - p.tile0)) {
    const dim3 grid(contraction_grid(p.ntiles - p.tile0, (p.batch + BTN - 1) / BTN, p.paired));
    if (rt == 1) return launch_forward_rt<T, 1, BTN>(p, grid, S, coeffs, s);
    if (rt == 2) return launch_forward_rt<T, 2, BTN>(p, grid, S, coeffs, s);
    return launch_forward_rt<T, 4, BTN>(p, grid, S, coeffs, s);
  }
  const dim3 grid(contraction_grid(p.ntiles - p.tile0, (p.batch + BTW - 1) / BTW, p.paired));
  if (rt == 1) return launch_forward_rt<T, 1, BTW>(p, grid, S, coeffs, s);
  if (rt == 2) return launch_forward_rt<T, 2, BTW>(p, grid, S, coeffs, s);
  return launch_forward_rt<T, 4, BTW>(p, grid, S, coeffs, s);
}

template <class T>
hipError_t launch_beta_inverse(const BetaParams<T>& p, const cpx<T>* coeffs, cpx<T>* S, hipStream_t s) {
  constexpr int BTW = BetaCfg<T>::BT;                             // widest signal tile
  constexpr int BTN = BTW > 16 ? 16 : BTW;                         // narrow tiles (narrow_tiles)
  const int bt = narrow_tiles(p, p.ntiles - p.tile0) ? BTN : BTW;
  const dim3 grid(contraction_grid(p.ntiles - p.tile0, (p.batch + bt - 1) / bt));
  const size_t smem = inverse_smem<T>();
  const int lq = beta_lq(p.B);
  hipError_t e;
#define SU2_INV_CASE(Q, BTC)                                                                             \
  if (lq == Q && bt == BTC) {                                                                            \
    constexpr int W = inverse_wpp<T>(Q);                                                                 \
    if ((e = set_smem(beta_inverse_kernel<T, Q, BTC, W>, smem)) != hipSuccess) return e;                 \
    hipLaunchKernelGGL((beta_inverse_kernel<T, Q, BTC, W>), grid, dim3(inverse_threads<W>()), smem, s, coeffs, \
                       S, p);                                                                            \
    return hipGetLastError();                                                                            \
  }
  SU2_INV_CASE(2, BTW)
  SU2_INV_CASE(4, BTW)
  SU2_INV_CASE(8, BTW)
  SU2_INV_CASE(16, BTW)
  if constexpr (BTN != BTW) {
    SU2_INV_CASE(2, BTN)
    SU2_INV_CASE(4, BTN)
    SU2_INV_CASE(8, BTN)
    SU2_INV_CASE(16, BTN)
  }
#undef SU2_INV_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_beta_forward<float>(const BetaParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_beta_forward<double>(const BetaParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);
template hipError_t launch_beta_inverse<float>(const BetaParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_beta_inverse<double>(const BetaParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);

}  // namespace su2
