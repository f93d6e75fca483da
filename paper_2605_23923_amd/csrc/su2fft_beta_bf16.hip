// Beta contraction in split bfloat16 ("BF16x3"): every FP32 operand x is
// carried as x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to
// nearest even), and a product A B is formed on the matrix cores as
// A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation (the lo*lo term,
// about 2^-16 relative, is dropped).  The contraction itself is the one of
// the FP32 path (the inner products <s, P^l_{nm}> of Section 4 for every
// pair); only the arithmetic of the matrix products changes.
//
// Instruction: V_MFMA_F32_16X16X32_BF16, A 16x32, B 32x16, lane l holding
// A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i = 0..7, and
// the accumulator D[4 (l / 16) + r][l % 16] (all measured).
//
// Tables (hi in the low 16 bits, lo in the high 16 bits of a 32-bit word):
//   forward: [tile][k / 8][column j = coff + i][k % 8]  (a lane's 8 nodes are
//            one aligned 32-byte load), rows k >= N zero;
//   inverse: the tile-major [tile][k][lsum] layout of the other paths.
#include "su2fft_internal.h"

namespace su2 {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_rne_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

__device__ __forceinline__ floatx4 mfma_bf16(u16x8 a, u16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                  0);
}

// split eight FP32 values into their bf16 hi and lo parts
__device__ __forceinline__ void split8(const float* v, u16x8& hi, u16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const unsigned short h = bf16_rne_bits(v[i]);
    hi[i] = h;
    lo[i] = bf16_rne_bits(v[i] - bf16_bits_to_f32(h));
  }
}

// eight table words -> hi and lo operands
__device__ __forceinline__ void unpack8(const unsigned* w, u16x8& hi, u16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    hi[i] = (unsigned short)(w[i] & 0xffffu);
    lo[i] = (unsigned short)(w[i] >> 16);
  }
}

constexpr int XB_THREADS = 512;
constexpr int XB_BT = 32;   // inverse: signals per workgroup (64 real columns)
constexpr int XBF_BT = 16;  // forward: signals per workgroup (a 32-node S chunk is 64 KB)
constexpr int XB_KC = 32;   // nodes per chunk = K of one matrix instruction

// Forward.  One workgroup per (pair tile, signal tile), in the order of
// contraction_slot; wave w owns pairs w and w + 8.
// S streams through LDS in chunks of 32 nodes with register prefetch; the
// table operand is read straight from the node-interleaved layout.
constexpr size_t XBF_SMEM = (size_t)XB_KC * (XBF_BT * (2 * PT + 2) + 16) * sizeof(float);
constexpr size_t XBI_SMEM = (size_t)16 * XB_BT * (2 * PT + 2) * sizeof(float);

// EARLY: the table operands of a chunk are requested together at its start.
// Measured at four row tiles (B = 128 batch 16: 0.495 -> 0.476 ms); at two
// (B = 64) the requests inside the tile loop are 1-2 % faster.  The
// work-list kernel of mixed plans, with less register room, keeps them there.
template <int RTMAX, bool EARLY = (RTMAX >= 4)>
__device__ __forceinline__ void beta_forward_bf16x3_body(const cpx<float>* __restrict__ S,
                                                         cpx<float>* __restrict__ coeffs, const BetaParams<float>& p,
                                                         const unsigned* __restrict__ tabf, int tile, int bt,
                                                         unsigned char* smem, int tid) {
  constexpr int BT = XBF_BT, CT = 2 * BT / 16, KC = XB_KC;
  constexpr int PB = 2 * PT + 2;
  constexpr int PK = BT * PB + 16;
  constexpr int VC = 2;                         // complex values per 16-byte load
  constexpr int SV = KC * BT * PT / VC;
  constexpr int SPT = SV / XB_THREADS;
  static_assert(SV % XB_THREADS == 0, "chunk split");
  float* sS = reinterpret_cast<float*>(smem);

  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  // the wave index is uniform: the pairs' descriptors load into scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lrow = lane & 15, lg = lane >> 4;
  const int N = p.N;
  const int NB8 = (N + 7) / 8;
  const PairInfo p0 = p.pairs[tile * PT];
  const int lsum = p0.lsum;
  // the node-interleaved table holds NB8 * 8 rows per tile: its tile block starts
  // at (tab / N) * NB8 * 8, tab being the tile offset in the [k][lsum] layout
  const unsigned* tb = tabf + (p0.tab / N) * (long long)NB8 * 8;

  PairInfo pi[2];
#pragma unroll
  for (int i = 0; i < 2; i++) {
    pi[i] = p.pairs[tile * PT + wave + 8 * i];
    if (p.real && mirrored_pair(pi[i].tm, pi[i].tn)) pi[i].L = 0;  // its coefficients come from the mirror
  }

  floatx4 acc[2][RTMAX][CT];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int rt = 0; rt < RTMAX; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++) acc[i][rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};

  // HALF: the next chunk's first half is requested before the current
  // chunk's products and its second half after them, so that the prefetch
  // holds half the registers
  constexpr bool HALF = RTMAX == 2 && !EARLY;
  constexpr int SH = HALF ? SPT / 2 : SPT;
  float4 sreg[SH];
  auto fetch = [&](int k0, int h) {
#pragma unroll
    for (int ii = 0; ii < SH; ii++) {
      const int i = h * SH + ii;
      const int v = tid + XB_THREADS * i;
      const int kk = v / (BT * PT / VC), rem = v - kk * (BT * PT / VC);
      const int bb = rem / (PT / VC), pv = rem - bb * (PT / VC);
      const int k = k0 + kk;
      if (k < N && bb < nb)
        sreg[ii] = *reinterpret_cast<const float4*>(S + (((size_t)tile * N + k) * p.batch + b0 + bb) * PT + pv * VC);
      else
        sreg[ii] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto commit = [&](int h) {
#pragma unroll
    for (int ii = 0; ii < SH; ii++) {
      const int i = h * SH + ii;
      const int v = tid + XB_THREADS * i;
      const int kk = v / (BT * PT / VC), rem = v - kk * (BT * PT / VC);
      const int bb = rem / (PT / VC), pv = rem - bb * (PT / VC);
      float* d = sS + kk * PK + bb * PB + 2 * pv * VC;
      d[0] = sreg[ii].x; d[1] = sreg[ii].y; d[2] = sreg[ii].z; d[3] = sreg[ii].w;
    }
  };

  const int nchunk = (N + KC - 1) / KC;
  fetch(0, 0);
  commit(0);
  if constexpr (HALF) {
    fetch(0, 1);
    commit(1);
  }
  for (int c = 0; c < nchunk; c++) {
    __syncthreads();
    if (c + 1 < nchunk) fetch((c + 1) * KC, 0);
    const int kb = c * (KC / 8) + lg;  // this lane's group of 8 nodes
    // the chunk's table operands of both pairs, requested together before
    // any of them is used (an index out of range reads the table's first
    // row and is masked to zero), so their latencies overlap
    uint4 tw[2][RTMAX][2];
    bool tok[2][RTMAX];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int rt = 0; rt < RTMAX; rt++) {
        const int l = rt * 16 + lrow;
        tok[i][rt] = l < pi[i].L && kb < NB8;
        if constexpr (EARLY) {
          const uint4* src = reinterpret_cast<const uint4*>(
              tok[i][rt] ? tb + ((size_t)kb * lsum + pi[i].coff + l) * 8 : tabf);
          tw[i][rt][0] = src[0];
          tw[i][rt][1] = src[1];
        }
      }
#pragma unroll
    for (int i = 0; i < 2; i++) {
      const int L = pi[i].L;
      if (L == 0) continue;
      const int pp = wave + 8 * i;
      // B operands: 8 consecutive nodes of one column, split into hi and lo
      u16x8 bhi[CT], blo[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int cc = ct * 16 + lrow;
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = sS[(8 * lg + q) * PK + (cc >> 1) * PB + 2 * pp + (cc & 1)];
        split8(v, bhi[ct], blo[ct]);
      }
#pragma unroll
      for (int rt = 0; rt < RTMAX; rt++) {
        if (rt * 16 < L) {
          u16x8 ahi, alo;
          if (tok[i][rt]) {
            if constexpr (!EARLY) {
              const uint4* src =
                  reinterpret_cast<const uint4*>(tb + ((size_t)kb * lsum + pi[i].coff + rt * 16 + lrow) * 8);
              tw[i][rt][0] = src[0];
              tw[i][rt][1] = src[1];
            }
            const uint4 w0 = tw[i][rt][0], w1 = tw[i][rt][1];
            const unsigned w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
            unpack8(w, ahi, alo);
          } else {
#pragma unroll
            for (int q = 0; q < 8; q++) { ahi[q] = 0; alo[q] = 0; }
          }
#pragma unroll
          for (int ct = 0; ct < CT; ct++) {
            acc[i][rt][ct] = mfma_bf16(ahi, bhi[ct], acc[i][rt][ct]);
            acc[i][rt][ct] = mfma_bf16(ahi, blo[ct], acc[i][rt][ct]);
            acc[i][rt][ct] = mfma_bf16(alo, bhi[ct], acc[i][rt][ct]);
          }
        }
      }
    }
    __syncthreads();
    if (c + 1 < nchunk) {
      commit(0);
      if constexpr (HALF) {
        fetch((c + 1) * KC, 1);
        commit(1);
      }
    }
  }

  // epilogue: the coefficients leave through LDS (CoefRound), 8 degrees of
  // all 16 pairs per round
  typedef CoefRound<float, BT, XB_THREADS> CR;
  static_assert(CR::ELEMS * sizeof(float) <= XBF_SMEM, "coefficient rounds fit");
  float* cst = reinterpret_cast<float*>(smem);
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
            const int row = 4 * lg + r - r0;
            if (row >= 0 && row < CR::JC) cst[(wave + 8 * h) * CR::PS + row * CR::CWP + ct * 16 + lrow] = acc[h][rt][ct][r];
          }
      }
    }
    __syncthreads();
    CR::store(coeffs, p, tile, j0, b0, nb, cst, tid);
  }
}

template <int RTMAX>
__global__ __launch_bounds__(XB_THREADS, RTMAX == 2 ? 4 : 1) void beta_forward_bf16x3_kernel(const cpx<float>* __restrict__ S,
                                                                         cpx<float>* __restrict__ coeffs,
                                                                         BetaParams<float> p,
                                                                         const unsigned* __restrict__ tabf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileSlot sl = contraction_slot(blockIdx.x, p.ntiles - p.tile0, (p.batch + XBF_BT - 1) / XBF_BT, p.paired);
  if (!sl.valid) return;
  beta_forward_bf16x3_body<RTMAX>(S, coeffs, p, tabf, p.tile0 + sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// Inverse.  One workgroup per (pair tile, signal tile), in the order of
// contraction_slot; wave w owns pairs w and w + 8 and
// keeps their split, scaled coefficients as B operands (32 degrees per
// instruction), gathered through LDS like the FP32 path's; the nodes are swept
// in blocks of 16 (the table words of the next block requested before the
// current block's products) and staged through LDS so that S is written in
// whole 16-pair rows, by buffer stores that stay in flight across the next
// block's products.  BT signals per workgroup: 32, or 16 for batches of at
// most 16, which would leave half of a 32-signal tile's columns empty.
template <int LQ, int BT = XB_BT>
__device__ __forceinline__ void beta_inverse_bf16x3_body(const cpx<float>* __restrict__ coeffs,
                                                         cpx<float>* __restrict__ S, const BetaParams<float>& p,
                                                         const unsigned* __restrict__ tabi, int tile, int bt,
                                                         unsigned char* smem, int tid) {
  constexpr int CT = 2 * BT / 16;
  static_assert(BT == 16 || BT == 32, "signal tile");
  constexpr int PB = 2 * PT + 2;
  float* stage = reinterpret_cast<float*>(smem);
  const int b0 = bt * BT;
  const int nb = min(BT, p.batch - b0);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lrow = lane & 15, lg = lane >> 4;
  const int N = p.N;
  const PairInfo p0 = p.pairs[tile * PT];
  const int lsum = p0.lsum;
  const unsigned* tb = tabi + p0.tab;

  PairInfo pi[2];
#pragma unroll
  for (int q = 0; q < 2; q++) {
    pi[q] = p.pairs[tile * PT + wave + 8 * q];
    if (p.real && mirrored_pair(pi[q].tm, pi[q].tn)) pi[q].L = 0;  // its spectra are never read
  }

  // B operands: lane (lrow, lg) holds degrees 32 s + 8 lg + i, i = 0..7, of
  // column ct * 16 + lrow; a round of 8 degrees (CoefRound) is exactly one
  // lane group's 8 degrees
  constexpr int J = 32 * LQ;
  typedef CoefRound<float, BT, XB_THREADS> CR;
  static_assert(CR::ELEMS * sizeof(float) <= XBI_SMEM && CR::JC == 8, "coefficient rounds fit in the stage buffer");
  u16x8 bhi[2][LQ][CT], blo[2][LQ][CT];
#pragma unroll
  for (int j0 = 0; j0 < J; j0 += 8) {
    CR::gather(coeffs, p, tile, j0, b0, nb, stage, tid);
    const int s = j0 / 32;
    if (8 * lg == j0 % 32) {
#pragma unroll
      for (int q = 0; q < 2; q++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
          float v[8];
#pragma unroll
          for (int i = 0; i < 8; i++) v[i] = stage[(wave + 8 * q) * CR::PS + i * CR::CWP + ct * 16 + lrow];
          split8(v, bhi[q][s][ct], blo[q][s][ct]);
        }
    }
    __syncthreads();
  }

  // table words of a block of 16 nodes: lane (lrow, lg) reads 8 consecutive
  // degrees of node k0 + lrow (rows past N read row N - 1 and are never
  // stored; degrees past L read the words that follow in the tile block, or
  // the zeroed table padding, and meet zero B operands)
  // The next block's words are requested before this block's products,
  // except with two 32-degree groups in 16-signal tiles (B = 128, batches of
  // at most 16): there they are requested after the products, so that one
  // register set suffices and two workgroups share a CU.
  constexpr bool EARLY = !(LQ == 2 && BT == 16);
  unsigned aw[2][LQ][8], awn[2][LQ][8];
  auto fetch_a = [&](unsigned (&dst)[2][LQ][8], int k0) {
    const int k = k0 + lrow < N ? k0 + lrow : N - 1;
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const unsigned* trow = tb + (size_t)k * lsum + pi[q].coff + 8 * lg;
#pragma unroll
      for (int s = 0; s < LQ; s++) {
#pragma unroll
        for (int i = 0; i < 8; i++) dst[q][s][i] = 0u;
        if (32 * s < pi[q].L) {  // wave-uniform branch
#pragma unroll
          for (int i = 0; i < 8; i++) dst[q][s][i] = trow[32 * s + i];
        }
      }
    }
  };
  constexpr int NV = 16 * BT * (PT / 2);  // 16-byte stores per block of 16 nodes
  static_assert(NV % XB_THREADS == 0, "store split");
  const long long slab = (long long)N * p.batch * PT;
  const __amdgpu_buffer_rsrc_t srsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(S + (size_t)tile * slab), (short)0, (int)(slab * (long long)sizeof(cpx<float>)), BUFFER_RSRC_WORD3);
  fetch_a(aw, 0);
  for (int k0 = 0; k0 < N; k0 += 16) {
    if constexpr (EARLY)
      if (k0 + 16 < N) fetch_a(awn, k0 + 16);
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const int L = pi[q].L;
      const int pp = wave + 8 * q;
      floatx4 acc[CT];
#pragma unroll
      for (int ct = 0; ct < CT; ct++) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < LQ; s++) {
        if (32 * s < L) {
          u16x8 ahi, alo;
          unpack8(aw[q][s], ahi, alo);
#pragma unroll
          for (int ct = 0; ct < CT; ct++) {
            acc[ct] = mfma_bf16(ahi, bhi[q][s][ct], acc[ct]);
            acc[ct] = mfma_bf16(ahi, blo[q][s][ct], acc[ct]);
            acc[ct] = mfma_bf16(alo, bhi[q][s][ct], acc[ct]);
          }
        }
      }
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int cc = ct * 16 + lrow;
        const int bb = cc >> 1, reim = cc & 1;
#pragma unroll
        for (int r = 0; r < 4; r++) stage[((4 * lg + r) * BT + bb) * PB + 2 * pp + reim] = acc[ct][r];
      }
    }
    if constexpr (!EARLY)
      if (k0 + 16 < N) fetch_a(aw, k0 + 16);  // in flight during the staging and the stores
    __syncthreads();
    // the thread index passes through an empty asm statement so that the
    // store addresses are formed here, not hoisted out of the node loop
    int tq = tid;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int i = 0; i < NV / XB_THREADS; i++) {
      const int v = tq + XB_THREADS * i;
      const int row = v / (PT / 2), pv = v - row * (PT / 2);
      const int kk = row / BT, bb = row - kk * BT;
      const int k = k0 + kk;
      const float* src = stage + row * PB + 4 * pv;
      u32x4 w;
      float* wd = reinterpret_cast<float*>(&w);
#pragma unroll
      for (int e = 0; e < 4; e++) wd[e] = src[e];
      const unsigned off = (k < N && bb < nb)
                               ? (unsigned)((((long long)k * p.batch + b0 + bb) * PT + 2 * pv) * (long long)sizeof(cpx<float>))
                               : 0x80000000u;  // past the slab: dropped by the range check
      __builtin_amdgcn_raw_buffer_store_b128(w, srsrc, off, 0, 0);
    }
    __syncthreads();
    if constexpr (EARLY) {
#pragma unroll
      for (int q = 0; q < 2; q++)
#pragma unroll
        for (int s = 0; s < LQ; s++)
#pragma unroll
          for (int i = 0; i < 8; i++) aw[q][s][i] = awn[q][s][i];
    }
  }
}

template <int LQ, int BT>
__global__ __launch_bounds__(XB_THREADS) void beta_inverse_bf16x3_kernel(const cpx<float>* __restrict__ coeffs,
                                                                         cpx<float>* __restrict__ S,
                                                                         BetaParams<float> p,
                                                                         const unsigned* __restrict__ tabi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileSlot sl = contraction_slot(blockIdx.x, p.ntiles - p.tile0, (p.batch + BT - 1) / BT);  // natural order
  if (!sl.valid) return;
  beta_inverse_bf16x3_body<LQ, BT>(coeffs, S, p, tabi, p.tile0 + sl.tile, sl.bt, smem_raw, threadIdx.x);
}

// Reorder the tile-major split table into the node-interleaved forward layout.
// Grid: (chunks of one tile block, tiles).
__global__ void interleave_bf16_table_kernel(int N, const PairInfo* __restrict__ pairs, const bf16x2_t* __restrict__ src,
                                             unsigned* __restrict__ dst) {
  const int NB8 = (N + 7) / 8;
  const PairInfo p0 = pairs[blockIdx.y * PT];
  if (!p0.towner) return;  // a mirror tile: its block is its mirror's
  const long long cnt = (long long)NB8 * 8 * p0.lsum;
  const long long base = (p0.tab / N) * (long long)NB8 * 8;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / p0.lsum), j = (int)(e - (long long)k * p0.lsum);
    unsigned w = 0u;
    if (k < N) {
      const bf16x2_t v = src[p0.tab + (long long)k * p0.lsum + j];
      w = (unsigned)v.hi | ((unsigned)v.lo << 16);
    }
    dst[base + ((long long)(k / 8) * p0.lsum + j) * 8 + (k % 8)] = w;
  }
}

template <class K>
static hipError_t set_smem_bf(K kern, size_t smem) {
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
}

hipError_t launch_beta_forward_bf16x3(const BetaParams<float>& p, const unsigned* tabf, const cpx<float>* S,
                                      cpx<float>* coeffs, hipStream_t s) {
  const dim3 grid(contraction_grid(p.ntiles - p.tile0, (p.batch + XBF_BT - 1) / XBF_BT, p.paired));
  const int rt = beta_rtmax(p.B);
  hipError_t e;
#define SU2_XBF_CASE(R)                                                                                           \
  if (rt == R) {                                                                                                  \
    if ((e = set_smem_bf(beta_forward_bf16x3_kernel<R>, XBF_SMEM)) != hipSuccess) return e;                       \
    hipLaunchKernelGGL((beta_forward_bf16x3_kernel<R>), grid, dim3(XB_THREADS), XBF_SMEM, s, S, coeffs, p, tabf); \
    return hipGetLastError();                                                                                     \
  }
  SU2_XBF_CASE(1)
  SU2_XBF_CASE(2)
  SU2_XBF_CASE(4)
#undef SU2_XBF_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_beta_inverse_bf16x3(const BetaParams<float>& p, const unsigned* tabi, const cpx<float>* coeffs,
                                      cpx<float>* S, hipStream_t s) {
  // 16-signal tiles for batches of at most 16, and where the widest would
  // leave fewer than 1.5 workgroups per CU (as for the FP32 contractions)
  const bool narrow =
      p.batch <= 16 || 2LL * (p.ntiles - p.tile0) * ((p.batch + XB_BT - 1) / XB_BT) < 3LL * device_cus();
  const int bt = narrow ? 16 : XB_BT;
  const dim3 grid(contraction_grid(p.ntiles - p.tile0, (p.batch + bt - 1) / bt));
  const int lq2 = beta_bf16_lq(p.B);
  hipError_t e;
#define SU2_XBI_CASE(Q, BTC)                                                                                  \
  if (lq2 == Q && bt == BTC) {                                                                                \
    if ((e = set_smem_bf(beta_inverse_bf16x3_kernel<Q, BTC>, XBI_SMEM)) != hipSuccess) return e;              \
    hipLaunchKernelGGL((beta_inverse_bf16x3_kernel<Q, BTC>), grid, dim3(XB_THREADS), XBI_SMEM, s, coeffs, S, p, \
                       tabi);                                                                                 \
    return hipGetLastError();                                                                                 \
  }
  SU2_XBI_CASE(1, XB_BT)
  SU2_XBI_CASE(2, XB_BT)
  SU2_XBI_CASE(1, 16)
  SU2_XBI_CASE(2, 16)
#undef SU2_XBI_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_interleave_bf16_table(int N, int ntiles, const PairInfo* pairs, const bf16x2_t* src, unsigned* dst,
                                        hipStream_t s) {
  hipLaunchKernelGGL(interleave_bf16_table_kernel, dim3(16, ntiles), dim3(256), 0, s, N, pairs, src, dst);
  return hipGetLastError();
}

}  // namespace su2
