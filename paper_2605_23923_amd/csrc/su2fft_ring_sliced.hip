// Ring FFT (stage 1, Proposition 4.2 / Proposition 6.1) for N = 256 nodes per
// angle in FP32, in one pass, with two workgroups per compute unit.
//
// A 256 x 256 ring (512 KB) is shared by four workgroups ("slices") that are
// dispatched side by side on one XCD (contraction_slot), so a ring's input
// comes from HBM once and from that XCD's L2 for the other slices.  Each
// slice keeps a 64 KB block in LDS and 64 KB in registers (512 threads x 16
// complex values), so that two slices share a compute unit and one's loads
// and stores overlap the other's arithmetic.  w_n = e^{2 pi i / n}.
//
// Forward, slice s holds the gamma frequencies q = 4 q' + s (q' < 64):
//   rows     G[j][q'] = sum_{l2 < 64} w64^{q' l2} w256^{s l2} sum_{l1 < 4} w4^{s l1} f[j][l2 + 64 l1]
//            (8 lanes per row: 8-point DFT, twiddle, exchange inside the wave, 8-point DFT)
//   split    the alpha sum over j = jl + 128 jh (jl < 128) by the parity of p:
//              E[jl] = h(jl) (G[jl] + i^delta G[jl + 128])              -> H[2 p'']
//              O[jl] = h(jl) w256^{jl} (G[jl] - i^delta G[jl + 128])    -> H[2 p'' + 1]
//            with h(j) = e^{i pi delta j / 256} the half-bin shift (delta = 1 on
//            odd q: half-integer n; never in SO(3) plans).  E goes to LDS, O
//            stays in registers.
//   columns  H[2 p'' + par][q] = sum_{jl < 128} w128^{p'' jl} (E or O)[jl]: a 16 x 8
//            transform per column (8 lanes), only p'' in [0, 32) and [96, 128),
//            i.e. the retained p in [0, 64) and [192, 256); E first, then O
//            moved into LDS and transformed the same way.  S_k = W_k i^e H.
// Inverse, slice s holds the rows j = 4 j' + s (j' < 64):
//   columns  G[4 j' + s][q] = h(4 j' + s)^* sum_{p' < 64} w64^{-p' j'} w256^{-p' s} (H[p'][q] + i^s H[p' + 192][q])
//            for every q (only p in [0, 64) and [192, 256) hold bins): odd q
//            first, kept in registers, then even q into LDS
//   rows     f[j][l] = A[l] + w256^{-l} B[l], f[j][l + 128] = A[l] - w256^{-l} B[l],
//            A, B the 128-point inverse transforms over the even and the odd q
//            (A from LDS, then the odd q moved into LDS for B).
// Every slice reads the whole ring (forward: samples; inverse: spectra), each
// once from HBM or L2, and writes its quarter of the output.
//
// LDS layout.  The block is row-major with 64 (forward: E[jl][q']) or 128
// (inverse: G[j'][q'']) complex words per row and the column index XORed
// with sw(row) = 8 (row mod 2) + (row mod 8 & 6).  A 64-bit LDS access serves
// 16 lanes at a time, one word in each of the 16 bank pairs (word w in pair w
// mod 16); with this swizzle every access below (row writes and reads,
// column writes and reads, and both in-wave exchanges, whose slot for value
// a of lane b is 8 a + ((a + b) mod 8)) meets 16 different bank pairs per 16
// lanes.  The in-wave exchanges need no workgroup barrier: a wave's LDS
// accesses take effect in program order.
#include "su2fft_internal.h"

namespace su2 {

constexpr int S4_NT = 512;   // threads per workgroup
constexpr int S4_N = 256;    // nodes per angle
constexpr int S4_SLC = 4;    // workgroups per ring
constexpr int S4_BW = 8192;  // complex words of the LDS block (64 KB)
constexpr size_t S4_SMEM = (size_t)(S4_BW + 2 * S4_N) * sizeof(cpx<float>);  // + e^{i pi t / 256}, t < 512
static_assert(2 * S4_SMEM <= 160 * 1024, "two workgroups per compute unit");

// orders this wave's LDS accesses before and after it (an exchange between
// lanes of one wave)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }

__device__ __forceinline__ int s4_sw(int row) { return ((row & 1) << 3) | (row & 6); }
// exchange slot of value a of lane b among the 8 lanes of a line
__device__ __forceinline__ int s4_slot(int a, int b) { return 8 * a + ((a + b) & 7); }

// v, hidden from the optimiser: twiddle reads indexed by it are issued where
// they are used instead of being hoisted out of the loops and held in
// registers (LDS reads are cheap; registers are the limit here)
__device__ __forceinline__ int s4_opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
// the same for a value known to lie in [0, R) (R a power of two): the mask
// hands the range back to the optimiser, so that tests on it still fold
template <int R>
__device__ __forceinline__ int s4_opaque_lt(int v) {
  return s4_opaque(v) & (R - 1);
}

// Element offset of pair index u in one ring's spectra (u >= -15: the
// offset of a pair 16 j further on is this plus j tile strides, also where
// u itself lies before the first pair)
__device__ __forceinline__ long long s4_off(int u, long long tile_stride) {
  return (long long)(u >> 4) * tile_stride + (u & 15);
}

// ---- forward ----

// The radix-4 step over l1 kept for slice SL: sum_{l1} w4^{SL l1} a_{l1}
template <int SL>
__device__ __forceinline__ cpx<float> s4_fold(cpx<float> a0, cpx<float> a1, cpx<float> a2, cpx<float> a3) {
  if constexpr (SL == 0) return cadd(cadd(a0, a1), cadd(a2, a3));
  else if constexpr (SL == 2) return csub(cadd(a0, a2), cadd(a1, a3));
  else if constexpr (SL == 1) return cadd(csub(a0, a2), mul_i(csub(a1, a3)));
  else return csub(csub(a0, a2), mul_i(csub(a1, a3)));
}

// Row phase of forward slice SL (a compile-time constant, so that the radix-4
// step and the twiddles take no branches): every row j of the ring, 8 lanes
// per row, rows jl and jl + 128 by the same lanes; E[jl] goes to the LDS
// block, O[jl] (two rows jl per thread) stays in registers.
template <bool REAL, int SL>
__device__ __forceinline__ void s4_rows_forward(const cpx<float>* __restrict__ samples, size_t x0, cpx<float>* E,
                                                const cpx<float>* tws, int t, int delta, cpx<float> (&O)[2][8]) {
  typedef float T;
  constexpr int N = S4_N;
  constexpr int M = 2 * N - 1;
  const int c = t & 7, rr = t >> 3;
#pragma unroll
  for (int hp = 0; hp < 2; hp++) {
    const int jl = rr + 64 * hp;
    cpx<T>* row = E + jl * 64;
    const int swr = s4_sw(jl);
    cpx<T> g[2][8];
#pragma unroll
    for (int half = 0; half < 2; half++) {
      const int j = jl + 128 * half;
      // the row's loads stay behind the previous row's transform (register budget)
      __builtin_amdgcn_sched_barrier(0);
      cpx<T> v[32];  // f[j][c + 8 m]
      if constexpr (REAL) {  // real samples (plain loads: the ring's other slices read them from L2)
        const T* xr = reinterpret_cast<const T*>(samples) + x0 + (size_t)j * N + c;
#pragma unroll
        for (int m = 0; m < 32; m++) v[m] = {xr[8 * m], opaque_zero<T>()};
      } else {
        const cpx<T>* xc = samples + x0 + (size_t)j * N + c;
#pragma unroll
        for (int m = 0; m < 32; m++) v[m] = xc[8 * m];
      }
      cpx<T> y[8];  // the radix-4 step over l1 kept for this slice: l2 = c + 8 m
#pragma unroll
      for (int m = 0; m < 8; m++) y[m] = s4_fold<SL>(v[m], v[m + 8], v[m + 16], v[m + 24]);
      // twiddle reads where they are used (register budget)
      __builtin_amdgcn_sched_barrier(0);
      const int cl = s4_opaque_lt<8>(c);
      if constexpr (SL != 0) {
#pragma unroll
        for (int m = 0; m < 8; m++) y[m] = cmul(y[m], tws[(2 * SL * (cl + 8 * m)) & M]);  // w256^{SL l2}
      }
      dftr<T, 8, 1>(y);  // y[k1] = sum_m y[m] w8^{k1 m}
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k1 = 1; k1 < 8; k1++) y[k1] = cmul(y[k1], tws[(8 * cl * k1) & M]);  // w64^{c k1}
      // LDS addresses formed per row (register budget)
      cpx<T>* rowx = E + s4_opaque_lt<128>(jl) * 64;
#pragma unroll
      for (int k1 = 0; k1 < 8; k1++) rowx[s4_slot(k1, cl) ^ swr] = y[k1];
      wave_lds_sync();
#pragma unroll
      for (int cc = 0; cc < 8; cc++) y[cc] = rowx[s4_slot(cl, cc) ^ swr];  // lane cc's k1 = c
      wave_lds_sync();
      dftr<T, 8, 1>(y);  // y[k2] = G[j][q' = c + 8 k2]
#pragma unroll
      for (int k2 = 0; k2 < 8; k2++) g[half][k2] = y[k2];
    }
    const cpx<T> hE = tws[(delta * jl) & M], hO = tws[((delta + 2) * jl) & M];
    const int cr = s4_opaque_lt<8>(c);
#pragma unroll
    for (int k2 = 0; k2 < 8; k2++) {
      const cpx<T> gb = delta ? mul_i(g[1][k2]) : g[1][k2];
      row[(cr + 8 * k2) ^ swr] = cmul(cadd(g[0][k2], gb), hE);
      O[hp][k2] = cmul(csub(g[0][k2], gb), hO);
      asm volatile("" : "+v"(O[hp][k2].re), "+v"(O[hp][k2].im));  // formed here, held as one value
    }
  }
}

// i^e s as a complex factor
__device__ __forceinline__ cpx<float> s4_ipow(int e, float s) {
  const float ss = (e & 2) ? -s : s;
  return (e & 1) ? cpx<float>{0.0f, ss} : cpx<float>{ss, 0.0f};
}

template <bool REAL>
__global__ __launch_bounds__(S4_NT, 4) void ring_forward_sliced4(const cpx<float>* __restrict__ samples,
                                                                 cpx<float>* __restrict__ S, FastRingParams<float> p) {
  typedef float T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* E = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = E + S4_BW;
  constexpr int N = S4_N;
  constexpr int M = 2 * N - 1;
  const int t = threadIdx.x;
  const TileSlot sl = contraction_slot(blockIdx.x, p.batch * N, S4_SLC);
  if (!sl.valid) return;
  const int ring = sl.tile, s = sl.bt;
  // rings node-major over the signals (as the N <= 128 forward rings): the
  // rings in flight together write whole rows of each spectra tile
  const int k = ring / p.batch, b = ring - k * p.batch;
  const size_t x0 = ring_offset(p.soff, b, N) + (size_t)k * N * N;
  for (int i = t; i < 2 * N; i += S4_NT) tws[i] = p.tw[i];
  __syncthreads();
  const int delta = ((s & 1) && !p.so3) ? 1 : 0;
  const int c = t & 7, rr = t >> 3;

  cpx<T> O[2][8];
  switch (s) {
    case 0: s4_rows_forward<REAL, 0>(samples, x0, E, tws, t, delta, O); break;
    case 1: s4_rows_forward<REAL, 1>(samples, x0, E, tws, t, delta, O); break;
    case 2: s4_rows_forward<REAL, 2>(samples, x0, E, tws, t, delta, O); break;
    default: s4_rows_forward<REAL, 3>(samples, x0, E, tws, t, delta, O); break;
  }

  // ---- columns: 8 lanes per column q', E (even p) then O (odd p); the E
  //      pass's outputs wait in registers so that both parities (adjacent
  //      pairs of S) are written together and every line of S is completed
  //      at once
  const int qc = t >> 3;
  const T Wk = p.W[k];
  cpx<T>* Sk = S + ((size_t)k * p.batch + b) * PT;
  const size_t tile_stride = (size_t)N * p.batch * PT;
  cpx<T> XE[8];  // E pass: [4 h + kk]
#pragma unroll
  for (int par = 0; par < 2; par++) {
    const int cp = s4_opaque_lt<8>(c), qp = s4_opaque_lt<64>(qc);  // LDS addresses formed per pass
    __syncthreads();
    if (par == 1) {  // every column of E read: O takes its place
      const int rp = s4_opaque_lt<64>(rr);
#pragma unroll
      for (int hp = 0; hp < 2; hp++) {
        const int jl = rp + 64 * hp;
#pragma unroll
        for (int k2 = 0; k2 < 8; k2++) E[jl * 64 + ((cp + 8 * k2) ^ s4_sw(jl))] = O[hp][k2];
      }
      __syncthreads();
    }
    cpx<T> a[16];  // rows jl = c + 8 i of column qc
#pragma unroll
    for (int i = 0; i < 16; i++) {
      const int jl = cp + 8 * i;
      a[i] = E[jl * 64 + (qp ^ s4_sw(jl))];
    }
    dftr<T, 16, 1>(a);  // a[k1] = sum_i a[i] w16^{k1 i}
    __builtin_amdgcn_sched_barrier(0);  // twiddles read after the transform (register budget)
    const int cl = s4_opaque_lt<8>(c);
#pragma unroll
    for (int k1 = 1; k1 < 16; k1++) a[k1] = cmul(a[k1], tws[(4 * cl * k1) & M]);  // w128^{c k1}
#pragma unroll
    for (int k1 = 0; k1 < 16; k1++) {
      const int jl = s4_slot(k1, cp);
      E[jl * 64 + (qp ^ s4_sw(jl))] = a[k1];
    }
    wave_lds_sync();
    cpx<T> lo[8], hi[8];  // lane cc's k1 = c and k1 = c + 8
#pragma unroll
    for (int cc = 0; cc < 8; cc++) {
      const int j0 = s4_slot(cp, cc), j1 = s4_slot(cp + 8, cc);
      lo[cc] = E[j0 * 64 + (qp ^ s4_sw(j0))];
      hi[cc] = E[j1 * 64 + (qp ^ s4_sw(j1))];
    }
    wave_lds_sync();
    dftr<T, 8, 1>(lo);  // lo[k2] = X[p'' = c + 16 k2]
    dftr<T, 8, 1>(hi);  // hi[k2] = X[p'' = c + 8 + 16 k2]
    if (par == 0) {
#pragma unroll
      for (int h = 0; h < 2; h++)
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const int k2 = kk < 2 ? kk : kk + 4;  // p'' in [0, 32) and [96, 128)
          XE[4 * h + kk] = h ? hi[k2] : lo[k2];
          asm volatile("" : "+v"(XE[4 * h + kk].re), "+v"(XE[4 * h + kk].im));
        }
    } else {
      // bins p = 2 p'' (E) and 2 p'' + 1 (O) of column q = 4 q' + s; the
      // phase exponent (3 p + e0) mod 4 is (6 c + 3 par + e0) mod 4 for every
      // bin of this lane.  The lane's bins are p = pb + 16 (h + 2 k) with
      // pb = 2 c (+ 1 for O) in the lower run and 192 + 2 c (+ 1) in the upper
      // one (k = k2 mod 6), so their pair indices step by 16, one tile
      const int4 ci = reinterpret_cast<const int4*>(p.cols)[S4_SLC * qp + s];
      const cpx<T> rE = s4_ipow((6 * cp + ci.w) & 3, Wk), rO = s4_ipow((6 * cp + 3 + ci.w) & 3, Wk);
      const bool valid = (ci.w >> 4) & 1;
      const bool first_hi = 192 + 2 * cp >= 192 + ((ci.w >> 2) & 3);  // E bin p = 192 + 2 c retained
      const long long ts = (long long)tile_stride;
      const long long oLE = s4_off(ci.z + 2 * cp, ts), oLO = s4_off(ci.z + 2 * cp + 1, ts);
      const long long oHE = s4_off(ci.x + 2 * cp, ts), oHO = s4_off(ci.x + 2 * cp + 1, ts);
      const long long oL0 = cp == 0 ? (long long)s4_off(ci.y, ts) : oLE;  // bin p = 0: pair ci.y
      if (valid) {
#pragma unroll
        for (int h = 0; h < 2; h++)
#pragma unroll
          for (int kk = 0; kk < 4; kk++) {
            const int k2 = kk < 2 ? kk : kk + 4;
            const long long j = (long long)(h + 2 * (kk & 1)) * ts;
            const cpx<T> xe = cmul(XE[4 * h + kk], rE), xo = cmul(h ? hi[k2] : lo[k2], rO);
            if (kk < 2) {
              Sk[(h == 0 && kk == 0 ? oL0 : oLE) + j] = xe;
              Sk[oLO + j] = xo;
            } else {
              if (h != 0 || kk != 2 || first_hi) Sk[oHE + j] = xe;
              Sk[oHO + j] = xo;
            }
          }
      }
    }
  }
}

// ---- inverse / adjoint ----

// One 128-point inverse transform per row of the LDS block: 8 lanes per row
// (row jr = t / 8), the row's values at columns c + 8 i; out[8 h + k2] is the
// output l = c + 8 h + 16 k2.
__device__ __forceinline__ void s4_rows_inverse(cpx<float>* row, int swr, int c, const cpx<float>* tws,
                                                cpx<float> (&out)[16]) {
  typedef float T;
  constexpr int M = 2 * S4_N - 1;
  c = s4_opaque_lt<8>(c);  // addresses formed per call (register budget)
  cpx<T> a[16];
#pragma unroll
  for (int i = 0; i < 16; i++) a[i] = row[(c + 8 * i) ^ swr];
  dftr<T, 16, -1>(a);
  __builtin_amdgcn_sched_barrier(0);  // twiddles read after the transform (register budget)
  const int cl = s4_opaque_lt<8>(c);
#pragma unroll
  for (int k1 = 1; k1 < 16; k1++) a[k1] = cmulc(a[k1], tws[(4 * cl * k1) & M]);  // w128^{-c k1}
#pragma unroll
  for (int k1 = 0; k1 < 16; k1++) row[s4_slot(k1, cl) ^ swr] = a[k1];
  wave_lds_sync();
  cpx<T> lo[8], hi[8];
#pragma unroll
  for (int cc = 0; cc < 8; cc++) {
    lo[cc] = row[s4_slot(cl, cc) ^ swr];
    hi[cc] = row[s4_slot(cl + 8, cc) ^ swr];
  }
  wave_lds_sync();
  dftr<T, 8, -1>(lo);
  dftr<T, 8, -1>(hi);
#pragma unroll
  for (int k2 = 0; k2 < 8; k2++) {
    out[k2] = lo[k2];
    out[8 + k2] = hi[k2];
  }
}

// Spectra of one column (q = 2 cq + odd) as this lane loads them: bins
// p' = c + 8 m and 192 + c + 8 m, m < 8.  Their pair indices run on from
// ci.z + c (lower run, p' >= 1; p' = 0 is pair ci.y) and ci.x + c (upper run),
// so they step by one tile every two m.  Every lane loads a valid address;
// bins that are not retained are zeroed when the column is transformed.
struct S4Gather {
  cpx<float> lo[8], hi[8];
  int4 ci;
};
__device__ __forceinline__ void s4_gather(const cpx<float>* __restrict__ Sk, long long ts, const int* __restrict__ cols,
                                          int q, int c, S4Gather& g) {
  g.ci = reinterpret_cast<const int4*>(cols)[q];
  const int4 ci = g.ci;
  const bool valid = (ci.w >> 4) & 1;
  const bool first_hi = c >= ((ci.w >> 2) & 3);  // upper bin p = 192 + c retained
  const long long oL[2] = {s4_off(ci.z + c, ts), s4_off(ci.z + c + 8, ts)};
  const long long oH[2] = {s4_off(ci.x + c, ts), s4_off(ci.x + c + 8, ts)};
  const long long oL0 = c == 0 ? s4_off(ci.y, ts) : oL[0];
#pragma unroll
  for (int m = 0; m < 8; m++) {
    const long long j = (long long)(m >> 1) * ts;
    const bool ok3 = valid && (m != 0 || first_hi);
    g.lo[m] = Sk[(m == 0 ? oL0 : oL[m & 1]) + j];
    g.hi[m] = Sk[ok3 ? oH[m & 1] + j : 0];
  }
}

// Column phase of inverse slice SL (rows j = 4 j' + SL; a compile-time
// constant, so that the radix-4 step takes no branches): 8 lanes per column
// q = 2 cq + odd for all 256 q, odd q first (kept in registers, godd), then
// even q into the LDS block; a column's 64 LDS words serve as its exchange
// slots.  The next column's spectra are requested before the current one is
// transformed.
template <int SL>
__device__ __forceinline__ void s4_cols_inverse(const cpx<float>* __restrict__ Sk, size_t tile_stride,
                                                const int* __restrict__ cols, float scale, int so3, cpx<float>* G,
                                                const cpx<float>* tws, int t, cpx<float> (&godd)[2][8]) {
  typedef float T;
  constexpr int M = 2 * S4_N - 1;
  const long long ts = (long long)tile_stride;
  S4Gather gs[2];
  s4_gather(Sk, ts, cols, 2 * (t >> 3) + 1, t & 7, gs[0]);
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int odd = r < 2 ? 1 : 0;
    const int c = s4_opaque_lt<8>(t);  // addresses formed per column (register budget)
    const int cq = s4_opaque_lt<64>(t >> 3) + 64 * (r & 1);
    if (r < 3) {
      const int rn = r + 1;
      s4_gather(Sk, ts, cols, 2 * (s4_opaque_lt<64>(t >> 3) + 64 * (rn & 1)) + (rn < 2 ? 1 : 0), c, gs[rn & 1]);
    }
    const S4Gather& g = gs[r & 1];
    const int4 ci = g.ci;
    // the conjugate phase times the scale: the exponent (3 p + e0) mod 4 is
    // (3 c + e0) mod 4 for every bin p = c + 8 m (+ 192) of this lane
    const cpx<T> rho = s4_ipow((4 - ((3 * c + ci.w) & 3)) & 3, scale);
    const bool valid = (ci.w >> 4) & 1;
    const bool first_hi = c >= ((ci.w >> 2) & 3);
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> x[8];  // p' = c + 8 m
#pragma unroll
    for (int m = 0; m < 8; m++) {
      const int p0 = c + 8 * m;
      const bool ok3 = valid && (m != 0 || first_hi);
      const cpx<T> v0 = valid ? cmul(g.lo[m], rho) : zero;
      const cpx<T> v3 = ok3 ? cmul(g.hi[m], rho) : zero;
      // i^SL on the upper bins, then w256^{-p' SL}
      cpx<T> u;
      if constexpr (SL == 0) u = cadd(v0, v3);
      else if constexpr (SL == 1) u = cadd(v0, mul_i(v3));
      else if constexpr (SL == 2) u = csub(v0, v3);
      else u = csub(v0, mul_i(v3));
      if constexpr (SL != 0) u = cmulc(u, tws[(2 * SL * p0) & M]);
      x[m] = u;
    }
    dftr<T, 8, -1>(x);  // x[j1] = sum_m x[m] w8^{-m j1}
#pragma unroll
    for (int j1 = 1; j1 < 8; j1++) x[j1] = cmulc(x[j1], tws[(8 * c * j1) & M]);  // w64^{-c j1}
#pragma unroll
    for (int j1 = 0; j1 < 8; j1++) {
      const int jp = s4_slot(j1, c);
      G[jp * 128 + (cq ^ s4_sw(jp))] = x[j1];
    }
    wave_lds_sync();
#pragma unroll
    for (int cc = 0; cc < 8; cc++) {
      const int jp = s4_slot(c, cc);
      x[cc] = G[jp * 128 + (cq ^ s4_sw(jp))];
    }
    wave_lds_sync();
    dftr<T, 8, -1>(x);  // x[j2]: j' = c + 8 j2
    if (odd) {
      const bool shift = !so3;  // e^{-i pi (4 j' + SL) / 256}
#pragma unroll
      for (int j2 = 0; j2 < 8; j2++) {
        const cpx<T> v = shift ? cmulc(x[j2], tws[(4 * (c + 8 * j2) + SL) & M]) : x[j2];
        godd[r][j2] = v;
        asm volatile("" : "+v"(godd[r][j2].re), "+v"(godd[r][j2].im));  // formed here, held as one value
      }
    } else {
#pragma unroll
      for (int j2 = 0; j2 < 8; j2++) {
        const int jp = c + 8 * j2;
        G[jp * 128 + (cq ^ s4_sw(jp))] = x[j2];
      }
    }
  }
}

template <bool REAL>
__global__ __launch_bounds__(S4_NT, 4) void ring_inverse_sliced4(const cpx<float>* __restrict__ S,
                                                                 cpx<float>* __restrict__ samples,
                                                                 FastRingParams<float> p) {
  typedef float T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* G = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = G + S4_BW;
  constexpr int N = S4_N;
  constexpr int M = 2 * N - 1;
  const int t = threadIdx.x;
  const TileSlot sl = contraction_slot(blockIdx.x, p.batch * N, S4_SLC);
  if (!sl.valid) return;
  const int ring = sl.tile, s = sl.bt;
  const int b = ring / N, k = ring - b * N;
  for (int i = t; i < 2 * N; i += S4_NT) tws[i] = p.tw[i];
  __syncthreads();
  const T scale = p.adjoint ? p.W[k] : T(1);
  const cpx<T>* Sk = S + ((size_t)k * p.batch + b) * PT;
  const size_t tile_stride = (size_t)N * p.batch * PT;
  const int c = t & 7, cq0 = t >> 3;

  cpx<T> godd[2][8];
  switch (s) {
    case 0: s4_cols_inverse<0>(Sk, tile_stride, p.cols, scale, p.so3, G, tws, t, godd); break;
    case 1: s4_cols_inverse<1>(Sk, tile_stride, p.cols, scale, p.so3, G, tws, t, godd); break;
    case 2: s4_cols_inverse<2>(Sk, tile_stride, p.cols, scale, p.so3, G, tws, t, godd); break;
    default: s4_cols_inverse<3>(Sk, tile_stride, p.cols, scale, p.so3, G, tws, t, godd); break;
  }

  // ---- rows: 8 lanes per row j', A over the even q, then B over the odd q
  const int jr = t >> 3;
  cpx<T>* row = G + jr * 128;
  const int swr = s4_sw(jr);
  __syncthreads();
  cpx<T> A[16], Bv[16];
  s4_rows_inverse(row, swr, c, tws, A);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 2; r++) {
    const int cq = cq0 + 64 * r;
#pragma unroll
    for (int j2 = 0; j2 < 8; j2++) {
      const int jp = c + 8 * j2;
      G[jp * 128 + (cq ^ s4_sw(jp))] = godd[r][j2];
    }
  }
  __syncthreads();
  s4_rows_inverse(row, swr, c, tws, Bv);
  const size_t xrow = ring_offset(p.soff, b, N) + (size_t)k * N * N + (size_t)(4 * jr + s) * N;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const int l = c + 8 * (i >> 3) + 16 * (i & 7);
    const cpx<T> wb = cmulc(Bv[i], tws[(2 * l) & M]);  // w256^{-l} B[l]
    const cpx<T> f0 = cadd(A[i], wb), f1 = csub(A[i], wb);
    st_sample(samples, xrow + l, f0, REAL);
    st_sample(samples, xrow + l + 128, f1, REAL);
  }
}

hipError_t launch_ring_sliced4(bool forward, const FastRingParams<float>& p, const cpx<float>* in, cpx<float>* out,
                               hipStream_t s) {
  if (p.N != S4_N || !p.cols) return hipErrorInvalidValue;
  const bool real = p.real_io != 0;
  const void* kern = forward ? (real ? (const void*)ring_forward_sliced4<true> : (const void*)ring_forward_sliced4<false>)
                             : (real ? (const void*)ring_inverse_sliced4<true> : (const void*)ring_inverse_sliced4<false>);
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)S4_SMEM);
  if (e != hipSuccess) return e;
  FastRingParams<float> pp = p;
  void* args[] = {(void*)&in, (void*)&out, (void*)&pp};
  return hipLaunchKernel(kern, dim3(contraction_grid(p.batch * S4_N, S4_SLC)), dim3(S4_NT), args, S4_SMEM, s);
}

}  // namespace su2
