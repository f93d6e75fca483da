// Ring FFT (stage 1, Proposition 4.2 / Proposition 6.1) for N = 256 nodes per
// angle (bandlimit 128).  A 256 x 256 ring (512 KB in FP32) does not fit in
// one compute unit's registers and LDS, so each direction runs as two passes
// over a chunk of rings with an intermediate G^T[ring][q][j] (the gamma
// transform of every row, stored transposed):
//   forward  rows:    G[j][q] = sum_l f[j][l] e^{+2 pi i q l / N}, written as G^T[q][j]
//            columns: H[p][q] = sum_j G[j][q] e^{i pi delta j / N} e^{+2 pi i p j / N}
//                     (delta = 1 for odd q, the half-bin shift of half-integer n),
//                     retained bins only, S_k(m, n) = W_k rho H[p][q]
//   inverse  columns: bins of S (conjugate phase, W_k for the adjoint) -> inverse
//                     alpha transform, shift undone -> G^T[q][j]
//            rows:    inverse gamma transform of every row -> samples.
// The chunk of rings is sized so that the intermediate (128 MB) can stay in
// the memory-side cache between the two passes.
//
// Every line (a row j, or a column q of G^T) is held by 16 lanes with 16
// values each and transformed as 256 = 16 x 16: a 16-point DFT in registers,
// twiddles, a transpose through LDS, a second 16-point DFT.  A workgroup
// holds 32 lines.
#include "su2fft_internal.h"

namespace su2 {

constexpr int LG_NT = 512;                    // threads per workgroup
constexpr int LG_N = 256;                     // nodes per angle
constexpr int LG_LINES = LG_NT / 16;          // lines per workgroup
constexpr int LG_XP = 17;                     // exchange pitch (16 + 1)
constexpr int LG_XBUF = LG_LINES * 16 * LG_XP;            // exchange buffers of all lines
constexpr int LG_TP = LG_LINES + 1;                       // transpose pitch
static_assert(LG_N * LG_TP <= LG_XBUF, "transpose fits in the exchange buffer");
constexpr int LG_BLOCKS = LG_N / LG_LINES;                // line blocks per ring

template <class T>
constexpr size_t large_smem() { return (size_t)(LG_XBUF + 2 * LG_N) * sizeof(cpx<T>); }

// 256-point DFT of one line held by 16 lanes.  On entry lane c holds x[c + 16 i]
// in v[i]; on exit it holds X[c + 16 o] in v[o], X[u] = sum_v x[v] e^{SIGN 2 pi i u v / 256}.
// xb is the line's exchange buffer; tw[t] = e^{i pi t / 256}.  Contains a
// workgroup barrier: every thread of the workgroup calls it together.
template <class T, int SIGN>
__device__ __forceinline__ void line_dft256(cpx<T>* v, int c, cpx<T>* xb, const cpx<T>* tw) {
  dftr<T, 16, SIGN>(v);  // over i: v[a] = y_c[a]
#pragma unroll
  for (int a = 1; a < 16; a++) {
    const cpx<T> w = tw[(2 * a * c) & (2 * LG_N - 1)];  // e^{SIGN 2 pi i a c / 256}
    v[a] = SIGN > 0 ? cmul(v[a], w) : cmulc(v[a], w);
  }
#pragma unroll
  for (int a = 0; a < 16; a++) xb[a * LG_XP + c] = v[a];
  __syncthreads();
#pragma unroll
  for (int c2 = 0; c2 < 16; c2++) v[c2] = xb[c * LG_XP + c2];
  dftr<T, 16, SIGN>(v);  // over c2: v[o] = X[c + 16 o]
}

// c ? a : b on complex values, as two scalar selects (a conditional on the
// structs themselves would select between addresses and keep the register
// arrays in memory)
template <class T>
__device__ __forceinline__ cpx<T> csel(bool c, cpx<T> a, cpx<T> b) {
  cpx<T> r;
  r.re = c ? a.re : b.re;
  r.im = c ? a.im : b.im;
  return r;
}

template <class T>
__device__ __forceinline__ void large_load_tw(cpx<T>* tws, const cpx<T>* tw, int t) {
  for (int i = t; i < 2 * LG_N; i += LG_NT) tws[i] = tw[i];
}

// ---- forward ----

template <class T>
__global__ __launch_bounds__(LG_NT) void ring_rows_forward_large(const cpx<T>* __restrict__ samples,
                                                                 LargeRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = buf + LG_XBUF;
  constexpr int N = LG_N;
  const int t = threadIdx.x;
  const int blk = blockIdx.x % LG_BLOCKS, rc = blockIdx.x / LG_BLOCKS;
  const int ring = p.ring0 + rc, b = ring / N, k = ring - b * N;
  const int line = t / 16, c = t % 16;
  const int j0 = blk * LG_LINES;
  const size_t x0 = ring_offset(p.f.soff, b, N) + ((size_t)k * N + j0 + line) * N;
  cpx<T> v[16];
#pragma unroll
  for (int i = 0; i < 16; i++) v[i] = ld_sample(samples, x0 + c + 16 * i, p.f.real_io);
  large_load_tw(tws, p.f.tw, t);
  __syncthreads();
  line_dft256<T, 1>(v, c, buf + line * 16 * LG_XP, tws);  // lane c: G[j][q = c + 16 o]
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 16; o++) buf[(c + 16 * o) * LG_TP + line] = v[o];
  __syncthreads();
  cpx<T>* G = p.G + (size_t)rc * N * N;
  const int jl = t % LG_LINES;
#pragma unroll
  for (int r = 0; r < N / (LG_NT / LG_LINES); r++) {
    const int q = t / LG_LINES + (LG_NT / LG_LINES) * r;
    G[(size_t)q * N + j0 + jl] = buf[q * LG_TP + jl];
  }
}

template <class T>
__global__ __launch_bounds__(LG_NT) void ring_cols_forward_large(cpx<T>* __restrict__ S, LargeRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = buf + LG_XBUF;
  constexpr int N = LG_N;
  const int t = threadIdx.x;
  const int blk = blockIdx.x % LG_BLOCKS, rc = blockIdx.x / LG_BLOCKS;
  const int ring = p.ring0 + rc, b = ring / N, k = ring - b * N;
  const int line = t / 16, c = t % 16;
  const int q = blk * LG_LINES + line;
  const cpx<T>* g = p.G + ((size_t)rc * N + q) * N;
  cpx<T> v[16];
#pragma unroll
  for (int i = 0; i < 16; i++) v[i] = g[c + 16 * i];
  int ent[8];  // bins of this lane's outputs that can be retained: p = c + 16 p1
#pragma unroll
  for (int i = 0; i < 8; i++) ent[i] = p.f.bins[q * N + c + 16 * kept_row<16>(i)];
  large_load_tw(tws, p.f.tw, t);
  __syncthreads();
  const bool odd = (q & 1) && !p.f.so3;  // half-integer n: input shifted by e^{i pi j / N}
#pragma unroll
  for (int i = 0; i < 16; i++) {
    v[i] = csel(odd, cmul(v[i], tws[c + 16 * i]), v[i]);
  }
  line_dft256<T, 1>(v, c, buf + line * 16 * LG_XP, tws);  // lane c: H[p = c + 16 o][q]
  const int pb = p.qrange[2 * blk], pe = p.qrange[2 * blk + 1];
  const T Wk = p.f.W[k];
  __syncthreads();
#pragma unroll
  for (int o = 0; o < 16; o++) {
    if (o >= 4 && o < 12) continue;  // never retained
    const int e = ent[o < 4 ? o : o - 8];
    if (e >= 0) buf[(e >> 2) - pb] = ipow_scale(v[o], e & 3, Wk);
  }
  __syncthreads();
  for (int pi = pb + t; pi < pe; pi += LG_NT) {
    const int tile = pi / PT;
    S[(((size_t)tile * N + k) * p.f.batch + b) * PT + (pi - tile * PT)] = buf[pi - pb];
  }
}

// ---- inverse / adjoint ----

template <class T>
__global__ __launch_bounds__(LG_NT) void ring_cols_inverse_large(const cpx<T>* __restrict__ S,
                                                                 LargeRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = buf + LG_XBUF;
  constexpr int N = LG_N;
  const int t = threadIdx.x;
  const int blk = blockIdx.x % LG_BLOCKS, rc = blockIdx.x / LG_BLOCKS;
  const int ring = p.ring0 + rc, b = ring / N, k = ring - b * N;
  const int line = t / 16, c = t % 16;
  const int q = blk * LG_LINES + line;
  const int pb = p.qrange[2 * blk], pe = p.qrange[2 * blk + 1];
  int ent[8];
#pragma unroll
  for (int i = 0; i < 8; i++) ent[i] = p.f.bins[q * N + c + 16 * kept_row<16>(i)];
  for (int pi = pb + t; pi < pe; pi += LG_NT) {
    const int tile = pi / PT;
    buf[pi - pb] = S[(((size_t)tile * N + k) * p.f.batch + b) * PT + (pi - tile * PT)];
  }
  large_load_tw(tws, p.f.tw, t);
  __syncthreads();
  const T scale = p.f.adjoint ? p.f.W[k] : T(1);
  cpx<T> v[16];
#pragma unroll
  for (int o = 0; o < 16; o++) {
    v[o] = {T(0), T(0)};
    if (o >= 4 && o < 12) continue;  // never retained
    const int e = ent[o < 4 ? o : o - 8];
    const cpx<T> val = ipow_scale(buf[e >= 0 ? (e >> 2) - pb : 0], (4 - (e & 3)) & 3, scale);
    v[o] = csel(e >= 0, val, cpx<T>{T(0), T(0)});
  }
  __syncthreads();
  line_dft256<T, -1>(v, c, buf + line * 16 * LG_XP, tws);  // lane c: y[j = c + 16 o]
  const bool odd = (q & 1) && !p.f.so3;
  cpx<T>* g = p.G + ((size_t)rc * N + q) * N;
#pragma unroll
  for (int o = 0; o < 16; o++) {
    g[c + 16 * o] = csel(odd, cmulc(v[o], tws[c + 16 * o]), v[o]);
  }
}

template <class T>
__global__ __launch_bounds__(LG_NT) void ring_rows_inverse_large(cpx<T>* __restrict__ samples,
                                                                 LargeRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tws = buf + LG_XBUF;
  constexpr int N = LG_N;
  const int t = threadIdx.x;
  const int blk = blockIdx.x % LG_BLOCKS, rc = blockIdx.x / LG_BLOCKS;
  const int ring = p.ring0 + rc, b = ring / N, k = ring - b * N;
  const int line = t / 16, c = t % 16;
  const int j0 = blk * LG_LINES;
  const cpx<T>* G = p.G + (size_t)rc * N * N;
  const int jl = t % LG_LINES;
#pragma unroll
  for (int r = 0; r < N / (LG_NT / LG_LINES); r++) {
    const int q = t / LG_LINES + (LG_NT / LG_LINES) * r;
    buf[q * LG_TP + jl] = G[(size_t)q * N + j0 + jl];
  }
  large_load_tw(tws, p.f.tw, t);
  __syncthreads();
  cpx<T> v[16];
#pragma unroll
  for (int i = 0; i < 16; i++) v[i] = buf[(c + 16 * i) * LG_TP + line];  // G[j][q = c + 16 i]
  __syncthreads();
  line_dft256<T, -1>(v, c, buf + line * 16 * LG_XP, tws);  // lane c: f[j][l = c + 16 o]
  const size_t x0 = ring_offset(p.f.soff, b, N) + ((size_t)k * N + j0 + line) * N;
#pragma unroll
  for (int o = 0; o < 16; o++) st_sample(samples, x0 + c + 16 * o, v[o], p.f.real_io);
}

// ---- forward in one pass, in slices (FP32) ----
//
// The FP32 forward runs in one pass instead: a ring is shared by SLC = 4
// workgroups that together hold its whole transform in LDS, a quarter each
// (145 KB with padding and tables), and each reads the ring's samples in
// full.  The four are dispatched back to back on one XCD (contraction_slot),
// so the samples come from HBM once and from that XCD's L2 three times, and
// nothing round-trips through memory between the two axes.  Slice s holds
// the gamma frequencies q = 4 q' + s (q' = 0..63):
//   rows     G[j][q'] = sum_{l2 < 64} w64^{q' l2} w256^{s l2} sum_{l1 < 4} i^{s l1} f[j][l2 + 64 l1]
//            (the first radix-4 step of the gamma DFT, kept for this s, then a
//            64-point DFT as 8 x 8 with one exchange inside a wave)
//   columns  H[p][q] = sum_j G[j][q'] e^{i pi delta j / N} w256^{p j}, retained p only
//            (16 x 16 with one exchange), written to S;
// w_n = e^{2 pi i / n}, delta = 1 on odd q (SU(2) half-integer n).
// (Slicing the inverse the same way, by rows j = 4 j' + s, measured slower
// than its two passes: every slice gathers all of the ring's bins.  Eight
// slices of 512 threads, two workgroups per CU, were slower in both
// directions: the single-output radix-8 step and the eightfold loads cost
// more vector instructions than the overlap gains.)
//
// LDS layout.  A 64-bit LDS access serves 16 lanes per cycle, one 8-byte word
// in each of the 16 bank pairs (word w in bank pair w mod 16).  Every
// position below is a per-lane base plus a compile-time offset, and every
// group of 16 lanes meets 16 different bank pairs in every access:
// G[j][q'] at 72 j + ((j / 2) mod 8) + q'.  Rows 2g and 2g + 1, which share a
// 16-lane group in the row phase, are 8 bank pairs apart; the row exchange
// uses row slots c + 9 k1 (distinct mod 8 both ways); the 16 lanes of a
// column, rows c + 16 i, land on bank pairs 8 (c mod 2) + c / 2.  The column
// exchange runs, after a barrier, in padded 16 x 17 buffers, one per column.
// The row and column exchanges stay inside one wave (the 8 or 16 lanes of a
// line), so they need no workgroup barrier: a wave's LDS accesses take effect
// in program order.  Twiddles come from small LDS tables.
constexpr int SLC = 4;                  // slices (workgroups) per ring
constexpr int SL_NT = 1024;             // threads per workgroup
constexpr int SL_L = LG_N / SLC;        // columns q' of a slice
constexpr int SL_PF = 72;               // row pitch (8 mod 16, room for slots up to 70)
constexpr int SL_XP = 17;               // padded exchange pitch
constexpr int SL_GW = LG_N * SL_PF;     // G words
constexpr int SL_T2 = 0, SL_T8 = 256, SL_TS = 320, SL_TX = 384, SL_TW = 640;  // table offsets
constexpr size_t SL_SMEM = ((size_t)SL_GW + SL_TW) * sizeof(cpx<float>);
static_assert(SL_SMEM <= 160 * 1024, "LDS");
static_assert(SL_L * 16 * SL_XP <= SL_GW, "padded exchange buffers fit in G");

// orders this wave's LDS accesses before and after it (an exchange between
// lanes of one wave)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }

// the twiddle tables of slice s (tw: e^{i pi t / 256} in global memory):
//   T2[16 a + c] = w256^{a c}, T8[8 k + c] = w64^{c k}, TS[8 m + c] = w256^{s (c + 8 m)},
//   TX[j] = e^{i pi j / 256}
__device__ __forceinline__ void sl_tables(cpx<float>* tb, const cpx<float>* __restrict__ tw, int s, int t) {
  constexpr int M = 2 * LG_N - 1;
  for (int e = t; e < SL_TW; e += SL_NT) {
    int idx;
    if (e < SL_T8) idx = 2 * (e >> 4) * (e & 15);
    else if (e < SL_TS) idx = 8 * ((e - SL_T8) >> 3) * (e & 7);
    else if (e < SL_TX) idx = 2 * s * ((e & 7) + 8 * ((e - SL_TS) >> 3));
    else idx = e - SL_TX;
    tb[e] = tw[idx & M];
  }
}

__global__ __launch_bounds__(SL_NT) void ring_forward_sliced(const cpx<float>* __restrict__ samples,
                                                             cpx<float>* __restrict__ S, FastRingParams<float> p) {
  typedef float T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* G = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tb = G + SL_GW;
  constexpr int N = LG_N;
  const int t = threadIdx.x;
  const TileSlot sl = contraction_slot(blockIdx.x, p.batch * N, SLC);
  if (!sl.valid) return;
  const int ring = sl.tile, s = sl.bt;
  const int b = ring / N, k = ring - b * N;
  const cpx<T>* x = samples + ring_offset(p.soff, b, N) + (size_t)k * N * N;
  const T* xr = reinterpret_cast<const T*>(samples) + ring_offset(p.soff, b, N) + (size_t)k * N * N;
  sl_tables(tb, p.tw, s, t);
  __syncthreads();

  // ---- rows: 8 lanes per row, 128 rows per round
  const int c = t % 8, rr = t / 8;
#pragma unroll 1
  for (int h = 0; h < 2; h++) {
    const int j = rr + 128 * h;
    cpx<T> v[32];  // f[j][c + 8 m], m = 0..31
    if (p.real_io) {  // real samples (plain loads: the ring's other slices read them from L2)
#pragma unroll
      for (int m = 0; m < 32; m++) v[m] = {xr[(size_t)j * N + c + 8 * m], T(0)};
    } else {
#pragma unroll
      for (int m = 0; m < 32; m++) v[m] = x[(size_t)j * N + c + 8 * m];
    }
    cpx<T> y[8];  // radix-4 step over l1 for this s: y[m] for l2 = c + 8 m
#pragma unroll
    for (int m = 0; m < 8; m++) {
      const cpx<T> a0 = v[m], a1 = v[m + 8], a2 = v[m + 16], a3 = v[m + 24];
      if (s == 0) y[m] = cadd(cadd(a0, a1), cadd(a2, a3));
      else if (s == 2) y[m] = csub(cadd(a0, a2), cadd(a1, a3));
      else if (s == 1) y[m] = cadd(csub(a0, a2), mul_i(csub(a1, a3)));
      else y[m] = csub(csub(a0, a2), mul_i(csub(a1, a3)));
    }
    if (s != 0) {  // w256^{s l2}, l2 = c + 8 m
#pragma unroll
      for (int m = 0; m < 8; m++) y[m] = cmul(y[m], tb[SL_TS + 8 * m + c]);
    }
    dftr<T, 8, 1>(y);  // y[k1] = sum_m y[m] w8^{k1 m}
#pragma unroll
    for (int k1 = 1; k1 < 8; k1++) y[k1] = cmul(y[k1], tb[SL_T8 + 8 * k1 + c]);  // w64^{c k1}
    cpx<T>* row = G + SL_PF * j;
#pragma unroll
    for (int k1 = 0; k1 < 8; k1++) row[c + 9 * k1] = y[k1];
    wave_lds_sync();
#pragma unroll
    for (int cc = 0; cc < 8; cc++) y[cc] = row[cc + 9 * c];  // lane c: k1 = c of lane cc
    wave_lds_sync();
    dftr<T, 8, 1>(y);  // y[k2] = G[j][q' = c + 8 k2]
    cpx<T>* gj = row + ((j >> 1) & 7) + c;
#pragma unroll
    for (int k2 = 0; k2 < 8; k2++) gj[8 * k2] = y[k2];
  }

  // ---- columns: 16 lanes per column q', all 64 columns at once
  const int qc = t / 16, c2 = t % 16;
  const int q = SLC * qc + s;
  int ent[8];  // bins of this lane's retained outputs p = c2 + 16 o, o in {0..3, 12..15}
#pragma unroll
  for (int i = 0; i < 8; i++) ent[i] = p.bins[q * N + c2 + 16 * kept_row<16>(i)];
  const T Wk = p.W[k];
  __syncthreads();
  cpx<T> a[16];
  const cpx<T>* gc = G + SL_PF * c2 + (c2 >> 1) + qc;  // rows c2 + 16 i of column qc
#pragma unroll
  for (int i = 0; i < 16; i++) a[i] = gc[16 * SL_PF * i];
  if ((s & 1) && !p.so3) {  // half-bin shift e^{i pi j / N}, j = c2 + 16 i
#pragma unroll
    for (int i = 0; i < 16; i++) a[i] = cmul(a[i], tb[SL_TX + c2 + 16 * i]);
  }
  dftr<T, 16, 1>(a);
#pragma unroll
  for (int a1 = 1; a1 < 16; a1++) a[a1] = cmul(a[a1], tb[SL_T2 + 16 * a1 + c2]);  // w256^{a1 c2}
  __syncthreads();  // every column read: G becomes the exchange buffers
  cpx<T>* xb = G + qc * 16 * SL_XP;
#pragma unroll
  for (int a1 = 0; a1 < 16; a1++) xb[SL_XP * a1 + c2] = a[a1];
  wave_lds_sync();
#pragma unroll
  for (int cc = 0; cc < 16; cc++) a[cc] = xb[SL_XP * c2 + cc];
  dftr<T, 16, 1>(a);  // a[o] = H[p = c2 + 16 o][q]
  cpx<T>* Sk = S + ((size_t)k * p.batch + b) * PT;
  const size_t tile_stride = (size_t)N * p.batch * PT;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const int e = ent[i];
    if (e >= 0) {
      const int pi = e >> 2;
      Sk[(size_t)(pi / PT) * tile_stride + (pi % PT)] = ipow_scale(a[kept_row<16>(i)], e & 3, Wk);
    }
  }
}

hipError_t launch_ring_forward_sliced(const FastRingParams<float>& p, const cpx<float>* samples, cpx<float>* S,
                                      hipStream_t s) {
  if (p.N != LG_N) return hipErrorInvalidValue;
  const void* kern = (const void*)ring_forward_sliced;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)SL_SMEM);
  if (e != hipSuccess) return e;
  FastRingParams<float> pp = p;
  void* args[] = {(void*)&samples, (void*)&S, (void*)&pp};
  return hipLaunchKernel(kern, dim3(contraction_grid(p.batch * LG_N, SLC)), dim3(SL_NT), args, SL_SMEM, s);
}

// ---- host ----

template <class T>
static hipError_t launch_large(bool forward, LargeRingParams<T> p, const cpx<T>* in, cpx<T>* out, hipStream_t s) {
  if (p.f.N != LG_N || p.chunk < 1) return hipErrorInvalidValue;
  const size_t smem = large_smem<T>();
  const void* k1 = forward ? (const void*)ring_rows_forward_large<T> : (const void*)ring_cols_inverse_large<T>;
  const void* k2 = forward ? (const void*)ring_cols_forward_large<T> : (const void*)ring_rows_inverse_large<T>;
  hipError_t e;
  if ((e = hipFuncSetAttribute(k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute(k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)) != hipSuccess) return e;
  const int total = p.f.batch * LG_N;
  for (int r0 = 0; r0 < total; r0 += p.chunk) {
    p.ring0 = r0;
    const int nr = total - r0 < p.chunk ? total - r0 : p.chunk;
    const dim3 grid((unsigned)(nr * LG_BLOCKS));
    if (forward) {
      hipLaunchKernelGGL(ring_rows_forward_large<T>, grid, dim3(LG_NT), smem, s, in, p);
      hipLaunchKernelGGL(ring_cols_forward_large<T>, grid, dim3(LG_NT), smem, s, out, p);
    } else {
      hipLaunchKernelGGL(ring_cols_inverse_large<T>, grid, dim3(LG_NT), smem, s, in, p);
      hipLaunchKernelGGL(ring_rows_inverse_large<T>, grid, dim3(LG_NT), smem, s, out, p);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

bool large_ring_supported(int N) { return N == LG_N; }
int large_ring_block() { return LG_LINES; }
int large_ring_slice_capacity() { return LG_XBUF; }

template <class T>
hipError_t launch_ring_forward_large(const LargeRingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s) {
  return launch_large<T>(true, p, samples, S, s);
}
template <class T>
hipError_t launch_ring_inverse_large(const LargeRingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s) {
  return launch_large<T>(false, p, S, samples, s);
}

template hipError_t launch_ring_forward_large<float>(const LargeRingParams<float>&, const cpx<float>*, cpx<float>*,
                                                     hipStream_t);
template hipError_t launch_ring_forward_large<double>(const LargeRingParams<double>&, const cpx<double>*,
                                                      cpx<double>*, hipStream_t);
template hipError_t launch_ring_inverse_large<float>(const LargeRingParams<float>&, const cpx<float>*, cpx<float>*,
                                                     hipStream_t);
template hipError_t launch_ring_inverse_large<double>(const LargeRingParams<double>&, const cpx<double>*,
                                                      cpx<double>*, hipStream_t);

}  // namespace su2
