// Ring FFT (stage 1, Proposition 4.2 / Proposition 6.1) for N = 256 nodes per
// angle (bandlimit 128) in FP64.  A 256 x 256 ring (1 MB in FP64) does not fit
// in one compute unit's registers and LDS, so each direction runs as two
// passes over a chunk of rings with an intermediate G^T[ring][q][j] (the gamma
// transform of every row, stored transposed; FP32 rings run in one pass,
// su2fft_ring_sliced.hip):
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

template <class T, bool REAL>
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
  for (int i = 0; i < 16; i++) v[i] = ld_sample(samples, x0 + c + 16 * i, REAL);
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

template <class T, bool REAL>
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
  for (int o = 0; o < 16; o++) st_sample(samples, x0 + c + 16 * o, v[o], REAL);
}

// ---- host ----

template <class T>
static hipError_t launch_large(bool forward, LargeRingParams<T> p, const cpx<T>* in, cpx<T>* out, hipStream_t s) {
  if (p.f.N != LG_N || p.chunk < 1) return hipErrorInvalidValue;
  const size_t smem = large_smem<T>();
  // real samples are a compile-time case: a run-time test around the sample
  // accesses lets the compiler merge the two access forms into one of scalar
  // loads with per-element addresses
  const bool real = p.f.real_io != 0;
  const void* rows_fwd = real ? (const void*)ring_rows_forward_large<T, true> : (const void*)ring_rows_forward_large<T, false>;
  const void* rows_inv = real ? (const void*)ring_rows_inverse_large<T, true> : (const void*)ring_rows_inverse_large<T, false>;
  const void* k1 = forward ? rows_fwd : (const void*)ring_cols_inverse_large<T>;
  const void* k2 = forward ? (const void*)ring_cols_forward_large<T> : rows_inv;
  hipError_t e;
  if ((e = hipFuncSetAttribute(k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute(k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)) != hipSuccess) return e;
  const int total = p.f.batch * LG_N;
  for (int r0 = 0; r0 < total; r0 += p.chunk) {
    p.ring0 = r0;
    const int nr = total - r0 < p.chunk ? total - r0 : p.chunk;
    const dim3 grid((unsigned)(nr * LG_BLOCKS));
    if (forward) {
      if (real) hipLaunchKernelGGL((ring_rows_forward_large<T, true>), grid, dim3(LG_NT), smem, s, in, p);
      else hipLaunchKernelGGL((ring_rows_forward_large<T, false>), grid, dim3(LG_NT), smem, s, in, p);
      hipLaunchKernelGGL(ring_cols_forward_large<T>, grid, dim3(LG_NT), smem, s, out, p);
    } else {
      hipLaunchKernelGGL(ring_cols_inverse_large<T>, grid, dim3(LG_NT), smem, s, in, p);
      if (real) hipLaunchKernelGGL((ring_rows_inverse_large<T, true>), grid, dim3(LG_NT), smem, s, out, p);
      else hipLaunchKernelGGL((ring_rows_inverse_large<T, false>), grid, dim3(LG_NT), smem, s, out, p);
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
