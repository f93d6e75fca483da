// Stage 1 of the separated transform (Section 4, Proposition 4.2; cost model of
// Proposition 6.1): on every beta ring, a 2D DFT over (alpha, gamma).
//
// Forward, per ring (signal b, node k), with w = e^{+2 pi i / N}:
//   G[j, q]  = sum_l f[k, j, l] w^{q l}                     (gamma, q = 2m mod N)
//   H[p, q]  = sum_j G[j, q] tw_q(j) w^{p j}                 (alpha; tw_q(j) = e^{i pi j / N}
//                                                            for odd q, i.e. half-integer n,
//                                                            p = (n - 1/2) mod N; 1 and
//                                                            p = n mod N otherwise)
//   S_k(m,n) = W_k rho_{mn} H[p, q],  rho_{mn} = i^{n-m} (-1)^{2m} e^{-i pi n}
// so that fhat(l)_{mn} = sum_k d^l_{nm}(beta_k) S_k(m, n) (the beta contraction).
// The phases come from the node offsets alpha_0 = -pi, gamma_0 = -2pi and
// from conj(P^l_{nm}) = i^{n-m} d^l_{nm}.
//
// One workgroup owns one ring.  The ring (or, when it does not fit in LDS, one
// class of gamma frequencies q = split*q' + r at a time, after a first
// decimation-in-frequency split of the gamma axis) is held in LDS; both
// transforms run in place as mixed-radix (2, 3, 4, 8) decimation-in-frequency
// passes, leaving the bins in digit-reversed order, which the epilogue
// reads through a per-pair position table.  The inverse runs the adjoint
// network (decimation in time with conjugate twiddles) from the scattered
// bins back to natural order.
#include "su2fft_internal.h"

namespace su2 {

// threads per workgroup of the generic ring kernels (one ring per workgroup)
constexpr int GENERIC_NT = 512;

template <class T, int R, int SIGN>
__device__ __forceinline__ void dft_small(cpx<T>* a) {
  if constexpr (R == 2) {
    cpx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (R == 3) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    cpx<T> t1 = cadd(a[1], a[2]);
    cpx<T> t2 = csub(a[1], a[2]);
    cpx<T> m1 = {a[0].re - T(0.5) * t1.re, a[0].im - T(0.5) * t1.im};
    cpx<T> m2 = {-T(SIGN) * h * t2.im, T(SIGN) * h * t2.re};
    a[0] = cadd(a[0], t1);
    a[1] = cadd(m1, m2);
    a[2] = csub(m1, m2);
  } else if constexpr (R == 4) {
    cpx<T> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    cpx<T> s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    cpx<T> jd13 = {-T(SIGN) * d13.im, T(SIGN) * d13.re};  // SIGN * i * d13
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, jd13);
    a[3] = csub(d02, jd13);
  } else if constexpr (R == 8) {
    cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
    dft_small<T, 4, SIGN>(e);
    dft_small<T, 4, SIGN>(o);
    const T r2 = T(0.70710678118654752440084436210485);
    // o[k] *= w8^k, w8 = e^{SIGN i pi / 4}
    cpx<T> o1 = {r2 * (o[1].re - T(SIGN) * o[1].im), r2 * (o[1].im + T(SIGN) * o[1].re)};
    cpx<T> o2 = {-T(SIGN) * o[2].im, T(SIGN) * o[2].re};
    cpx<T> o3 = {r2 * (-o[3].re - T(SIGN) * o[3].im), r2 * (-o[3].im + T(SIGN) * o[3].re)};
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
}

// One in-place decimation-in-frequency pass of radix R over `nlines` lines of
// length L (element stride es, line stride ls).  Ls is the current
// sub-transform length; outputs k of each butterfly are multiplied by
// w_Ls^{k * off} with w_Ls = e^{+2 pi i / Ls} = tw[(2N / Ls) * ...].
template <class T, int R>
__device__ void dif_pass(cpx<T>* X, int nlines, int L, int Ls, int es, int ls, bool line_fast,
                         const cpx<T>* tw, int twoN) {
  const int M = Ls / R;
  const int per_line = L / R;
  const int total = nlines * per_line;
  const int tstep = twoN / Ls;
  for (int bf = threadIdx.x; bf < total; bf += blockDim.x) {
    int line, u;
    if (line_fast) { line = bf % nlines; u = bf / nlines; }
    else { line = bf / per_line; u = bf - line * per_line; }
    const int block = u / M, off = u - block * M;
    const int base = line * ls + (block * Ls + off) * es;
    cpx<T> a[R];
#pragma unroll
    for (int i = 0; i < R; i++) a[i] = X[base + i * M * es];
    dft_small<T, R, 1>(a);
#pragma unroll
    for (int i = 1; i < R; i++) {
      int e = (i * off * tstep) % twoN;
      a[i] = cmul(a[i], tw[e]);
    }
#pragma unroll
    for (int i = 0; i < R; i++) X[base + i * M * es] = a[i];
  }
}

// The adjoint of dif_pass: conjugate twiddles first, then the radix-R DFT with
// the negative sign.  Running the passes in reverse order computes the
// unnormalised inverse DFT from digit-reversed input into natural order.
template <class T, int R>
__device__ void dit_pass(cpx<T>* X, int nlines, int L, int Ls, int es, int ls, bool line_fast,
                         const cpx<T>* tw, int twoN) {
  const int M = Ls / R;
  const int per_line = L / R;
  const int total = nlines * per_line;
  const int tstep = twoN / Ls;
  for (int bf = threadIdx.x; bf < total; bf += blockDim.x) {
    int line, u;
    if (line_fast) { line = bf % nlines; u = bf / nlines; }
    else { line = bf / per_line; u = bf - line * per_line; }
    const int block = u / M, off = u - block * M;
    const int base = line * ls + (block * Ls + off) * es;
    cpx<T> a[R];
#pragma unroll
    for (int i = 0; i < R; i++) a[i] = X[base + i * M * es];
#pragma unroll
    for (int i = 1; i < R; i++) {
      int e = (i * off * tstep) % twoN;
      a[i] = cmulc(a[i], tw[e]);
    }
    dft_small<T, R, -1>(a);
#pragma unroll
    for (int i = 0; i < R; i++) X[base + i * M * es] = a[i];
  }
}

template <class T>
__device__ void run_dif(cpx<T>* X, int nlines, int L, int es, int ls, bool line_fast, const int* rad, int nrad,
                        const cpx<T>* tw, int twoN) {
  int Ls = L;
  for (int s = 0; s < nrad; s++) {
    const int R = rad[s];
    if (R == 8) dif_pass<T, 8>(X, nlines, L, Ls, es, ls, line_fast, tw, twoN);
    else if (R == 4) dif_pass<T, 4>(X, nlines, L, Ls, es, ls, line_fast, tw, twoN);
    else if (R == 3) dif_pass<T, 3>(X, nlines, L, Ls, es, ls, line_fast, tw, twoN);
    else dif_pass<T, 2>(X, nlines, L, Ls, es, ls, line_fast, tw, twoN);
    Ls /= R;
    __syncthreads();
  }
}

template <class T>
__device__ void run_dit(cpx<T>* X, int nlines, int L, int es, int ls, bool line_fast, const int* rad, int nrad,
                        const cpx<T>* tw, int twoN) {
  int Ls_list[MAX_RADICES];
  int Ls = L;
  for (int s = 0; s < nrad; s++) { Ls_list[s] = Ls; Ls /= rad[s]; }
  for (int s = nrad - 1; s >= 0; s--) {
    const int R = rad[s];
    if (R == 8) dit_pass<T, 8>(X, nlines, L, Ls_list[s], es, ls, line_fast, tw, twoN);
    else if (R == 4) dit_pass<T, 4>(X, nlines, L, Ls_list[s], es, ls, line_fast, tw, twoN);
    else if (R == 3) dit_pass<T, 3>(X, nlines, L, Ls_list[s], es, ls, line_fast, tw, twoN);
    else dit_pass<T, 2>(X, nlines, L, Ls_list[s], es, ls, line_fast, tw, twoN);
    __syncthreads();
  }
}

// sample idx of a buffer of complex samples, or (real_io) of real samples
template <class T>
__device__ __forceinline__ cpx<T> ring_sample(const cpx<T>* __restrict__ x, size_t idx, int real_io) {
  if (real_io) return {reinterpret_cast<const T*>(x)[idx], T(0)};
  return x[idx];
}

// Body of one ring (signal b, node k): the ring's N x N input block starts at
// element x0 of the sample buffer xs (complex, or real for real_io plans);
// smem holds N * Nc + 2N complex values.
template <class T>
__device__ void ring_forward_body(const cpx<T>* __restrict__ xs, size_t x0, cpx<T>* __restrict__ S,
                                  const RingParams<T>& p, int b, int k, unsigned char* smem_raw) {
  const int N = p.N, Nc = p.Nc, R = p.split, twoN = 2 * N;
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = X + N * Nc;
  for (int t = threadIdx.x; t < twoN; t += blockDim.x) tw[t] = p.tw[t];
  const T Wk = p.W[k];
  for (int r = 0; r < R; r++) {
    __syncthreads();
    // first split of the gamma axis: y_r[j][c] = w^{r c} sum_i x[j][c + i Nc] e^{2 pi i r i / R}
    for (int e = threadIdx.x; e < N * Nc; e += blockDim.x) {
      const int j = e / Nc, c = e - j * Nc;
      cpx<T> v;
      if (R == 1) {
        v = ring_sample(xs, x0 + (size_t)j * N + c, p.real_io);
      } else {
        v = {T(0), T(0)};
        for (int i = 0; i < R; i++) {
          cpx<T> xi = ring_sample(xs, x0 + (size_t)j * N + c + i * Nc, p.real_io);
          v = cadd(v, cmul(xi, tw[((twoN / R) * r * i) % twoN]));
        }
        v = cmul(v, tw[(2 * r * c) % twoN]);
      }
      X[e] = v;
    }
    __syncthreads();
    // gamma: rows j, length Nc
    run_dif<T>(X, N, Nc, 1, Nc, false, p.rad_c, p.nrad_c, tw, twoN);
    // half-bin twist e^{i pi j / N} on columns whose q is odd (half-integer n;
    // none in SO(3) plans, whose n are integers)
    for (int e = threadIdx.x; e < N * Nc; e += blockDim.x) {
      const int j = e / Nc, c = e - j * Nc;
      const int q = R * p.colq[c] + r;
      if ((q & 1) && !p.so3) X[e] = cmul(X[e], tw[j]);
    }
    __syncthreads();
    // alpha: columns, length N
    run_dif<T>(X, Nc, N, Nc, 1, true, p.rad_n, p.nrad_n, tw, twoN);
    // epilogue: the retained bins of this class, times W_k rho_{mn}
    for (int pi = p.cls_begin[r] + threadIdx.x; pi < p.cls_end[r]; pi += blockDim.x) {
      cpx<T> v = cscale(cmul(X[p.fftpos[pi]], p.rho[pi]), Wk);
      const int tile = pi / PT;
      S[(((size_t)tile * N + k) * p.batch + b) * PT + (pi - tile * PT)] = v;
    }
  }
}

// ---- compile-time forms for the 3-smooth sizes N = 48 and N = 96 ----
//
// The same passes as run_dif / run_dit, and the same bodies for rings held
// whole in LDS (split 1), with every size, radix, stride and index known to
// the compiler: the per-butterfly divisions and remainders by run-time sizes
// of the forms above become constants.  The radix sequence is radix_plan's
// (8s, then 4 or 2, then 3s), which the host's bin positions assume.

constexpr int ct_nrad(int L) {
  int p2 = 0, p3 = 0;
  while (L % 2 == 0) { L /= 2; p2++; }
  while (L % 3 == 0) { L /= 3; p3++; }
  return p2 / 3 + (p2 % 3 ? 1 : 0) + p3;
}
constexpr int ct_rad(int L, int s) {
  int p2 = 0, p3 = 0;
  while (L % 2 == 0) { L /= 2; p2++; }
  while (L % 3 == 0) { L /= 3; p3++; }
  const int n8 = p2 / 3, n42 = p2 % 3 ? 1 : 0;
  if (s < n8) return 8;
  if (s < n8 + n42) return p2 % 3 == 2 ? 4 : 2;
  return 3;
}
// sub-transform length entering pass s
constexpr int ct_ls(int L, int s) {
  int Ls = L;
  for (int t = 0; t < s; t++) Ls /= ct_rad(L, t);
  return Ls;
}

template <class T, int R, int NLINES, int L, int LS, int ES, int LSTR, bool LINE_FAST, int TWON, bool DIF>
__device__ __forceinline__ void pass_ct(cpx<T>* X, const cpx<T>* tw) {
  constexpr int M = LS / R, PER_LINE = L / R, TOTAL = NLINES * PER_LINE, TSTEP = TWON / LS;
  for (int bf = threadIdx.x; bf < TOTAL; bf += GENERIC_NT) {
    int line, u;
    if constexpr (LINE_FAST) {
      line = bf % NLINES;
      u = bf / NLINES;
    } else {
      line = bf / PER_LINE;
      u = bf - line * PER_LINE;
    }
    const int block = u / M, off = u - block * M;
    const int base = line * LSTR + (block * LS + off) * ES;
    cpx<T> a[R];
#pragma unroll
    for (int i = 0; i < R; i++) a[i] = X[base + i * M * ES];
    if constexpr (DIF) {
      dft_small<T, R, 1>(a);
#pragma unroll
      for (int i = 1; i < R; i++) a[i] = cmul(a[i], tw[(i * off * TSTEP) % TWON]);
    } else {
#pragma unroll
      for (int i = 1; i < R; i++) a[i] = cmulc(a[i], tw[(i * off * TSTEP) % TWON]);
      dft_small<T, R, -1>(a);
    }
#pragma unroll
    for (int i = 0; i < R; i++) X[base + i * M * ES] = a[i];
  }
}

template <class T, int NLINES, int L, int ES, int LSTR, bool LINE_FAST, int TWON, int S = 0>
__device__ __forceinline__ void run_dif_ct(cpx<T>* X, const cpx<T>* tw) {
  if constexpr (S < ct_nrad(L)) {
    pass_ct<T, ct_rad(L, S), NLINES, L, ct_ls(L, S), ES, LSTR, LINE_FAST, TWON, true>(X, tw);
    __syncthreads();
    run_dif_ct<T, NLINES, L, ES, LSTR, LINE_FAST, TWON, S + 1>(X, tw);
  }
}

template <class T, int NLINES, int L, int ES, int LSTR, bool LINE_FAST, int TWON, int S = ct_nrad(L) - 1>
__device__ __forceinline__ void run_dit_ct(cpx<T>* X, const cpx<T>* tw) {
  if constexpr (S >= 0) {
    pass_ct<T, ct_rad(L, S), NLINES, L, ct_ls(L, S), ES, LSTR, LINE_FAST, TWON, false>(X, tw);
    __syncthreads();
    run_dit_ct<T, NLINES, L, ES, LSTR, LINE_FAST, TWON, S - 1>(X, tw);
  }
}

// ring_forward_body for N held whole in LDS (split 1); N a compile-time size
template <class T, int N>
__device__ void ring_forward_body_ct(const cpx<T>* __restrict__ xs, size_t x0, cpx<T>* __restrict__ S,
                                     const RingParams<T>& p, int b, int k, unsigned char* smem_raw) {
  constexpr int twoN = 2 * N;
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = X + N * N;
  for (int t = threadIdx.x; t < twoN; t += GENERIC_NT) tw[t] = p.tw[t];
  const T Wk = p.W[k];
  __syncthreads();
  for (int e = threadIdx.x; e < N * N; e += GENERIC_NT) X[e] = ring_sample(xs, x0 + e, p.real_io);
  __syncthreads();
  run_dif_ct<T, N, N, 1, N, false, twoN>(X, tw);  // gamma: rows j
  for (int e = threadIdx.x; e < N * N; e += GENERIC_NT) {
    const int j = e / N, c = e - j * N;
    const int q = p.colq[c];
    if ((q & 1) && !p.so3) X[e] = cmul(X[e], tw[j]);
  }
  __syncthreads();
  run_dif_ct<T, N, N, N, 1, true, twoN>(X, tw);  // alpha: columns
  for (int pi = p.cls_begin[0] + threadIdx.x; pi < p.cls_end[0]; pi += GENERIC_NT) {
    cpx<T> v = cscale(cmul(X[p.fftpos[pi]], p.rho[pi]), Wk);
    const int tile = pi / PT;
    S[(((size_t)tile * N + k) * p.batch + b) * PT + (pi - tile * PT)] = v;
  }
}

// ring_inverse_body for N held whole in LDS (split 1); N a compile-time size
template <class T, int N>
__device__ void ring_inverse_body_ct(const cpx<T>* __restrict__ S, cpx<T>* __restrict__ xs, size_t x0,
                                     const RingParams<T>& p, int b, int k, unsigned char* smem_raw) {
  constexpr int twoN = 2 * N;
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = X + N * N;
  for (int t = threadIdx.x; t < twoN; t += GENERIC_NT) tw[t] = p.tw[t];
  const T scale = p.adjoint ? p.W[k] : T(1);
  __syncthreads();
  for (int e = threadIdx.x; e < N * N; e += GENERIC_NT) X[e] = {T(0), T(0)};
  __syncthreads();
  for (int pi = p.cls_begin[0] + threadIdx.x; pi < p.cls_end[0]; pi += GENERIC_NT) {
    const int tile = pi / PT;
    cpx<T> v = S[(((size_t)tile * N + k) * p.batch + b) * PT + (pi - tile * PT)];
    X[p.fftpos[pi]] = cscale(cmulc(v, p.rho[pi]), scale);
  }
  __syncthreads();
  run_dit_ct<T, N, N, N, 1, true, twoN>(X, tw);  // alpha: columns
  for (int e = threadIdx.x; e < N * N; e += GENERIC_NT) {
    const int j = e / N, c = e - j * N;
    const int q = p.colq[c];
    if ((q & 1) && !p.so3) X[e] = cmulc(X[e], tw[j]);
  }
  __syncthreads();
  run_dit_ct<T, N, N, 1, N, false, twoN>(X, tw);  // gamma: rows j
  T* xr = reinterpret_cast<T*>(xs);
  for (int e = threadIdx.x; e < N * N; e += GENERIC_NT) {
    const size_t o = x0 + e;
    if (p.real_io) xr[o] = X[e].re;
    else xs[o] = X[e];
  }
}

// the bodies above for the sizes they are built for, the run-time forms otherwise
template <class T>
__device__ __forceinline__ void ring_forward_any(const cpx<T>* __restrict__ xs, size_t x0, cpx<T>* __restrict__ S,
                                                 const RingParams<T>& p, int b, int k, unsigned char* smem) {
  if (p.split == 1 && p.N == 96) ring_forward_body_ct<T, 96>(xs, x0, S, p, b, k, smem);
  else if (p.split == 1 && p.N == 48) ring_forward_body_ct<T, 48>(xs, x0, S, p, b, k, smem);
  else ring_forward_body<T>(xs, x0, S, p, b, k, smem);
}
template <class T>
__device__ __forceinline__ void ring_inverse_any(const cpx<T>* __restrict__ S, cpx<T>* __restrict__ xs, size_t x0,
                                                 const RingParams<T>& p, int b, int k, unsigned char* smem) {
  if (p.split == 1 && p.N == 96) ring_inverse_body_ct<T, 96>(S, xs, x0, p, b, k, smem);
  else if (p.split == 1 && p.N == 48) ring_inverse_body_ct<T, 48>(S, xs, x0, p, b, k, smem);
  else ring_inverse_body<T>(S, xs, x0, p, b, k, smem);
}

template <class T>
__global__ __launch_bounds__(GENERIC_NT) void ring_forward_kernel(const cpx<T>* __restrict__ samples,
                                                                   cpx<T>* __restrict__ S, RingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ring = blockIdx.x;
  const int b = ring / p.N, k = ring - b * p.N;
  ring_forward_any<T>(samples, ring_offset(p.soff, b, p.N) + (size_t)k * p.N * p.N, S, p, b, k, smem_raw);
}

// The ring's N x N output block starts at element x0 of the sample buffer xs
// (complex, or real for real_io plans: the real part is written).
template <class T>
__device__ void ring_inverse_body(const cpx<T>* __restrict__ S, cpx<T>* __restrict__ xs, size_t x0,
                                  const RingParams<T>& p, int b, int k, unsigned char* smem_raw) {
  const int N = p.N, Nc = p.Nc, R = p.split, twoN = 2 * N;
  cpx<T>* X = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = X + N * Nc;
  for (int t = threadIdx.x; t < twoN; t += blockDim.x) tw[t] = p.tw[t];
  const T scale = p.adjoint ? p.W[k] : T(1);
  for (int r = 0; r < R; r++) {
    __syncthreads();
    for (int e = threadIdx.x; e < N * Nc; e += blockDim.x) X[e] = {T(0), T(0)};
    __syncthreads();
    for (int pi = p.cls_begin[r] + threadIdx.x; pi < p.cls_end[r]; pi += blockDim.x) {
      const int tile = pi / PT;
      cpx<T> v = S[(((size_t)tile * N + k) * p.batch + b) * PT + (pi - tile * PT)];
      X[p.fftpos[pi]] = cscale(cmulc(v, p.rho[pi]), scale);
    }
    __syncthreads();
    run_dit<T>(X, Nc, N, Nc, 1, true, p.rad_n, p.nrad_n, tw, twoN);
    for (int e = threadIdx.x; e < N * Nc; e += blockDim.x) {
      const int j = e / Nc, c = e - j * Nc;
      const int q = R * p.colq[c] + r;
      if ((q & 1) && !p.so3) X[e] = cmulc(X[e], tw[j]);
    }
    __syncthreads();
    run_dit<T>(X, N, Nc, 1, Nc, false, p.rad_c, p.nrad_c, tw, twoN);
    // undo the gamma split: x[j][c + i Nc] += e^{-2 pi i r i / R} w^{-r c} y_r[j][c].
    // Each output element is read and written by the same thread in every class.
    T* xr = reinterpret_cast<T*>(xs);
    for (int e = threadIdx.x; e < N * Nc; e += blockDim.x) {
      const int j = e / Nc, c = e - j * Nc;
      if (R == 1) {
        const size_t o = x0 + (size_t)j * N + c;
        if (p.real_io) xr[o] = X[e].re;
        else xs[o] = X[e];
      } else {
        cpx<T> y = cmulc(X[e], tw[(2 * r * c) % twoN]);
        for (int i = 0; i < R; i++) {
          cpx<T> v = cmulc(y, tw[((twoN / R) * r * i) % twoN]);
          const size_t o = x0 + (size_t)j * N + c + i * Nc;
          if (p.real_io) xr[o] = (r == 0) ? v.re : xr[o] + v.re;
          else xs[o] = (r == 0) ? v : cadd(xs[o], v);
        }
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(GENERIC_NT) void ring_inverse_kernel(const cpx<T>* __restrict__ S,
                                                                   cpx<T>* __restrict__ samples, RingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ring = blockIdx.x;
  const int b = ring / p.N, k = ring - b * p.N;
  ring_inverse_any<T>(S, samples, ring_offset(p.soff, b, p.N) + (size_t)k * p.N * p.N, p, b, k, smem_raw);
}

template <class T>
size_t ring_smem_bytes(const RingParams<T>& p) {
  return (size_t)(p.N * p.Nc + 2 * p.N) * sizeof(cpx<T>);
}

template <class T>
hipError_t launch_ring_forward(const RingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s) {
  const size_t smem = ring_smem_bytes(p);
  hipError_t e = hipFuncSetAttribute((const void*)ring_forward_kernel<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ring_forward_kernel<T>, dim3(p.batch * p.N), dim3(GENERIC_NT), smem, s, samples, S, p);
  return hipGetLastError();
}

template <class T>
hipError_t launch_ring_inverse(const RingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s) {
  const size_t smem = ring_smem_bytes(p);
  hipError_t e = hipFuncSetAttribute((const void*)ring_inverse_kernel<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ring_inverse_kernel<T>, dim3(p.batch * p.N), dim3(GENERIC_NT), smem, s, S, samples, p);
  return hipGetLastError();
}

template size_t ring_smem_bytes<float>(const RingParams<float>&);
template size_t ring_smem_bytes<double>(const RingParams<double>&);
template hipError_t launch_ring_forward<float>(const RingParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_ring_forward<double>(const RingParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);
template hipError_t launch_ring_inverse<float>(const RingParams<float>&, const cpx<float>*, cpx<float>*, hipStream_t);
template hipError_t launch_ring_inverse<double>(const RingParams<double>&, const cpx<double>*, cpx<double>*,
                                                hipStream_t);

}  // namespace su2
