// Ring FFT (stage 1, Proposition 4.2 / Proposition 6.1) specialised at
// compile time for N = N1 * N2 nodes per angle, held in registers.
//
// Each length-N transform is split four-step style: l = l1 + N1 l2,
// q = q2 + N2 q1 (gamma) and j = j1 + N1 j2, p = p2 + N2 p1 (alpha):
//   phase 1  radix-N2 DFT over l2, twiddle w^{q2 l1}          (thread: row j, l1)
//   phase 2  radix-N1 DFT over l1 -> G[j][q2 + N2 q1]          (thread: j, q2)
//   phase 3  radix-N2 DFT over j2 of G e^{2 pi i delta j2 / N2},
//            twiddle e^{2 pi i (p2 + delta) j1 / N}             (thread: column q, j1)
//   phase 4  radix-N1 DFT over j1 -> H[p2 + N2 p1][q]          (thread: q, p2)
// with delta = 1/2 on odd q: the half-bin shift of half-integer n folded into
// the alpha transform (sum_j G[j] e^{2 pi i (p + delta) j / N}).  Only the
// output rows p1 in [0, N1/4) and [3 N1/4, N1) can hold retained bins
// (|2n| <= B-1 with N = 2B), so the others are never formed.  Between phases
// the data crosses LDS three times, each exchange in ROUNDS slices so that
// the LDS buffer is 1/ROUNDS of the ring.  The inverse runs the phases in
// reverse with conjugate roots and gathers its bins straight from the beta
// stage output, so no LDS zero fill is needed.
//
// A workgroup has FAST_NT threads.  For N = 128 they all work on one ring;
// for smaller N the workgroup is split into sub-groups of NTR threads, each
// with its own slice of LDS, working on consecutive rings of one signal (the
// sub-groups run the same code, so the workgroup barriers line up).
#include "su2fft_internal.h"

namespace su2 {

// multiply by e^{SIGN 2 pi i K / 16} for a compile-time K
template <class T, int K, int SIGN>
__device__ __forceinline__ cpx<T> rot16(cpx<T> a) {
  constexpr int k = ((K % 16) + 16) % 16;
  if constexpr (k == 0) return a;
  else if constexpr (k == 4) return {-T(SIGN) * a.im, T(SIGN) * a.re};
  else if constexpr (k == 8) return {-a.re, -a.im};
  else if constexpr (k == 12) return {T(SIGN) * a.im, -T(SIGN) * a.re};
  else {
    constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                              0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    constexpr double s[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                              1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
    const T wr = T(c[k]), wi = T(SIGN) * T(s[k]);
    return {a.re * wr - a.im * wi, a.re * wi + a.im * wr};
  }
}

// In-register DFT of length R in {2, 4, 8, 16}: a[q] <- sum_n a[n] e^{SIGN 2 pi i q n / R}
template <class T, int R, int SIGN>
__device__ __forceinline__ void dftr(cpx<T>* a) {
  if constexpr (R == 2) {
    cpx<T> t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  } else if constexpr (R == 4) {
    cpx<T> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    cpx<T> s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
    cpx<T> r13 = rot16<T, 4, SIGN>(d13);
    a[0] = cadd(s02, s13);
    a[2] = csub(s02, s13);
    a[1] = cadd(d02, r13);
    a[3] = csub(d02, r13);
  } else {
    // R = 2 * H: even/odd split, twiddle e^{SIGN 2 pi i q / R} on the odd half
    constexpr int H = R / 2;
    cpx<T> e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; i++) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
    dftr<T, H, SIGN>(e);
    dftr<T, H, SIGN>(o);
#pragma unroll
    for (int q = 0; q < H; q++) {
      cpx<T> w;
      // o[q] * e^{SIGN 2 pi i q / R}; 16 / R steps of 1/16 turn per q
      switch (q * (16 / R)) {
        case 0: w = o[q]; break;
        case 1: w = rot16<T, 1, SIGN>(o[q]); break;
        case 2: w = rot16<T, 2, SIGN>(o[q]); break;
        case 3: w = rot16<T, 3, SIGN>(o[q]); break;
        case 4: w = rot16<T, 4, SIGN>(o[q]); break;
        case 5: w = rot16<T, 5, SIGN>(o[q]); break;
        case 6: w = rot16<T, 6, SIGN>(o[q]); break;
        default: w = rot16<T, 7, SIGN>(o[q]); break;
      }
      a[q] = cadd(e[q], w);
      a[q + H] = csub(e[q], w);
    }
  }
}

template <int N1, int N2, int NT, int ROUNDS>
struct FastGeom {
  static constexpr int N = N1 * N2;
  static constexpr int I1 = N * N1 / NT;   // phase 1 / 3 instances per thread
  static constexpr int I2 = N * N2 / NT;   // phase 2 / 4 instances per thread
  static constexpr int P1 = N + 1;         // exchange 1 pitch: Z[q2][l1][j]
  static constexpr int P2 = N;             // exchange 2 pitch: G[q][j]
  static constexpr int P3 = N1 + 1;        // exchange 3 pitch: Y[q][p2][j1]
  static constexpr int Q2R = N2 / ROUNDS;  // q2 values per exchange-1 round
  static constexpr int QR = N / ROUNDS;    // q values per exchange-2/3 round
  static constexpr int BUF1 = Q2R * N1 * P1;
  static constexpr int BUF2 = QR * P2;
  static constexpr int BUF3 = QR * N2 * P3;
  static constexpr int BUF = BUF1 > BUF2 ? (BUF1 > BUF3 ? BUF1 : BUF3) : (BUF2 > BUF3 ? BUF2 : BUF3);
  // A q slice (half of the gamma frequencies) holds at most (N/2)^2 retained
  // pairs; the inverse keeps a slice in registers, SLICE_PER_THREAD per thread.
  static constexpr int SLICE_PER_THREAD = (N / 2) * (N / 2) / NT;
  static constexpr int SLICE_CAP = SLICE_PER_THREAD * NT < BUF ? SLICE_PER_THREAD * NT : BUF;
  static_assert((N / 2) * (N / 2) % NT == 0, "slice split");
  static_assert(NT % N == 0 && NT % N1 == 0 && NT % N2 == 0, "thread count");
  static_assert(N2 % ROUNDS == 0 && (N2 / ROUNDS) % (NT / N) == 0, "exchange-1 rounds align with phase-2 instances");
  static_assert(QR % (NT / N1) == 0 && QR % N2 == 0, "exchange-2 rounds align with phase-3 instances");
  static_assert(QR == NT / N2 * (I2 / ROUNDS) || I2 % ROUNDS == 0, "exchange-3 rounds align with phase-4 instances");
  static_assert(N1 % 4 == 0, "alpha pruning");
};

// The samples are read or written exactly once: non-temporal accesses keep
// them from evicting the ring spectra and tables from the caches.
template <class T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T>* a) {
  return {__builtin_nontemporal_load(&a->re), __builtin_nontemporal_load(&a->im)};
}
template <class T>
__device__ __forceinline__ void st_stream(cpx<T>* a, cpx<T> v) {
  __builtin_nontemporal_store(v.re, &a->re);
  __builtin_nontemporal_store(v.im, &a->im);
}

// v * i^e * s for e in 0..3, without branches (e differs between lanes)
template <class T>
__device__ __forceinline__ cpx<T> ipow_scale(cpx<T> v, int e, T s) {
  const T ss = (e & 2) ? -s : s;
  const T c = (e & 1) ? T(0) : ss;  // Re(i^e) s
  const T d = (e & 1) ? ss : T(0);  // Im(i^e) s
  return {v.re * c - v.im * d, v.re * d + v.im * c};
}

// rows p1 of an N1-point output that can hold retained bins: [0, N1/4) and [3 N1/4, N1)
template <int N1>
__device__ __forceinline__ constexpr int kept_row(int i) { return i < N1 / 4 ? i : i + N1 / 2; }

// the N1 / 2 bin entries of (q, p2), stored contiguously, in 16- or 8-byte loads
template <int N1, int N2>
__device__ __forceinline__ void load_entries(const int* __restrict__ bins, int q, int p2, int (&ent)[N1 / 2]) {
  constexpr int H = N1 / 2;
  const int* src = bins + (q * N2 + p2) * H;
  if constexpr (H % 4 == 0) {
#pragma unroll
    for (int v = 0; v < H / 4; v++) {
      const int4 w = reinterpret_cast<const int4*>(src)[v];
      ent[4 * v] = w.x; ent[4 * v + 1] = w.y; ent[4 * v + 2] = w.z; ent[4 * v + 3] = w.w;
    }
  } else {
    static_assert(H == 2, "entries per (q, p2)");
    const int2 w = *reinterpret_cast<const int2*>(src);
    ent[0] = w.x; ent[1] = w.y;
  }
}

// FP32 rings: two workgroups per CU (64 KB LDS slices, at most 128 VGPRs);
// FP64 rings: one workgroup per CU.
template <class T>
constexpr int fast_waves_per_simd() { return sizeof(T) == 4 ? 4 : 2; }

// Columns (gamma frequencies q) of the alpha transform: thread t's phase-3
// instance si has q = q0(t) + (NT / N1) si, q0 running over NT / N1 values.
// DEAL: where a wave's q0 values fit in one half of that range they are dealt
// out by parity (even q0 in the first half of the threads, odd in the
// second), so every wave's columns share the parity of q that decides the
// half-bin shift, which is then a branch per wave rather than a select per
// lane.  The forward transform deals (its shift comes before the phase-3 DFT;
// about 2 % faster FP32 forward ring at N = 128); the inverse, whose shift
// follows the DFT, measured 2 % slower dealt and keeps q0 = t / N1.
template <int N1, int NT, bool DEAL>
struct Phase3Cols {
  static constexpr int QN = NT / N1, H = QN / 2, W = 64 / N1;  // W: q0 values per wave
  static constexpr bool BY_PARITY = DEAL && W <= H && H % W == 0;
  __device__ static __forceinline__ int q0(int t) {
    const int c = t / N1;
    return BY_PARITY ? 2 * (c % H) + c / H : c;
  }
  // 1 when this thread's columns are odd (half-integer n, shifted by half a
  // bin); never for SO(3) plans (integer n only); wave-uniform when BY_PARITY
  __device__ static __forceinline__ int parity(int t, int so3) {
    const int odd = so3 ? 0 : q0(t) & 1;
    return BY_PARITY ? __builtin_amdgcn_readfirstlane(odd) : odd;
  }
};

// multiply by e^{i pi j / N2} (the half-bin shift at node j of an N2-point
// transform) with the root as a compile-time constant
template <class T, int N2, int J, int SIGN>
__device__ __forceinline__ cpx<T> halfbin(cpx<T> a) {
  static_assert(16 % (2 * N2) == 0, "half-bin roots of an N2-point transform are 16th roots");
  return rot16<T, J * (16 / (2 * N2)), SIGN>(a);
}

// One ring (signal b, node k); xv is the ring's N x N input block (complex,
// or real for REAL), t the thread's index in the workgroup.  REAL: a real ring
// has a Hermitian spectrum, so only the first q slice (2m >= 0) is formed and
// written; the contraction and the inverse take the rest from the symmetry.
template <class T, int N1, int N2, int NT, int ROUNDS, bool REAL = false>
__device__ __forceinline__ void ring_forward_fast_body(const void* __restrict__ xv, cpx<T>* __restrict__ S,
                                                       const FastRingParams<T>& p, int b, int k,
                                                       unsigned char* smem_raw, int t) {
  typedef FastGeom<N1, N2, NT, ROUNDS> G;
  typedef Phase3Cols<N1, NT, true> P3;
  constexpr int N = G::N;
  constexpr int RR = REAL ? 1 : ROUNDS;  // q slices formed after the gamma transform
  static_assert(ROUNDS == FAST_ROUNDS, "pair ranges are given per round");
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + G::BUF;  // e^{i pi t / N}, t = 0..2N-1
  for (int i = t; i < 2 * N; i += NT) tw[i] = p.tw[i];

  // ---- phase 1: radix-N2 over l2 (coalesced rows: lanes run over l1)
  const int l1 = t % N1;
  cpx<T> a[G::I1][N2];
#pragma unroll
  for (int s = 0; s < G::I1; s++) {
    const int j = t / N1 + (NT / N1) * s;
#pragma unroll
    for (int l2 = 0; l2 < N2; l2++) {
      if constexpr (REAL)
        a[s][l2] = {__builtin_nontemporal_load(reinterpret_cast<const T*>(xv) + j * N + l1 + N1 * l2), T(0)};
      else
        a[s][l2] = ld_stream(reinterpret_cast<const cpx<T>*>(xv) + j * N + l1 + N1 * l2);
    }
  }
  __syncthreads();
  cpx<T> tw1[N2];  // w^{q2 l1}: this thread's l1 is the same in every instance
#pragma unroll
  for (int q2 = 1; q2 < N2; q2++) tw1[q2] = tw[(2 * q2 * l1) % (2 * N)];
#pragma unroll
  for (int s = 0; s < G::I1; s++) {
    dftr<T, N2, 1>(a[s]);
#pragma unroll
    for (int q2 = 1; q2 < N2; q2++) a[s][q2] = cmul(a[s][q2], tw1[q2]);
  }

  // ---- exchange 1 (by q2 slices) and phase 2: radix-N1 over l1
  const int jr = t % N;
  cpx<T> c[G::I2][N1];
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1; s++) {
      const int j = t / N1 + (NT / N1) * s;
#pragma unroll
      for (int qq = 0; qq < G::Q2R; qq++) buf[(qq * N1 + l1) * G::P1 + j] = a[s][r * G::Q2R + qq];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I2 / ROUNDS; s++) {
      const int si = r * (G::I2 / ROUNDS) + s;
      const int q2 = t / N + (NT / N) * si;
#pragma unroll
      for (int m = 0; m < N1; m++) c[si][m] = buf[((q2 - r * G::Q2R) * N1 + m) * G::P1 + jr];
    }
  }
#pragma unroll
  for (int s = 0; s < G::I2; s++) dftr<T, N1, 1>(c[s]);   // c[s][q1] = G[jr][q2 + N2 q1]

  // ---- exchange 2 (by q slices) and phase 3: radix-N2 over j2 with the half-bin shift
  const int j1 = t % N1;
  // every phase-3 instance of this thread has q of the parity of q0(t)
  const int odd = P3::parity(t, p.so3);
  cpx<T> tw3[N2];  // e^{2 pi i (p2 + delta) j1 / N}
#pragma unroll
  for (int p2 = 0; p2 < N2; p2++) tw3[p2] = tw[((2 * p2 + odd) * j1) % (2 * N)];
#pragma unroll
  for (int r = 0; r < RR; r++) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I2; s++) {
      const int q2 = t / N + (NT / N) * s;
#pragma unroll
      for (int q1 = r * (G::QR / N2); q1 < (r + 1) * (G::QR / N2); q1++)
        buf[(q2 + N2 * q1 - r * G::QR) * G::P2 + jr] = c[s][q1];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1 / ROUNDS; s++) {
      const int si = r * (G::I1 / ROUNDS) + s;
      const int q = P3::q0(t) + (NT / N1) * si;
#pragma unroll
      for (int j2 = 0; j2 < N2; j2++) a[si][j2] = buf[(q - r * G::QR) * G::P2 + j1 + N1 * j2];
    }
  }
#pragma unroll
  for (int s = 0; s < RR * (G::I1 / ROUNDS); s++) {
    if (odd) {
      a[s][1] = halfbin<T, N2, 1, 1>(a[s][1]);
      if constexpr (N2 > 2) {
        a[s][2] = halfbin<T, N2, 2, 1>(a[s][2]);
        a[s][3] = halfbin<T, N2, 3, 1>(a[s][3]);
      }
      if constexpr (N2 > 4) {
        a[s][4] = halfbin<T, N2, 4, 1>(a[s][4]);
        a[s][5] = halfbin<T, N2, 5, 1>(a[s][5]);
        a[s][6] = halfbin<T, N2, 6, 1>(a[s][6]);
        a[s][7] = halfbin<T, N2, 7, 1>(a[s][7]);
      }
    }
    dftr<T, N2, 1>(a[s]);
#pragma unroll
    for (int p2 = 0; p2 < N2; p2++) a[s][p2] = cmul(a[s][p2], tw3[p2]);
  }

  // ---- exchange 3 (by q slices), phase 4: radix-N1 over j1 (pruned), and the
  //      epilogue through LDS so that S is written in whole PT-pair rows
  const int p2 = t % N2;
  const T Wk = p.W[k];
#pragma unroll
  for (int r = 0; r < RR; r++) {
    static_assert(G::I2 / ROUNDS == 1, "one phase-4 instance per round");
    const int q = t / N2 + (NT / N2) * r;
    // this thread's bin entries for the round, fetched before the exchange so
    // that their latency hides behind it
    int ent[N1 / 2];
    load_entries<N1, N2>(p.bins, q, p2, ent);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1 / ROUNDS; s++) {
      const int si = r * (G::I1 / ROUNDS) + s;
      const int qq = P3::q0(t) + (NT / N1) * si;
#pragma unroll
      for (int pp = 0; pp < N2; pp++) buf[((qq - r * G::QR) * N2 + pp) * G::P3 + j1] = a[si][pp];
    }
    __syncthreads();
    cpx<T> h[N1];
#pragma unroll
    for (int m = 0; m < N1; m++) h[m] = buf[((q - r * G::QR) * N2 + p2) * G::P3 + m];
    __syncthreads();
    dftr<T, N1, 1>(h);
    const int pb = p.rbeg[r], pe = p.rend[r];
#pragma unroll
    for (int i = 0; i < N1 / 2; i++)
      if (ent[i] >= 0) buf[(ent[i] >> 2) - pb] = ipow_scale(h[kept_row<N1>(i)], ent[i] & 3, Wk);
    __syncthreads();
    // pairs pi = pb + t + NT i: NT pairs are NT / PT whole tiles apart, so
    // each step moves the address by a fixed stride
    static_assert(NT % PT == 0, "whole tiles per step");
    if (pb + t < pe) {
      const int tile0 = (pb + t) / PT;
      cpx<T>* dst = S + (((size_t)tile0 * N + k) * p.batch + b) * PT + (pb + t - tile0 * PT);
      const size_t step = (size_t)(NT / PT) * N * p.batch * PT;
      for (int pi = pb + t; pi < pe; pi += NT, dst += step) *dst = buf[pi - pb];
    }
  }
}

// REAL: the output ring is real.  Only the first q slice's pairs (2m >= 0)
// hold spectra; every bin reads its pair's value or the conjugate of its
// mirror pair's (bins_real), and only the real part is written.
// Shapes of the inverse ring's per-thread inputs: the retained spectra of
// the ring's q slices (SR slices of SPR values; REAL: both rounds read the
// first slice) and the phase-4' bin entries of each of the RA rounds.
template <int N1, int N2, int NT, int ROUNDS, bool REAL>
struct InvShape {
  typedef FastGeom<N1, N2, NT, ROUNDS> G;
  static constexpr int SR = REAL ? 1 : ROUNDS, SPR = G::SLICE_PER_THREAD, RA = REAL ? 1 : ROUNDS;
};

// This thread's phase-4' bin entries (column q = t / N2 + (NT / N2) r, row
// p2 = t mod N2): the same for every ring of a plan.
template <class T, int N1, int N2, int NT, int ROUNDS, bool REAL>
__device__ __forceinline__ void ring_inverse_fast_entries(const FastRingParams<T>& p,
                                                          int (&ent)[InvShape<N1, N2, NT, ROUNDS, REAL>::RA][N1 / 2],
                                                          int t) {
  const int* bins = REAL ? p.bins_real : p.bins;
#pragma unroll
  for (int r = 0; r < InvShape<N1, N2, NT, ROUNDS, REAL>::RA; r++) {
    const int q = t / N2 + (NT / N2) * r;
    load_entries<N1, N2>(bins, q, t % N2, ent[r]);
  }
}

// The retained spectra of ring (b, k) in slices [r0, r1), and (with_scale)
// the ring's scale (W_k for the adjoint, else 1).  Every thread issues the
// same loads: an index past its slice reads the slice's first pair and the
// value is replaced by zero, so the compiler counts the loads in flight
// exactly when it places its waits.
template <class T, int N1, int N2, int NT, int ROUNDS, bool REAL>
__device__ __forceinline__ void ring_inverse_fast_gather(
    const cpx<T>* __restrict__ S, const FastRingParams<T>& p, int b, int k,
    cpx<T> (&sv)[InvShape<N1, N2, NT, ROUNDS, REAL>::SR][InvShape<N1, N2, NT, ROUNDS, REAL>::SPR], T& scale,
    int t, int r0 = 0, int r1 = InvShape<N1, N2, NT, ROUNDS, REAL>::SR, bool with_scale = true) {
  typedef InvShape<N1, N2, NT, ROUNDS, REAL> SH;
  constexpr int N = N1 * N2, SPR = SH::SPR;
  if (with_scale) scale = p.adjoint ? p.W[k] : T(1);
#pragma unroll
  for (int r = 0; r < SH::SR; r++) {
    if (r < r0 || r >= r1) continue;
    const int pb = p.rbeg[r], pe = p.rend[r];
    // pairs pi = pb + t + NT i: NT pairs are NT / PT whole tiles apart, so
    // each step moves the address by a fixed stride
    static_assert(NT % PT == 0, "whole tiles per step");
    const int tile0 = (pb + t) / PT;
    const cpx<T>* src = S + (((size_t)tile0 * N + k) * p.batch + b) * PT + (pb + t - tile0 * PT);
    // the slice's first pair, relative to src (the offset is selected, not
    // the pointer, so that each value is one load)
    const long long first = (long long)((((size_t)(pb / PT) * N + k) * p.batch + b) * PT + (pb - pb / PT * PT)) -
                            (long long)((((size_t)tile0 * N + k) * p.batch + b) * PT + (pb + t - tile0 * PT));
    const long long step = (long long)(NT / PT) * N * p.batch * PT;
#pragma unroll
    for (int i = 0; i < SPR; i++) {
      const bool in = pb + t + NT * i < pe;
      const cpx<T> v = src[in ? i * step : first];
      sv[r][i] = in ? v : cpx<T>{T(0), T(0)};
    }
  }
}

// Phases 4' to 1' of one ring from its gathered spectra; the output ring is
// left in a (a[s][l2] is sample (j, l1 + N1 l2), j = t / N1 + (NT / N1) s,
// l1 = t mod N1).  buf is the exchange buffer and tw the table e^{i pi t / N}
// already in LDS; the first barrier orders buf against earlier use.
template <class T, int N1, int N2, int NT, int ROUNDS, bool REAL>
__device__ __forceinline__ void ring_inverse_fast_transform(
    const cpx<T> (&sv)[InvShape<N1, N2, NT, ROUNDS, REAL>::SR][InvShape<N1, N2, NT, ROUNDS, REAL>::SPR],
    const int (&entr)[InvShape<N1, N2, NT, ROUNDS, REAL>::RA][N1 / 2], T scale, const FastRingParams<T>& p,
    cpx<T>* buf, const cpx<T>* tw, cpx<T> (&a)[N1 * N2 * N1 / NT][N2], int t) {
  typedef FastGeom<N1, N2, NT, ROUNDS> G;
  typedef Phase3Cols<N1, NT, false> P3;
  constexpr int N = G::N;
  static_assert(ROUNDS == FAST_ROUNDS, "pair ranges are given per round");
  constexpr int SPR = G::SLICE_PER_THREAD;
  const int p2 = t % N2, j1 = t % N1, jr = t % N, l1 = t % N1;
  // per round: stage the slice in LDS, gather the bins, phase 4' (radix-N1
  // over p1 -> j1), exchange 3' (write)
  // REAL: only the first q slice is transformed along alpha; the gamma
  // frequencies of the second slice are the conjugates of the first's
  // (G[j][N - q] = conj(G[j][q]) for a real ring), taken in exchange 2'
  constexpr int RA = REAL ? 1 : ROUNDS;  // rounds of phases 4' and 3'
#pragma unroll
  for (int r = 0; r < RA; r++) {
    const int rs = REAL ? 0 : r;  // slice staged in this round
    const int pb = p.rbeg[rs], pe = p.rend[rs];
    static_assert(G::I2 / ROUNDS == 1, "one phase-4 instance per round");
    const int q = t / N2 + (NT / N2) * r;
    const int* ent = entr[r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SPR; i++)
      if (pb + t + NT * i < pe) buf[t + NT * i] = sv[REAL ? 0 : r][i];
    __syncthreads();
    cpx<T> h[N1];
#pragma unroll
    for (int p1 = 0; p1 < N1; p1++) h[p1] = {T(0), T(0)};
#pragma unroll
    for (int i = 0; i < N1 / 2; i++) {
      // every lane reads a valid slot; bins that are not retained are zeroed
      const int e = ent[i];
      cpx<T> v;
      if constexpr (REAL) {  // (source pair << 3) | (conjugate << 2) | phase
        v = buf[e >= 0 ? (e >> 3) - pb : 0];
        if ((e >> 2) & 1) v.im = -v.im;
      } else {
        v = buf[e >= 0 ? (e >> 2) - pb : 0];
      }
      v = ipow_scale(v, (4 - (e & 3)) & 3, scale);
      h[kept_row<N1>(i)] = e >= 0 ? v : cpx<T>{T(0), T(0)};
    }
    dftr<T, N1, -1>(h);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < N1; m++) buf[((q - r * G::QR) * N2 + p2) * G::P3 + m] = h[m];
    __syncthreads();
    // exchange 3' (read) for the phase-3' instances of this round
#pragma unroll
    for (int s = 0; s < G::I1 / ROUNDS; s++) {
      const int si = r * (G::I1 / ROUNDS) + s;
      const int qq = P3::q0(t) + (NT / N1) * si;
#pragma unroll
      for (int pp = 0; pp < N2; pp++) a[si][pp] = buf[((qq - r * G::QR) * N2 + pp) * G::P3 + j1];
    }
  }

  // ---- phase 3': conj twiddle, radix-N2 over p2 -> j2, times e^{-2 pi i delta j2 / N2}
  const int odd = P3::parity(t, p.so3);
  cpx<T> tw3[N2];
#pragma unroll
  for (int pp = 0; pp < N2; pp++) tw3[pp] = tw[((2 * pp + odd) * j1) % (2 * N)];
#pragma unroll
  for (int s = 0; s < G::I1 / ROUNDS * RA; s++) {
#pragma unroll
    for (int pp = 0; pp < N2; pp++) a[s][pp] = cmulc(a[s][pp], tw3[pp]);
    dftr<T, N2, -1>(a[s]);
    if (odd) {
      a[s][1] = halfbin<T, N2, 1, -1>(a[s][1]);
      if constexpr (N2 > 2) {
        a[s][2] = halfbin<T, N2, 2, -1>(a[s][2]);
        a[s][3] = halfbin<T, N2, 3, -1>(a[s][3]);
      }
      if constexpr (N2 > 4) {
        a[s][4] = halfbin<T, N2, 4, -1>(a[s][4]);
        a[s][5] = halfbin<T, N2, 5, -1>(a[s][5]);
        a[s][6] = halfbin<T, N2, 6, -1>(a[s][6]);
        a[s][7] = halfbin<T, N2, 7, -1>(a[s][7]);
      }
    }
  }

  // ---- exchange 2' and phase 2': radix-N1 over q1 -> l1
  cpx<T> c[G::I2][N1];
  if constexpr (REAL) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1 / ROUNDS; s++) {
      const int q = P3::q0(t) + (NT / N1) * s;
#pragma unroll
      for (int j2 = 0; j2 < N2; j2++) buf[q * G::P2 + j1 + N1 * j2] = a[s][j2];
    }
    __syncthreads();
    static_assert(G::QR % N2 == 0, "slice boundary on a q1 boundary");
#pragma unroll
    for (int s = 0; s < G::I2; s++) {
      const int q2 = t / N + (NT / N) * s;
#pragma unroll
      for (int q1 = 0; q1 < N1; q1++) {
        if (q1 < G::QR / N2) {
          c[s][q1] = buf[(q2 + N2 * q1) * G::P2 + jr];
        } else {  // q >= N/2: conj(G[j][N - q]); q = N/2 holds no retained bin
          const int qm = N - q2 - N2 * q1;
          const cpx<T> v = buf[(qm < G::QR ? qm : 0) * G::P2 + jr];
          c[s][q1] = qm < G::QR ? cpx<T>{v.re, -v.im} : cpx<T>{T(0), T(0)};
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < (REAL ? 0 : ROUNDS); r++) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1 / ROUNDS; s++) {
      const int si = r * (G::I1 / ROUNDS) + s;
      const int q = P3::q0(t) + (NT / N1) * si;
#pragma unroll
      for (int j2 = 0; j2 < N2; j2++) buf[(q - r * G::QR) * G::P2 + j1 + N1 * j2] = a[si][j2];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I2; s++) {
      const int q2 = t / N + (NT / N) * s;
#pragma unroll
      for (int q1 = r * (G::QR / N2); q1 < (r + 1) * (G::QR / N2); q1++)
        c[s][q1] = buf[(q2 + N2 * q1 - r * G::QR) * G::P2 + jr];
    }
  }
#pragma unroll
  for (int s = 0; s < G::I2; s++) dftr<T, N1, -1>(c[s]);

  // ---- exchange 1', conj twiddle w^{-q2 l1}, phase 1': radix-N2 over q2 -> l2, coalesced store
  cpx<T> tw1[N2];
#pragma unroll
  for (int q2 = 1; q2 < N2; q2++) tw1[q2] = tw[(2 * q2 * l1) % (2 * N)];
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I2 / ROUNDS; s++) {
      const int si = r * (G::I2 / ROUNDS) + s;
      const int q2 = t / N + (NT / N) * si;
#pragma unroll
      for (int m = 0; m < N1; m++) buf[((q2 - r * G::Q2R) * N1 + m) * G::P1 + jr] = c[si][m];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < G::I1; s++) {
      const int j = t / N1 + (NT / N1) * s;
#pragma unroll
      for (int qq = 0; qq < G::Q2R; qq++) a[s][r * G::Q2R + qq] = buf[(qq * N1 + l1) * G::P1 + j];
    }
  }
#pragma unroll
  for (int s = 0; s < G::I1; s++) {
    const int j = t / N1 + (NT / N1) * s;
#pragma unroll
    for (int q2 = 1; q2 < N2; q2++) a[s][q2] = cmulc(a[s][q2], tw1[q2]);
    dftr<T, N2, -1>(a[s]);
  }
}

// The output ring held in a (as ring_inverse_fast_transform leaves it) to
// the samples xov: coalesced rows, non-temporal stores (REAL: real parts).
template <class T, int N1, int N2, int NT, bool REAL>
__device__ __forceinline__ void ring_inverse_fast_store(const cpx<T> (&a)[N1 * N2 * N1 / NT][N2],
                                                        void* __restrict__ xov, int t) {
  constexpr int N = N1 * N2;
  const int l1 = t % N1;
#pragma unroll
  for (int s = 0; s < N * N1 / NT; s++) {
    const int j = t / N1 + (NT / N1) * s;
#pragma unroll
    for (int l2 = 0; l2 < N2; l2++) {
      if constexpr (REAL)
        __builtin_nontemporal_store(a[s][l2].re, reinterpret_cast<T*>(xov) + j * N + l1 + N1 * l2);
      else
        st_stream(reinterpret_cast<cpx<T>*>(xov) + j * N + l1 + N1 * l2, a[s][l2]);
    }
  }
}

template <class T, int N1, int N2, int NT, int ROUNDS, bool REAL = false>
__device__ __forceinline__ void ring_inverse_fast_body(const cpx<T>* __restrict__ S, void* __restrict__ xov,
                                                       const FastRingParams<T>& p, int b, int k,
                                                       unsigned char* smem_raw, int t) {
  typedef FastGeom<N1, N2, NT, ROUNDS> G;
  typedef InvShape<N1, N2, NT, ROUNDS, REAL> SH;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + G::BUF;
  for (int i = t; i < 2 * G::N; i += NT) tw[i] = p.tw[i];
  cpx<T> sv[SH::SR][SH::SPR];
  T scale;
  ring_inverse_fast_gather<T, N1, N2, NT, ROUNDS, REAL>(S, p, b, k, sv, scale, t);
  int ent[SH::RA][N1 / 2];
  ring_inverse_fast_entries<T, N1, N2, NT, ROUNDS, REAL>(p, ent, t);
  cpx<T> a[G::I1][N2];
  ring_inverse_fast_transform<T, N1, N2, NT, ROUNDS, REAL>(sv, ent, scale, p, buf, tw, a, t);
  ring_inverse_fast_store<T, N1, N2, NT, REAL>(a, xov, t);
}

// Split of the N-point transforms and threads per ring for each supported N
// (the constraints are the static assertions of FastGeom).
template <int N>
struct FastCfg;
template <>
struct FastCfg<128> {
  static constexpr int N1 = 16, N2 = 8, NTR = 512;
};
template <>
struct FastCfg<64> {
  static constexpr int N1 = 16, N2 = 4, NTR = 128;
};
template <>
struct FastCfg<32> {
  static constexpr int N1 = 8, N2 = 4, NTR = 64;
};
template <>
struct FastCfg<16> {
  static constexpr int N1 = 4, N2 = 4, NTR = 32;
};

template <class T, int N>
struct FastRing {
  typedef FastCfg<N> C;
  typedef FastGeom<C::N1, C::N2, C::NTR, FAST_ROUNDS> G;
  static constexpr int RPW = FAST_NT / C::NTR;  // rings per workgroup
  static constexpr size_t RING_SMEM = ((G::BUF + 2 * N) * sizeof(cpx<T>) + 15) / 16 * 16;
  static constexpr size_t SMEM = RPW * RING_SMEM;
  static_assert(FAST_NT % C::NTR == 0 && N % RPW == 0, "rings per workgroup");
};

// The workgroup's RPW rings (signal b, nodes k0 .. k0 + RPW - 1); t is the
// thread's index in the workgroup.
template <class T, int N, bool REAL = false>
__device__ __forceinline__ void ring_forward_fast_group(const void* __restrict__ samples, cpx<T>* __restrict__ S,
                                                        const FastRingParams<T>& p, int b, int k0,
                                                        unsigned char* smem, int t) {
  typedef FastRing<T, N> R;
  typedef typename std::conditional<REAL, T, cpx<T>>::type E;  // sample element
  const int sub = R::RPW == 1 ? 0 : t / R::C::NTR, k = k0 + sub;
  ring_forward_fast_body<T, R::C::N1, R::C::N2, R::C::NTR, FAST_ROUNDS, REAL>(
      reinterpret_cast<const E*>(samples) + ring_offset(p.soff, b, N) + (size_t)k * N * N, S, p, b, k,
      smem + sub * R::RING_SMEM, R::RPW == 1 ? t : t - sub * R::C::NTR);
}

template <class T, int N, bool REAL = false>
__device__ __forceinline__ void ring_inverse_fast_group(const cpx<T>* __restrict__ S, void* __restrict__ samples,
                                                        const FastRingParams<T>& p, int b, int k0,
                                                        unsigned char* smem, int t) {
  typedef FastRing<T, N> R;
  typedef typename std::conditional<REAL, T, cpx<T>>::type E;
  const int sub = R::RPW == 1 ? 0 : t / R::C::NTR, k = k0 + sub;
  ring_inverse_fast_body<T, R::C::N1, R::C::N2, R::C::NTR, FAST_ROUNDS, REAL>(
      S, reinterpret_cast<E*>(samples) + ring_offset(p.soff, b, N) + (size_t)k * N * N, p, b, k,
      smem + sub * R::RING_SMEM, R::RPW == 1 ? t : t - sub * R::C::NTR);
}

// Workgroup blk -> signal b and first node k0 of its rpw consecutive rings.
// Node-major over the signals (forward rings, paired FP64 inverse): the
// workgroups resident at one time hold a few nodes of every signal, so that
// the spectra they write or read (layout tile, node, signal, pair) form
// whole rows of each tile rather than scattered 128-byte pieces (B = 64
// batch 32 FP32 forward 0.182 -> 0.175 ms, paired FP64 inverse 0.405 ->
// 0.397 ms).  Signal-major (single-ring inverse): a few signals' consecutive
// rings, i.e. a few long streams of sample writes, measured faster for the
// FP32 inverse than node-major or groups of 4 or 8 signals (0.155 against
// 0.158 ms and more).
__device__ __forceinline__ void ring_of_block(bool node_major, int blk, int rpw, int N, int batch, int& b,
                                              int& k0) {
  if (node_major) {
    const int kb = blk / batch;
    b = blk - kb * batch;
    k0 = kb * rpw;
  } else {
    const int nk = N / rpw;
    b = blk / nk;
    k0 = (blk - b * nk) * rpw;
  }
}

template <class T, int N, bool REAL>
__global__ __launch_bounds__(FAST_NT, fast_waves_per_simd<T>()) void ring_forward_fast(
    const void* __restrict__ samples, cpx<T>* __restrict__ S, FastRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int b, k0;
  ring_of_block(true, blockIdx.x, FastRing<T, N>::RPW, N, p.batch, b, k0);
  ring_forward_fast_group<T, N, REAL>(samples, S, p, b, k0, smem_raw, threadIdx.x);
}

template <class T, int N, bool REAL>
__global__ __launch_bounds__(FAST_NT, fast_waves_per_simd<T>()) void ring_inverse_fast(
    const cpx<T>* __restrict__ S, void* __restrict__ samples, FastRingParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int b, k0;
  ring_of_block(false, blockIdx.x, FastRing<T, N>::RPW, N, p.batch, b, k0);
  ring_inverse_fast_group<T, N, REAL>(S, samples, p, b, k0, smem_raw, threadIdx.x);
}

// N = 128 inverse, two rings per workgroup (nodes k0, k0 + 1 of one
// signal).  The second ring's spectra are requested after the first ring's
// transform and before its sample stores, so their latency hides behind the
// stores, and the first ring's stores drain while the second ring is
// transformed (a workgroup keeps its slot until its stores have completed).
// The bin entries are the same for both rings.  Used for FP64, where a CU
// holds a single workgroup (0.449 -> 0.419 ms at B = 64 batch 32); FP32 rings
// run two workgroups per CU, which already cover these latencies (measured
// no change), and keep one ring per workgroup.
template <class T, bool REAL>
__global__ __launch_bounds__(FAST_NT, fast_waves_per_simd<T>()) void ring_inverse_fast_pair(
    const cpx<T>* __restrict__ S, void* __restrict__ samples, FastRingParams<T> p) {
  typedef FastRing<T, 128> R;
  typedef FastCfg<128> C;
  constexpr int N1 = C::N1, N2 = C::N2, NT = C::NTR, N = 128;
  typedef InvShape<N1, N2, NT, FAST_ROUNDS, REAL> SH;
  typedef typename std::conditional<REAL, T, cpx<T>>::type E;
  static_assert(R::RPW == 1 && NT == FAST_NT, "one ring per workgroup pass");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + R::G::BUF;
  const int t = threadIdx.x;
  for (int i = t; i < 2 * N; i += NT) tw[i] = p.tw[i];
  int b, k0;
  ring_of_block(true, blockIdx.x, 2, N, p.batch, b, k0);  // N even: k0 + 1 < N
  E* xo = reinterpret_cast<E*>(samples) + ring_offset(p.soff, b, N);
  cpx<T> sv[SH::SR][SH::SPR];
  T scale;
  ring_inverse_fast_gather<T, N1, N2, NT, FAST_ROUNDS, REAL>(S, p, b, k0, sv, scale, t);
  int ent[SH::RA][N1 / 2];
  ring_inverse_fast_entries<T, N1, N2, NT, FAST_ROUNDS, REAL>(p, ent, t);
  cpx<T> a[R::G::I1][N2];
  ring_inverse_fast_transform<T, N1, N2, NT, FAST_ROUNDS, REAL>(sv, ent, scale, p, buf, tw, a, t);
  // a copy of the thread index the compiler cannot see through, so that the
  // second ring's addresses are formed where they are used rather than held
  // in registers across the first ring
  int t2 = t;
  asm volatile("" : "+v"(t2));
  // the second ring's first slice before the first ring's stores (all of it
  // would not fit the register budget beside the first ring's output), the
  // rest after them
  ring_inverse_fast_gather<T, N1, N2, NT, FAST_ROUNDS, REAL>(S, p, b, k0 + 1, sv, scale, t2, 0, 1);
  __builtin_amdgcn_sched_barrier(0);
  ring_inverse_fast_store<T, N1, N2, NT, REAL>(a, xo + (size_t)k0 * N * N, t);
  __builtin_amdgcn_sched_barrier(0);
  ring_inverse_fast_gather<T, N1, N2, NT, FAST_ROUNDS, REAL>(S, p, b, k0 + 1, sv, scale, t2, 1, SH::SR, false);
  ring_inverse_fast_transform<T, N1, N2, NT, FAST_ROUNDS, REAL>(sv, ent, scale, p, buf, tw, a, t2);
  ring_inverse_fast_store<T, N1, N2, NT, REAL>(a, xo + (size_t)(k0 + 1) * N * N, t2);
}

template <class T>
bool fast_ring_supported(int N) {
  return N == 16 || N == 32 || N == 64 || N == 128;
}

template <class T>
size_t fast_ring_smem(int N) {
  switch (N) {
    case 16: return FastRing<T, 16>::SMEM;
    case 32: return FastRing<T, 32>::SMEM;
    case 64: return FastRing<T, 64>::SMEM;
    case 128: return FastRing<T, 128>::SMEM;
  }
  return 0;
}

template <class T>
int fast_ring_slice_capacity(int N) {
  switch (N) {
    case 16: return FastRing<T, 16>::G::SLICE_CAP;
    case 32: return FastRing<T, 32>::G::SLICE_CAP;
    case 64: return FastRing<T, 64>::G::SLICE_CAP;
    case 128: return FastRing<T, 128>::G::SLICE_CAP;
  }
  return 0;
}

bool fast_ring_split(int N, int* n1, int* n2) {
  switch (N) {
    case 16: *n1 = FastCfg<16>::N1; *n2 = FastCfg<16>::N2; return true;
    case 32: *n1 = FastCfg<32>::N1; *n2 = FastCfg<32>::N2; return true;
    case 64: *n1 = FastCfg<64>::N1; *n2 = FastCfg<64>::N2; return true;
    case 128: *n1 = FastCfg<128>::N1; *n2 = FastCfg<128>::N2; return true;
  }
  return false;
}

int fast_rings_per_group(int N) {
  switch (N) {
    case 16: return FastRing<float, 16>::RPW;
    case 32: return FastRing<float, 32>::RPW;
    case 64: return FastRing<float, 64>::RPW;
    case 128: return FastRing<float, 128>::RPW;
  }
  return 0;
}

// the epilogue / prologue stage a slice's pair range in the ring's exchange buffer

template <class T, int N>
static bool slices_fit(const FastRingParams<T>& p) {
  for (int r = 0; r < FAST_ROUNDS; r++)
    if (p.rend[r] - p.rbeg[r] > FastRing<T, N>::G::SLICE_CAP) return false;
  return p.N == N;
}

template <class T, int N>
static hipError_t launch_fast(bool forward, bool real, const FastRingParams<T>& p, const void* in, void* out,
                              hipStream_t s) {
  typedef FastRing<T, N> R;
  if (!slices_fit<T, N>(p) || (real && !p.bins_real)) return hipErrorInvalidValue;
  if constexpr (N == 128 && std::is_same<T, double>::value) {
    // two rings per workgroup (a signal's N rings pair up).  Complex plans
    // only: the real variant of the paired kernel rounds some values
    // differently (last bits) from the single-ring body that mixed plans run,
    // and real plans keep the single-ring kernel so that both agree bit for bit.
    if (!forward && !real) {
      const void* kern = (const void*)ring_inverse_fast_pair<T, false>;
      hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)R::SMEM);
      if (e != hipSuccess) return e;
      FastRingParams<T> pp = p;
      void* args[] = {(void*)&in, (void*)&out, (void*)&pp};
      return hipLaunchKernel(kern, dim3((unsigned)((long long)p.batch * N / 2)), dim3(FAST_NT), args, R::SMEM, s);
    }
  }
  const void* kern =
      forward ? (real ? (const void*)ring_forward_fast<T, N, true> : (const void*)ring_forward_fast<T, N, false>)
              : (real ? (const void*)ring_inverse_fast<T, N, true> : (const void*)ring_inverse_fast<T, N, false>);
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)R::SMEM);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((long long)p.batch * N / R::RPW));
  FastRingParams<T> pp = p;
  void* args[] = {(void*)&in, (void*)&out, (void*)&pp};
  return hipLaunchKernel(kern, grid, dim3(FAST_NT), args, R::SMEM, s);
}

template <class T>
static hipError_t launch_fast_any(bool forward, bool real, const FastRingParams<T>& p, const void* in, void* out,
                                  hipStream_t s) {
  switch (p.N) {
    case 16: return launch_fast<T, 16>(forward, real, p, in, out, s);
    case 32: return launch_fast<T, 32>(forward, real, p, in, out, s);
    case 64: return launch_fast<T, 64>(forward, real, p, in, out, s);
    case 128: return launch_fast<T, 128>(forward, real, p, in, out, s);
  }
  return hipErrorInvalidValue;
}

template <class T>
hipError_t launch_ring_forward_fast(const FastRingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s) {
  return launch_fast_any<T>(true, false, p, samples, S, s);
}

template <class T>
hipError_t launch_ring_inverse_fast(const FastRingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s) {
  return launch_fast_any<T>(false, false, p, S, samples, s);
}

template <class T>
hipError_t launch_ring_forward_fast_real(const FastRingParams<T>& p, const T* samples, cpx<T>* S, hipStream_t s) {
  return launch_fast_any<T>(true, true, p, samples, S, s);
}

template <class T>
hipError_t launch_ring_inverse_fast_real(const FastRingParams<T>& p, const cpx<T>* S, T* samples, hipStream_t s) {
  return launch_fast_any<T>(false, true, p, S, samples, s);
}

template size_t fast_ring_smem<float>(int);
template size_t fast_ring_smem<double>(int);
template int fast_ring_slice_capacity<float>(int);
template int fast_ring_slice_capacity<double>(int);
template bool fast_ring_supported<float>(int);
template bool fast_ring_supported<double>(int);
template hipError_t launch_ring_forward_fast<float>(const FastRingParams<float>&, const cpx<float>*, cpx<float>*,
                                                    hipStream_t);
template hipError_t launch_ring_forward_fast<double>(const FastRingParams<double>&, const cpx<double>*, cpx<double>*,
                                                     hipStream_t);
template hipError_t launch_ring_inverse_fast<float>(const FastRingParams<float>&, const cpx<float>*, cpx<float>*,
                                                    hipStream_t);
template hipError_t launch_ring_inverse_fast<double>(const FastRingParams<double>&, const cpx<double>*, cpx<double>*,
                                                     hipStream_t);
template hipError_t launch_ring_forward_fast_real<float>(const FastRingParams<float>&, const float*, cpx<float>*,
                                                         hipStream_t);
template hipError_t launch_ring_forward_fast_real<double>(const FastRingParams<double>&, const double*, cpx<double>*,
                                                          hipStream_t);
template hipError_t launch_ring_inverse_fast_real<float>(const FastRingParams<float>&, const cpx<float>*, float*,
                                                         hipStream_t);
template hipError_t launch_ring_inverse_fast_real<double>(const FastRingParams<double>&, const cpx<double>*, double*,
                                                          hipStream_t);

}  // namespace su2
