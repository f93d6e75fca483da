// Internal declarations shared by the su2fft host code and its HIP kernels.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/su2fft.h"

namespace su2 {

// Pairs (m, n) are processed in tiles of PT consecutive pairs.  The
// intermediate ring spectra live in the plan workspace as
//   S[tile][k][b][PT]   (complex),
// so that a ring (b, k) writes PT contiguous values per tile and a beta
// contraction over one tile reads, for each k, a contiguous [b][PT] slab.
constexpr int PT = 16;
constexpr int MAX_RADICES = 8;
constexpr int MAX_SPLIT = 8;
constexpr int FFT_THREADS = 256;
constexpr int GEMM_THREADS = 256;

template <class T>
struct cpx {
  T re, im;
};

template <class T>
__host__ __device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__host__ __device__ inline cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <class T>
__host__ __device__ inline cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__host__ __device__ inline cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__host__ __device__ inline cpx<T> cscale(cpx<T> a, T s) { return {a.re * s, a.im * s}; }

// Per-pair data used by the beta contraction.  The Wigner-d table is stored
// tile-major: the PT pairs of a tile share rows k of length lsum = sum of
// their L, so that the table slice of one tile and one node range is a single
// contiguous block:  d^{l0 + i}_{nm}(beta_k) = tab[tab + k * lsum + coff + i].
//
// Symmetry-reduced tables.  d^l_{-n,-m} = d^l_{mn} = (-1)^{m-n} d^l_{nm}: the
// pair (-m, -n) has the table of (m, n) times (-1)^{m-n}.  Plans whose pair
// list is laid out point-symmetrically (position i holds the mirror of
// position P_pad - 1 - i, so tile t is the mirror of tile ntiles - 1 - t with
// its pairs in reverse order) store the blocks of the lower tiles only; a
// pair of an upper tile points at its mirror's column (tab, lsum, coff, itab)
// with tsign = (-1)^{m-n}, and the contractions multiply the values they
// read from a stored table by tsign.
struct PairInfo {
  int tm, tn;     // doubled m, n
  int tl0;        // doubled lowest degree: max(|tm|, |tn|)
  int L;          // number of degrees l (0 for padding pairs)
  long long tab;  // offset of the pair's tile block (in table elements)
  int lsum;       // row length of the tile block
  int coff;       // column offset of this pair inside a row
  long long itab; // offset of the pair's values in the inverse-layout table (elements)
  int tsign;      // the stored column holds tsign x this pair's values (+1 or -1)
  int towner;     // 1: the column was generated for this pair; 0: it is its mirror's
};

// Inverse-layout table: the values one wave of the inverse contraction loads
// as matrix-core A operands, in lane order.  For a pair with L degrees,
// S = ceil(L / 4) groups of 4 degrees and NB = ceil(N / 16) blocks of 16
// nodes: element ((kb * S + s) * 64 + lane) holds d^l(beta_k) with
// k = 16 kb + lane % 16 and l = 4 s + lane / 16 (zero past N or L), so one
// load instruction reads 64 consecutive values.
__host__ __device__ inline long long inverse_table_elems(int L, int N) {
  return (long long)((L + 3) / 4) * ((N + 15) / 16) * 64;
}

// Parameters of the ring-FFT kernels (one workgroup per ring (signal, k)).
template <class T>
struct RingParams {
  int N;          // nodes per angle
  int Nc;         // columns held in LDS at once: N / split
  int split;      // number of gamma-frequency classes processed one after another
  int batch;
  int ntiles;     // pair tiles
  int nrad_c, nrad_n;
  int rad_c[MAX_RADICES];   // radix sequence of the length-Nc gamma transform
  int rad_n[MAX_RADICES];   // radix sequence of the length-N alpha transform
  int cls_begin[MAX_SPLIT], cls_end[MAX_SPLIT];  // pair ranges per class
  const cpx<T>* tw;         // e^{+i pi t / N}, t = 0..2N-1
  const T* W;               // beta weights W_k
  const int* fftpos;        // per pair: LDS position (row * Nc + column) of its bin
  const cpx<T>* rho;        // per pair: phase i^{n-m} (-1)^{2m} e^{-i pi n}
  const int* colq;          // per LDS column c': q' with pos(q') = c'
  int adjoint;              // inverse chain: 0 -> plain, 1 -> multiply by W_k
  const long long* soff;    // per signal: offset of its samples (complex values), or null: b * N^3
  int so3;                  // SO(3) plan: integer n only, no half-bin shift on any q
  int real_io;              // real samples: the forward reads reals, the inverse writes the real part
};

// start of signal b's samples: an explicit offset table (batches of signals with
// different bandlimits share one buffer) or the dense stride N^3
__host__ __device__ inline size_t ring_offset(const long long* soff, int b, int N) {
  return soff ? (size_t)soff[b] : (size_t)b * N * N * N;
}

// Parameters of the register-resident ring FFT kernels (compile-time N).  The
// kernels process the gamma frequencies q in FAST_ROUNDS equal slices; the
// retained pairs of slice r occupy the index range [rbeg[r], rend[r]).
constexpr int FAST_ROUNDS = 2;
constexpr int FAST_NT = 512;  // threads per workgroup
template <class T>
struct FastRingParams {
  int N, batch;
  const cpx<T>* tw;   // e^{+i pi t / N}, t = 0..2N-1
  const T* W;         // beta weights W_k
  // bin (p, q): (pair << 2) | e with rho = i^e, or -1 if the bin is not
  // retained.  For the N of the register-resident kernels (split N = N1 N2,
  // p = p2 + N2 p1) stored in the order they read it: entry
  // ((q N2 + p2) (N1 / 2) + i) is the bin of row p1 = kept_row(i), so a
  // thread's entries are contiguous; for N = 256, at q * N + p
  const int* bins;
  int adjoint;        // inverse chain: 0 -> plain, 1 -> multiply by W_k
  int rbeg[FAST_ROUNDS], rend[FAST_ROUNDS];
  const long long* soff;  // per signal sample offsets, or null
  // real signals (inverse): (source pair << 3) | (conjugate << 2) | e, the
  // source being the bin's own pair (2m >= 0) or its mirror (-m, -n); same order as bins
  const int* bins_real;
  int so3;            // SO(3) plan: integer n only, no half-bin shift on any q
  int real_io;        // N = 256 kernels: real samples in (forward) or the real part out (inverse)
  // N = 256 one-pass kernels: per gamma frequency q, 4 ints (the pair index of
  // bin p = 192, of p = 0, of p = 1 minus 1; e0 | (first retained p >= 192,
  // minus 192) << 2 | (column retained) << 4): bin (p, q) is retained for p in
  // [0, 64) and [192 + ((w >> 2) & 3), 256) of a retained column, its pair
  // index runs on from those bases and its phase exponent is (3 p + e0) mod 4
  const int* cols;
};

// Sample access of the ring kernels.  Element idx of a signal buffer: complex,
// or (real_io) the real sample at the same index of a real buffer, read as a
// complex value with zero imaginary part; stores keep only the real part.
// Samples are read or written exactly once: non-temporal accesses keep them
// from evicting the ring spectra and tables from the caches.
// A zero the compiler cannot see: real samples enter the transforms with this
// imaginary part, so that they are computed exactly as complex samples with a
// zero imaginary part (a known zero would be folded away and change which
// products become FMAs, and with them the rounding).
template <class T>
__device__ __forceinline__ T opaque_zero() {
  T z = T(0);
  asm volatile("" : "+v"(z));
  return z;
}
template <class T>
__device__ __forceinline__ cpx<T> ld_sample(const cpx<T>* base, size_t idx, int real_io) {
  if (real_io) return {__builtin_nontemporal_load(reinterpret_cast<const T*>(base) + idx), opaque_zero<T>()};
  return {__builtin_nontemporal_load(&base[idx].re), __builtin_nontemporal_load(&base[idx].im)};
}
template <class T>
__device__ __forceinline__ void st_sample(cpx<T>* base, size_t idx, cpx<T> v, int real_io) {
  if (real_io) {
    // the imaginary part is formed all the same, so that the compiler builds
    // the real part exactly as in the complex case (a dead imaginary part
    // changes which products it fuses into FMAs, and with them the rounding)
    asm volatile("" ::"v"(v.im));
    __builtin_nontemporal_store(v.re, reinterpret_cast<T*>(base) + idx);
  } else {
    __builtin_nontemporal_store(v.re, &base[idx].re);
    __builtin_nontemporal_store(v.im, &base[idx].im);
  }
}

// Parameters of the two-pass ring kernels (N = 256): the register-resident
// kernels' parameters plus the pair range of every block of gamma frequencies
// and the intermediate buffer of a chunk of rings.
template <class T>
struct LargeRingParams {
  FastRingParams<T> f;
  const int* qrange;  // [2 * block]: begin, end of the retained pairs of q in [32 block, 32 block + 32)
  cpx<T>* G;          // chunk * N * N complex values
  int chunk;          // rings per chunk
  int ring0;          // first ring (signal * N + node) of the chunk being processed
};

// Parameters of the beta contraction kernels.
template <class T>
struct BetaParams {
  int B, N, batch, ntiles;
  long long ncoef;          // coefficients per signal
  const PairInfo* pairs;
  const T* tab;             // Wigner-d table, tile-major (see PairInfo)
  const T* tabi;            // the same values in the inverse layout (see PairInfo::itab)
  int scale_mode;           // inverse: 0 -> (2l+1) weights, 1 -> none (adjoint)
  const long long* coff;    // per signal: offset of its coefficients (complex values), or null: b * ncoef
  // real signals: only pairs with 2m > 0, or 2m = 0 and 2n >= 0, are contracted;
  // the forward also writes the mirror coefficient (-1)^{m-n} conj(fhat(l)_{mn})
  // at (-m, -n), the inverse reads the Hermitian part of the coefficients
  int real;
  int tile0;                // first pair tile launched (grid x = ntiles - tile0)
  int so3;                  // SO(3) plan: integer-l coefficient layout
  int table_signs;          // stored tables with mirror columns: multiply read values by PairInfo::tsign
  int paired;               // mirror tiles t, ntiles - 1 - t share a table block: the forward launches them side by side
};

// flat coefficient index of (2l, 2m, 2n): the SU(2) layout (2l-major blocks of
// every l in {0, 1/2, 1, ...}) or, for SO(3) plans, blocks of integer l only
// starting at l (2l-1)(2l+1) / 3
__host__ __device__ inline int coef_index_of(int so3, int tl, int tm, int tn) {
  // inside a block both layouts are (2l+1) x (2l+1), row (tm + tl) / 2, column
  // (tn + tl) / 2; only the block start differs (32-bit: at most 707264 values)
  const int start = so3 ? (tl >> 1) * (tl - 1) * (tl + 1) / 3 : tl * (tl + 1) * (2 * tl + 1) / 6;
  return start + ((tm + tl) >> 1) * (tl + 1) + ((tn + tl) >> 1);
}

// pair (m, n) of a real-signal plan whose values come from its mirror (-m, -n)
__host__ __device__ inline bool mirrored_pair(int tm, int tn) { return tm < 0 || (tm == 0 && tn < 0); }

// Tables generated inside the contraction kernels ("on the fly"): the FP64
// three-term recurrence in l runs per (pair, node) from its seed; only
// per-pair and per-node scalars are stored.
//   seed:  d^{l0}_{nm}(beta_k) = seedc[pair] cos^{pc}(beta_k / 2) sin^{ps}(beta_k / 2)
//   step:  d^{l0+i} = (rc[0] x_k - rc[1]) d^{l0+i-1} - rc[2] d^{l0+i-2},  x_k = cos beta_k,
//          rc = rcoef + 3 (tile_row0 + coff + i), tile_row0 = (tile table offset) / N
template <class T>
struct OtfParams {
  BetaParams<T> b;
  const double* seedc;  // per pair
  const double* rcoef;  // 3 per (pair, degree index i >= 1), tile-major like the table rows
  const double* xk;     // cos(beta_k)
  const double* ck;     // cos(beta_k / 2)
  const double* sk;     // sin(beta_k / 2)
};

// Exponents of the single surviving term of Wigner's sum at l0 = max(|a|, |b|)
// (doubled indices t0, ta, tb): d^{l0}_{ab} = (-1)^neg sqrt(C(t0, top)) cos^pc sin^ps.
__host__ __device__ inline void wigner_seed_form(int t0, int ta, int tb, int* top, int* pc, int* ps, int* neg) {
  *neg = 0;
  if (t0 == ta) {
    *top = (t0 + tb) / 2; *pc = (t0 + tb) / 2; *ps = (t0 - tb) / 2;
    *neg = ((t0 - tb) / 2) & 1;
  } else if (t0 == -ta) {
    *top = (t0 + tb) / 2; *pc = (t0 - tb) / 2; *ps = (t0 + tb) / 2;
  } else if (t0 == tb) {
    *top = (t0 + ta) / 2; *pc = (t0 + ta) / 2; *ps = (t0 - ta) / 2;
  } else {  // t0 == -tb
    *top = (t0 + ta) / 2; *pc = (t0 - ta) / 2; *ps = (t0 + ta) / 2;
    *neg = ((t0 + ta) / 2) & 1;
  }
}

__host__ __device__ inline size_t coef_offset(const long long* coff, int b, long long ncoef) {
  return coff ? (size_t)coff[b] : (size_t)b * ncoef;
}

// Launch order of the contraction workgroups.  The dispatcher hands
// workgroup ids to the eight XCDs round robin (id % 8), and the ids one XCD
// receives start in order, side by side.  Every workgroup that reads the same
// table block (the signal tiles of one pair tile, and with `paired` those of
// its mirror tile ntl - 1 - tile as well) therefore gets consecutive slots of
// one XCD: the first brings the block into that XCD's L2 and the others read
// it there at about the same time.  Units (tiles, or mirror pairs of tiles)
// go to the XCDs round robin (unit % 8), so the ragged per-tile costs stay
// balanced over them.  A one-dimensional grid of contraction_grid()
// workgroups covers ntl pair tiles x nbt signal tiles; the few slots past the
// last unit (and the mirror slot of a self-mirror middle tile) return at once.
constexpr int NXCD = 8;
struct TileSlot {
  int tile, bt;
  bool valid;
};
__host__ __device__ inline TileSlot contraction_slot(int id, int ntl, int nbt, int paired = 0) {
  const int per = paired ? 2 * nbt : nbt;
  const int nunits = paired ? (ntl + 1) / 2 : ntl;
  const int x = id % NXCD, r = id / NXCD;
  const int u = (r / per) * NXCD + x, w = r % per;
  const int member = w / nbt;
  TileSlot s;
  s.tile = member ? ntl - 1 - u : u;
  s.bt = w - member * nbt;
  s.valid = u < nunits && !(member && s.tile == u);
  return s;
}
__host__ __device__ inline unsigned contraction_grid(int ntl, int nbt, int paired = 0) {
  const int nunits = paired ? (ntl + 1) / 2 : ntl;
  return (unsigned)(((nunits + NXCD - 1) / NXCD) * NXCD * (paired ? 2 * nbt : nbt));
}

// bf16 split table entry (hi, lo) for the split-precision contraction
struct bf16x2_t {
  unsigned short hi, lo;
};

// ---- kernel launchers (defined in the .hip files) ----
template <class T>
hipError_t launch_ring_forward(const RingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s);
template <class T>
hipError_t launch_ring_inverse(const RingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s);
template <class T>
hipError_t launch_beta_forward(const BetaParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, hipStream_t s);
template <class T>
hipError_t launch_beta_inverse(const BetaParams<T>& p, const cpx<T>* coeffs, cpx<T>* S, hipStream_t s);
template <class T>
hipError_t launch_beta_forward_otf(const OtfParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, hipStream_t s);
template <class T>
hipError_t launch_beta_inverse_otf(const OtfParams<T>& p, const cpx<T>* coeffs, cpx<T>* S, hipStream_t s);
// forward contraction in the shifted-recurrence (divide-and-conquer) form;
// depth 1 or 2 (coarse step blk in {2, 4, 8}); B <= 64
bool shifted_supported(int B);
template <class T>
hipError_t launch_beta_forward_shifted(const OtfParams<T>& p, const cpx<T>* S, cpx<T>* coeffs, int depth, int blk,
                                       hipStream_t s);
hipError_t launch_beta_forward_bf16x3(const BetaParams<float>& p, const unsigned* tabf, const cpx<float>* S,
                                      cpx<float>* coeffs, hipStream_t s);
hipError_t launch_beta_inverse_bf16x3(const BetaParams<float>& p, const unsigned* tabi, const cpx<float>* coeffs,
                                      cpx<float>* S, hipStream_t s);
// N = 256 rings in FP32 in one pass, four workgroups per ring, two per CU
// (forward: samples -> S; inverse / adjoint: S -> samples)
hipError_t launch_ring_sliced4(bool forward, const FastRingParams<float>& p, const cpx<float>* in, cpx<float>* out,
                               hipStream_t s);
hipError_t launch_interleave_bf16_table(int N, int ntiles, const PairInfo* pairs, const bf16x2_t* src, unsigned* dst,
                                        hipStream_t s);

// compile-time shapes of the contraction kernels for bandlimit B:
// row blocks of 16 degrees (forward) and groups of 4 degrees (inverse)
inline int beta_rtmax(int B) {
  const int lmax = (B + 1) / 2;
  return lmax <= 16 ? 1 : (lmax <= 32 ? 2 : 4);
}
inline int beta_lq(int B) {
  const int lmax = (B + 1) / 2;
  return lmax <= 8 ? 2 : (lmax <= 16 ? 4 : (lmax <= 32 ? 8 : 16));
}
// split-BF16 inverse: groups of 32 degrees
inline int beta_bf16_lq(int B) { return (B + 1) / 2 <= 32 ? 1 : 2; }

template <class T>
bool fast_ring_supported(int N);
// dynamic LDS bytes of one workgroup of the register-resident ring kernels,
// and the number of rings (consecutive nodes of one signal) it transforms
template <class T>
size_t fast_ring_smem(int N);
int fast_rings_per_group(int N);
// the register-resident kernels' split N = N1 N2 (false if N has none)
bool fast_ring_split(int N, int* n1, int* n2);
// pairs of one q slice that the kernels can stage in LDS
template <class T>
int fast_ring_slice_capacity(int N);
template <class T>
hipError_t launch_ring_forward_fast(const FastRingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s);
template <class T>
hipError_t launch_ring_inverse_fast(const FastRingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s);
// real signals: real samples in or out; only the pairs with 2m >= 0 carry spectra
template <class T>
hipError_t launch_ring_forward_fast_real(const FastRingParams<T>& p, const T* samples, cpx<T>* S, hipStream_t s);
template <class T>
hipError_t launch_ring_inverse_fast_real(const FastRingParams<T>& p, const cpx<T>* S, T* samples, hipStream_t s);

bool large_ring_supported(int N);
int large_ring_block();           // gamma frequencies per block (pair ranges are given per block)
int large_ring_slice_capacity();  // pairs of one block the kernels can stage in LDS
template <class T>
hipError_t launch_ring_forward_large(const LargeRingParams<T>& p, const cpx<T>* samples, cpx<T>* S, hipStream_t s);
template <class T>
hipError_t launch_ring_inverse_large(const LargeRingParams<T>& p, const cpx<T>* S, cpx<T>* samples, hipStream_t s);

// d-table generation: FP64 three-term recurrence in l, one thread per (pair, k).
hipError_t launch_dtable(int B, int N, int npairs, const PairInfo* pairs, const double* beta, double* tab64,
                         hipStream_t s);
hipError_t launch_round_table_f32(long long n, const double* src, float* dst, hipStream_t s);
template <class T>
hipError_t launch_inverse_table(int N, int npairs, const PairInfo* pairs, const double* tab64, T* dst, hipStream_t s);
hipError_t launch_split_table_bf16(long long n, const double* src, bf16x2_t* dst, hipStream_t s);

}  // namespace su2
