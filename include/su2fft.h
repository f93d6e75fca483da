/*
 * su2fft -- separated Fourier transform on SU(2) for MI355X (gfx950).
 *
 * C ABI.  No C++ or framework types cross it: plain integers, plain host or
 * device pointers, and the HIP stream handle (hipStream_t, itself an opaque
 * pointer; the header includes HIP's C runtime API header for its type).
 *
 * The transform (Section 3, Definition 3.4 and the Peter-Weyl series; the
 * separation of Section 4, Proposition 4.2, with the contraction over beta of
 * Section 4 generalised to every (m, n) pair):
 *
 *   forward  fhat(l)_{mn} = sum_{k,j,l'} W_k f(alpha_j, beta_k, gamma_l') conj(t^l_{nm})
 *   inverse  f(alpha_j, beta_k, gamma_l') = sum_{2l<B} (2l+1) sum_{m,n} fhat(l)_{mn} t^l_{nm}
 *   adjoint  (F^H c)(alpha_j, beta_k, gamma_l') = W_k sum_{l,m,n} c_{lmn} t^l_{nm}
 *
 * with t^l_{nm}(alpha, beta, gamma) = P^l_{nm}(cos beta) exp(-i(n alpha + m gamma))
 * (the index-swapped basis of Section 3), l running over {0, 1/2, 1, ...,
 * (B-1)/2} and m, n over -l..l with l-m, l-n integer.
 *
 * Grid (Definition 4.1 as read for an exact quadrature), N = 2B nodes per angle:
 *   alpha_j = -pi + 2 pi j / N,  beta_k = pi k / (N-1),  gamma_l = -2 pi + 4 pi l / N,
 *   W_k = w_k / (2 N^2), w_k the Clenshaw-Curtis weights on cos(beta_k).
 * For a bandlimited f (all coefficients with 2l >= B zero) forward(inverse(c)) = c
 * up to rounding.
 *
 * Layouts (per signal; signals of a batch are consecutive):
 *   samples       [k: beta][j: alpha][l: gamma], row-major, N^3 complex values;
 *   coefficients  2l-major blocks; the block of 2l = tl starts at tl(tl+1)(2tl+1)/6
 *                 and is the (2l+1)x(2l+1) matrix fhat(l), row-major over
 *                 m = -l..l (rows) and n = -l..l (columns); B(B+1)(2B+1)/6 values.
 *   Complex values are interleaved (re, im): double for SU2_C128, float otherwise.
 *
 * Ownership and concurrency:
 *   The plan owns its device tables and workspace, allocated on the device that
 *   is current at su2_plan_create and freed by su2_plan_destroy.  The caller
 *   owns every data pointer (device memory of that device, aligned to the
 *   element size, inputs and outputs not overlapping); inputs are never written
 *   and every output element is written.  Calls enqueue work on `stream`
 *   (a hipStream_t; NULL = the null stream) and return without synchronising;
 *   a kernel fault surfaces at the caller's next synchronisation.  A plan holds
 *   one workspace: two calls with the same plan must not run concurrently
 *   (different plans are independent).
 *
 * Errors: arguments are validated before any HIP call; no exception crosses
 * the ABI.  On SU2_ERR_HIP the HIP error code is kept in a thread-local slot
 * read by su2_last_hip_error().
 */
#ifndef SU2FFT_H
#define SU2FFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SU2_OK = 0,
  SU2_ERR_INVALID_VALUE = 1, /* null pointer, B < 1, batch < 1, unknown dtype, null plan */
  SU2_ERR_UNSUPPORTED = 2,   /* B > 128, N = 2B not of the form 2^a 3^b, or a batch so
                                large that N x batch x 16 ring-spectrum values of one
                                pair tile exceed 2^31 - 1 bytes (batch > 131072 at
                                B = 64 in SU2_C64) */
  SU2_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed; nothing is leaked */
  SU2_ERR_HIP = 4,           /* a HIP call or kernel launch failed (see su2_last_hip_error) */
  SU2_ERR_NO_DEVICE = 5      /* no usable GPU */
} su2_status_t;

typedef enum {
  SU2_C128 = 0,       /* complex double in and out; FP64 FFT, FP64 MFMA beta contraction */
  SU2_C64 = 1,        /* complex float in and out; FP32 FFT, FP32 MFMA beta contraction  */
  SU2_C64_BF16X3 = 2  /* complex float in and out; FP32 FFT; beta contraction in split
                         bfloat16 (x = hi + lo, three products hi*hi + hi*lo + lo*hi)
                         with FP32 accumulation */
} su2_dtype_t;

typedef struct su2_plan_s* su2_plan_t;

/* Create a plan for `batch` signals of bandlimit B (2l < B) in `dtype`.
 * Section 4, Definition 4.1 (grid) and Proposition 4.2 (the separation the
 * plan's kernels carry out).  Allocates the Wigner-d tables (generated on the
 * GPU by the FP64 three-term recurrence in l; Lemma 4.3 is its m = n = 0 case)
 * and the workspace, on the current device; synchronises once.
 * *out receives the plan (NULL on error). */
su2_status_t su2_plan_create(int32_t B, int32_t batch, su2_dtype_t dtype, su2_plan_t* out);

/* Plan options (bit flags) for su2_plan_create_ex. */
enum {
  /* Generate the Wigner-d values inside the beta-contraction kernels instead of
   * storing the table: the FP64 three-term recurrence in l (Section 4; Lemma 4.3
   * is its m = n = 0 case) runs per (pair, node) from its single-term seed in
   * every call, and only per-pair and per-node scalars are kept (about 3 C(B)
   * doubles instead of C(B) * 2B table values: 724 MB of FP32 at B = 128).
   * Same results as the stored table up to rounding.  SU2_C128 and SU2_C64
   * only (SU2_ERR_UNSUPPORTED for SU2_C64_BF16X3). */
  SU2_PLAN_TABLES_ON_THE_FLY = 1u,
  /* Real signals.  The samples are real (double for SU2_C128, float for
   * SU2_C64 and SU2_C64_BF16X3; N^3 values per signal, same order), the
   * coefficients complex as usual.  A real f has
   * fhat(l)_{-m,-n} = (-1)^{m-n} conj(fhat(l)_{mn}) (Definition 3.4 with
   * conj(t^l_{nm}) = (-1)^{m-n} t^l_{-n,-m}).  su2_forward writes every
   * coefficient; su2_inverse and su2_adjoint return the real part of the
   * complex result, i.e. of the transform of the Hermitian part
   * (c_{mn} + (-1)^{m-n} conj(c_{-m,-n})) / 2 of the coefficients (the adjoint
   * is then the adjoint of the real-input forward map).  At B in
   * {8, 16, 32, 64} both stages run only for the pairs with 2m > 0, or 2m = 0
   * and 2n >= 0 (the forward writes the others by the symmetry, exactly); at
   * other bandlimits the complex kernels run with real samples in and the real
   * part out (the forward then computes both halves, Hermitian to rounding).
   * Every mode and bandlimit; SU2_ERR_UNSUPPORTED with
   * SU2_PLAN_TABLES_ON_THE_FLY or SU2_PLAN_SO3.  su2_beta_forward_shifted does
   * not accept real-signal plans. */
  SU2_PLAN_REAL_SIGNALS = 2u,
  /* SO(3) transform: the group the paper's grid (Definition 4.1, phi and psi
   * both over [-pi, pi]) covers, on which only integer l occur.  Integer
   * l with 2l < B, N = 2B periodic nodes per angle, alpha_j = -pi + 2 pi j / N,
   * gamma_l = -pi + 2 pi l / N, beta_k and W_k as for SU(2) (normalisation
   * 1/(8 pi^2), so W_k = w_k / (2 N^2) again).  Same definitions of forward,
   * inverse and adjoint with t^l_{nm} for integer l, m, n.  Samples: N^3
   * complex values as for SU(2); coefficients: blocks of integer l only, the
   * block of l starting at l(2l-1)(2l+1)/3, row-major over m then n
   * (su2_so3_num_coeffs, su2_so3_coeff_index).  Every mode and bandlimit;
   * SU2_ERR_UNSUPPORTED with any other flag. */
  SU2_PLAN_SO3 = 4u
};

/* su2_plan_create with options: `flags` is a bitwise or of SU2_PLAN_* values
 * (0 gives su2_plan_create's plan).  Unknown bits: SU2_ERR_INVALID_VALUE. */
su2_status_t su2_plan_create_ex(int32_t B, int32_t batch, su2_dtype_t dtype, uint32_t flags, su2_plan_t* out);

/* Plan for a batch of signals with individual bandlimits B_per_signal[0..batch-1]
 * (each 1..128, N = 2B of the form 2^a 3^b).  Signals are concatenated in order
 * in the sample and coefficient buffers: signal s starts at the prefix sum of
 * the per-signal sizes (su2_num_samples / su2_num_coeffs of its B).  A call
 * runs as work-list launches covering every signal (ring FFTs, then
 * contractions, or the reverse); they are captured into a HIP graph the
 * first time a (direction, input, output, stream) combination is used, and
 * the graph is replayed on later calls with the same buffers and stream (the
 * plan keeps up to 16 such graphs).  Results are bit-identical to single-B
 * plans of each signal (B = 128 groups run the single-B plan's N = 256 ring
 * kernels beside the work lists).  B_per_signal is a host array, read only
 * during the call.  su2_run_stage and su2_plan_dtable do not accept mixed
 * plans. */
su2_status_t su2_plan_create_mixed(const int32_t* B_per_signal, int32_t batch, su2_dtype_t dtype,
                                   su2_plan_t* out);

/* su2_plan_create_mixed with options: flags SU2_PLAN_REAL_SIGNALS (real
 * samples, N^3 per signal at the same offsets as complex ones, with
 * su2_plan_create_ex's real-signal semantics per signal) or SU2_PLAN_SO3
 * (coefficients of each signal: su2_so3_num_coeffs of its B, concatenated);
 * 0 gives su2_plan_create_mixed's plan.  SU2_PLAN_TABLES_ON_THE_FLY, or both
 * flags together: SU2_ERR_UNSUPPORTED; unknown bits: SU2_ERR_INVALID_VALUE. */
su2_status_t su2_plan_create_mixed_ex(const int32_t* B_per_signal, int32_t batch, su2_dtype_t dtype, uint32_t flags,
                                      su2_plan_t* out);

/* Release the plan's device memory.  Waits for work the plan enqueued.
 * NULL is accepted and ignored. */
su2_status_t su2_plan_destroy(su2_plan_t plan);

/* Forward transform (analysis), Definition 3.4 with the separation of
 * Proposition 4.2: a 2D FFT over (alpha, gamma) on every beta ring, then the
 * contraction over beta for every (m, n) pair.
 * d_samples: device, batch x N^3 complex; d_coeffs: device, batch x C(B) complex. */
su2_status_t su2_forward(su2_plan_t plan, const void* d_samples, void* d_coeffs, hipStream_t stream);

/* Inverse transform (synthesis), the Peter-Weyl series of Section 3 evaluated
 * as the transpose chain of the forward: contraction over l per (m, n), then an
 * inverse 2D FFT per ring.  d_coeffs: device input; d_samples: device output. */
su2_status_t su2_inverse(su2_plan_t plan, const void* d_coeffs, void* d_samples, hipStream_t stream);

/* Adjoint (conjugate transpose) of su2_forward: the inverse chain with the
 * weight W_k in place of (2l+1).  This is the backward map of the forward
 * transform for gradient computation. */
su2_status_t su2_adjoint(su2_plan_t plan, const void* d_coeffs, void* d_samples, hipStream_t stream);

/* su2_forward for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Same
 * plan, kernels and result as su2_forward (bitwise); the ring spectra between
 * the two stages go to the library's static device scratch instead of the
 * plan's workspace, and the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  The scratch is a file-scope device array of
 * SU2_NOALLOC_SCRATCH_BYTES (64 MiB), one per GPU the library runs on, held
 * until the process ends; its address on a device is looked up once, at the
 * first plan creation on that device.  The plan's ring spectra must fit:
 * bytes = 16 (SU2_C128) or 8 (other dtypes) x 2B x batch x P16, P16 being the
 * retained (m, n) pairs rounded up to a multiple of 16 (SU(2): P = 2B^2 - 2B + 1;
 * SO(3) plans: (2L - 1)^2 with L = floor((B - 1) / 2) + 1), e.g. B = 64 in
 * SU2_C64 up to batch 8, B = 128 in SU2_C64 at batch 1.  Larger plans, and
 * B = 128 plans in SU2_C128 (whose two-pass rings use a second workspace),
 * return SU2_ERR_UNSUPPORTED before any device work.
 * SU2_ERR_INVALID_VALUE for a null argument, a mixed plan, or a current
 * device other than the plan's.  Every call on a GPU shares that GPU's
 * scratch: calls that overlap in time on one GPU (different streams, or
 * threads) race and must be serialised by the caller.  Nothing in the scratch
 * needs clearing: a call reads only values it wrote itself.  The scratch keeps
 * the last call's ring spectra. */
#define SU2_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
su2_status_t su2_forward_noalloc(su2_plan_t plan, const void* d_samples, void* d_coeffs, hipStream_t stream);

/* The kernels behind su2_forward / su2_inverse / su2_adjoint, one at a time,
 * for timing and profiling a single stage.  The intermediate ring spectra stay
 * in the plan's workspace:
 *   SU2_STAGE_RING_FORWARD  in = samples -> workspace      (out unused)
 *   SU2_STAGE_BETA_FORWARD  workspace -> out = coefficients (in unused)
 *   SU2_STAGE_BETA_INVERSE  in = coefficients -> workspace  (out unused)
 *   SU2_STAGE_RING_INVERSE  workspace -> out = samples      (in unused)
 *   SU2_STAGE_BETA_ADJOINT, SU2_STAGE_RING_ADJOINT: the same for su2_adjoint.
 * su2_forward is exactly RING_FORWARD then BETA_FORWARD on the same stream;
 * su2_inverse is BETA_INVERSE then RING_INVERSE; su2_adjoint is BETA_ADJOINT
 * then RING_ADJOINT.  Single-B plans only. */
typedef enum {
  SU2_STAGE_RING_FORWARD = 0,
  SU2_STAGE_BETA_FORWARD = 1,
  SU2_STAGE_BETA_INVERSE = 2,
  SU2_STAGE_RING_INVERSE = 3,
  SU2_STAGE_BETA_ADJOINT = 4,
  SU2_STAGE_RING_ADJOINT = 5
} su2_stage_t;
su2_status_t su2_run_stage(su2_plan_t plan, su2_stage_t stage, const void* in, void* out, hipStream_t stream);

/* Sizes and indexing (pure host functions, no device needed).
 * su2_num_samples: points of the grid of Definition 4.1 (read with N = 2B
 * periodic nodes per angle): (2B)^3, or -1 if B < 1.
 * su2_num_coeffs: entries of the coefficient matrices fhat(l) of Definition
 * 3.4 over every l with 2l < B, i.e. sum over 2l = 0..B-1 of (2l+1)^2 =
 * B(B+1)(2B+1)/6, or -1 if B < 1.
 * su2_coeff_index: flat index of fhat(l)_{mn} (doubled indices, the matrix
 * entry of Definition 3.4 at row m, column n) in the layout described at the
 * top of this file; -1 unless 0 <= two_l, |two_m|, |two_n| <= two_l and
 * two_l - two_m, two_l - two_n are even. */
int64_t su2_num_samples(int32_t B);
int64_t su2_num_coeffs(int32_t B);
int64_t su2_coeff_index(int32_t two_l, int32_t two_m, int32_t two_n);
/* SO(3) plans (SU2_PLAN_SO3): coefficients per signal (integer l, 2l < B), and
 * the flat index of fhat(l)_{mn} from plain integers l, m, n (-1 if invalid). */
int64_t su2_so3_num_coeffs(int32_t B);
int64_t su2_so3_coeff_index(int32_t l, int32_t m, int32_t n);

/* Grid nodes and beta weights of the plan's quadrature: Definition 4.1 read
 * as an exact rule (periodic alpha and gamma nodes, the printed theta nodes
 * beta_k = pi k / (2B - 1), Clenshaw-Curtis weights on cos(beta_k), gamma over
 * [-2 pi, 2 pi) so that half-integer l are resolved; see the grid formula at
 * the top of this file).  Host arrays of 2B doubles each; any pointer may be
 * NULL to skip it.  w_beta receives W_k = w_k / (2 N^2).  SU2_ERR_INVALID_VALUE
 * if B < 1, SU2_ERR_UNSUPPORTED where su2_plan_create would refuse B (B > 128,
 * or 2B not of the form 2^a 3^b). */
su2_status_t su2_grid(int32_t B, double* alpha, double* beta, double* gamma, double* w_beta);

/* Mixed plans: the grid size, in workgroups per compute unit, that the
 * autotuner chose at plan creation for each of the four work-list kernels
 * (ring forward, contraction forward, contraction inverse/adjoint, ring
 * inverse/adjoint), written to workgroups_per_cu[0..3]: one of 1, 2, 3, 4, 6,
 * 8 (a persistent grid whose workgroups walk the task list in a static stride)
 * or 0 (one workgroup per task).  The choice does not change any result.
 * Environment, read at plan creation: SU2_AUTOTUNE=0 skips the search (default
 * 2 each); SU2_AUTOTUNE_CACHE names a text file that caches choices across
 * processes; SU2_GRID="a,b,c,d" pins the four values (each one of the above),
 * over the search and the cache.  SU2_ERR_INVALID_VALUE for a single-B plan. */
su2_status_t su2_plan_tuning(su2_plan_t plan, int32_t* workgroups_per_cu);

/* Mixed plans: the contraction tile shapes the autotuner chose at plan
 * creation, four int32 per bandlimit group in increasing B: B, signals per
 * forward contraction tile, signals per inverse/adjoint contraction tile, beta
 * nodes per forward chunk.  The search times, per group, 16-signal tiles
 * against the widest (32 in FP32 forward and inverse, 32 in the split-BF16
 * inverse; FP64 tiles are 16 wide, the split-BF16 forward 16) and, per plan,
 * 4-node against 8-node forward chunks (FP32 and FP64; split BF16 works in
 * 32-node chunks).  No shape changes any result: every signal's sums over beta
 * run in node order whatever the tile.  out receives at most capacity int32
 * (whole groups only; out may be NULL to query the count), *count the number of
 * groups.  Environment, read at plan creation: SU2_AUTOTUNE=0 keeps the default
 * shapes (16-signal tiles for FP32 groups of at most 16 signals, the widest
 * otherwise; 4-node FP32 and 8-node FP64 chunks); SU2_TILE_SHAPES="kc,fwd,inv"
 * pins chunk and tile widths wherever the mode has them.  Results are cached
 * with the grid sizes of su2_plan_tuning.  SU2_ERR_INVALID_VALUE for a single-B
 * plan or a NULL count. */
su2_status_t su2_plan_tile_shapes(su2_plan_t plan, int32_t* out, int32_t capacity, int32_t* count);

/* Plan queries: bandlimit (-1 for mixed plans), batch, dtype, device bytes held. */
su2_status_t su2_plan_info(su2_plan_t plan, int32_t* B, int32_t* batch, int32_t* dtype,
                           int64_t* device_bytes);

/* The contraction stage of the forward transform in the divide-and-conquer
 * form of Section 4 (the shifted three-term recurrence: the matrix-recurrence
 * and composition-rule propositions, Theorem 4.7, and its worked example for
 * depth 2), generalised from the Legendre case to the Wigner-d recurrence of
 * every (m, n) pair, instead of against the stored table.  For a pair with
 * degrees l0 .. l0+L-1 and base level Lb = l0 + 1 it forms the stored products
 * s^{Lb} = S d^{l0+1}, s^{Lb-1} = S d^{l0} of the pair's ring spectrum S and
 *   depth 1:  fhat(l0+1+r) = <s^{Lb}, A_r^{Lb}> + <s^{Lb-1}, B_r^{Lb}>,
 *   depth 2:  r = n1 + n2 with n1 a multiple of `block` (2, 4, 8 or 16;
 *             ignored at depth 1) and the four terms <s^{Lb}, A_{n2}^{Lb+n1} A_{n1}^{Lb}> +
 *             <s^{Lb}, B_{n2}^{Lb+n1} A_{n1-1}^{Lb}> + <s^{Lb-1}, A_{n2}^{Lb+n1} B_{n1}^{Lb}> +
 *             <s^{Lb-1}, B_{n2}^{Lb+n1} B_{n1-1}^{Lb}>,
 * with the shifted polynomials A, B generated per node in FP64.  Depth 1 and
 * depth 2 with block 16 (the matrix-core row tile: the fine chains of the two
 * row tiles run side by side) contract on the FP64 matrix cores; blocks 2, 4
 * and 8 run on the vector ALUs.  Reads the
 * ring spectra that su2_run_stage(SU2_STAGE_RING_FORWARD) left in the plan and
 * writes d_coeffs exactly like su2_run_stage(SU2_STAGE_BETA_FORWARD) (same
 * values up to rounding).  Arithmetic in FP64 for every dtype (the method's
 * stored products leave the FP32 range near the poles).  Single-B plans with
 * B <= 64 (SU2_ERR_UNSUPPORTED above); SU2_ERR_INVALID_VALUE for bad depth or
 * block, mixed plans or null pointers. */
su2_status_t su2_beta_forward_shifted(su2_plan_t plan, int32_t depth, int32_t block, void* d_coeffs, hipStream_t stream);

/* Diagnostic: copy to host the FP64 Wigner-d table a single-B plan generated
 * for the pair (m, n) (doubled indices): host_out[k * L + i] = d^{l0+i}_{nm}(beta_k),
 * l0 = max(|m|, |n|), k = 0..2B-1, with *L = number of degrees l (may be NULL
 * to query L only when host_out is NULL).  SU2_ERR_INVALID_VALUE if the pair is
 * not retained (|2m|, |2n| > B-1 or 2m, 2n of different parity);
 * SU2_ERR_UNSUPPORTED for a plan without a stored table.  Synchronous. */
su2_status_t su2_plan_dtable(su2_plan_t plan, int32_t two_m, int32_t two_n, double* host_out, int32_t* L);

const char* su2_status_string(su2_status_t status);
int32_t su2_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SU2FFT_H */
