// Host-side plan structure shared by the single-bandlimit and the mixed
// (work-list) paths of the su2fft library.
#pragma once

#include <string.h>

#include <type_traits>
#include <vector>

#include "su2fft_internal.h"

struct MixedState;  // mixed-bandlimit plans: groups, work lists, graphs, tuning

using namespace su2;

struct su2_plan_s {
  int B = 0, N = 0, batch = 0;
  su2_dtype_t dtype = SU2_C128;
  int split = 1, Nc = 0;
  int P = 0, P_pad = 0, ntiles = 0;
  int nrad_c = 0, nrad_n = 0, rad_c[MAX_RADICES] = {0}, rad_n[MAX_RADICES] = {0};
  int cls_begin[MAX_SPLIT] = {0}, cls_end[MAX_SPLIT] = {0};
  long long ncoef = 0;
  long long tab_elems = 0;
  int device = 0;
  int64_t bytes = 0;
  // device memory
  PairInfo* d_pairs = nullptr;
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  double* d_tabi64 = nullptr;   // inverse-layout copies (c128 / c64 plans with stored tables)
  float* d_tabi32 = nullptr;
  long long itab_elems = 0;
  bf16x2_t* d_tabbf = nullptr;
  unsigned* d_tabbf_fwd = nullptr;
  int* d_fftpos = nullptr;
  int* d_colq = nullptr;
  int* d_bins = nullptr;
  bool fast = false;
  int rbeg[FAST_ROUNDS] = {0}, rend[FAST_ROUNDS] = {0};
  // two-pass ring kernels (N = 256): pair ranges per q block, intermediate
  // tables generated inside the contraction kernels: per-pair seed constants,
  // recurrence coefficients, node values
  bool otf = false;
  bool sym = false;             // point-symmetric pair layout, upper tiles share the lower tiles' table blocks
  bool real = false;            // real-signal plan
  // real-signal plan on the complex kernels (rings without a half-spectrum
  // form: generic and N = 256): real samples in, real part out, every pair
  // contracted; otherwise a real plan forms and contracts only the pairs
  // with 2m > 0, or 2m = 0 and 2n >= 0
  bool real_io = false;
  bool so3 = false;             // SO(3) plan: integer l, gamma over [-pi, pi)
  int* d_bins_real = nullptr;
  double* d_seedc = nullptr;
  double* d_rcoef = nullptr;
  double* d_nodes = nullptr;  // [3][N]: cos(beta_k), cos(beta_k / 2), sin(beta_k / 2)
  bool large = false;            // N = 256: two-pass ring kernels through an intermediate (d_G)
  bool sliced = false;          // N = 256 in FP32: both ring directions run in one pass, four workgroups per ring
  int* d_cols = nullptr;        // N = 256 in FP32: per-column bin bases of the one-pass rings (null: not usable)
  int* d_qrange = nullptr;
  void* d_G = nullptr;
  int large_chunk = 0;
  void* d_rho = nullptr;
  void* d_tw = nullptr;
  void* d_W = nullptr;
  void* d_S = nullptr;
  std::vector<void*> allocs;
  std::vector<PairInfo> h_pairs;
  // signals of a mixed plan that this (group) plan serves: their offsets in the
  // caller's concatenated buffers (device), or null for a dense batch
  const long long* d_soff = nullptr;
  const long long* d_coff = nullptr;
  MixedState* mixed = nullptr;

  hipError_t alloc(void** p, size_t n) {
    hipError_t e = hipMalloc(p, n == 0 ? 16 : n);
    if (e == hipSuccess) { allocs.push_back(*p); bytes += (int64_t)n; }
    return e;
  }
  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
  }
};


namespace su2 {

su2_status_t hip_fail(hipError_t e);
void set_last_hip_error(hipError_t e);
bool only_2_3(int n);
su2_status_t build_plan(su2_plan_s* pl);
// mixed-bandlimit plans (su2fft_kernels.hip)
su2_status_t create_mixed(const int32_t* Bs, int32_t batch, su2_dtype_t dtype, bool real, bool so3, su2_plan_s* pl);
void release_mixed(su2_plan_s* pl);
su2_status_t run_mixed(su2_plan_s* pl, int dir, const void* in, void* out, hipStream_t stream);
void mixed_tuning(const su2_plan_s* pl, int32_t* knobs);
int mixed_shapes(const su2_plan_s* pl, int32_t* out, int32_t capacity);  // groups; fills 4 int32 per group

template <class T>
RingParams<T> ring_params(const su2_plan_s* pl, int adjoint) {
  RingParams<T> r;
  memset(&r, 0, sizeof(r));
  r.N = pl->N; r.Nc = pl->Nc; r.split = pl->split; r.batch = pl->batch; r.ntiles = pl->ntiles;
  r.nrad_c = pl->nrad_c; r.nrad_n = pl->nrad_n;
  for (int i = 0; i < MAX_RADICES; i++) { r.rad_c[i] = pl->rad_c[i]; r.rad_n[i] = pl->rad_n[i]; }
  for (int i = 0; i < MAX_SPLIT; i++) { r.cls_begin[i] = pl->cls_begin[i]; r.cls_end[i] = pl->cls_end[i]; }
  r.tw = (const cpx<T>*)pl->d_tw;
  r.W = (const T*)pl->d_W;
  r.fftpos = pl->d_fftpos;
  r.rho = (const cpx<T>*)pl->d_rho;
  r.colq = pl->d_colq;
  r.adjoint = adjoint;
  r.soff = pl->d_soff;
  r.so3 = pl->so3 ? 1 : 0;
  r.real_io = pl->real_io ? 1 : 0;
  return r;
}

template <class T>
FastRingParams<T> fast_params(const su2_plan_s* pl, int adjoint) {
  FastRingParams<T> r;
  memset(&r, 0, sizeof(r));  // every field not set below (offset tables) is null
  r.N = pl->N; r.batch = pl->batch;
  r.tw = (const cpx<T>*)pl->d_tw;
  r.W = (const T*)pl->d_W;
  r.bins = pl->d_bins;
  r.adjoint = adjoint;
  for (int i = 0; i < FAST_ROUNDS; i++) { r.rbeg[i] = pl->rbeg[i]; r.rend[i] = pl->rend[i]; }
  r.soff = pl->d_soff;
  r.bins_real = pl->d_bins_real;
  r.so3 = pl->so3 ? 1 : 0;
  r.real_io = pl->real_io ? 1 : 0;
  r.cols = pl->d_cols;
  return r;
}

template <class T>
LargeRingParams<T> large_params(const su2_plan_s* pl, int adjoint) {
  LargeRingParams<T> r;
  memset(&r, 0, sizeof(r));
  r.f = fast_params<T>(pl, adjoint);
  r.qrange = pl->d_qrange;
  r.G = (cpx<T>*)pl->d_G;
  r.chunk = pl->large_chunk;
  return r;
}

template <class T>
BetaParams<T> beta_params(const su2_plan_s* pl, const T* tab, int scale_mode);

template <class T>
OtfParams<T> otf_params(const su2_plan_s* pl, int scale_mode) {
  OtfParams<T> r;
  memset(&r, 0, sizeof(r));
  r.b = beta_params<T>(pl, nullptr, scale_mode);
  // kernels on these parameters generate each pair's own values (its own
  // seed): no stored column, no mirror sign, no shared blocks to pair up
  r.b.table_signs = 0;
  r.b.paired = 0;
  r.seedc = pl->d_seedc;
  r.rcoef = pl->d_rcoef;
  r.xk = pl->d_nodes;
  r.ck = pl->d_nodes + pl->N;
  r.sk = pl->d_nodes + 2 * pl->N;
  return r;
}

template <class T>
BetaParams<T> beta_params(const su2_plan_s* pl, const T* tab, int scale_mode) {
  BetaParams<T> b;
  memset(&b, 0, sizeof(b));  // every field not set below (offset tables) is null
  b.B = pl->B; b.N = pl->N; b.batch = pl->batch; b.ntiles = pl->ntiles;
  b.ncoef = pl->ncoef;
  b.pairs = pl->d_pairs;
  b.tab = tab;
  b.tabi = std::is_same<T, double>::value ? reinterpret_cast<const T*>(pl->d_tabi64)
                                          : reinterpret_cast<const T*>(pl->d_tabi32);
  b.scale_mode = scale_mode;
  b.coff = pl->d_coff;
  const bool half = pl->real && !pl->real_io;  // half-spectrum real plan
  b.real = half ? 1 : 0;
  b.tile0 = half ? pl->rbeg[0] / PT : 0;
  b.so3 = pl->so3 ? 1 : 0;
  b.table_signs = pl->sym ? 1 : 0;
  b.paired = (pl->sym && b.tile0 == 0) ? 1 : 0;
  return b;
}


}  // namespace su2
