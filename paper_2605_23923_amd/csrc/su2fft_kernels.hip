// All device code of su2fft in one translation unit, plus batches of signals
// with different bandlimits ("mixed" plans).
//
// A mixed plan groups its signals by bandlimit B.  Each group has the tables
// and the ring-spectrum workspace of a single-B plan; its signals stay where
// the caller put them (concatenated in order), reached through per-signal
// offset tables.  A transform runs as work lists: one of (group, signal,
// node) ring tasks per ring kernel family, and the (group, pair tile, signal
// tile) contraction tasks split by contraction shape class and tile width, each launch
// calling the same kernel bodies as the single-B launches (so every signal's
// result is bit-identical to a single-B plan's); the rings of N = 256 groups
// run the single-B plan's own N = 256 kernels beside the work lists.  Tasks
// are ordered by decreasing cost and taken in a static stride by a grid of
// `knob x CUs` workgroups, or (knob 0) one workgroup per task; the knob of
// each kernel is chosen by timing the candidates at plan creation
// (autotuner, cached per device, mode and bandlimit mix, optionally on
// disk).  The launches of a call are captured once into a HIP graph per
// (direction, buffers, stream) and replayed.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <type_traits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "su2fft_ring.hip"
#include "su2fft_ring_fast.hip"
#include "su2fft_ring_large.hip"
#include "su2fft_ring_sliced.hip"
#include "su2fft_beta.hip"
#include "su2fft_beta_bf16.hip"
#include "su2fft_beta_otf.hip"
#include "su2fft_beta_shifted.hip"
#include "su2fft_plan.h"

namespace su2 {

struct WorkItem {
  int g;     // group
  int a, b;  // ring task: (signal in group, first node); contraction task: (pair tile, signal tile)
};

template <class T>
struct GroupDev {
  int fast;               // register-resident ring kernels
  int rtmax, lq, lq2;     // contraction shapes of the group's bandlimit
  int narrow_f, narrow_i; // 16-signal contraction tiles (forward, inverse) instead of the widest
  RingParams<T> rp[3];    // generic ring kernels: forward, inverse, adjoint
  FastRingParams<T> fp[3];
  BetaParams<T> bp[3];    // contraction: forward, inverse, adjoint
  const unsigned* tabf_bf;  // split-BF16 tables (forward / inverse layouts)
  const unsigned* tabi_bf;
  cpx<T>* S;
};

// ---- work-list kernels ----

// Ring tasks come in two lists, one per ring kernel family, and every
// contraction launch carries one shape class (row tiles RTC, degree groups
// LQC / LQ2C) and holds only that class's bodies, so that each work-list
// kernel keeps the register budget of its single-B counterpart.  W is the
// set of signal-tile widths a launch holds: 1 the 16-signal body, 2 the
// widest, 3 both (each task takes its group's width).
// dir 0: forward (in = samples -> workspaces); 1: inverse, 2: adjoint (workspaces -> out = samples)
// REAL: real-signal plans (the half-spectrum form of the register-resident rings)
template <class T, bool FWD, bool REAL>
__global__ __launch_bounds__(FAST_NT, fast_waves_per_simd<T>()) void ring_fast_worklist_kernel(
    const WorkItem* __restrict__ items, int n, const GroupDev<T>* __restrict__ groups, const cpx<T>* __restrict__ in,
    cpx<T>* __restrict__ out, int dir) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];   // (signal, first node)
    const FastRingParams<T>& p = groups[w.g].fp[dir];
    cpx<T>* S = groups[w.g].S;
    // The thread index passes through an empty asm statement so that the
    // per-thread twiddle and index set-up stays inside the loop instead of
    // being hoisted in front of it, where it would hold registers for the
    // whole loop and spill.
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
#define SU2_FAST_CASE(NN)                                                    \
  case NN:                                                                   \
    if constexpr (FWD)                                                       \
      ring_forward_fast_group<T, NN, REAL>(in, S, p, w.a, w.b, smem, t);     \
    else                                                                     \
      ring_inverse_fast_group<T, NN, REAL>(S, out, p, w.a, w.b, smem, t);    \
    break;
    switch (p.N) {
      SU2_FAST_CASE(16)
      SU2_FAST_CASE(32)
      SU2_FAST_CASE(64)
      SU2_FAST_CASE(128)
    }
#undef SU2_FAST_CASE
    __syncthreads();
  }
}

template <class T, bool FWD>
__global__ __launch_bounds__(GENERIC_NT) void ring_generic_worklist_kernel(const WorkItem* __restrict__ items, int n,
                                                                            const GroupDev<T>* __restrict__ groups,
                                                                            const cpx<T>* __restrict__ in,
                                                                            cpx<T>* __restrict__ out, int dir) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    const RingParams<T>& p = groups[w.g].rp[dir];
    if constexpr (FWD)
      ring_forward_any<T>(in, ring_offset(p.soff, w.a, p.N) + (size_t)w.b * p.N * p.N, groups[w.g].S, p, w.a, w.b,
                          smem);
    else
      ring_inverse_any<T>(groups[w.g].S, out, ring_offset(p.soff, w.a, p.N) + (size_t)w.b * p.N * p.N, p, w.a, w.b,
                          smem);
    __syncthreads();
  }
}

template <class T, int RTC, int KC, int W>
__global__ __launch_bounds__(FWD_THREADS) void beta_forward_worklist_kernel(const WorkItem* __restrict__ items, int n,
                                                                            const GroupDev<T>* __restrict__ groups,
                                                                            cpx<T>* __restrict__ coeffs) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));   // keep per-thread set-up inside the loop (see the ring work list)
    const GroupDev<T>& g = groups[w.g];
    if (g.rtmax == RTC) {
      if constexpr ((W & 1) != 0)
        if (g.narrow_f) beta_forward_body<T, RTC, KC, 16>(g.S, coeffs, g.bp[0], w.a, w.b, smem, t);
      if constexpr ((W & 2) != 0)
        if (!g.narrow_f) beta_forward_body<T, RTC, KC>(g.S, coeffs, g.bp[0], w.a, w.b, smem, t);
    }
    __syncthreads();
  }
}

template <class T, int LQC, int W>
__global__ __launch_bounds__(inverse_threads<inverse_wpp<T>(LQC)>()) void beta_inverse_worklist_kernel(
    const WorkItem* __restrict__ items, int n, const GroupDev<T>* __restrict__ groups, const cpx<T>* __restrict__ coeffs,
    int dir) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));   // keep per-thread set-up inside the loop (see the ring work list)
    const GroupDev<T>& g = groups[w.g];
    if (g.lq == LQC) {
      constexpr int WPP = inverse_wpp<T>(LQC);
      if constexpr ((W & 1) != 0)
        if (g.narrow_i) beta_inverse_body<T, LQC, 16, WPP>(coeffs, g.S, g.bp[dir], w.a, w.b, smem, t);
      if constexpr ((W & 2) != 0)
        if (!g.narrow_i) beta_inverse_body<T, LQC, BetaCfg<T>::BT, WPP>(coeffs, g.S, g.bp[dir], w.a, w.b, smem, t);
    }
    __syncthreads();
  }
}

template <int RTC>
__global__ __launch_bounds__(XB_THREADS) void beta_forward_bf16x3_worklist_kernel(
    const WorkItem* __restrict__ items, int n, const GroupDev<float>* __restrict__ groups, cpx<float>* __restrict__ coeffs) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));   // keep per-thread set-up inside the loop (see the ring work list)
    const GroupDev<float>& g = groups[w.g];
    if constexpr (RTC == 1)
      if (g.rtmax == 1) beta_forward_bf16x3_body<1>(g.S, coeffs, g.bp[0], g.tabf_bf, w.a, w.b, smem, t);
    if constexpr (RTC == 2)
      if (g.rtmax == 2) beta_forward_bf16x3_body<2>(g.S, coeffs, g.bp[0], g.tabf_bf, w.a, w.b, smem, t);
    if constexpr (RTC == 4)
      if (g.rtmax == 4) beta_forward_bf16x3_body<4, false>(g.S, coeffs, g.bp[0], g.tabf_bf, w.a, w.b, smem, t);
    __syncthreads();
  }
}

template <int LQ2C, int W>
__global__ __launch_bounds__(XB_THREADS) void beta_inverse_bf16x3_worklist_kernel(
    const WorkItem* __restrict__ items, int n, const GroupDev<float>* __restrict__ groups,
    const cpx<float>* __restrict__ coeffs, int dir) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const WorkItem w = items[it];
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));   // keep per-thread set-up inside the loop (see the ring work list)
    const GroupDev<float>& g = groups[w.g];
    if (g.lq2 == LQ2C) {
      if constexpr ((W & 1) != 0)
        if (g.narrow_i) beta_inverse_bf16x3_body<LQ2C, 16>(coeffs, g.S, g.bp[dir], g.tabi_bf, w.a, w.b, smem, t);
      if constexpr ((W & 2) != 0)
        if (!g.narrow_i) beta_inverse_bf16x3_body<LQ2C>(coeffs, g.S, g.bp[dir], g.tabi_bf, w.a, w.b, smem, t);
    }
    __syncthreads();
  }
}

}  // namespace su2

// ---- mixed plans (host) ----

struct MixedGraph {
  int dir;
  const void* in;
  void* out;
  hipStream_t stream;
  hipGraphExec_t exec;
};

struct MixedState {
  std::vector<su2_plan_s*> groups;  // one single-B plan per distinct bandlimit
  std::vector<int> group_B;
  long long total_samples = 0, total_coeffs = 0;
  void* d_groups = nullptr;         // GroupDev<T>[groups]
  su2::WorkItem* d_ringf = nullptr;   // ring tasks of the register-resident N = 128 kernels
  su2::WorkItem* d_ringg = nullptr;   // ring tasks of the generic kernels
  su2::WorkItem* d_betaf = nullptr;
  su2::WorkItem* d_betai = nullptr;
  int n_ringf = 0, n_ringg = 0, n_betaf = 0, n_betai = 0;
  // groups whose rings (N = 256) run the single-B plan's dedicated kernels
  // (one-pass sliced in FP32, two-pass in FP64) instead of a work list
  std::vector<int> dedicated;
  // the contraction lists in runs of one shape class (forward: row tiles;
  // inverse: degrees per group), largest class first: a run is one launch of
  // the kernel built for exactly that class, so that the small bandlimits
  // keep the registers, and the occupancy, of their single-B kernels.  A
  // class whose groups use both signal-tile widths runs as one launch
  // holding both bodies, unless that kernel fits fewer than two workgroups
  // per CU and the 16-signal body alone fits more: then the two widths are
  // two runs (the 32-signal body takes 195 VGPRs in the FP32 forward of
  // 65-128 degrees, the 16-signal one 119)
  struct Run {
    int cls, w, begin, n;  // w: tile widths held (1: 16 signals, 2: widest, 3: both)
  };
  std::vector<Run> runs_f, runs_i;
  size_t smem_ringf = 0, smem_ringg = 0, smem_betaf = 0, smem_betai = 0;
  int rtmax = 1;                    // largest forward row-tile count present (LDS check)
  int num_cu = 0;
  // workgroups per CU (0: one per task): ring forward, contraction forward,
  // contraction inverse, ring inverse
  int knob[4] = {2, 2, 2, 2};
  // tile shapes (autotuned): nodes per forward chunk, and per group 16-signal
  // contraction tiles (1) or the widest (0) in the forward and the inverse
  int kc = 4;
  std::vector<int> narrow_f, narrow_i;
  int max_betaf = 0, max_betai = 0;  // work-list capacities (every group in 16-signal tiles)
  hipStream_t cap = nullptr;          // capture stream
  hipStream_t side = nullptr;         // second branch: generic and N = 256 rings beside the fast ones
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<MixedGraph> graphs;
  std::vector<void*> allocs;
};

namespace {

using namespace su2;

hipError_t mixed_alloc(MixedState* ms, void** p, size_t n) {
  hipError_t e = hipMalloc(p, n == 0 ? 16 : n);
  if (e == hipSuccess) ms->allocs.push_back(*p);
  return e;
}

// kernel selection by the plan's largest shapes
template <class T>
void* ringf_kernel_ptr(bool fwd, bool real) {
  if (real) return fwd ? (void*)ring_fast_worklist_kernel<T, true, true> : (void*)ring_fast_worklist_kernel<T, false, true>;
  return fwd ? (void*)ring_fast_worklist_kernel<T, true, false> : (void*)ring_fast_worklist_kernel<T, false, false>;
}
template <class T>
void* ringg_kernel_ptr(bool fwd) {
  return fwd ? (void*)ring_generic_worklist_kernel<T, true> : (void*)ring_generic_worklist_kernel<T, false>;
}

template <class T, int KC, int W>
void* betaf_kernel_ptr_w(int rtmax) {
  if (rtmax <= 1) return (void*)beta_forward_worklist_kernel<T, 1, KC, W>;
  if (rtmax <= 2) return (void*)beta_forward_worklist_kernel<T, 2, KC, W>;
  return (void*)beta_forward_worklist_kernel<T, 4, KC, W>;
}
template <class T, int KC>
void* betaf_kernel_ptr_k(int rtmax, int w) {
  if constexpr (BetaCfg<T>::BT == 16) return betaf_kernel_ptr_w<T, KC, 2>(rtmax);  // one width
  else
    return w == 1 ? betaf_kernel_ptr_w<T, KC, 1>(rtmax)
                  : (w == 2 ? betaf_kernel_ptr_w<T, KC, 2>(rtmax) : betaf_kernel_ptr_w<T, KC, 3>(rtmax));
}
template <class T>
void* betaf_kernel_ptr(int rtmax, int kc, int w) {
  return kc == 8 ? betaf_kernel_ptr_k<T, 8>(rtmax, w) : betaf_kernel_ptr_k<T, 4>(rtmax, w);
}
template <class T>
size_t betaf_smem(int rtmax, int kc) {
  if (kc == 8)
    return rtmax <= 1 ? FwdGeom<T, 1, 8>::SMEM : (rtmax <= 2 ? FwdGeom<T, 2, 8>::SMEM : FwdGeom<T, 4, 8>::SMEM);
  return rtmax <= 1 ? FwdGeom<T, 1, 4>::SMEM : (rtmax <= 2 ? FwdGeom<T, 2, 4>::SMEM : FwdGeom<T, 4, 4>::SMEM);
}
template <class T, int W>
void* betai_kernel_ptr_w(int lq) {
  if (lq <= 2) return (void*)beta_inverse_worklist_kernel<T, 2, W>;
  if (lq <= 4) return (void*)beta_inverse_worklist_kernel<T, 4, W>;
  if (lq <= 8) return (void*)beta_inverse_worklist_kernel<T, 8, W>;
  return (void*)beta_inverse_worklist_kernel<T, 16, W>;
}
// threads of the inverse work-list kernel of degree class lq (the class's
// kernel is built for exactly that class, lq in {2, 4, 8, 16})
template <class T>
int betai_threads(int lq) {
  return inverse_wpp<T>(lq) == 1 ? inverse_threads<1>() : inverse_threads<2>();
}
template <class T>
void* betai_kernel_ptr(int lq, int w) {
  if constexpr (BetaCfg<T>::BT == 16) return betai_kernel_ptr_w<T, 2>(lq);  // one width
  else
    return w == 1 ? betai_kernel_ptr_w<T, 1>(lq) : (w == 2 ? betai_kernel_ptr_w<T, 2>(lq) : betai_kernel_ptr_w<T, 3>(lq));
}
void* betaf_bf16_kernel_ptr(int rtmax) {
  if (rtmax <= 1) return (void*)beta_forward_bf16x3_worklist_kernel<1>;
  if (rtmax <= 2) return (void*)beta_forward_bf16x3_worklist_kernel<2>;
  return (void*)beta_forward_bf16x3_worklist_kernel<4>;
}
template <int W>
void* betai_bf16_kernel_ptr_w(int lq2) {
  return lq2 <= 1 ? (void*)beta_inverse_bf16x3_worklist_kernel<1, W> : (void*)beta_inverse_bf16x3_worklist_kernel<2, W>;
}
void* betai_bf16_kernel_ptr(int lq2, int w) {
  return w == 1 ? betai_bf16_kernel_ptr_w<1>(lq2) : (w == 2 ? betai_bf16_kernel_ptr_w<2>(lq2) : betai_bf16_kernel_ptr_w<3>(lq2));
}

// workgroups of `threads` threads with `smem` bytes of LDS that one CU holds
// of kernel f (0 if the runtime cannot tell)
int wgs_per_cu(const void* f, int threads, size_t smem, int device) {
  int max_lds = 0, n = 0;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, threads, smem) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// the rings of an N = 256 group with the single-B plan's kernels (d: 0
// forward, 1 inverse, 2 adjoint); the ring spectra are the group's workspace
template <class T>
hipError_t launch_rings_256(su2_plan_s* gp, bool fwd, int d, const void* in, void* out, hipStream_t s) {
  cpx<T>* S = (cpx<T>*)gp->d_S;
  if (gp->sliced) {
    if constexpr (std::is_same<T, float>::value)
      return fwd ? launch_ring_sliced4(true, fast_params<T>(gp, 0), (const cpx<T>*)in, S, s)
                 : launch_ring_sliced4(false, fast_params<T>(gp, d == 2), S, (cpx<T>*)out, s);
    return hipErrorInvalidValue;
  }
  return fwd ? launch_ring_forward_large<T>(large_params<T>(gp, 0), (const cpx<T>*)in, S, s)
             : launch_ring_inverse_large<T>(large_params<T>(gp, d == 2), S, (cpx<T>*)out, s);
}

// enqueue one work-list launch: which = 0 ring forward, 1 contraction forward,
// 2 contraction inverse/adjoint, 3 ring inverse/adjoint
template <class T>
hipError_t enqueue(su2_plan_s* pl, int which, int dir, const void* in, void* out, hipStream_t s, int knob) {
  MixedState* ms = pl->mixed;
  const GroupDev<T>* g = (const GroupDev<T>*)ms->d_groups;
  const bool bf = pl->dtype == SU2_C64_BF16X3;
  auto grid_of = [&](int n) { return dim3((unsigned)std::max(1, knob > 0 ? std::min(n, knob * ms->num_cu) : n)); };
  switch (which) {
    case 0:
    case 3: {
      // the generic list and the N = 256 groups run on a second branch beside
      // the register-resident list (fork/join through events, also inside a
      // stream capture)
      const bool side_work = ms->n_ringg > 0 || !ms->dedicated.empty();
      const bool both = ms->n_ringf > 0 && side_work;
      hipStream_t sg = both ? ms->side : s;
      hipError_t e;
      if (both) {
        if ((e = hipEventRecord(ms->fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ms->side, ms->fork, 0)) != hipSuccess) return e;
      }
      int d = which == 0 ? 0 : dir;
      const cpx<T>* xin = (const cpx<T>*)in;
      cpx<T>* xout = (cpx<T>*)out;
      void* args[] = {nullptr, nullptr, (void*)&g, (void*)&xin, (void*)&xout, (void*)&d};
      if (ms->n_ringg > 0) {
        args[0] = (void*)&ms->d_ringg;
        args[1] = (void*)&ms->n_ringg;
        if ((e = hipLaunchKernel(ringg_kernel_ptr<T>(which == 0), grid_of(ms->n_ringg), dim3(GENERIC_NT), args,
                                 ms->smem_ringg, sg)) != hipSuccess)
          return e;
      }
      for (int gi : ms->dedicated)
        if ((e = launch_rings_256<T>(ms->groups[gi], which == 0, d, in, out, sg)) != hipSuccess) return e;
      if (ms->n_ringf > 0) {
        args[0] = (void*)&ms->d_ringf;
        args[1] = (void*)&ms->n_ringf;
        if ((e = hipLaunchKernel(ringf_kernel_ptr<T>(which == 0, pl->real), grid_of(ms->n_ringf), dim3(FAST_NT), args,
                                 ms->smem_ringf, s)) != hipSuccess)
          return e;
      }
      if (both) {
        if ((e = hipEventRecord(ms->join, ms->side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, ms->join, 0)) != hipSuccess) return e;
      }
      break;
    }
    case 1:
    case 2: {
      // the largest class on the call's stream, the others one after another
      // on the second branch, so that the launches' tails overlap
      const std::vector<MixedState::Run>& runs = which == 1 ? ms->runs_f : ms->runs_i;
      const bool split = runs.size() > 1;
      hipError_t e;
      if (split) {
        if ((e = hipEventRecord(ms->fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ms->side, ms->fork, 0)) != hipSuccess) return e;
      }
      for (size_t ri = 0; ri < runs.size(); ri++) {
        const MixedState::Run& r = runs[ri];
        hipStream_t rs = ri == 0 ? s : ms->side;
        if (which == 1) {
          const WorkItem* items = ms->d_betaf + r.begin;
          void* args[] = {(void*)&items, (void*)&r.n, (void*)&g, (void*)&out};
          e = bf ? hipLaunchKernel(betaf_bf16_kernel_ptr(r.cls), grid_of(r.n), dim3(XB_THREADS), args, XBF_SMEM, rs)
                 : hipLaunchKernel(betaf_kernel_ptr<T>(r.cls, ms->kc, r.w), grid_of(r.n), dim3(FWD_THREADS), args,
                                   betaf_smem<T>(r.cls, ms->kc), rs);
        } else {
          const WorkItem* items = ms->d_betai + r.begin;
          void* args[] = {(void*)&items, (void*)&r.n, (void*)&g, (void*)&in, (void*)&dir};
          e = bf ? hipLaunchKernel(betai_bf16_kernel_ptr(r.cls, r.w), grid_of(r.n), dim3(XB_THREADS), args,
                                   ms->smem_betai, rs)
                 : hipLaunchKernel(betai_kernel_ptr<T>(r.cls, r.w), grid_of(r.n), dim3(betai_threads<T>(r.cls)), args,
                                   ms->smem_betai, rs);
        }
        if (e != hipSuccess) return e;
      }
      if (split) {
        if ((e = hipEventRecord(ms->join, ms->side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, ms->join, 0)) != hipSuccess) return e;
      }
      break;
    }
  }
  return hipGetLastError();
}

hipError_t enqueue_any(su2_plan_s* pl, int which, int dir, const void* in, void* out, hipStream_t s, int knob) {
  return pl->dtype == SU2_C128 ? enqueue<double>(pl, which, dir, in, out, s, knob)
                               : enqueue<float>(pl, which, dir, in, out, s, knob);
}

hipError_t enqueue_call(su2_plan_s* pl, int dir, const void* in, void* out, hipStream_t s) {
  MixedState* ms = pl->mixed;
  hipError_t e;
  if (dir == 0) {
    if ((e = enqueue_any(pl, 0, 0, in, nullptr, s, ms->knob[0])) != hipSuccess) return e;
    return enqueue_any(pl, 1, 0, nullptr, out, s, ms->knob[1]);
  }
  if ((e = enqueue_any(pl, 2, dir, in, nullptr, s, ms->knob[2])) != hipSuccess) return e;
  return enqueue_any(pl, 3, dir, nullptr, out, s, ms->knob[3]);
}

// The dynamic-LDS limit is a property of the kernel function, shared by every
// plan: raise it to the device maximum (each launch still asks only for what
// its plan needs).
template <class T>
hipError_t set_worklist_smem(su2_plan_s* pl) {
  MixedState* ms = pl->mixed;
  const bool bf = pl->dtype == SU2_C64_BF16X3;
  int max_lds = 0;
  hipError_t e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device);
  if (e != hipSuccess) return e;
  if (ms->smem_ringf > (size_t)max_lds || ms->smem_ringg > (size_t)max_lds || ms->smem_betaf > (size_t)max_lds ||
      ms->smem_betai > (size_t)max_lds)
    return hipErrorInvalidValue;
  for (const MixedState::Run& r : ms->runs_f)
    if ((e = hipFuncSetAttribute(bf ? betaf_bf16_kernel_ptr(r.cls) : betaf_kernel_ptr<T>(r.cls, ms->kc, r.w),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, max_lds)) != hipSuccess)
      return e;
  for (const MixedState::Run& r : ms->runs_i)
    if ((e = hipFuncSetAttribute(bf ? betai_bf16_kernel_ptr(r.cls, r.w) : betai_kernel_ptr<T>(r.cls, r.w),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, max_lds)) != hipSuccess)
      return e;
  for (int fwd = 0; fwd < 2; fwd++) {
    if ((e = hipFuncSetAttribute(ringf_kernel_ptr<T>(fwd, pl->real), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 max_lds)) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute(ringg_kernel_ptr<T>(fwd), hipFuncAttributeMaxDynamicSharedMemorySize, max_lds)) !=
        hipSuccess)
      return e;
  }
  return hipSuccess;
}

// build the per-group device descriptors, work lists and LDS sizes from the
// plan's tile shapes (ms->kc, ms->narrow_f, ms->narrow_i); only_group >= 0
// keeps only that group's contraction tasks (the autotuner times one group's
// shapes at a time).  The device lists are allocated once, at the capacity of
// every group in 16-signal tiles, and refilled on later calls.
template <class T>
su2_status_t build_worklists(su2_plan_s* pl, int only_group = -1) {
  MixedState* ms = pl->mixed;
  const bool bf = pl->dtype == SU2_C64_BF16X3;
  const int ng = (int)ms->groups.size();
  const bool first = ms->d_groups == nullptr;
  if (first) {
    // default shapes: FP32 groups of at most 16 signals take 16-signal tiles
    // (as single-B plans do); FP32 forward chunks of 4 nodes, FP64 of 8
    ms->narrow_f.assign(ng, 0);
    ms->narrow_i.assign(ng, 0);
    for (int gi = 0; gi < ng; gi++)
      ms->narrow_f[gi] = ms->narrow_i[gi] = sizeof(T) == 4 && ms->groups[gi]->batch <= 16 ? 1 : 0;
    ms->kc = fwd_kc_default<T>();
  }
  std::vector<GroupDev<T>> hg(ng);
  std::vector<std::pair<double, WorkItem>> ringf, ringg, betaf, betai;
  int cap_f = 0, cap_i = 0;
  ms->rtmax = 1;
  ms->dedicated.clear();
  for (int gi = 0; gi < ng; gi++) {
    su2_plan_s* gp = ms->groups[gi];
    GroupDev<T>& d = hg[gi];
    memset(&d, 0, sizeof(d));
    d.fast = gp->fast ? 1 : 0;
    d.rtmax = beta_rtmax(gp->B);
    d.lq = beta_lq(gp->B);
    d.lq2 = beta_bf16_lq(gp->B);
    d.narrow_f = ms->narrow_f[gi];
    d.narrow_i = ms->narrow_i[gi];
    const T* tab = std::is_same<T, double>::value ? (const T*)gp->d_tab64 : (const T*)gp->d_tab32;
    for (int dir = 0; dir < 3; dir++) {
      d.rp[dir] = ring_params<T>(gp, dir == 2);
      d.fp[dir] = fast_params<T>(gp, dir == 2);
      d.bp[dir] = beta_params<T>(gp, tab, dir == 2);
    }
    d.tabf_bf = gp->d_tabbf_fwd;
    d.tabi_bf = (const unsigned*)gp->d_tabbf;
    d.S = (cpx<T>*)gp->d_S;
    ms->rtmax = std::max(ms->rtmax, d.rtmax);
    const int N = gp->N;
    // ring LDS
    const double ring_cost = (double)N * N * (N > 1 ? std::log2((double)N) : 1.0);
    if (gp->large) {
      ms->dedicated.push_back(gi);  // launched whole by launch_rings_256
    } else if (gp->fast) {
      // one task per workgroup's worth of consecutive rings of a signal
      ms->smem_ringf = std::max(ms->smem_ringf, fast_ring_smem<T>(N));
      const int rpw = fast_rings_per_group(N);
      for (int i = 0; i < gp->batch; i++)
        for (int k = 0; k < N; k += rpw) ringf.push_back({ring_cost * rpw, WorkItem{gi, i, k}});
    } else {
      ms->smem_ringg = std::max(ms->smem_ringg, ring_smem_bytes<T>(d.rp[0]));
      for (int i = 0; i < gp->batch; i++)
        for (int k = 0; k < N; k++) ringg.push_back({ring_cost, WorkItem{gi, i, k}});
    }
    const int btf = bf ? XBF_BT : (d.narrow_f ? 16 : BetaCfg<T>::BT);
    const int bti = d.narrow_i ? 16 : (bf ? XB_BT : BetaCfg<T>::BT);
    cap_f += gp->ntiles * ((gp->batch + 15) / 16);
    cap_i += gp->ntiles * ((gp->batch + 15) / 16);
    if (only_group >= 0 && gi != only_group) continue;
    for (int t = d.bp[0].tile0; t < gp->ntiles; t++) {
      const double tile_cost = (double)N * std::max(1, gp->h_pairs[t * PT].lsum);
      for (int b = 0; b * btf < gp->batch; b++)
        betaf.push_back({tile_cost * std::min(btf, gp->batch - b * btf), WorkItem{gi, t, b}});
      for (int b = 0; b * bti < gp->batch; b++)
        betai.push_back({tile_cost * std::min(bti, gp->batch - b * bti), WorkItem{gi, t, b}});
    }
  }
  if (bf) {
    ms->smem_betaf = XBF_SMEM;
    ms->smem_betai = XBI_SMEM;
  } else {
    ms->smem_betaf = betaf_smem<T>(ms->rtmax, ms->kc);
    ms->smem_betai = inverse_smem<T>();
  }
  auto by_cost = [](const std::pair<double, WorkItem>& x, const std::pair<double, WorkItem>& y) {
    return x.first > y.first;
  };
  hipError_t e;
  if (first) {
    ms->max_betaf = cap_f;
    ms->max_betai = cap_i;
    if ((e = mixed_alloc(ms, &ms->d_groups, sizeof(GroupDev<T>) * ng)) != hipSuccess) return hip_fail(e);
    if ((e = mixed_alloc(ms, (void**)&ms->d_ringf, sizeof(WorkItem) * ringf.size())) != hipSuccess) return hip_fail(e);
    if ((e = mixed_alloc(ms, (void**)&ms->d_ringg, sizeof(WorkItem) * ringg.size())) != hipSuccess) return hip_fail(e);
    if ((e = mixed_alloc(ms, (void**)&ms->d_betaf, sizeof(WorkItem) * cap_f)) != hipSuccess) return hip_fail(e);
    if ((e = mixed_alloc(ms, (void**)&ms->d_betai, sizeof(WorkItem) * cap_i)) != hipSuccess) return hip_fail(e);
  }
  if ((int)betaf.size() > ms->max_betaf || (int)betai.size() > ms->max_betai) return SU2_ERR_INVALID_VALUE;
  if ((e = hipMemcpy(ms->d_groups, hg.data(), sizeof(GroupDev<T>) * ng, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  // each list: sorted by decreasing cost, uploaded
  auto upload = [&](std::vector<std::pair<double, WorkItem>>& lst, WorkItem* dst, int* n) -> hipError_t {
    std::stable_sort(lst.begin(), lst.end(), by_cost);
    std::vector<WorkItem> v;
    for (auto& x : lst) v.push_back(x.second);
    *n = (int)v.size();
    return v.empty() ? hipSuccess : hipMemcpy(dst, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice);
  };
  if ((e = upload(ringf, ms->d_ringf, &ms->n_ringf)) != hipSuccess) return hip_fail(e);
  if ((e = upload(ringg, ms->d_ringg, &ms->n_ringg)) != hipSuccess) return hip_fail(e);
  // contraction lists: by class (largest first), then by tile width where a
  // class is split (widest first), then by decreasing cost; one run per class
  // and width set
  auto upload_runs = [&](std::vector<std::pair<double, WorkItem>>& lst, WorkItem* dst, int* n,
                         std::vector<MixedState::Run>& runs, bool fwd) -> hipError_t {
    auto cls = [&](const WorkItem& w) { return fwd ? hg[w.g].rtmax : (bf ? hg[w.g].lq2 : hg[w.g].lq); };
    auto narrow = [&](const WorkItem& w) { return fwd ? (!bf && hg[w.g].narrow_f) : hg[w.g].narrow_i != 0; };
    int present[17] = {0};  // per class: 1 = 16-signal tasks, 2 = widest
    for (auto& x : lst) present[cls(x.second)] |= narrow(x.second) ? 1 : 2;
    bool split[17] = {false};
    for (int c = 1; c <= 16; c++) {
      if (present[c] != 3) continue;
      const void* both = fwd ? betaf_kernel_ptr<T>(c, ms->kc, 3) : (bf ? betai_bf16_kernel_ptr(c, 3) : betai_kernel_ptr<T>(c, 3));
      const void* one = fwd ? betaf_kernel_ptr<T>(c, ms->kc, 1) : (bf ? betai_bf16_kernel_ptr(c, 1) : betai_kernel_ptr<T>(c, 1));
      const int threads = fwd ? FWD_THREADS : (bf ? XB_THREADS : betai_threads<T>(c));
      const size_t smem = fwd ? betaf_smem<T>(c, ms->kc) : (bf ? XBI_SMEM : inverse_smem<T>());
      const int nb = wgs_per_cu(both, threads, smem, pl->device), n1 = wgs_per_cu(one, threads, smem, pl->device);
      split[c] = nb < 2 && n1 > nb;
    }
    auto wset = [&](const WorkItem& w) {
      const int c = cls(w);
      return present[c] == 3 && !split[c] ? 3 : (narrow(w) ? 1 : 2);
    };
    std::stable_sort(lst.begin(), lst.end(), [&](const std::pair<double, WorkItem>& x,
                                                 const std::pair<double, WorkItem>& y) {
      const int cx = cls(x.second), cy = cls(y.second);
      if (cx != cy) return cx > cy;
      const int wx = wset(x.second), wy = wset(y.second);
      return wx != wy ? wx > wy : x.first > y.first;
    });
    runs.clear();
    std::vector<WorkItem> v;
    for (auto& x : lst) {
      const int c = cls(x.second), a = wset(x.second);
      if (runs.empty() || runs.back().cls != c || runs.back().w != a) runs.push_back({c, a, (int)v.size(), 0});
      runs.back().n++;
      v.push_back(x.second);
    }
    *n = (int)v.size();
    return v.empty() ? hipSuccess : hipMemcpy(dst, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice);
  };
  if ((e = upload_runs(betaf, ms->d_betaf, &ms->n_betaf, ms->runs_f, true)) != hipSuccess) return hip_fail(e);
  if ((e = upload_runs(betai, ms->d_betai, &ms->n_betai, ms->runs_i, false)) != hipSuccess) return hip_fail(e);
  if ((e = set_worklist_smem<T>(pl)) != hipSuccess) return hip_fail(e);
  return SU2_OK;
}

su2_status_t rebuild_worklists(su2_plan_s* pl, int only_group = -1) {
  return pl->dtype == SU2_C128 ? build_worklists<double>(pl, only_group) : build_worklists<float>(pl, only_group);
}

// ---- autotuner: tile shapes and persistent grid sizes ----
//
// At plan creation each mixed plan chooses, by timing its own work lists on
// scratch buffers (HIP events, best of two after a warm-up):
//   1. per bandlimit group, the signals per contraction tile: 16 or the
//      widest (32 in FP32) in the forward (FP32) and in the inverse (FP32 and
//      split BF16), timing that group's contraction tasks alone;
//   2. the nodes per forward chunk, 4 or 8 (FP32 and FP64);
//   3. the grid of each of the four work-list kernels, 1, 2, 3, 4, 6 or 8
//      workgroups per CU walking the list, or one workgroup per task.
//      SU2_GRID="a,b,c,d" pins them (0 for one per task) over the search.
// None of them changes a result (every signal's sums run in the same order).
// Choices are cached per (device, mode, bandlimit mix) in the process and,
// with SU2_AUTOTUNE_CACHE naming a text file, across processes.
// SU2_AUTOTUNE=0 keeps the defaults (16-signal tiles for FP32 groups of at
// most 16 signals, the widest otherwise; 4-node FP32 and 8-node FP64 chunks;
// 2 workgroups per CU).  SU2_TILE_SHAPES="kc,fwd,inv" (e.g. "8,16,32") pins
// the shapes of every group where they apply and skips steps 1 and 2.

std::mutex g_tune_mu;
std::map<std::string, std::vector<int>> g_tune_cache;
std::string g_tune_file_loaded;   // cache file already read into g_tune_cache

// the grid candidates of the autotuner, in workgroups per CU (0: one
// workgroup per task, no task loop)
constexpr int GRID_CANDS[] = {1, 2, 3, 4, 6, 8, 0};
bool grid_candidate(int v) {
  for (int c : GRID_CANDS)
    if (v == c) return true;
  return false;
}

// SU2_GRID="a,b,c,d": the four work-list grids pinned (each a candidate)
bool pinned_grid(int (&k)[4]) {
  const char* env = getenv("SU2_GRID");
  if (!env || sscanf(env, "%d,%d,%d,%d", &k[0], &k[1], &k[2], &k[3]) != 4) return false;
  for (int v : k)
    if (!grid_candidate(v)) return false;
  return true;
}

// shapes pinned through SU2_TILE_SHAPES ("kc,fwd,inv"); false if unset or malformed
bool pinned_shapes(int* kc, int* fwd, int* inv) {
  const char* env = getenv("SU2_TILE_SHAPES");
  if (!env) return false;
  return sscanf(env, "%d,%d,%d", kc, fwd, inv) == 3;
}

std::string tune_key(const su2_plan_s* pl) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, pl->device) == hipSuccess) arch = prop.gcnArchName;
  std::string k = arch + ":" + std::to_string((int)pl->dtype) + (pl->real ? "r" : "") + (pl->so3 ? "s" : "");
  const MixedState* ms = pl->mixed;
  for (size_t g = 0; g < ms->groups.size(); g++)
    k += ":" + std::to_string(ms->group_B[g]) + "x" + std::to_string(ms->groups[g]->batch);
  int kc, f, i;
  if (pinned_shapes(&kc, &f, &i)) k += ":pinned" + std::to_string(kc) + "," + std::to_string(f) + "," + std::to_string(i);
  return k;
}

void load_tune_file() {
  const char* path = getenv("SU2_AUTOTUNE_CACHE");
  if (!path || g_tune_file_loaded == path) return;
  g_tune_file_loaded = path;
  FILE* f = fopen(path, "r");
  if (!f) return;
  static char line[1 << 16];
  while (fgets(line, sizeof(line), f)) {
    char* p = line;
    while (*p && *p != ' ' && *p != '\n') p++;
    if (*p != ' ') continue;
    *p++ = 0;
    std::vector<int> v;
    char* end = nullptr;
    for (long x = strtol(p, &end, 10); end != p; x = strtol(p, &end, 10)) {
      v.push_back((int)x);
      p = end;
    }
    if (v.size() >= 5) g_tune_cache[line] = v;
  }
  fclose(f);
}

void store_tune_file(const std::string& key, const std::vector<int>& v) {
  const char* path = getenv("SU2_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s", key.c_str());
  for (int x : v) fprintf(f, " %d", x);
  fprintf(f, "\n");
  fclose(f);
}

su2_status_t autotune(su2_plan_s* pl) {
  MixedState* ms = pl->mixed;
  const bool bf = pl->dtype == SU2_C64_BF16X3, dbl = pl->dtype == SU2_C128;
  const int ng = (int)ms->groups.size();
  su2_status_t st;
  int pk = 0, pf = 0, pi = 0;
  const bool pinned = pinned_shapes(&pk, &pf, &pi);
  if (pinned) {
    if (!bf && (pk == 4 || pk == 8)) ms->kc = pk;
    for (int g = 0; g < ng; g++) {
      if (!bf && !dbl && (pf == 16 || pf == 32)) ms->narrow_f[g] = pf == 16;
      if (!dbl && (pi == 16 || pi == 32)) ms->narrow_i[g] = pi == 16;
    }
    if ((st = rebuild_worklists(pl)) != SU2_OK) return st;
  }
  const char* env = getenv("SU2_AUTOTUNE");
  if (env && env[0] == '0') return SU2_OK;  // keep the defaults (or the pinned shapes)
  const std::string key = tune_key(pl);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    // an entry is used only if every value is one the search could have chosen
    auto valid = [&](const std::vector<int>& v) {
      if (v.size() != (size_t)(5 + 2 * ng)) return false;
      for (int i = 0; i < 4; i++)
        if (!grid_candidate(v[i])) return false;
      if (v[4] != 4 && v[4] != 8) return false;
      for (int g = 0; g < 2 * ng; g++)
        if (v[5 + g] != 0 && (v[5 + g] != 1 || dbl)) return false;
      return true;
    };
    if (it != g_tune_cache.end() && valid(it->second)) {
      const std::vector<int>& v = it->second;
      for (int i = 0; i < 4; i++) ms->knob[i] = v[i];
      ms->kc = v[4];
      for (int g = 0; g < ng; g++) {
        ms->narrow_f[g] = v[5 + g];
        ms->narrow_i[g] = v[5 + ng + g];
      }
      return rebuild_worklists(pl);
    }
  }
  const size_t cb = pl->dtype == SU2_C128 ? 16 : 8;
  void *din = nullptr, *dout = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&din, cb * (size_t)ms->total_samples)) != hipSuccess) return hip_fail(e);
  if ((e = hipMalloc(&dout, cb * (size_t)std::max(ms->total_samples, ms->total_coeffs))) != hipSuccess) {
    (void)hipFree(din);
    return hip_fail(e);
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipMemset(din, 0, cb * (size_t)ms->total_samples);
  (void)hipMemset(dout, 0, cb * (size_t)std::max(ms->total_samples, ms->total_coeffs));
  // stage order: ring forward (samples -> S), contraction forward, contraction inverse, ring inverse
  const void* ins[4] = {din, nullptr, dout, nullptr};
  void* outs[4] = {nullptr, dout, nullptr, din};
  const int dirs[4] = {0, 0, 1, 1};
  st = SU2_OK;
  // fastest of two timed launches after a warm-up; 1e30 on an error (st set)
  auto time_launch = [&](int which, int kn) -> float {
    float tmin = 1e30f;
    for (int rep = 0; rep < 3 && st == SU2_OK; rep++) {
      (void)hipEventRecord(e0, ms->cap);
      if ((e = enqueue_any(pl, which, dirs[which], ins[which], outs[which], ms->cap, kn)) != hipSuccess) {
        st = hip_fail(e);
        break;
      }
      (void)hipEventRecord(e1, ms->cap);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        st = hip_fail(e);
        break;
      }
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (rep > 0) tmin = std::min(tmin, t);
    }
    return tmin;
  };
  if (!pinned) {
    // 1. per group: signals per contraction tile (forward, then inverse)
    for (int g = 0; g < ng && st == SU2_OK; g++) {
      for (int which = 1; which <= 2 && st == SU2_OK; which++) {
        if (dbl || (bf && which == 1)) continue;  // one tile width only
        std::vector<int>& nar = which == 1 ? ms->narrow_f : ms->narrow_i;
        float best = 1e30f;
        int best_c = nar[g];
        for (int cand = 1; cand >= 0 && st == SU2_OK; cand--) {
          nar[g] = cand;
          if ((st = rebuild_worklists(pl, g)) != SU2_OK) break;
          const float t = time_launch(which, 2);
          if (t < best) { best = t; best_c = cand; }
        }
        nar[g] = best_c;
      }
    }
    // 2. nodes per forward chunk
    if (!bf && st == SU2_OK) {
      float best = 1e30f;
      int best_c = ms->kc;
      for (int cand : {4, 8}) {
        ms->kc = cand;
        if ((st = rebuild_worklists(pl)) != SU2_OK) break;
        const float t = time_launch(1, 2);
        if (t < best) { best = t; best_c = cand; }
      }
      ms->kc = best_c;
    }
  }
  if (st == SU2_OK) st = rebuild_worklists(pl);
  // 3. persistent grid size of each work-list kernel
  for (int which = 0; which < 4 && st == SU2_OK; which++) {
    float best = 1e30f;
    int best_k = ms->knob[which];
    for (int kn : GRID_CANDS) {
      const float t = time_launch(which, kn);
      if (st != SU2_OK) break;
      if (t < best) { best = t; best_k = kn; }
    }
    ms->knob[which] = best_k;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(din);
  (void)hipFree(dout);
  if (st != SU2_OK) return st;
  std::vector<int> v = {ms->knob[0], ms->knob[1], ms->knob[2], ms->knob[3], ms->kc};
  v.insert(v.end(), ms->narrow_f.begin(), ms->narrow_f.end());
  v.insert(v.end(), ms->narrow_i.begin(), ms->narrow_i.end());
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = v;
  store_tune_file(key, v);
  return SU2_OK;
}

void destroy_mixed(su2_plan_s* pl) {
  MixedState* ms = pl->mixed;
  if (!ms) return;
  for (auto& g : ms->graphs) (void)hipGraphExecDestroy(g.exec);
  ms->graphs.clear();
  for (su2_plan_s* gp : ms->groups) {
    gp->release();
    delete gp;
  }
  ms->groups.clear();
  for (void* p : ms->allocs) (void)hipFree(p);
  ms->allocs.clear();
  if (ms->fork) (void)hipEventDestroy(ms->fork);
  if (ms->join) (void)hipEventDestroy(ms->join);
  if (ms->side) (void)hipStreamDestroy(ms->side);
  if (ms->cap) (void)hipStreamDestroy(ms->cap);
  delete ms;
  pl->mixed = nullptr;
}

}  // namespace

namespace su2 {

su2_status_t create_mixed(const int32_t* Bs, int32_t batch, su2_dtype_t dtype, bool real, bool so3, su2_plan_s* pl) {
  MixedState* ms = new (std::nothrow) MixedState();
  if (!ms) return SU2_ERR_OUT_OF_MEMORY;
  pl->mixed = ms;
  pl->dtype = dtype;
  pl->real = real;
  pl->so3 = so3;
  pl->batch = batch;
  pl->B = -1;
  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e);
  pl->device = dev;
  if ((e = hipDeviceGetAttribute(&ms->num_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return hip_fail(e);
  // signal offsets in the concatenated buffers, and the groups
  std::vector<long long> soff(batch), coff(batch);
  std::map<int, std::vector<int>> by_B;
  for (int s = 0; s < batch; s++) {
    const long long N = 2LL * Bs[s];
    soff[s] = ms->total_samples;
    coff[s] = ms->total_coeffs;
    ms->total_samples += N * N * N;
    const long long L = (Bs[s] - 1) / 2;  // SO(3): largest integer l
    ms->total_coeffs += so3 ? (L + 1) * (2 * L + 1) * (2 * L + 3) / 3 : (long long)Bs[s] * (Bs[s] + 1) * (2 * Bs[s] + 1) / 6;
    by_B[Bs[s]].push_back(s);
  }
  for (auto& kv : by_B) {
    su2_plan_s* gp = new (std::nothrow) su2_plan_s();
    if (!gp) return SU2_ERR_OUT_OF_MEMORY;
    ms->groups.push_back(gp);
    ms->group_B.push_back(kv.first);
    gp->B = kv.first;
    gp->batch = (int)kv.second.size();
    gp->dtype = dtype;
    gp->real = real;
    gp->so3 = so3;
    std::vector<long long> so, co;
    for (int s : kv.second) { so.push_back(soff[s]); co.push_back(coff[s]); }
    long long *dso = nullptr, *dco = nullptr;
    if ((e = gp->alloc((void**)&dso, sizeof(long long) * so.size())) != hipSuccess) return hip_fail(e);
    if ((e = gp->alloc((void**)&dco, sizeof(long long) * co.size())) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(dso, so.data(), sizeof(long long) * so.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipMemcpy(dco, co.data(), sizeof(long long) * co.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e);
    gp->d_soff = dso;
    gp->d_coff = dco;
    su2_status_t st = build_plan(gp);
    if (st != SU2_OK) return st;
    pl->bytes += gp->bytes;
  }
  su2_status_t st = rebuild_worklists(pl);
  if (st != SU2_OK) return st;
  if ((e = hipStreamCreateWithFlags(&ms->cap, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamCreateWithFlags(&ms->side, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);
  if ((e = hipEventCreateWithFlags(&ms->fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e);
  if ((e = hipEventCreateWithFlags(&ms->join, hipEventDisableTiming)) != hipSuccess) return hip_fail(e);
  st = autotune(pl);
  if (st != SU2_OK) return st;
  int pk[4];
  if (pinned_grid(pk))  // overrides the search and the cache (not stored)
    for (int i = 0; i < 4; i++) ms->knob[i] = pk[i];
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e);
  return SU2_OK;
}

void release_mixed(su2_plan_s* pl) { destroy_mixed(pl); }

su2_status_t run_mixed(su2_plan_s* pl, int dir, const void* in, void* out, hipStream_t stream) {
  MixedState* ms = pl->mixed;
  for (auto& g : ms->graphs)
    if (g.dir == dir && g.in == in && g.out == out && g.stream == stream) {
      hipError_t e = hipGraphLaunch(g.exec, stream);
      return e == hipSuccess ? SU2_OK : hip_fail(e);
    }
  hipError_t e;
  hipGraph_t graph = nullptr;
  if ((e = hipStreamBeginCapture(ms->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(e);
  hipError_t le = enqueue_call(pl, dir, in, out, ms->cap);
  e = hipStreamEndCapture(ms->cap, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(le);
  }
  if (e != hipSuccess) return hip_fail(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e);
  if (ms->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(ms->graphs.front().exec);
    ms->graphs.erase(ms->graphs.begin());
  }
  ms->graphs.push_back(MixedGraph{dir, in, out, stream, exec});
  e = hipGraphLaunch(exec, stream);
  return e == hipSuccess ? SU2_OK : hip_fail(e);
}

void mixed_tuning(const su2_plan_s* pl, int32_t* knobs) {
  for (int i = 0; i < 4; i++) knobs[i] = pl->mixed ? pl->mixed->knob[i] : 0;
}

int mixed_shapes(const su2_plan_s* pl, int32_t* out, int32_t capacity) {
  const MixedState* ms = pl->mixed;
  const int ng = (int)ms->groups.size();
  const bool bf = pl->dtype == SU2_C64_BF16X3;
  const int wide = pl->dtype == SU2_C128 ? BetaCfg<double>::BT : BetaCfg<float>::BT;
  for (int g = 0; g < ng && out && 4 * g + 3 < capacity; g++) {
    out[4 * g] = ms->group_B[g];
    out[4 * g + 1] = bf ? XBF_BT : (ms->narrow_f[g] ? 16 : wide);
    out[4 * g + 2] = ms->narrow_i[g] ? 16 : (bf ? XB_BT : wide);
    out[4 * g + 3] = bf ? XB_KC : ms->kc;
  }
  return ng;
}

}  // namespace su2
