// Host side of the su2fft C ABI: argument validation, grid and quadrature,
// the pair ordering and FFT bin map, plan tables and workspace, dispatch.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "su2fft_plan.h"

using namespace su2;

static thread_local int32_t g_last_hip_error = 0;

// ---- scratch of the allocation-free forward (su2_forward_noalloc) ----
// The ring spectra of a su2_forward_noalloc call live in this file-scope
// device array: one copy per GPU, held while the process runs.  On the host
// the array's name only stands for the symbol; host code uses the device
// address hipGetSymbolAddress returns on each GPU (scratch_address), never
// the name itself.
static __device__ __align__(256) unsigned char scratch[SU2_NOALLOC_SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, which must be current.
// Resolved once per device (at the first plan creation or noalloc call on it).
static hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

namespace su2 {

void set_last_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

su2_status_t hip_fail(hipError_t e) {
  g_last_hip_error = (int32_t)e;
  // a failed runtime call also sets HIP's per-thread "last error"; reset it so
  // that it is not reported again by the next launch check of a later call
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SU2_ERR_OUT_OF_MEMORY;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return SU2_ERR_NO_DEVICE;
  return SU2_ERR_HIP;
}

bool only_2_3(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// radix sequence for a length that is a product of 2s and 3s: 8s first, then
// a 4 or a 2 for the rest of the power of two, then 3s.
}  // namespace su2

namespace {

int radix_plan(int L, int* rad) {
  int n = 0;
  int p2 = 0, p3 = 0;
  while (L % 2 == 0) { L /= 2; p2++; }
  while (L % 3 == 0) { L /= 3; p3++; }
  while (p2 >= 3) { rad[n++] = 8; p2 -= 3; }
  if (p2 == 2) rad[n++] = 4;
  if (p2 == 1) rad[n++] = 2;
  for (int i = 0; i < p3; i++) rad[n++] = 3;
  return n;
}

// position of frequency q after in-place decimation-in-frequency passes with
// the given radix sequence on a length-L line
int dif_position(int q, int L, const int* rad, int nrad) {
  int pos = 0;
  for (int s = 0; s < nrad; s++) {
    const int R = rad[s];
    L /= R;
    pos += (q % R) * L;
    q /= R;
  }
  return pos;
}

int imod(int a, int n) { return ((a % n) + n) % n; }

// Clenshaw-Curtis weights on the n+1 Chebyshev extreme points cos(k pi / n)
// (closed endpoint weights plus a cosine sum for the interior), long double.
void clenshaw_curtis(int n, std::vector<long double>& w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  w.assign(n + 1, 0.0L);
  if (n == 1) { w[0] = w[1] = 1.0L; return; }
  const bool even = (n % 2 == 0);
  const long double wend = even ? 1.0L / ((long double)n * n - 1.0L) : 1.0L / ((long double)n * n);
  w[0] = w[n] = wend;
  for (int i = 1; i < n; i++) {
    const long double th = pi * i / n;
    long double v = 1.0L;
    const int kmax = even ? n / 2 - 1 : (n - 1) / 2;
    for (int k = 1; k <= kmax; k++) v -= 2.0L * cosl(2.0L * k * th) / (4.0L * k * k - 1.0L);
    if (even) v -= cosl(n * th) / ((long double)n * n - 1.0L);
    w[i] = 2.0L * v / n;
  }
}

void grid_ld(int B, std::vector<long double>& alpha, std::vector<long double>& beta, std::vector<long double>& gamma,
             std::vector<long double>& W, bool so3 = false) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const int N = 2 * B;
  alpha.resize(N); beta.resize(N); gamma.resize(N);
  std::vector<long double> w;
  clenshaw_curtis(N - 1, w);
  W.resize(N);
  for (int i = 0; i < N; i++) {
    alpha[i] = -pi + 2.0L * pi * i / N;
    beta[i] = pi * i / (N - 1);
    // SU(2): psi over [-2 pi, 2 pi); SO(3): the paper's [-pi, pi)
    gamma[i] = so3 ? -pi + 2.0L * pi * i / N : -2.0L * pi + 4.0L * pi * i / N;
    W[i] = w[i] / (2.0L * N * N);
  }
}

}  // namespace

namespace {

template <class T>
hipError_t upload_typed(su2_plan_s* pl, const std::vector<long double>& W, const std::vector<long double>& twr,
                        const std::vector<long double>& twi, const std::vector<int>& rho_e) {
  const int N = pl->N;
  std::vector<T> hW(N);
  for (int i = 0; i < N; i++) hW[i] = (T)W[i];
  std::vector<cpx<T>> htw(2 * N);
  for (int i = 0; i < 2 * N; i++) htw[i] = {(T)twr[i], (T)twi[i]};
  std::vector<cpx<T>> hrho(pl->P_pad);
  const T ir[4] = {1, 0, -1, 0}, ii[4] = {0, 1, 0, -1};  // i^e
  for (int p = 0; p < pl->P_pad; p++) hrho[p] = {ir[rho_e[p]], ii[rho_e[p]]};
  hipError_t e;
  if ((e = pl->alloc(&pl->d_W, sizeof(T) * N)) != hipSuccess) return e;
  if ((e = pl->alloc(&pl->d_tw, sizeof(cpx<T>) * 2 * N)) != hipSuccess) return e;
  if ((e = pl->alloc(&pl->d_rho, sizeof(cpx<T>) * pl->P_pad)) != hipSuccess) return e;
  if ((e = hipMemcpy(pl->d_W, hW.data(), sizeof(T) * N, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(pl->d_tw, htw.data(), sizeof(cpx<T>) * 2 * N, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(pl->d_rho, hrho.data(), sizeof(cpx<T>) * pl->P_pad, hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  return hipSuccess;
}

}  // namespace

namespace su2 {

// Scalars of the on-the-fly tables: per pair the seed constant
// (-1)^neg sqrt(C(2 l0, top)), per (pair, degree index i >= 1) the three
// coefficients of the step that produces degree l0 + i from l0 + i - 1 and
// l0 + i - 2 (tile-major rows, like the table), and per node cos beta,
// cos beta/2, sin beta/2.  Computed in long double, stored as double.
hipError_t upload_otf_scalars(su2_plan_s* pl, const std::vector<long double>& beta) {
  const int N = pl->N;
  const std::vector<PairInfo>& pairs = pl->h_pairs;
  std::vector<double> seedc(pl->P_pad, 0.0), rc((size_t)3 * (pl->tab_elems / N + 1), 0.0), nodes(3 * (size_t)N);
  for (int p = 0; p < pl->P_pad; p++) {
    const PairInfo& q = pairs[p];
    if (q.L == 0) continue;
    int top, pc, ps, neg;
    wigner_seed_form(q.tl0, q.tn, q.tm, &top, &pc, &ps, &neg);
    long double lb = lgammal(q.tl0 + 1.0L) - lgammal(top + 1.0L) - lgammal(q.tl0 - top + 1.0L);
    seedc[p] = (double)((neg ? -1.0L : 1.0L) * expl(0.5L * lb));
    const long long row = q.tab / N + q.coff;
    const long double a = 0.5L * q.tn, b = 0.5L * q.tm;
    for (int i = 1; i < q.L; i++) {
      const long double l = 0.5L * (q.tl0 + 2 * (i - 1)), lp1 = l + 1.0L;  // step l -> l + 1
      const long double pre = lp1 * (2.0L * l + 1.0L) / sqrtl((lp1 * lp1 - a * a) * (lp1 * lp1 - b * b));
      long double c1 = 0.0L, c2 = 0.0L;
      if (l != 0.0L) {
        c1 = pre * a * b / (l * lp1);
        c2 = pre * sqrtl((l * l - a * a) * (l * l - b * b)) / (l * (2.0L * l + 1.0L));
      }
      rc[3 * (row + i)] = (double)pre;
      rc[3 * (row + i) + 1] = (double)c1;
      rc[3 * (row + i) + 2] = (double)c2;
    }
  }
  for (int k = 0; k < N; k++) {
    nodes[k] = (double)cosl(beta[k]);
    nodes[N + k] = (double)cosl(0.5L * beta[k]);
    nodes[2 * N + k] = (double)sinl(0.5L * beta[k]);
  }
  hipError_t e;
  if ((e = pl->alloc((void**)&pl->d_seedc, sizeof(double) * seedc.size())) != hipSuccess) return e;
  if ((e = pl->alloc((void**)&pl->d_rcoef, sizeof(double) * rc.size())) != hipSuccess) return e;
  if ((e = pl->alloc((void**)&pl->d_nodes, sizeof(double) * nodes.size())) != hipSuccess) return e;
  if ((e = hipMemcpy(pl->d_seedc, seedc.data(), sizeof(double) * seedc.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  if ((e = hipMemcpy(pl->d_rcoef, rc.data(), sizeof(double) * rc.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  return hipMemcpy(pl->d_nodes, nodes.data(), sizeof(double) * nodes.size(), hipMemcpyHostToDevice);
}

su2_status_t build_plan(su2_plan_s* pl) {
  const int B = pl->B, N = 2 * B;
  const bool so3 = pl->so3;
  pl->N = N;
  // the contraction kernels address one pair tile's ring spectra (N nodes x
  // batch x 16 pairs) with 32-bit byte offsets
  if ((size_t)N * (size_t)pl->batch * PT * (pl->dtype == SU2_C128 ? 16 : 8) > (size_t)INT32_MAX)
    return SU2_ERR_UNSUPPORTED;
  pl->ncoef = so3 ? (long long)((B - 1) / 2 + 1) * (2 * ((B - 1) / 2) + 1) * (2 * ((B - 1) / 2) + 3) / 3
                  : (long long)B * (B + 1) * (2 * B + 1) / 6;
  // ring bins of a pair (doubled indices): gamma frequency q, alpha frequency p,
  // and the exponent e of the phase rho = i^e that the ring kernels apply.
  //   SU(2): gamma_0 = -2 pi, alpha_0 = -pi: q = 2m, p = n (or n - 1/2 for
  //          half-integer n, with the half-bin shift), rho = i^{n-m} (-1)^{2m} e^{-i pi n}
  //   SO(3): gamma_0 = alpha_0 = -pi, integer m, n: q = m, p = n,
  //          rho = i^{n-m} e^{-i pi m} e^{-i pi n} = i^{3n + m}
  auto bin_q = [&](int tm) { return so3 ? imod(tm / 2, N) : imod(tm, N); };
  auto bin_p = [&](int tn) { return so3 ? imod(tn / 2, N) : imod((tn & 1) ? (tn - 1) / 2 : tn / 2, N); };
  auto phase_e = [&](int tm, int tn) {
    return so3 ? imod((3 * tn + tm) / 2, 4) : imod((tn - tm) / 2 + 2 * tm + 3 * tn, 4);
  };
  const size_t cb = (pl->dtype == SU2_C128) ? 16 : 8;

  hipError_t e;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e);
  pl->device = dev;
  {
    // set-up of the noalloc scratch on this device (once per device)
    void* scr = nullptr;
    if ((e = scratch_address(dev, &scr)) != hipSuccess) return hip_fail(e);
  }
  int max_lds = 0;
  if ((e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
    return hip_fail(e);

  // gamma-frequency classes: the smallest divisor of N whose class fits in LDS
  int split = 0;
  for (int s = 1; s <= MAX_SPLIT; s++) {
    if (N % s) continue;
    const size_t need = ((size_t)N * (N / s) + 2 * (size_t)N) * cb;
    if (need <= (size_t)max_lds) { split = s; break; }
  }
  if (split == 0) return SU2_ERR_UNSUPPORTED;
  // the register-resident ring kernels handle the whole ring themselves and
  // want the pairs ordered by 2m alone
  pl->fast = (pl->dtype == SU2_C128) ? fast_ring_supported<double>(N) : fast_ring_supported<float>(N);
  const bool n256 = !pl->fast && large_ring_supported(N);
  pl->sliced = n256 && pl->dtype != SU2_C128;
  pl->large = n256;
  // only the register-resident rings have a half-spectrum form for real signals
  pl->real_io = pl->real && !pl->fast;
  if (pl->fast || n256) split = 1;
  pl->split = split;
  pl->Nc = N / split;
  pl->nrad_c = radix_plan(pl->Nc, pl->rad_c);
  pl->nrad_n = radix_plan(N, pl->rad_n);

  // pairs (m, n): grouped by class r = (2m mod N) mod split, then 2m, then 2n
  std::vector<PairInfo> pairs;
  std::vector<int> fftpos, rho_e;
  long long tab = 0;
  for (int r = 0; r < split; r++) {
    pl->cls_begin[r] = (int)pairs.size();
    for (int tm = -(B - 1); tm <= B - 1; tm++) {
      if (so3 && (tm & 1)) continue;  // SO(3): integer m only
      const int q = bin_q(tm);
      if (q % split != r) continue;
      const int qp = q / split;
      const int ccol = dif_position(qp, pl->Nc, pl->rad_c, pl->nrad_c);
      for (int tn = -(B - 1); tn <= B - 1; tn++) {
        if ((tn - tm) & 1) continue;
        if (so3 && (tn & 1)) continue;
        PairInfo pi;
        pi.tm = tm; pi.tn = tn;
        pi.tl0 = abs(tm) > abs(tn) ? abs(tm) : abs(tn);
        pi.L = (B - 1 - pi.tl0) / 2 + 1;
        pi.tab = 0;
        pi.lsum = 0;
        pi.coff = 0;
        pi.itab = 0;
        pairs.push_back(pi);
        const int palpha = bin_p(tn);
        const int jrow = dif_position(palpha, N, pl->rad_n, pl->nrad_n);
        fftpos.push_back(jrow * pl->Nc + ccol);
        rho_e.push_back(phase_e(tm, tn));
      }
    }
    pl->cls_end[r] = (int)pairs.size();
  }
  pl->P = (int)pairs.size();
  // Layout of the pair list.  Point-symmetric where the ring kernels take the
  // pairs in one class ordered by (2m, 2n) (the list is then centrally
  // symmetric: its mirror (-m, -n) of position i sits at P - 1 - i), the plan
  // keeps a table (the on-the-fly plans keep none) and the padding fits the
  // ring kernels' slices: the pairs with 2m < 0, padded to whole tiles; the
  // 2m = 0 run with one pad right after (0, 0) and as many pads on both ends
  // as whole tiles need; the pads of the first part again; the pairs with
  // 2m > 0.  Position i then mirrors position P_pad - 1 - i, tile t mirrors
  // tile ntiles - 1 - t, and the upper tiles share the lower tiles' table
  // blocks (PairInfo::tsign).  Otherwise the pairs keep their order and the
  // list is padded at the end.
  auto pad_pair = []() {
    PairInfo pi;
    pi.tm = 0; pi.tn = 0; pi.tl0 = 0; pi.L = 0; pi.tab = 0; pi.lsum = 0; pi.coff = 0; pi.itab = 0;
    pi.tsign = 1; pi.towner = 1;
    return pi;
  };
  std::vector<int> order;  // index into `pairs` per position, -1 for a pad
  bool sym = split == 1 && !pl->otf && (pl->fast || n256);  // not the generic ring kernel (class ranges)
  if (sym) {
    int nA = 0, R0 = 0;
    for (const PairInfo& q : pairs) { nA += q.tm < 0; R0 += q.tm == 0; }
    const int nA16 = (nA + PT - 1) / PT * PT;
    int R16 = R0 + 1;                       // R0 is odd: the run is symmetric about (0, 0)
    while (R16 % PT) R16 += 2;
    const int a2 = (R16 - R0 - 1) / 2;
    for (int i = 0; i < nA; i++) order.push_back(i);
    for (int i = nA; i < nA16 + a2; i++) order.push_back(-1);
    for (int i = 0; i <= R0 / 2; i++) order.push_back(nA + i);      // (0, n <= 0)
    order.push_back(-1);                                            // the mirror of (0, 0)
    for (int i = R0 / 2 + 1; i < R0; i++) order.push_back(nA + i);  // (0, n > 0)
    for (int i = 0; i < a2 + nA16 - nA; i++) order.push_back(-1);
    for (int i = nA + R0; i < pl->P; i++) order.push_back(i);
    // check the mirror property position by position (pads pair with pads or (0, 0))
    const int T = (int)order.size();
    for (int i = 0; i < T && sym; i++) {
      const int a = order[i], b = order[T - 1 - i];
      if (a < 0 || b < 0) {
        const int o = a < 0 ? b : a;
        sym = o < 0 || (pairs[o].tm == 0 && pairs[o].tn == 0);
      } else {
        sym = pairs[a].tm == -pairs[b].tm && pairs[a].tn == -pairs[b].tn;
      }
    }
    if (T % PT) sym = false;
    // the slices of the register-resident ring kernels must still fit
    if (sym && pl->fast) {
      const int cap = pl->dtype == SU2_C128 ? fast_ring_slice_capacity<double>(N) : fast_ring_slice_capacity<float>(N);
      int rb[FAST_ROUNDS], re[FAST_ROUNDS];
      for (int r = 0; r < FAST_ROUNDS; r++) { rb[r] = T; re[r] = 0; }
      for (int i = 0; i < T; i++) {
        if (order[i] < 0) continue;
        const int r = bin_q(pairs[order[i]].tm) / (N / FAST_ROUNDS);
        rb[r] = std::min(rb[r], i);
        re[r] = std::max(re[r], i + 1);
      }
      for (int r = 0; r < FAST_ROUNDS; r++)
        if (re[r] > rb[r] && re[r] - rb[r] > cap) sym = false;
    }
  }
  if (!sym) {
    order.clear();
    for (int i = 0; i < pl->P; i++) order.push_back(i);
    while (order.size() % PT) order.push_back(-1);
  }
  pl->sym = sym;
  {
    std::vector<PairInfo> np;
    std::vector<int> nf, nr;
    for (int o : order) {
      if (o < 0) {
        np.push_back(pad_pair());
        nf.push_back(0);
        nr.push_back(0);
      } else {
        PairInfo q = pairs[o];
        q.tsign = 1;
        q.towner = 1;
        np.push_back(q);
        nf.push_back(fftpos[o]);
        nr.push_back(rho_e[o]);
      }
    }
    pairs.swap(np);
    fftpos.swap(nf);
    rho_e.swap(nr);
  }
  pl->P_pad = (int)pairs.size();
  pl->ntiles = pl->P_pad / PT;
  // tile-major table blocks; with the symmetric layout the upper tiles point
  // at their mirrors' blocks
  long long itab = 0;
  for (int t = 0; t < pl->ntiles; t++) {
    const int t0 = t * PT, tm_ = pl->ntiles - 1 - t;
    if (sym && tm_ < t) {
      const int m0 = tm_ * PT;
      for (int i = 0; i < PT; i++) {
        PairInfo& q = pairs[t0 + i];
        const PairInfo& mq = pairs[m0 + PT - 1 - i];
        q.tab = mq.tab;
        q.lsum = mq.lsum;
        q.coff = mq.coff;
        q.itab = mq.itab;
        q.towner = 0;
        q.tsign = (q.L > 0 && (((q.tm - q.tn) / 2) & 1)) ? -1 : 1;
      }
      continue;
    }
    int lsum = 0;
    for (int i = 0; i < PT; i++) { pairs[t0 + i].coff = lsum; lsum += pairs[t0 + i].L; }
    for (int i = 0; i < PT; i++) {
      pairs[t0 + i].tab = tab;
      pairs[t0 + i].lsum = lsum;
      pairs[t0 + i].itab = itab;
      itab += inverse_table_elems(pairs[t0 + i].L, N);
    }
    tab += (long long)N * lsum;
  }
  pl->tab_elems = tab;
  pl->itab_elems = itab;
  pl->h_pairs = pairs;
  // bin -> pair map for the register-resident ring kernels, and the pair range
  // of each slice of q values they process together
  std::vector<int> bins((size_t)N * N, -1);
  for (int r = 0; r < FAST_ROUNDS; r++) { pl->rbeg[r] = pl->P_pad; pl->rend[r] = 0; }
  for (int pidx = 0; pidx < pl->P_pad; pidx++) {
    if (pairs[pidx].L == 0) continue;  // padding
    const int tm = pairs[pidx].tm, tn = pairs[pidx].tn;
    const int q = bin_q(tm);
    const int palpha = bin_p(tn);
    bins[(size_t)q * N + palpha] = (pidx << 2) | rho_e[pidx];
    const int r = q / (N / FAST_ROUNDS);
    pl->rbeg[r] = pidx < pl->rbeg[r] ? pidx : pl->rbeg[r];
    pl->rend[r] = pidx + 1 > pl->rend[r] ? pidx + 1 : pl->rend[r];
  }
  // real signals: every bin's source pair (its own, or the mirror (-m, -n)
  // with a conjugate) for the inverse ring kernel
  std::vector<int> bins_real;
  if (pl->real && !pl->real_io) {
    std::vector<int> at((size_t)(2 * B - 1) * (2 * B - 1), -1);
    for (int pidx = 0; pidx < pl->P_pad; pidx++)
      if (pairs[pidx].L > 0) at[(size_t)(pairs[pidx].tm + B - 1) * (2 * B - 1) + pairs[pidx].tn + B - 1] = pidx;
    bins_real.assign((size_t)N * N, -1);
    for (int pidx = 0; pidx < pl->P_pad; pidx++) {
      if (pairs[pidx].L == 0) continue;
      const int tm = pairs[pidx].tm, tn = pairs[pidx].tn;
      const int q = imod(tm, N);
      const int palpha = imod((tn & 1) ? (tn - 1) / 2 : tn / 2, N);
      const bool mir = mirrored_pair(tm, tn);
      const int src = mir ? at[(size_t)(-tm + B - 1) * (2 * B - 1) + (-tn + B - 1)] : pidx;
      if (src < 0) return SU2_ERR_UNSUPPORTED;
      bins_real[(size_t)q * N + palpha] = (src << 3) | ((mir ? 1 : 0) << 2) | rho_e[pidx];
    }
  }
  for (int r = 0; r < FAST_ROUNDS; r++) {
    if (pl->rend[r] < pl->rbeg[r]) pl->rbeg[r] = pl->rend[r] = 0;
    const int cap = pl->dtype == SU2_C128 ? fast_ring_slice_capacity<double>(N) : fast_ring_slice_capacity<float>(N);
    if (pl->fast && pl->rend[r] - pl->rbeg[r] > cap) return SU2_ERR_UNSUPPORTED;
  }
  // one-pass N = 256 kernels (FP32): per gamma frequency q the bases from
  // which the kernels compute every bin's pair and phase (FastRingParams::cols),
  // checked here against the bin map; if the pair layout does not follow them,
  // the plan keeps the two-pass kernels
  std::vector<int> cols;
  if (pl->sliced) {
    cols.assign((size_t)4 * N, 0);
    bool ok = true;
    for (int q = 0; q < N && ok; q++) {
      const int* bq = &bins[(size_t)q * N];
      int* cq = &cols[(size_t)4 * q];
      const bool valid = bq[0] >= 0;
      if (valid) {
        int hi_first = 192;
        while (hi_first < N && bq[hi_first] < 0) hi_first++;
        if (hi_first > 195 || bq[1] < 0) { ok = false; break; }
        cq[0] = (bq[hi_first] >> 2) - (hi_first - 192);
        cq[1] = bq[0] >> 2;
        cq[2] = (bq[1] >> 2) - 1;
        cq[3] = (bq[0] & 3) | ((hi_first - 192) << 2) | (1 << 4);
      }
      for (int pp = 0; pp < N && ok; pp++) {
        const bool kept = valid && (pp < 64 || pp >= 192 + ((cq[3] >> 2) & 3));
        if (!kept) { ok = bq[pp] < 0; continue; }
        const int pidx = pp < 64 ? (pp == 0 ? cq[1] : cq[2] + pp) : cq[0] + (pp - 192);
        const int ee = (3 * pp + (cq[3] & 3)) & 3;
        ok = bq[pp] == ((pidx << 2) | ee);
      }
    }
    if (!ok) {
      cols.clear();
      pl->sliced = false;
    }
  }
  // two-pass kernels: pair range of every block of gamma frequencies
  std::vector<int> qrange;
  if (pl->large) {
    const int qb = large_ring_block(), nblk = N / qb;
    qrange.assign(2 * nblk, 0);
    for (int blk = 0; blk < nblk; blk++) { qrange[2 * blk] = pl->P_pad; qrange[2 * blk + 1] = 0; }
    for (int pidx = 0; pidx < pl->P_pad; pidx++) {
      if (pairs[pidx].L == 0) continue;
      const int blk = bin_q(pairs[pidx].tm) / qb;
      qrange[2 * blk] = std::min(qrange[2 * blk], pidx);
      qrange[2 * blk + 1] = std::max(qrange[2 * blk + 1], pidx + 1);
    }
    for (int blk = 0; blk < nblk; blk++) {
      if (qrange[2 * blk + 1] < qrange[2 * blk]) qrange[2 * blk] = qrange[2 * blk + 1] = 0;
      if (qrange[2 * blk + 1] - qrange[2 * blk] > large_ring_slice_capacity()) return SU2_ERR_UNSUPPORTED;
    }
  }
  std::vector<int> colq(pl->Nc);
  for (int qp = 0; qp < pl->Nc; qp++) colq[dif_position(qp, pl->Nc, pl->rad_c, pl->nrad_c)] = qp;

  std::vector<long double> alpha, beta, gamma, W;
  grid_ld(B, alpha, beta, gamma, W, so3);
  std::vector<long double> twr(2 * N), twi(2 * N);
  const long double pi_l = 3.141592653589793238462643383279502884L;
  for (int t = 0; t < 2 * N; t++) { twr[t] = cosl(pi_l * t / N); twi[t] = sinl(pi_l * t / N); }
  std::vector<double> hbeta(N);
  for (int i = 0; i < N; i++) hbeta[i] = (double)beta[i];

  // device tables
  double* d_beta = nullptr;
  if ((e = pl->alloc((void**)&pl->d_pairs, sizeof(PairInfo) * pl->P_pad)) != hipSuccess) return hip_fail(e);
  if ((e = pl->alloc((void**)&pl->d_fftpos, sizeof(int) * pl->P_pad)) != hipSuccess) return hip_fail(e);
  if ((e = pl->alloc((void**)&pl->d_colq, sizeof(int) * pl->Nc)) != hipSuccess) return hip_fail(e);
  if ((e = pl->alloc((void**)&d_beta, sizeof(double) * N)) != hipSuccess) return hip_fail(e);
  // the bin maps in the register-resident kernels' reading order: the
  // entries of (q, p2) for the kept rows p1 of the alpha split, contiguous
  int n1 = 0, n2 = 0;
  auto thread_order = [&](std::vector<int>& b) {
    if (!fast_ring_split(N, &n1, &n2)) return;
    std::vector<int> v((size_t)N * N, -1);
    const int h = n1 / 2;
    for (int q = 0; q < N; q++)
      for (int p2 = 0; p2 < n2; p2++)
        for (int i = 0; i < h; i++) {
          const int p1 = i < n1 / 4 ? i : i + n1 / 2;  // rows [0, N1/4) and [3 N1/4, N1)
          v[((size_t)q * n2 + p2) * h + i] = b[(size_t)q * N + p2 + n2 * p1];
        }
    b.swap(v);
  };
  thread_order(bins);
  if (pl->real && !pl->real_io) thread_order(bins_real);
  if ((e = pl->alloc((void**)&pl->d_bins, sizeof(int) * (size_t)N * N)) != hipSuccess) return hip_fail(e);
  if ((e = hipMemcpy(pl->d_bins, bins.data(), sizeof(int) * (size_t)N * N, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if (!cols.empty()) {
    if ((e = pl->alloc((void**)&pl->d_cols, sizeof(int) * cols.size())) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(pl->d_cols, cols.data(), sizeof(int) * cols.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e);
  }
  if (pl->real && !pl->real_io) {
    if ((e = pl->alloc((void**)&pl->d_bins_real, sizeof(int) * (size_t)N * N)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(pl->d_bins_real, bins_real.data(), sizeof(int) * (size_t)N * N, hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e);
  }
  if ((e = hipMemcpy(pl->d_pairs, pairs.data(), sizeof(PairInfo) * pl->P_pad, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipMemcpy(pl->d_fftpos, fftpos.data(), sizeof(int) * pl->P_pad, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipMemcpy(pl->d_colq, colq.data(), sizeof(int) * pl->Nc, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipMemcpy(d_beta, hbeta.data(), sizeof(double) * N, hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if (pl->dtype == SU2_C128)
    e = upload_typed<double>(pl, W, twr, twi, rho_e);
  else
    e = upload_typed<float>(pl, W, twr, twi, rho_e);
  if (e != hipSuccess) return hip_fail(e);

  // per-pair and per-node recurrence scalars: the on-the-fly tables and the
  // shifted-recurrence contraction use them (a few MB)
  if ((e = upload_otf_scalars(pl, beta)) != hipSuccess) return hip_fail(e);
  if (!pl->otf) {
    // tables are padded by 64 bytes of zeros: the contraction kernels read
    // whole 16-byte vectors, and up to 3 elements past a pair's row segment
    // (multiplied by zero operands)
    if ((e = pl->alloc((void**)&pl->d_tab64, sizeof(double) * (size_t)tab + 64)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemset(pl->d_tab64 + tab, 0, 64)) != hipSuccess) return hip_fail(e);
    if ((e = launch_dtable(B, N, pl->P_pad, pl->d_pairs, d_beta, pl->d_tab64, 0)) != hipSuccess) return hip_fail(e);
    // the inverse-layout copy read by the inverse and adjoint contractions
    if (pl->dtype == SU2_C128) {
      if ((e = pl->alloc((void**)&pl->d_tabi64, sizeof(double) * (size_t)pl->itab_elems + 64)) != hipSuccess)
        return hip_fail(e);
      if ((e = launch_inverse_table<double>(N, pl->P_pad, pl->d_pairs, pl->d_tab64, pl->d_tabi64, 0)) != hipSuccess)
        return hip_fail(e);
    } else if (pl->dtype == SU2_C64) {
      if ((e = pl->alloc((void**)&pl->d_tabi32, sizeof(float) * (size_t)pl->itab_elems + 64)) != hipSuccess)
        return hip_fail(e);
      if ((e = launch_inverse_table<float>(N, pl->P_pad, pl->d_pairs, pl->d_tab64, pl->d_tabi32, 0)) != hipSuccess)
        return hip_fail(e);
    }
  }
  if (pl->otf) {
    // no stored table
  } else if (pl->dtype == SU2_C64) {
    if ((e = pl->alloc((void**)&pl->d_tab32, sizeof(float) * (size_t)tab + 64)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemset(pl->d_tab32 + tab, 0, 64)) != hipSuccess) return hip_fail(e);
    if ((e = launch_round_table_f32(tab, pl->d_tab64, pl->d_tab32, 0)) != hipSuccess) return hip_fail(e);
  } else if (pl->dtype == SU2_C64_BF16X3) {
    // 256 bytes of zeros after the last block: the split inverse reads up to
    // 31 words past a pair's row segment (against zero operands)
    if ((e = pl->alloc((void**)&pl->d_tabbf, sizeof(bf16x2_t) * (size_t)tab + 256)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemset(pl->d_tabbf + tab, 0, 256)) != hipSuccess) return hip_fail(e);
    if ((e = launch_split_table_bf16(tab, pl->d_tab64, pl->d_tabbf, 0)) != hipSuccess) return hip_fail(e);
    const long long fwd_words = tab / N * (long long)((N + 7) / 8) * 8;
    if ((e = pl->alloc((void**)&pl->d_tabbf_fwd, sizeof(unsigned) * (size_t)fwd_words + 64)) != hipSuccess)
      return hip_fail(e);
    if ((e = launch_interleave_bf16_table(N, pl->ntiles, pl->d_pairs, pl->d_tabbf, pl->d_tabbf_fwd, 0)) != hipSuccess)
      return hip_fail(e);
  }
  if ((e = pl->alloc(&pl->d_S, cb * (size_t)pl->P_pad * N * pl->batch)) != hipSuccess) return hip_fail(e);
  if (pl->large && !pl->sliced) {
    // intermediate of the two-pass ring kernels: a chunk of rings, at most 128 MB
    const size_t ring_bytes = cb * (size_t)N * N;
    pl->large_chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)pl->batch * N, (128u << 20) / ring_bytes));
    if ((e = pl->alloc(&pl->d_G, ring_bytes * pl->large_chunk)) != hipSuccess) return hip_fail(e);
    if ((e = pl->alloc((void**)&pl->d_qrange, sizeof(int) * qrange.size())) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpy(pl->d_qrange, qrange.data(), sizeof(int) * qrange.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(e);
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e);
  return SU2_OK;
}

}  // namespace su2

namespace {

template <class T>
const T* table_of(const su2_plan_s* pl) {
  return std::is_same<T, double>::value ? (const T*)pl->d_tab64 : (const T*)pl->d_tab32;
}

template <class T>
su2_status_t run_stage_t(su2_plan_s* pl, su2_stage_t stage, const void* in, void* out, hipStream_t s, void* S) {
  hipError_t e = hipSuccess;
  switch (stage) {
    case SU2_STAGE_RING_FORWARD:
      if (pl->real && !pl->real_io)
        e = launch_ring_forward_fast_real<T>(fast_params<T>(pl, 0), (const T*)in, (cpx<T>*)S, s);
      else if (pl->sliced) {
        if constexpr (std::is_same<T, float>::value)
          e = launch_ring_sliced4(true, fast_params<T>(pl, 0), (const cpx<T>*)in, (cpx<T>*)S, s);
        else
          e = hipErrorInvalidValue;
      } else if (pl->large)
        e = launch_ring_forward_large<T>(large_params<T>(pl, 0), (const cpx<T>*)in, (cpx<T>*)S, s);
      else if (pl->fast)
        e = launch_ring_forward_fast<T>(fast_params<T>(pl, 0), (const cpx<T>*)in, (cpx<T>*)S, s);
      else
        e = launch_ring_forward<T>(ring_params<T>(pl, 0), (const cpx<T>*)in, (cpx<T>*)S, s);
      break;
    case SU2_STAGE_BETA_FORWARD:
      if (pl->otf)
        e = launch_beta_forward_otf<T>(otf_params<T>(pl, 0), (const cpx<T>*)S, (cpx<T>*)out, s);
      else
        e = launch_beta_forward<T>(beta_params<T>(pl, table_of<T>(pl), 0), (const cpx<T>*)S, (cpx<T>*)out, s);
      break;
    case SU2_STAGE_BETA_INVERSE:
    case SU2_STAGE_BETA_ADJOINT:
      if (pl->otf)
        e = launch_beta_inverse_otf<T>(otf_params<T>(pl, stage == SU2_STAGE_BETA_ADJOINT), (const cpx<T>*)in,
                                       (cpx<T>*)S, s);
      else
        e = launch_beta_inverse<T>(beta_params<T>(pl, table_of<T>(pl), stage == SU2_STAGE_BETA_ADJOINT),
                                   (const cpx<T>*)in, (cpx<T>*)S, s);
      break;
    case SU2_STAGE_RING_INVERSE:
    case SU2_STAGE_RING_ADJOINT:
      if (pl->real && !pl->real_io)
        e = launch_ring_inverse_fast_real<T>(fast_params<T>(pl, stage == SU2_STAGE_RING_ADJOINT),
                                             (const cpx<T>*)S, (T*)out, s);
      else if (pl->sliced) {
        if constexpr (std::is_same<T, float>::value)
          e = launch_ring_sliced4(false, fast_params<T>(pl, stage == SU2_STAGE_RING_ADJOINT), (const cpx<T>*)S,
                                  (cpx<T>*)out, s);
        else
          e = hipErrorInvalidValue;
      } else if (pl->large)
        e = launch_ring_inverse_large<T>(large_params<T>(pl, stage == SU2_STAGE_RING_ADJOINT),
                                         (const cpx<T>*)S, (cpx<T>*)out, s);
      else if (pl->fast)
        e = launch_ring_inverse_fast<T>(fast_params<T>(pl, stage == SU2_STAGE_RING_ADJOINT), (const cpx<T>*)S,
                                        (cpx<T>*)out, s);
      else
        e = launch_ring_inverse<T>(ring_params<T>(pl, stage == SU2_STAGE_RING_ADJOINT), (const cpx<T>*)S,
                                   (cpx<T>*)out, s);
      break;
    default:
      return SU2_ERR_INVALID_VALUE;
  }
  if (e != hipSuccess) return hip_fail(e);
  return SU2_OK;
}

// `S` holds the ring spectra between the two stages of a call: the plan's
// workspace, or (su2_forward_noalloc) the library's static scratch
su2_status_t run_stage(su2_plan_s* pl, su2_stage_t stage, const void* in, void* out, hipStream_t s,
                       void* S = nullptr) {
  if (!S) S = pl->d_S;
  if (pl->dtype == SU2_C128) return run_stage_t<double>(pl, stage, in, out, s, S);
  if (pl->dtype == SU2_C64_BF16X3) {
    hipError_t e = hipSuccess;
    if (stage == SU2_STAGE_BETA_FORWARD) {
      e = launch_beta_forward_bf16x3(beta_params<float>(pl, nullptr, 0), pl->d_tabbf_fwd,
                                     (const cpx<float>*)S, (cpx<float>*)out, s);
    } else if (stage == SU2_STAGE_BETA_INVERSE || stage == SU2_STAGE_BETA_ADJOINT) {
      e = launch_beta_inverse_bf16x3(beta_params<float>(pl, nullptr, stage == SU2_STAGE_BETA_ADJOINT),
                                     (const unsigned*)pl->d_tabbf, (const cpx<float>*)in, (cpx<float>*)S, s);
    } else {
      return run_stage_t<float>(pl, stage, in, out, s, S);
    }
    if (e != hipSuccess) return hip_fail(e);
    return SU2_OK;
  }
  return run_stage_t<float>(pl, stage, in, out, s, S);
}

su2_status_t run_pair(su2_plan_s* pl, su2_stage_t first, su2_stage_t second, const void* in, void* out,
                      hipStream_t s, void* S = nullptr) {
  su2_status_t st = run_stage(pl, first, in, nullptr, s, S);
  if (st != SU2_OK) return st;
  return run_stage(pl, second, nullptr, out, s, S);
}

su2_status_t check_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    g_last_hip_error = (int32_t)e;
    return SU2_ERR_NO_DEVICE;
  }
  return SU2_OK;
}

}  // namespace

extern "C" {

int64_t su2_num_samples(int32_t B) {
  if (B < 1) return -1;
  const int64_t N = 2 * (int64_t)B;
  return N * N * N;
}

int64_t su2_num_coeffs(int32_t B) {
  if (B < 1) return -1;
  return (int64_t)B * (B + 1) * (2 * B + 1) / 6;
}

int64_t su2_coeff_index(int32_t tl, int32_t tm, int32_t tn) {
  if (tl < 0 || tm < -tl || tm > tl || tn < -tl || tn > tl) return -1;
  if (((tl - tm) & 1) || ((tl - tn) & 1)) return -1;
  return (int64_t)tl * (tl + 1) * (2 * tl + 1) / 6 + (int64_t)((tm + tl) / 2) * (tl + 1) + (tn + tl) / 2;
}

su2_status_t su2_grid(int32_t B, double* alpha, double* beta, double* gamma, double* w_beta) {
  if (B < 1) return SU2_ERR_INVALID_VALUE;
  if (B > 128 || !only_2_3(2 * B)) return SU2_ERR_UNSUPPORTED;
  std::vector<long double> a, b, g, W;
  grid_ld(B, a, b, g, W);
  for (int i = 0; i < 2 * B; i++) {
    if (alpha) alpha[i] = (double)a[i];
    if (beta) beta[i] = (double)b[i];
    if (gamma) gamma[i] = (double)g[i];
    if (w_beta) w_beta[i] = (double)W[i];
  }
  return SU2_OK;
}

su2_status_t su2_plan_create(int32_t B, int32_t batch, su2_dtype_t dtype, su2_plan_t* out) {
  return su2_plan_create_ex(B, batch, dtype, 0u, out);
}

su2_status_t su2_plan_create_ex(int32_t B, int32_t batch, su2_dtype_t dtype, uint32_t flags, su2_plan_t* out) {
  if (!out) return SU2_ERR_INVALID_VALUE;
  *out = nullptr;
  if (B < 1 || batch < 1) return SU2_ERR_INVALID_VALUE;
  if (dtype != SU2_C128 && dtype != SU2_C64 && dtype != SU2_C64_BF16X3) return SU2_ERR_INVALID_VALUE;
  if (flags & ~(uint32_t)(SU2_PLAN_TABLES_ON_THE_FLY | SU2_PLAN_REAL_SIGNALS | SU2_PLAN_SO3))
    return SU2_ERR_INVALID_VALUE;
  if (B > 128 || !only_2_3(2 * B)) return SU2_ERR_UNSUPPORTED;
  if ((size_t)2 * B * (size_t)batch * PT * (dtype == SU2_C128 ? 16 : 8) > (size_t)INT32_MAX)
    return SU2_ERR_UNSUPPORTED;  // see build_plan
  if ((flags & SU2_PLAN_TABLES_ON_THE_FLY) && dtype == SU2_C64_BF16X3) return SU2_ERR_UNSUPPORTED;
  // real signals and SO(3): every mode and bandlimit, with stored tables, not together
  if ((flags & (SU2_PLAN_REAL_SIGNALS | SU2_PLAN_SO3)) && (flags & SU2_PLAN_TABLES_ON_THE_FLY))
    return SU2_ERR_UNSUPPORTED;
  if ((flags & SU2_PLAN_REAL_SIGNALS) && (flags & SU2_PLAN_SO3)) return SU2_ERR_UNSUPPORTED;
  su2_status_t st = check_device();
  if (st != SU2_OK) return st;
  su2_plan_s* pl = new (std::nothrow) su2_plan_s();
  if (!pl) return SU2_ERR_OUT_OF_MEMORY;
  pl->B = B;
  pl->batch = batch;
  pl->dtype = dtype;
  pl->otf = (flags & SU2_PLAN_TABLES_ON_THE_FLY) != 0;
  pl->real = (flags & SU2_PLAN_REAL_SIGNALS) != 0;
  pl->so3 = (flags & SU2_PLAN_SO3) != 0;
  st = build_plan(pl);
  if (st != SU2_OK) {
    (void)hipDeviceSynchronize();
    pl->release();
    delete pl;
    return st;
  }
  *out = pl;
  return SU2_OK;
}

su2_status_t su2_plan_create_mixed(const int32_t* B_per_signal, int32_t batch, su2_dtype_t dtype, su2_plan_t* out) {
  return su2_plan_create_mixed_ex(B_per_signal, batch, dtype, 0u, out);
}

su2_status_t su2_plan_create_mixed_ex(const int32_t* B_per_signal, int32_t batch, su2_dtype_t dtype, uint32_t flags,
                                      su2_plan_t* out) {
  if (!out || !B_per_signal) return SU2_ERR_INVALID_VALUE;
  *out = nullptr;
  if (batch < 1) return SU2_ERR_INVALID_VALUE;
  if (dtype != SU2_C128 && dtype != SU2_C64 && dtype != SU2_C64_BF16X3) return SU2_ERR_INVALID_VALUE;
  if (flags & ~(uint32_t)(SU2_PLAN_TABLES_ON_THE_FLY | SU2_PLAN_REAL_SIGNALS | SU2_PLAN_SO3))
    return SU2_ERR_INVALID_VALUE;
  if ((flags & SU2_PLAN_TABLES_ON_THE_FLY) || flags == (uint32_t)(SU2_PLAN_REAL_SIGNALS | SU2_PLAN_SO3))
    return SU2_ERR_UNSUPPORTED;
  for (int i = 0; i < batch; i++) {
    if (B_per_signal[i] < 1) return SU2_ERR_INVALID_VALUE;
    if (B_per_signal[i] > 128 || !only_2_3(2 * B_per_signal[i])) return SU2_ERR_UNSUPPORTED;
  }
  su2_status_t st = check_device();
  if (st != SU2_OK) return st;
  su2_plan_s* pl = new (std::nothrow) su2_plan_s();
  if (!pl) return SU2_ERR_OUT_OF_MEMORY;
  st = create_mixed(B_per_signal, batch, dtype, (flags & SU2_PLAN_REAL_SIGNALS) != 0, (flags & SU2_PLAN_SO3) != 0, pl);
  if (st != SU2_OK) {
    (void)hipDeviceSynchronize();
    release_mixed(pl);
    pl->release();
    delete pl;
    return st;
  }
  *out = pl;
  return SU2_OK;
}

su2_status_t su2_plan_destroy(su2_plan_t plan) {
  if (!plan) return SU2_OK;
  hipError_t e = hipDeviceSynchronize();
  release_mixed(plan);
  plan->release();
  delete plan;
  if (e != hipSuccess) return hip_fail(e);
  return SU2_OK;
}

su2_status_t su2_plan_tuning(su2_plan_t plan, int32_t* workgroups_per_cu) {
  if (!plan || !workgroups_per_cu) return SU2_ERR_INVALID_VALUE;
  if (!plan->mixed) return SU2_ERR_INVALID_VALUE;
  mixed_tuning(plan, workgroups_per_cu);
  return SU2_OK;
}

su2_status_t su2_plan_tile_shapes(su2_plan_t plan, int32_t* out, int32_t capacity, int32_t* count) {
  if (!plan || !count || !plan->mixed || capacity < 0) return SU2_ERR_INVALID_VALUE;
  *count = mixed_shapes(plan, out, capacity);
  return SU2_OK;
}

su2_status_t su2_plan_info(su2_plan_t plan, int32_t* B, int32_t* batch, int32_t* dtype, int64_t* device_bytes) {
  if (!plan) return SU2_ERR_INVALID_VALUE;
  if (B) *B = plan->B;
  if (batch) *batch = plan->batch;
  if (dtype) *dtype = (int32_t)plan->dtype;
  if (device_bytes) *device_bytes = plan->bytes;
  return SU2_OK;
}

su2_status_t su2_forward(su2_plan_t plan, const void* d_samples, void* d_coeffs, hipStream_t stream) {
  if (!plan || !d_samples || !d_coeffs) return SU2_ERR_INVALID_VALUE;
  if (plan->mixed) return run_mixed(plan, 0, d_samples, d_coeffs, stream);
  return run_pair(plan, SU2_STAGE_RING_FORWARD, SU2_STAGE_BETA_FORWARD, d_samples, d_coeffs, stream);
}

su2_status_t su2_inverse(su2_plan_t plan, const void* d_coeffs, void* d_samples, hipStream_t stream) {
  if (!plan || !d_samples || !d_coeffs) return SU2_ERR_INVALID_VALUE;
  if (plan->mixed) return run_mixed(plan, 1, d_coeffs, d_samples, stream);
  return run_pair(plan, SU2_STAGE_BETA_INVERSE, SU2_STAGE_RING_INVERSE, d_coeffs, d_samples, stream);
}

su2_status_t su2_adjoint(su2_plan_t plan, const void* d_coeffs, void* d_samples, hipStream_t stream) {
  if (!plan || !d_samples || !d_coeffs) return SU2_ERR_INVALID_VALUE;
  if (plan->mixed) return run_mixed(plan, 2, d_coeffs, d_samples, stream);
  return run_pair(plan, SU2_STAGE_BETA_ADJOINT, SU2_STAGE_RING_ADJOINT, d_coeffs, d_samples, stream);
}

su2_status_t su2_forward_noalloc(su2_plan_t plan, const void* d_samples, void* d_coeffs, hipStream_t stream) {
  if (!plan || !d_samples || !d_coeffs || plan->mixed) return SU2_ERR_INVALID_VALUE;
  // the two-pass forward ring (N = 256 in FP64) keeps a second plan-owned buffer
  if (plan->large && !plan->sliced) return SU2_ERR_UNSUPPORTED;
  const size_t need = (plan->dtype == SU2_C128 ? 16 : 8) * (size_t)plan->P_pad * plan->N * plan->batch;
  if (need > SU2_NOALLOC_SCRATCH_BYTES) return SU2_ERR_UNSUPPORTED;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev != plan->device) return SU2_ERR_INVALID_VALUE;
  void* S = nullptr;
  if ((e = scratch_address(dev, &S)) != hipSuccess) return hip_fail(e);
  return run_pair(plan, SU2_STAGE_RING_FORWARD, SU2_STAGE_BETA_FORWARD, d_samples, d_coeffs, stream, S);
}

su2_status_t su2_run_stage(su2_plan_t plan, su2_stage_t stage, const void* in, void* out, hipStream_t stream) {
  if (!plan || plan->mixed) return SU2_ERR_INVALID_VALUE;
  if ((int)stage < 0 || (int)stage > (int)SU2_STAGE_RING_ADJOINT) return SU2_ERR_INVALID_VALUE;
  const bool needs_in = stage == SU2_STAGE_RING_FORWARD || stage == SU2_STAGE_BETA_INVERSE ||
                        stage == SU2_STAGE_BETA_ADJOINT;
  if (needs_in ? !in : !out) return SU2_ERR_INVALID_VALUE;
  return run_stage(plan, stage, in, out, stream);
}

su2_status_t su2_plan_dtable(su2_plan_t plan, int32_t two_m, int32_t two_n, double* host_out, int32_t* L) {
  if (!plan || plan->mixed || (!host_out && !L)) return SU2_ERR_INVALID_VALUE;
  if (plan->otf && host_out) return SU2_ERR_UNSUPPORTED;
  for (int p = 0; p < plan->P_pad; p++) {
    const PairInfo& pi = plan->h_pairs[p];
    if (pi.L == 0 || pi.tm != two_m || pi.tn != two_n) continue;
    if (L) *L = pi.L;
    if (host_out) {
      std::vector<double> rows((size_t)plan->N * pi.lsum);
      hipError_t e = hipMemcpy(rows.data(), plan->d_tab64 + pi.tab, sizeof(double) * rows.size(),
                               hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e);
      for (int k = 0; k < plan->N; k++)
        for (int i = 0; i < pi.L; i++)
          host_out[(size_t)k * pi.L + i] = pi.tsign * rows[(size_t)k * pi.lsum + pi.coff + i];
    }
    return SU2_OK;
  }
  return SU2_ERR_INVALID_VALUE;
}

su2_status_t su2_beta_forward_shifted(su2_plan_t plan, int32_t depth, int32_t block, void* d_coeffs, hipStream_t stream) {
  if (!plan || plan->mixed || plan->real || plan->so3 || !d_coeffs) return SU2_ERR_INVALID_VALUE;
  if (depth != 1 && depth != 2) return SU2_ERR_INVALID_VALUE;
  if (depth == 2 && block != 2 && block != 4 && block != 8 && block != 16) return SU2_ERR_INVALID_VALUE;
  if (!shifted_supported(plan->B)) return SU2_ERR_UNSUPPORTED;
  hipError_t e;
  if (plan->dtype == SU2_C128)
    e = launch_beta_forward_shifted<double>(otf_params<double>(plan, 0), (const cpx<double>*)plan->d_S,
                                            (cpx<double>*)d_coeffs, depth, block, stream);
  else
    e = launch_beta_forward_shifted<float>(otf_params<float>(plan, 0), (const cpx<float>*)plan->d_S,
                                           (cpx<float>*)d_coeffs, depth, block, stream);
  return e == hipSuccess ? SU2_OK : hip_fail(e);
}

int64_t su2_so3_num_coeffs(int32_t B) {
  if (B < 1) return -1;
  const int64_t L = (B - 1) / 2 + 1;  // integer degrees 0 .. L-1
  return L * (2 * L - 1) * (2 * L + 1) / 3;
}

int64_t su2_so3_coeff_index(int32_t l, int32_t m, int32_t n) {
  if (l < 0 || m < -l || m > l || n < -l || n > l) return -1;
  return coef_index_of(1, 2 * l, 2 * m, 2 * n);
}

const char* su2_status_string(su2_status_t status) {
  switch (status) {
    case SU2_OK: return "SU2_OK";
    case SU2_ERR_INVALID_VALUE: return "SU2_ERR_INVALID_VALUE: invalid argument";
    case SU2_ERR_UNSUPPORTED: return "SU2_ERR_UNSUPPORTED: unsupported bandlimit or mode";
    case SU2_ERR_OUT_OF_MEMORY: return "SU2_ERR_OUT_OF_MEMORY: device allocation failed";
    case SU2_ERR_HIP: return "SU2_ERR_HIP: HIP runtime error";
    case SU2_ERR_NO_DEVICE: return "SU2_ERR_NO_DEVICE: no usable GPU";
  }
  return "unknown status";
}

int32_t su2_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"
