/*
 * Reference oracle for the Fourier transform on SU(2) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP library under
 * paper_2605_23923_amd/) never calls, links or imports anything here, and this
 * file shares no code, table or constant generator with it.
 *
 * What it computes, in plain double precision, term by term:
 *
 *   forward  (Definition 3.4, discretised as in Theorem 5.1):
 *       fhat(l)_{mn} = sum_{k,j,l'} W_k f(alpha_j, beta_k, gamma_l')
 *                      * conj( t^l_{nm}(alpha_j, beta_k, gamma_l') )
 *   inverse  (the Peter-Weyl series of Section 3):
 *       f(alpha_j, beta_k, gamma_l') = sum_{2l<B} (2l+1) sum_{m,n} fhat(l)_{mn} t^l_{nm}(...)
 *   adjoint  (conjugate transpose of the forward map):
 *       (F^H c)(alpha_j, beta_k, gamma_l') = W_k sum_{l,m,n} c_{lmn} t^l_{nm}(...)
 *
 * with the basis of Section 3 (the index-swapped form, Euler angles)
 *       t^l_{nm}(alpha, beta, gamma) = P^l_{nm}(cos beta) exp(-i (n alpha + m gamma)),
 *       P^l_{nm}(cos beta) = i^{m-n} d^l_{nm}(beta),
 * d being Wigner's small-d function.  The phase relation between the paper's
 * Rodrigues-type P^l_{mn} and Wigner's d is a reading that the tests pin
 * against the paper's own formulas (Theorem 3.2 and the Euler-angle form).
 *
 * d is evaluated through the Jacobi-polynomial form (the route the paper
 * points to at the end of Section 4): sin^a(b/2) cos^b(b/2) P^{(a,b)}_s(cos b)
 * times a factorial normalisation, with P^{(a,b)}_s from its three-term
 * degree recurrence and the normalisation through lgamma.  No l-recurrence of
 * normalised d values is used here.
 *
 * Grid (Definition 4.1, read so that the quadrature is exact; every reading
 * is listed with its reason in the design notes):
 *   N = 2B nodes per angle,
 *   alpha_j = -pi + 2 pi j / N            (periodic nodes, duplicate endpoint dropped),
 *   beta_k  = pi k / (N - 1)              (the paper's theta nodes, k = 0..N-1),
 *   gamma_l = -2 pi + 4 pi l / N          (psi over [-2pi, 2pi): SU(2), not SO(3)),
 *   W_k     = w_k / (2 N^2),  w_k the Clenshaw-Curtis weights on x_k = cos beta_k
 *             (replacing the paper's sin(theta_k) Riemann weights).
 *
 * Layouts (shared with the C-ABI by contract, not by code):
 *   samples      [k][j][l]  complex (interleaved re, im), N^3 values;
 *   coefficients ell-major: the block for 2l = tl starts at tl(tl+1)(2tl+1)/6,
 *                row-major over m = -l..l (rows), n = -l..l (columns).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (no -ffast-math: IEEE semantics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct { double re, im; } cplx;

static cplx c_mul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static cplx c_conj(cplx a) { cplx r = {a.re, -a.im}; return r; }
static cplx c_scale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }

/* i^k for integer k */
static cplx i_pow(int k) {
  int r = ((k % 4) + 4) % 4;
  cplx v[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  return v[r];
}

int64_t orc_num_coeffs(int B) { return (int64_t)B * (B + 1) * (2 * B + 1) / 6; }

int64_t orc_block_offset(int tl) { return (int64_t)tl * (tl + 1) * (2 * tl + 1) / 6; }

/* flat index of fhat(l)_{mn} from doubled indices; -1 if the triple is not valid */
int64_t orc_coeff_index(int tl, int tm, int tn) {
  if (tl < 0 || tm < -tl || tm > tl || tn < -tl || tn > tl) return -1;
  if (((tl - tm) & 1) || ((tl - tn) & 1)) return -1;
  int dim = tl + 1;
  return orc_block_offset(tl) + (int64_t)((tm + tl) / 2) * dim + (tn + tl) / 2;
}

/* inverse of orc_coeff_index */
void orc_coeff_triple(int64_t idx, int* tl, int* tm, int* tn) {
  int t = 0;
  while (orc_block_offset(t + 1) <= idx) t++;
  int64_t r = idx - orc_block_offset(t);
  int dim = t + 1;
  *tl = t;
  *tm = 2 * (int)(r / dim) - t;
  *tn = 2 * (int)(r % dim) - t;
}

/* Clenshaw-Curtis weight w_k on the n+1 nodes x_k = cos(k pi / n), exact for
 * polynomials of degree <= n on [-1, 1] (Clenshaw & Curtis 1960, in the
 * cosine-sum form).  n = 0 (a single node) is not used: B >= 1 gives n >= 1. */
double orc_cc_weight(int n, int k) {
  double ck = (k == 0 || k == n) ? 1.0 : 2.0;
  double s = 0.0;
  for (int j = 1; j <= n / 2; j++) {
    double bj = (2 * j == n) ? 1.0 : 2.0;
    s += bj / (4.0 * j * j - 1.0) * cos(2.0 * j * k * M_PI / n);
  }
  return ck / n * (1.0 - s);
}

void orc_grid(int B, double* alpha, double* beta, double* gamma, double* W) {
  int N = 2 * B;
  for (int i = 0; i < N; i++) {
    if (alpha) alpha[i] = -M_PI + 2.0 * M_PI * i / N;
    if (beta) beta[i] = M_PI * i / (N - 1);
    if (gamma) gamma[i] = -2.0 * M_PI + 4.0 * M_PI * i / N;
    if (W) W[i] = orc_cc_weight(N - 1, i) / (2.0 * (double)N * (double)N);
  }
}

/* Jacobi polynomial P^{(a,b)}_s(x) by its degree recurrence (DLMF 18.9.1):
 *   2n(n+a+b)(2n+a+b-2) P_n = (2n+a+b-1)[(2n+a+b)(2n+a+b-2) x + a^2 - b^2] P_{n-1}
 *                             - 2(n+a-1)(n+b-1)(2n+a+b) P_{n-2},
 *   P_0 = 1,  P_1 = (a+1) + (a+b+2)(x-1)/2. */
double orc_jacobi(int s, int a, int b, double x) {
  if (s == 0) return 1.0;
  double p0 = 1.0;
  double p1 = (a + 1) + 0.5 * (a + b + 2) * (x - 1.0);
  for (int n = 2; n <= s; n++) {
    double c = 2.0 * n + a + b;
    double lhs = 2.0 * n * (n + a + b) * (c - 2.0);
    double p2 = ((c - 1.0) * (c * (c - 2.0) * x + (double)a * a - (double)b * b) * p1 -
                 2.0 * (n + a - 1.0) * (n + b - 1.0) * c * p0) / lhs;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

/* log of the binomial coefficient C(n, k) */
static double log_binom(int n, int k) { return lgamma(n + 1.0) - lgamma(k + 1.0) - lgamma(n - k + 1.0); }

/* Wigner small-d  d^j_{m' m}(beta), arguments doubled: tl = 2j, ta = 2m', tb = 2m.
 * Jacobi form: with kk = min(j+m, j-m, j+m', j-m'),
 *   kk = j+m  -> a = m'-m, lambda = m'-m;   kk = j-m  -> a = m-m', lambda = 0;
 *   kk = j+m' -> a = m-m', lambda = 0;      kk = j-m' -> a = m'-m, lambda = m'-m;
 *   b = 2j - 2kk - a,
 *   d = (-1)^lambda sqrt( C(2j-kk, kk+a) / C(kk+b, b) ) sin^a(beta/2) cos^b(beta/2) P^{(a,b)}_kk(cos beta).
 * Returns 0 for an invalid triple. */
double orc_wigner_d(int tl, int ta, int tb, double beta) {
  if (tl < 0 || ta < -tl || ta > tl || tb < -tl || tb > tl) return 0.0;
  if (((tl - ta) & 1) || ((tl - tb) & 1)) return 0.0;
  /* all quantities below are integers: j+m etc. */
  int jpm = (tl + tb) / 2, jmm = (tl - tb) / 2, jpmp = (tl + ta) / 2, jmmp = (tl - ta) / 2;
  int kk = jpm, a, lam;
  int mp_minus_m = (ta - tb) / 2;
  if (kk <= jmm && kk <= jpmp && kk <= jmmp) { a = mp_minus_m; lam = mp_minus_m; }
  else if (jmm <= jpmp && jmm <= jmmp) { kk = jmm; a = -mp_minus_m; lam = 0; }
  else if (jpmp <= jmmp) { kk = jpmp; a = -mp_minus_m; lam = 0; }
  else { kk = jmmp; a = mp_minus_m; lam = mp_minus_m; }
  int b = tl - 2 * kk - a;
  double lognorm = 0.5 * (log_binom(tl - kk, kk + a) - log_binom(kk + b, b));
  double sh = sin(0.5 * beta), ch = cos(0.5 * beta);
  double pa = (a == 0) ? 1.0 : pow(sh, a);
  double pb = (b == 0) ? 1.0 : pow(ch, b);
  double sign = (lam & 1) ? -1.0 : 1.0;
  return sign * exp(lognorm) * pa * pb * orc_jacobi(kk, a, b, cos(beta));
}

/* d^l_{ab}(beta) for n independent argument tuples (doubled indices), in
 * parallel; used to fill the tables of the CPU FFT-based baseline. */
void orc_wigner_d_many(int64_t n, const int* tl, const int* ta, const int* tb, const double* beta, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) out[i] = orc_wigner_d(tl[i], ta[i], tb[i], beta[i]);
}

/* P^l_{nm}(cos beta) = i^{m-n} d^l_{nm}(beta) (doubled indices) */
static cplx basis_P(int tl, int tm, int tn, double beta) {
  return c_scale(i_pow((tm - tn) / 2), orc_wigner_d(tl, tn, tm, beta));
}

/* Exported view of the basis used by the sums below: P^l_{nm}(cos beta) as
 * (re, im), doubled indices (tl, tm, tn). */
void orc_basis(int tl, int tm, int tn, double beta, double* re_im) {
  cplx p = basis_P(tl, tm, tn, beta);
  re_im[0] = p.re;
  re_im[1] = p.im;
}

/* Forward transform: selected coefficients (flat indices sel[0..nsel-1], or all
 * C(B) when sel is NULL) of the samples f ([k][j][l], interleaved complex).
 * out holds one complex value per selected coefficient. */
void orc_forward(int B, const double* f, int64_t nsel, const int64_t* sel, double* out) {
  int N = 2 * B;
  double* alpha = (double*)malloc(sizeof(double) * N);
  double* beta = (double*)malloc(sizeof(double) * N);
  double* gamma = (double*)malloc(sizeof(double) * N);
  double* W = (double*)malloc(sizeof(double) * N);
  orc_grid(B, alpha, beta, gamma, W);
  int64_t count = sel ? nsel : orc_num_coeffs(B);
  const cplx* fs = (const cplx*)f;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < count; s++) {
    int tl, tm, tn;
    orc_coeff_triple(sel ? sel[s] : s, &tl, &tm, &tn);
    cplx* Ea = (cplx*)malloc(sizeof(cplx) * N);
    cplx* Eg = (cplx*)malloc(sizeof(cplx) * N);
    cplx* Pk = (cplx*)malloc(sizeof(cplx) * N);
    for (int i = 0; i < N; i++) {
      /* exp(-i n alpha_j) and exp(-i m gamma_l) with n = tn/2, m = tm/2 */
      double pa = -0.5 * tn * alpha[i], pg = -0.5 * tm * gamma[i];
      Ea[i].re = cos(pa); Ea[i].im = sin(pa);
      Eg[i].re = cos(pg); Eg[i].im = sin(pg);
      Pk[i] = basis_P(tl, tm, tn, beta[i]);
    }
    cplx acc = {0.0, 0.0};
    for (int k = 0; k < N; k++)
      for (int j = 0; j < N; j++)
        for (int l = 0; l < N; l++) {
          cplx t = c_mul(c_mul(Pk[k], Ea[j]), Eg[l]);         /* t^l_{nm}(alpha_j, beta_k, gamma_l) */
          cplx term = c_scale(c_mul(fs[((int64_t)k * N + j) * N + l], c_conj(t)), W[k]);
          acc.re += term.re;
          acc.im += term.im;
        }
    out[2 * s] = acc.re;
    out[2 * s + 1] = acc.im;
    free(Ea); free(Eg); free(Pk);
  }
  free(alpha); free(beta); free(gamma); free(W);
}

/* Synthesis at selected sample points (flat index (k*N + j)*N + l, or all N^3
 * when sel is NULL).  mode 0: inverse, weight (2l+1) per term;
 * mode 1: adjoint, weight W_k per term. */
void orc_synth(int B, const double* c, int mode, int64_t nsel, const int64_t* sel, double* out) {
  int N = 2 * B;
  int64_t C = orc_num_coeffs(B);
  double* alpha = (double*)malloc(sizeof(double) * N);
  double* beta = (double*)malloc(sizeof(double) * N);
  double* gamma = (double*)malloc(sizeof(double) * N);
  double* W = (double*)malloc(sizeof(double) * N);
  orc_grid(B, alpha, beta, gamma, W);
  int64_t count = sel ? nsel : (int64_t)N * N * N;
  const cplx* cs = (const cplx*)c;
  /* basis values P^l_{nm}(cos beta_k) for every coefficient, at each ring k
   * that a selected point lies on (the cost model treats basis values as
   * precomputed lookups). */
  char* need = (char*)calloc(N, 1);
  for (int64_t s = 0; s < count; s++) need[(sel ? sel[s] : s) / ((int64_t)N * N)] = 1;
  cplx** Ptab = (cplx**)calloc(N, sizeof(cplx*));
  for (int k = 0; k < N; k++) {
    if (!need[k]) continue;
    Ptab[k] = (cplx*)malloc(sizeof(cplx) * C);
  }
#pragma omp parallel for schedule(dynamic, 64) collapse(2)
  for (int k = 0; k < N; k++)
    for (int64_t q = 0; q < C; q++) {
      if (!need[k]) continue;
      int tl, tm, tn;
      orc_coeff_triple(q, &tl, &tm, &tn);
      Ptab[k][q] = basis_P(tl, tm, tn, beta[k]);
    }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < count; s++) {
    int64_t pt = sel ? sel[s] : s;
    int k = (int)(pt / ((int64_t)N * N));
    int j = (int)((pt / N) % N);
    int l = (int)(pt % N);
    /* exp(-i n alpha_j) and exp(-i m gamma_l) for every doubled index 2n, 2m
     * in [-(B-1), B-1] (per-axis tables at this point) */
    cplx* Ea = (cplx*)malloc(sizeof(cplx) * (2 * B - 1));
    cplx* Eg = (cplx*)malloc(sizeof(cplx) * (2 * B - 1));
    for (int t2 = -(B - 1); t2 <= B - 1; t2++) {
      double pa = -0.5 * t2 * alpha[j], pg = -0.5 * t2 * gamma[l];
      Ea[t2 + B - 1].re = cos(pa); Ea[t2 + B - 1].im = sin(pa);
      Eg[t2 + B - 1].re = cos(pg); Eg[t2 + B - 1].im = sin(pg);
    }
    cplx acc = {0.0, 0.0};
    for (int64_t q = 0; q < C; q++) {
      int tl, tm, tn;
      orc_coeff_triple(q, &tl, &tm, &tn);
      cplx t = c_mul(c_mul(Ptab[k][q], Ea[tn + B - 1]), Eg[tm + B - 1]);  /* t^l_{nm} at the point */
      double wgt = (mode == 0) ? (double)(tl + 1) : W[k];
      cplx term = c_scale(c_mul(cs[q], t), wgt);
      acc.re += term.re;
      acc.im += term.im;
    }
    out[2 * s] = acc.re;
    out[2 * s + 1] = acc.im;
    free(Ea); free(Eg);
  }
  for (int k = 0; k < N; k++) free(Ptab[k]);
  free(Ptab); free(need);
  free(alpha); free(beta); free(gamma); free(W);
}

/* Number of OpenMP threads the oracle runs with (0 when built without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 0;
#endif
}

/* Set the number of OpenMP threads of later calls (n >= 1; ignored without
 * OpenMP).  Timing only: results do not depend on it. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
