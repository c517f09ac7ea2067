/*
 * oracle.c -- plain, slow, FP64 CPU reference for the exact magic of pure state vectors.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (little-endian): a qubit state psi has 2^n complex amplitudes, basis index
 * x = sum_k x_k 2^k; a qutrit state has 3^n amplitudes, x = sum_k x_k 3^k.  Complex arrays are
 * interleaved (re, im) doubles.  Every sum is Neumaier-compensated and per-thread partial sums
 * are merged in thread order, so results are deterministic for a fixed thread count.
 *
 * Two independent families:
 *   A. "direct": every Pauli string / phase-space point operator is built from its definition
 *      and its expectation value evaluated on psi (the work of the naive Algorithms 1 and 3,
 *      without the Gray-code ordering).  O(8^n) / O(n 27^n).
 *   B. "fast": Algorithm 2 (one Walsh-Hadamard transform per X-shift) and Algorithm 4 (one
 *      Z_3^n Fourier transform per shift), written plainly.  O(n 4^n) / O(n 9^n).
 *
 * Readings of the paper used here (the paper is silent or inconsistent on these points):
 *   R1  Algorithm 2 accumulates chi_b^{2q}; chi_b = <psi|X_a Z_b|psi> is imaginary when a.b is
 *       odd, so the sum is taken over |chi_b|^{2q} = <P>^{2q} with P the Hermitian Pauli string.
 *   R2  M_1 is the q->1 limit of Eq. (sre): M_1 = -2^{-n} sum_P <P>^2 log2 <P>^2 (0 log 0 = 0).
 *   R3  Algorithms 3 and 4 return log2(m); Eq. (mana2) divides by 3^n.  Mana = log2(m / 3^n).
 *   R4  The gradient is returned in the torch convention g = dM/dRe(psi) + i dM/dIm(psi).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

#define OR_OK 0
#define OR_EARG 1
#define OR_ENOMEM 2
#define OR_ENOTMONOMIAL 3

/* ------------------------------------------------------------------------------------------ */
/* compensated summation                                                                       */
/* ------------------------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;

static inline void ks_add(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static inline double ks_val(const ksum *k) { return k->s + k->c; }

static int n_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
static int thread_id(void) {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
int oracle_get_threads(void) { return n_threads(); }

/* Sums kept per Renyi index: slot 0 = sum <P>^2 (normalisation, lost_norm); slot 1+i = sum <P>^{2 q_i}
 * (or, for q_i == 1, sum <P>^2 log2 <P>^2).  MAXQ bounds the number of indices. */
#define MAXQ 8

static inline void add_term(ksum *acc, double e2, const double *q, int nq) {
  ks_add(&acc[0], e2);
  for (int i = 0; i < nq; i++) {
    if (q[i] == 1.0) ks_add(&acc[1 + i], e2 > 0.0 ? e2 * log2(e2) : 0.0);
    else ks_add(&acc[1 + i], pow(e2, q[i]));
  }
}

static int check_q(const double *q, int nq) {
  if (nq < 1 || nq > MAXQ || !q) return 0;
  for (int i = 0; i < nq; i++)
    if (!(q[i] > 0.0) || isnan(q[i]) || isinf(q[i])) return 0;
  return 1;
}

/* Eq. (sre): M_q = log2(S_q / 2^n) / (1 - q); R2 for q == 1; lost_norm = 1 - S_1 / 2^n. */
void oracle_sre_finalize(int n, const double *q, int nq, const double *sums, double *out) {
  double D = ldexp(1.0, n);
  for (int i = 0; i < nq; i++) {
    if (q[i] == 1.0) out[i] = -sums[1 + i] / D;
    else out[i] = log2(sums[1 + i] / D) / (1.0 - q[i]);
  }
  out[nq] = 1.0 - sums[0] / D;
}

/* ------------------------------------------------------------------------------------------ */
/* A. direct Pauli strings (Sec. 2, Eq. (sre); the work of Algorithm 1)                        */
/* ------------------------------------------------------------------------------------------ */
/* Pauli string s in base 4: digit k in {0:I, 1:X, 2:Y, 3:Z} acts on qubit k.  With
 * X|x> = |1-x>, Y|x> = i(-1)^x |1-x>, Z|x> = (-1)^x |x>, the string maps |x> to
 * i^{nY} (-1)^{popcount(x & (Ymask|Zmask))} |x ^ (Xmask|Ymask)>. */
typedef struct { uint64_t flip, signmask; int ny; } pauli_t;

static pauli_t pauli_from_digits(uint64_t s, int n) {
  pauli_t p = {0, 0, 0};
  for (int k = 0; k < n; k++) {
    int dgt = (int)((s >> (2 * k)) & 3u);
    if (dgt == 1) p.flip |= 1ull << k;
    else if (dgt == 2) { p.flip |= 1ull << k; p.signmask |= 1ull << k; p.ny++; }
    else if (dgt == 3) p.signmask |= 1ull << k;
  }
  return p;
}

/* <psi|P|psi> = sum_x conj(psi[x ^ flip]) * phase(x) * psi[x]; returns re and im separately. */
static void pauli_expect(const cplx *psi, uint64_t D, pauli_t p, double *re, double *im) {
  ksum sr = {0, 0}, si = {0, 0};
  for (uint64_t x = 0; x < D; x++) {
    cplx t = conj(psi[x ^ p.flip]) * psi[x];
    if (__builtin_popcountll(x & p.signmask) & 1) t = -t;
    ks_add(&sr, creal(t));
    ks_add(&si, cimag(t));
  }
  cplx e = ks_val(&sr) + I * ks_val(&si);
  static const cplx ipow[4] = {1.0, I, -1.0, -I};
  e *= ipow[p.ny & 3];
  *re = creal(e);
  *im = cimag(e);
}

/* Raw sums over all 4^n Pauli strings (slot layout as add_term).  Also reports max |Im <P>|. */
int oracle_sre_direct_sums(const double *psi_in, int n, const double *q, int nq, double *sums,
                           double *max_imag) {
  if (n < 1 || n > 14 || !psi_in || !sums || !check_q(q, nq)) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = 1ull << n, NP = 1ull << (2 * n);
  int T = n_threads();
  ksum *part = calloc((size_t)T * (MAXQ + 1), sizeof(ksum));
  double *pim = calloc((size_t)T, sizeof(double));
  if (!part || !pim) { free(part); free(pim); return OR_ENOMEM; }
#pragma omp parallel
  {
    int t = thread_id();
    ksum *acc = part + (size_t)t * (MAXQ + 1);
#pragma omp for schedule(static)
    for (int64_t s = 0; s < (int64_t)NP; s++) {
      double re, im;
      pauli_expect(psi, D, pauli_from_digits((uint64_t)s, n), &re, &im);
      if (fabs(im) > pim[t]) pim[t] = fabs(im);
      add_term(acc, re * re, q, nq);
    }
  }
  for (int k = 0; k <= nq; k++) {
    ksum tot = {0, 0};
    for (int t = 0; t < T; t++) ks_add(&tot, ks_val(&part[(size_t)t * (MAXQ + 1) + k]));
    sums[k] = ks_val(&tot);
  }
  if (max_imag) {
    double m = 0;
    for (int t = 0; t < T; t++) m = pim[t] > m ? pim[t] : m;
    *max_imag = m;
  }
  free(part);
  free(pim);
  return OR_OK;
}

int oracle_sre_direct(const double *psi, int n, const double *q, int nq, double *out) {
  double sums[MAXQ + 1];
  int st = oracle_sre_direct_sums(psi, n, q, nq, sums, NULL);
  if (st) return st;
  oracle_sre_finalize(n, q, nq, sums, out);
  return OR_OK;
}

/* <P_{a,b}> for the Hermitian Pauli string whose X-part is a and Z-part is b (per qubit
 * (a_k,b_k) = (0,0) I, (1,0) X, (0,1) Z, (1,1) Y), for every b of one X-row a. */
int oracle_sre_row_values_direct(const double *psi_in, int n, uint64_t a, double *out) {
  if (n < 1 || n > 20 || !psi_in || !out) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = 1ull << n;
  if (a >= D) return OR_EARG;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < (int64_t)D; b++) {
    uint64_t s = 0;
    for (int k = 0; k < n; k++) {
      int ak = (int)((a >> k) & 1), bk = (int)(((uint64_t)b >> k) & 1);
      uint64_t dgt = ak ? (bk ? 2 : 1) : (bk ? 3 : 0);
      s |= dgt << (2 * k);
    }
    double re, im;
    pauli_expect(psi, D, pauli_from_digits(s, n), &re, &im);
    out[b] = re;
  }
  return OR_OK;
}

/* Direct gradient: dS_q/dpsi*_y = sum_P 2q <P>^{2q-1} (P psi)_y and, by Eq. (sre),
 * g = 2 dM_q/dpsi* = 2 dS_q/dpsi* / ((1-q) S_q ln 2)  (R4).  q != 1. */
int oracle_sre_grad_direct(const double *psi_in, int n, double q, double *out, double *grad) {
  if (n < 1 || n > 12 || !psi_in || !out || !grad || !(q > 0) || q == 1.0) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = 1ull << n, NP = 1ull << (2 * n);
  int T = n_threads();
  cplx *G = calloc((size_t)T * D, sizeof(cplx));
  ksum *part = calloc((size_t)T * 2, sizeof(ksum));
  if (!G || !part) { free(G); free(part); return OR_ENOMEM; }
  static const cplx ipow[4] = {1.0, I, -1.0, -I};
#pragma omp parallel
  {
    int t = thread_id();
    cplx *g = G + (size_t)t * D;
#pragma omp for schedule(static)
    for (int64_t s = 0; s < (int64_t)NP; s++) {
      pauli_t p = pauli_from_digits((uint64_t)s, n);
      double re, im;
      pauli_expect(psi, D, p, &re, &im);
      ks_add(&part[2 * t], re * re);
      ks_add(&part[2 * t + 1], pow(re * re, q));
      double w = 2.0 * q * pow(fabs(re), 2.0 * q - 1.0) * (re < 0 ? -1.0 : 1.0);
      if (w == 0.0) continue;
      /* (P psi)_y: P|x> = phase(x)|x^flip>, so (P psi)_{x^flip} = phase(x) psi_x */
      for (uint64_t x = 0; x < D; x++) {
        cplx v = ipow[p.ny & 3] * psi[x];
        if (__builtin_popcountll(x & p.signmask) & 1) v = -v;
        g[x ^ p.flip] += w * v;
      }
    }
  }
  ksum s1 = {0, 0}, sq = {0, 0};
  for (int t = 0; t < T; t++) { ks_add(&s1, ks_val(&part[2 * t])); ks_add(&sq, ks_val(&part[2 * t + 1])); }
  double S1 = ks_val(&s1), Sq = ks_val(&sq), Dd = (double)D;
  out[0] = log2(Sq / Dd) / (1.0 - q);
  out[1] = 1.0 - S1 / Dd;
  double scale = 2.0 / ((1.0 - q) * Sq * log(2.0));
  cplx *gout = (cplx *)grad;
  for (uint64_t y = 0; y < D; y++) {
    cplx acc = 0;
    for (int t = 0; t < T; t++) acc += G[(size_t)t * D + y];
    gout[y] = scale * acc;
  }
  free(G);
  free(part);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* B. Algorithm 2: one Walsh-Hadamard transform per X-shift (Eqs. Z_FT_qubits, Z_ovN)         */
/* ------------------------------------------------------------------------------------------ */
/* In-place unnormalised H_2^{(x)n}, H_2 = [[1,1],[1,-1]] (Fino-Algazi butterflies). */
static void fwht(cplx *v, uint64_t D) {
  for (uint64_t h = 1; h < D; h <<= 1)
    for (uint64_t i = 0; i < D; i += 2 * h)
      for (uint64_t j = i; j < i + h; j++) {
        cplx u = v[j], w = v[j + h];
        v[j] = u + w;
        v[j + h] = u - w;
      }
}

/* chi_b(a) = sum_x beta_x^* alpha_x (-1)^{b.x} with alpha = psi, beta = X_a psi (beta_x = psi_{x^a}). */
static void row_transform(const cplx *psi, uint64_t D, uint64_t a, cplx *v) {
  for (uint64_t x = 0; x < D; x++) v[x] = conj(psi[x ^ a]) * psi[x];
  fwht(v, D);
}

static void row_sums(const cplx *psi, uint64_t D, uint64_t a, const double *q, int nq, cplx *v,
                     ksum *acc) {
  row_transform(psi, D, a, v);
  for (uint64_t b = 0; b < D; b++) {
    double e2 = creal(v[b]) * creal(v[b]) + cimag(v[b]) * cimag(v[b]); /* R1: |chi_b|^2 */
    add_term(acc, e2, q, nq);
  }
}

/* Raw sums over shifts a in [a0, a1) (slot layout as add_term). */
int oracle_sre_fwht_sums(const double *psi_in, int n, const double *q, int nq, uint64_t a0,
                         uint64_t a1, double *sums) {
  if (n < 1 || n > 30 || !psi_in || !sums || !check_q(q, nq)) return OR_EARG;
  uint64_t D = 1ull << n;
  if (a0 > a1 || a1 > D) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  int T = n_threads();
  ksum *part = calloc((size_t)T * (MAXQ + 1), sizeof(ksum));
  if (!part) return OR_ENOMEM;
  int fail = 0;
#pragma omp parallel
  {
    int t = thread_id();
    cplx *v = malloc(D * sizeof(cplx));
    if (!v) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp barrier
    if (!fail) {
      ksum *acc = part + (size_t)t * (MAXQ + 1);
#pragma omp for schedule(static)
      for (int64_t a = (int64_t)a0; a < (int64_t)a1; a++) row_sums(psi, D, (uint64_t)a, q, nq, v, acc);
    }
    free(v);
  }
  if (fail) { free(part); return OR_ENOMEM; }
  for (int k = 0; k <= nq; k++) {
    ksum tot = {0, 0};
    for (int t = 0; t < T; t++) ks_add(&tot, ks_val(&part[(size_t)t * (MAXQ + 1) + k]));
    sums[k] = ks_val(&tot);
  }
  free(part);
  return OR_OK;
}

int oracle_sre_fwht(const double *psi, int n, const double *q, int nq, double *out) {
  double sums[MAXQ + 1];
  int st = oracle_sre_fwht_sums(psi, n, q, nq, 0, 1ull << n, sums);
  if (st) return st;
  oracle_sre_finalize(n, q, nq, sums, out);
  return OR_OK;
}

/* Per-row sums for an explicit list of X-strings: row_sums[r*(nq+1) + slot]. */
int oracle_sre_fwht_rows(const double *psi_in, int n, const uint64_t *rows, int64_t n_rows,
                         const double *q, int nq, double *out) {
  if (n < 1 || n > 30 || !psi_in || !out || (n_rows > 0 && !rows) || n_rows < 0 || !check_q(q, nq))
    return OR_EARG;
  uint64_t D = 1ull << n;
  for (int64_t r = 0; r < n_rows; r++)
    if (rows[r] >= D) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  int fail = 0;
#pragma omp parallel
  {
    cplx *v = malloc(D * sizeof(cplx));
    if (!v) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp barrier
    if (!fail) {
#pragma omp for schedule(dynamic, 1)
      for (int64_t r = 0; r < n_rows; r++) {
        ksum acc[MAXQ + 1];
        memset(acc, 0, sizeof(acc));
        row_sums(psi, D, rows[r], q, nq, v, acc);
        for (int k = 0; k <= nq; k++) out[r * (nq + 1) + k] = ks_val(&acc[k]);
      }
    }
    free(v);
  }
  return fail ? OR_ENOMEM : OR_OK;
}

/* Signed real <P_{a,b}> of one X-row from the fast form: <P_{a,b}> = i^{popcount(a&b)} chi_b. */
int oracle_sre_row_values_fwht(const double *psi_in, int n, uint64_t a, double *out, double *max_imag) {
  if (n < 1 || n > 30 || !psi_in || !out) return OR_EARG;
  uint64_t D = 1ull << n;
  if (a >= D) return OR_EARG;
  cplx *v = malloc(D * sizeof(cplx));
  if (!v) return OR_ENOMEM;
  row_transform((const cplx *)psi_in, D, a, v);
  static const cplx ipow[4] = {1.0, I, -1.0, -I};
  double mi = 0;
  for (uint64_t b = 0; b < D; b++) {
    cplx e = ipow[__builtin_popcountll(a & b) & 3] * v[b];
    out[b] = creal(e);
    if (fabs(cimag(e)) > mi) mi = fabs(cimag(e));
  }
  if (max_imag) *max_imag = mi;
  free(v);
  return OR_OK;
}

/* Gradient from the fast form.  Differentiating chi_b(a) = sum_x conj(psi_{x^a}) psi_x (-1)^{b.x}
 * and using that chi_b(a) is real for even a.b and imaginary for odd a.b gives
 * dS_q/dpsi*_y = sum_a psi_{y^a} * 2q * [H^{(x)n} w_a]_y with w_a[b] = |chi_b|^{2q-2} chi_b. */
int oracle_sre_grad_fwht(const double *psi_in, int n, double q, double *out, double *grad) {
  if (n < 1 || n > 24 || !psi_in || !out || !grad || !(q > 0) || q == 1.0) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = 1ull << n;
  int T = n_threads();
  cplx *G = calloc((size_t)T * D, sizeof(cplx));
  ksum *part = calloc((size_t)T * 2, sizeof(ksum));
  if (!G || !part) { free(G); free(part); return OR_ENOMEM; }
  int fail = 0;
#pragma omp parallel
  {
    int t = thread_id();
    cplx *v = malloc(D * sizeof(cplx));
    if (!v) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp barrier
    if (!fail) {
      cplx *g = G + (size_t)t * D;
#pragma omp for schedule(static)
      for (int64_t a = 0; a < (int64_t)D; a++) {
        row_transform(psi, D, (uint64_t)a, v);
        for (uint64_t b = 0; b < D; b++) {
          double e2 = creal(v[b]) * creal(v[b]) + cimag(v[b]) * cimag(v[b]);
          ks_add(&part[2 * t], e2);
          ks_add(&part[2 * t + 1], pow(e2, q));
          v[b] = (e2 > 0 ? pow(e2, q - 1.0) : (q > 1 ? 0.0 : 0.0)) * v[b];
        }
        fwht(v, D);
        for (uint64_t y = 0; y < D; y++) g[y] += 2.0 * q * psi[y ^ (uint64_t)a] * v[y];
      }
    }
    free(v);
  }
  if (fail) { free(G); free(part); return OR_ENOMEM; }
  ksum s1 = {0, 0}, sq = {0, 0};
  for (int t = 0; t < T; t++) { ks_add(&s1, ks_val(&part[2 * t])); ks_add(&sq, ks_val(&part[2 * t + 1])); }
  double S1 = ks_val(&s1), Sq = ks_val(&sq), Dd = (double)D;
  out[0] = log2(Sq / Dd) / (1.0 - q);
  out[1] = 1.0 - S1 / Dd;
  double scale = 2.0 / ((1.0 - q) * Sq * log(2.0));
  cplx *gout = (cplx *)grad;
  for (uint64_t y = 0; y < D; y++) {
    cplx acc = 0;
    for (int t = 0; t < T; t++) acc += G[(size_t)t * D + y];
    gout[y] = scale * acc;
  }
  free(G);
  free(part);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Qutrits                                                                                     */
/* ------------------------------------------------------------------------------------------ */
static uint64_t pow3(int n) { uint64_t p = 1; while (n-- > 0) p *= 3; return p; }

/* Single-qutrit phase-space point operators from Eqs. (clock_and_shift), (pauli_qudit) and
 * (phase-space): omega = e^{2 pi i/3}, X|k> = |k+1>, Z|k> = omega^k |k>,
 * T_{ab} = omega^{-2^{-1} a b} Z^a X^b with 2^{-1} = 2 in Z_3,
 * A_0 = (1/3) sum_{a,b} T_{ab},  A_{(a,b)} = T_{ab} A_0 T_{ab}^dagger.
 * The N-qutrit operators are tensor products of these (A_0 factorises because T_u does).
 * Each single-qutrit A is checked to be monomial (one non-zero per column): A|x> = c_x |pi(x)>. */
typedef struct { int perm[9][3]; cplx coef[9][3]; } qutrit_ops_t;

static void mat3_mul(const cplx *A, const cplx *B, cplx *C) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      cplx s = 0;
      for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

static int build_qutrit_ops(qutrit_ops_t *ops) {
  const double tp = 2.0 * M_PI / 3.0;
  cplx w[3] = {1.0, cos(tp) + I * sin(tp), cos(2 * tp) + I * sin(2 * tp)};
  cplx X[9] = {0}, Z[9] = {0}, Id[9] = {0};
  for (int k = 0; k < 3; k++) {
    X[3 * ((k + 1) % 3) + k] = 1.0; /* X|k> = |k+1>: row k+1, column k */
    Z[3 * k + k] = w[k];
    Id[3 * k + k] = 1.0;
  }
  cplx Tm[9][9], A0[9] = {0};
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      cplx Za[9], Xb[9], t[9];
      memcpy(Za, Id, sizeof(Za));
      memcpy(Xb, Id, sizeof(Xb));
      for (int r = 0; r < a; r++) { mat3_mul(Za, Z, t); memcpy(Za, t, sizeof(t)); }
      for (int r = 0; r < b; r++) { mat3_mul(Xb, X, t); memcpy(Xb, t, sizeof(t)); }
      mat3_mul(Za, Xb, t);
      int e = (-2 * a * b) % 3; /* omega^{-2^{-1} a b}, 2^{-1} = 2 */
      e = ((e % 3) + 3) % 3;
      for (int i = 0; i < 9; i++) Tm[3 * a + b][i] = w[e] * t[i];
      for (int i = 0; i < 9; i++) A0[i] += Tm[3 * a + b][i] / 3.0;
    }
  for (int u = 0; u < 9; u++) {
    cplx Td[9], t[9], A[9];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) Td[3 * i + j] = conj(Tm[u][3 * j + i]);
    mat3_mul(Tm[u], A0, t);
    mat3_mul(t, Td, A);
    for (int col = 0; col < 3; col++) {
      int nz = 0;
      for (int row = 0; row < 3; row++) {
        if (cabs(A[3 * row + col]) > 1e-12) {
          nz++;
          ops->perm[u][col] = row;
          ops->coef[u][col] = A[3 * row + col];
        }
      }
      if (nz != 1) return OR_ENOTMONOMIAL;
    }
  }
  return OR_OK;
}

/* Direct mana: for every u in Z_3^{2n}, e_u = <psi|A_u|psi> with A_u = (x)_k A_{u_k};
 * out = {log2(sum_u |e_u| / 3^n) (R3), sum_u W_u, 3^n sum_u W_u^2} with W_u = e_u / 3^n. */
int oracle_mana_direct(const double *psi_in, int n, double *out) {
  if (n < 1 || n > 8 || !psi_in || !out) return OR_EARG;
  qutrit_ops_t ops;
  int st = build_qutrit_ops(&ops);
  if (st) return st;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = pow3(n), NU = D * D;
  int T = n_threads();
  ksum *part = calloc((size_t)T * 3, sizeof(ksum));
  if (!part) return OR_ENOMEM;
#pragma omp parallel
  {
    int t = thread_id();
    int *dig = malloc(sizeof(int) * (size_t)n);
    int uk[32];
#pragma omp for schedule(static)
    for (int64_t u = 0; u < (int64_t)NU; u++) {
      uint64_t uu = (uint64_t)u;
      for (int k = 0; k < n; k++) { uk[k] = (int)(uu % 9); uu /= 9; }
      ksum er = {0, 0};
      for (uint64_t x = 0; x < D; x++) {
        uint64_t xx = x, y = 0, p3 = 1;
        cplx c = 1.0;
        for (int k = 0; k < n; k++) {
          int xk = (int)(xx % 3);
          xx /= 3;
          dig[k] = xk;
          y += (uint64_t)ops.perm[uk[k]][xk] * p3;
          c *= ops.coef[uk[k]][xk];
          p3 *= 3;
        }
        ks_add(&er, creal(conj(psi[y]) * c * psi[x]));
      }
      double e = ks_val(&er);
      ks_add(&part[3 * t], fabs(e));
      ks_add(&part[3 * t + 1], e);
      ks_add(&part[3 * t + 2], e * e);
    }
    free(dig);
  }
  ksum m = {0, 0}, s = {0, 0}, s2 = {0, 0};
  for (int t = 0; t < T; t++) {
    ks_add(&m, ks_val(&part[3 * t]));
    ks_add(&s, ks_val(&part[3 * t + 1]));
    ks_add(&s2, ks_val(&part[3 * t + 2]));
  }
  double Dd = (double)D;
  out[0] = log2(ks_val(&m) / Dd);
  out[1] = ks_val(&s) / Dd;
  out[2] = ks_val(&s2) / Dd;
  free(part);
  return OR_OK;
}

/* In-place F_3^{(x)n} with (F_3)_{jk} = omega^{2jk} (Eq. F3_unnorm_def). */
static void fft3(cplx *v, uint64_t D, int n) {
  const double tp = 2.0 * M_PI / 3.0;
  cplx w1 = cos(tp) + I * sin(tp), w2 = cos(2 * tp) + I * sin(2 * tp);
  uint64_t h = 1;
  for (int k = 0; k < n; k++, h *= 3)
    for (uint64_t i = 0; i < D; i += 3 * h)
      for (uint64_t j = i; j < i + h; j++) {
        cplx x0 = v[j], x1 = v[j + h], x2 = v[j + 2 * h];
        v[j] = x0 + x1 + x2;           /* k = 0 */
        v[j + h] = x0 + w2 * x1 + w1 * x2;     /* k = 1: omega^{2j} */
        v[j + 2 * h] = x0 + w1 * x1 + w2 * x2; /* k = 2: omega^{4j} = omega^{j} */
      }
}

/* digit-wise (x + s*a) mod 3 with s in {+1,-1} and sign of x sx in {+1,-1} */
static uint64_t digitwise(uint64_t x, int sx, uint64_t a, int sa, int n) {
  uint64_t y = 0, p3 = 1;
  for (int k = 0; k < n; k++) {
    int xd = (int)(x % 3), ad = (int)(a % 3);
    x /= 3;
    a /= 3;
    int r = ((sx * xd + sa * ad) % 3 + 3) % 3;
    y += (uint64_t)r * p3;
    p3 *= 3;
  }
  return y;
}

/* Algorithm 4: for each a, alpha = X_a psi (alpha_x = psi_{x-a}), v_x = conj(alpha_x) alpha_{-x},
 * chi = F_3^{(x)n} v (Eq. mana_FT); m += sum_b |chi_b|.  Sums over shifts [a0, a1):
 * sums = {sum |chi|, sum chi, sum |chi|^2}. */
int oracle_mana_fft_sums(const double *psi_in, int n, uint64_t a0, uint64_t a1, double *sums) {
  if (n < 1 || n > 16 || !psi_in || !sums) return OR_EARG;
  const cplx *psi = (const cplx *)psi_in;
  uint64_t D = pow3(n);
  if (a0 > a1 || a1 > D) return OR_EARG;
  int T = n_threads();
  ksum *part = calloc((size_t)T * 3, sizeof(ksum));
  if (!part) return OR_ENOMEM;
  int fail = 0;
#pragma omp parallel
  {
    int t = thread_id();
    cplx *v = malloc(D * sizeof(cplx));
    if (!v) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp barrier
    if (!fail) {
#pragma omp for schedule(static)
      for (int64_t a = (int64_t)a0; a < (int64_t)a1; a++) {
        for (uint64_t x = 0; x < D; x++) {
          cplx ax = psi[digitwise(x, +1, (uint64_t)a, -1, n)];  /* alpha_x = psi_{x-a} */
          cplx amx = psi[digitwise(x, -1, (uint64_t)a, -1, n)]; /* alpha_{-x} = psi_{-x-a} */
          v[x] = conj(ax) * amx;
        }
        fft3(v, D, n);
        for (uint64_t b = 0; b < D; b++) {
          ks_add(&part[3 * t], cabs(v[b]));
          ks_add(&part[3 * t + 1], creal(v[b]));
          ks_add(&part[3 * t + 2], creal(v[b]) * creal(v[b]) + cimag(v[b]) * cimag(v[b]));
        }
      }
    }
    free(v);
  }
  if (fail) { free(part); return OR_ENOMEM; }
  for (int k = 0; k < 3; k++) {
    ksum tot = {0, 0};
    for (int t = 0; t < T; t++) ks_add(&tot, ks_val(&part[3 * t + k]));
    sums[k] = ks_val(&tot);
  }
  free(part);
  return OR_OK;
}

int oracle_mana_fft(const double *psi, int n, double *out) {
  double sums[3];
  int st = oracle_mana_fft_sums(psi, n, 0, pow3(n), sums);
  if (st) return st;
  double Dd = (double)pow3(n);
  out[0] = log2(sums[0] / Dd); /* R3 */
  out[1] = sums[1] / Dd;
  out[2] = sums[2] / Dd;
  return OR_OK;
}

/* Per-shift mana row sums {sum_b |chi_b|, sum_b chi_b, sum_b |chi_b|^2} for explicit shifts. */
int oracle_mana_fft_rows(const double *psi_in, int n, const uint64_t *rows, int64_t n_rows, double *out) {
  if (n < 1 || n > 16 || !psi_in || !out || n_rows < 0 || (n_rows > 0 && !rows)) return OR_EARG;
  for (int64_t r = 0; r < n_rows; r++) {
    double s[3];
    int st = oracle_mana_fft_sums(psi_in, n, rows[r], rows[r] + 1, s);
    if (st) return st;
    memcpy(out + 3 * r, s, sizeof(s));
  }
  return OR_OK;
}
