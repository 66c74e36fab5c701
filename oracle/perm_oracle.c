/*
 * CPU oracle for the matrix permanent -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library, and it includes nothing from it.
 *
 * Storage: column-major with leading dimension ld, a(i,j) = A[i + j*ld]
 * (0-based i, j).  Complex matrices are interleaved (re, im) pairs, so
 * a(i,j) = A[2*(i+j*ld)] + i*A[2*(i+j*ld)+1].  0/1 matrices are bytes.
 *
 * Four routes, each written from the paper (Lundow & Markstrom,
 * "Efficient computation of permanents, with applications to Boson sampling
 * and random matrices"):
 *
 *   O1 oracle_brute_*      The definition: sum over all n! permutations of
 *                          the product of one entry per row (Sec. I, Eq. per).
 *   O2 oracle_ryser_*      Ryser's inclusion-exclusion over all 2^n column
 *                          subsets J (Sec. II.A, Eq. ryser), the subsets
 *                          visited in Gray-code order (Sec. II.A), the terms
 *                          added with Kahan summation (App. A, Kahan) in
 *                          long double, partial sums of the threads stored in
 *                          an array and added afterwards in a fixed order
 *                          (Sec. II.B).
 *   O3 oracle_ryser_i128   O2 on integer matrices with exact arithmetic
 *                          modulo 2^128 (exact whenever |per| < 2^127).
 *   O4 oracle_chunk_*      The half-range partial sum of App. A
 *                          (subpermanent) over an explicit Gray-index range,
 *                          every term's row-sum vector formed directly from
 *                          the Gray code (App. A, Gray unranking), with no
 *                          walk, so there is no drift.  Sign convention as in
 *                          App. A: term g carries (-1)^(g+1), and
 *                          per(A) = 2 (-1)^n * (sum over all 2^(n-1) terms).
 *   O5 oracle_ryser2_*     Ryser's formula for a matrix whose columns repeat
 *                          (Sec. II.A, Eq. ryser2): distinct columns c_k with
 *                          multiplicities m_k, a sum over all vectors f with
 *                          0 <= f_k <= m_k of (-1)^(sum f) prod_k C(m_k, f_k)
 *                          prod_i sum_k f_k c_k(i), per = (-1)^n * sum.  The
 *                          whole sum runs over f in counting order; the range
 *                          form runs over f in reflected mixed-radix Gray
 *                          order (the paper fixes no order for Eq. ryser2),
 *                          every term formed directly from f.
 *   O7 oracle_sparse_*     The sparse form of Ryser's formula (App. B):
 *                          greedypartition picks rows of least degree with
 *                          pairwise disjoint column sets S_1..S_d; the sum of
 *                          Eq. ryser runs only over column sets J that meet
 *                          every S_l (a nonempty subset of each S_l times any
 *                          subset of the rest T), which drops only zero terms.
 *   O6 oracle_band_*       The band transfer matrix of App. C (bandpermanent)
 *                          for a_ij = 0 when |i-j| > k: the product of the
 *                          row forms C_i = sum_j a_ij x_j, kept as a
 *                          polynomial in the column variables with
 *                          x_j^2 = 0, the variable of the column that leaves
 *                          the band set to 1 after each row, and all of
 *                          them set to 1 at the end.
 *
 * Threads (pthreads) only split index ranges evenly (App. A, distribute);
 * every thread's partial result lands in an array that is added in index
 * order, so the result does not depend on scheduling.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef unsigned __int128 u128;

#define ORACLE_MAX_N 64
#define ORACLE_MAX_THREADS 256

/* ------------------------------------------------------------------------ */
/* Small utilities                                                           */
/* ------------------------------------------------------------------------ */

/* Kahan summation in long double (App. A, Kahan). */
typedef struct {
  long double s, b;
} kahan_ld;

static void kahan_add(kahan_ld* k, long double a) {
  long double c = a - k->b;
  long double t = k->s + c;
  k->b = (t - k->s) - c;
  k->s = t;
}

/* Split a long double into an unevaluated pair of doubles hi + lo. */
static void ld_to_pair(long double x, double* out) {
  double hi = (double)x;
  out[0] = hi;
  out[1] = (double)(x - (long double)hi);
}

static void u128_to_pair(u128 x, uint64_t* out) {
  out[0] = (uint64_t)x;
  out[1] = (uint64_t)(x >> 64);
}

/* App. A, distribute: cut a sequence of length total into m near-equal
 * consecutive parts; part i starts at k and has length len. */
static void distribute(uint64_t total, uint64_t m, uint64_t i, uint64_t* k,
                       uint64_t* len) {
  uint64_t q = total / m;
  uint64_t r = total % m;
  *k = i * q + (i < r ? i : r);
  *len = q + (i < r ? 1 : 0);
}

static int pick_threads(int requested, uint64_t work_items) {
  int t = requested;
  if (t <= 0) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    t = c > 0 ? (int)c : 1;
  }
  if (t > ORACLE_MAX_THREADS) t = ORACLE_MAX_THREADS;
  if ((uint64_t)t > work_items) t = work_items > 0 ? (int)work_items : 1;
  return t;
}

/* Gray code of k (App. A, Gray unranking). */
static uint64_t gray(uint64_t k) { return k ^ (k >> 1); }

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

/* ------------------------------------------------------------------------ */
/* O1: the definition, all n! permutations (Sec. I, Eq. per)                 */
/* ------------------------------------------------------------------------ */

/* Visit every permutation of {0..n-1} once (Heap's method). */
typedef void (*perm_visitor)(const int* p, int n, void* ctx);

static void for_each_permutation(int n, perm_visitor visit, void* ctx) {
  int p[ORACLE_MAX_N], c[ORACLE_MAX_N];
  for (int i = 0; i < n; ++i) {
    p[i] = i;
    c[i] = 0;
  }
  visit(p, n, ctx);
  int i = 1;
  while (i < n) {
    if (c[i] < i) {
      int a = (i % 2 == 0) ? 0 : c[i];
      int t = p[a];
      p[a] = p[i];
      p[i] = t;
      visit(p, n, ctx);
      c[i] += 1;
      i = 1;
    } else {
      c[i] = 0;
      i += 1;
    }
  }
}

typedef struct {
  const double* A;
  int ld;
  kahan_ld re, im;
  u128 acc;
  const uint8_t* B;
} brute_ctx;

static void visit_real(const int* p, int n, void* vctx) {
  brute_ctx* x = (brute_ctx*)vctx;
  long double prod = 1.0L;
  for (int i = 0; i < n; ++i) prod *= (long double)x->A[i + (size_t)p[i] * x->ld];
  kahan_add(&x->re, prod);
}

static void visit_complex(const int* p, int n, void* vctx) {
  brute_ctx* x = (brute_ctx*)vctx;
  long double pr = 1.0L, pi = 0.0L;
  for (int i = 0; i < n; ++i) {
    size_t o = 2 * (i + (size_t)p[i] * x->ld);
    long double ar = x->A[o], ai = x->A[o + 1];
    long double nr = pr * ar - pi * ai;
    long double ni = pr * ai + pi * ar;
    pr = nr;
    pi = ni;
  }
  kahan_add(&x->re, pr);
  kahan_add(&x->im, pi);
}

static void visit_int(const int* p, int n, void* vctx) {
  brute_ctx* x = (brute_ctx*)vctx;
  u128 prod = 1;
  for (int i = 0; i < n; ++i) prod *= (u128)x->B[i + (size_t)p[i] * x->ld];
  x->acc += prod;
}

/* out[0..1]: per(A) as hi + lo.  Returns 0, or -1 on bad arguments. */
int oracle_brute_real(const double* A, int n, int ld, double* out) {
  if (n < 0 || n > 12 || ld < n) return -1;
  brute_ctx x;
  memset(&x, 0, sizeof x);
  x.A = A;
  x.ld = ld;
  for_each_permutation(n, visit_real, &x);
  ld_to_pair(x.re.s, out);
  return 0;
}

/* out[0..3]: re hi, re lo, im hi, im lo. */
int oracle_brute_complex(const double* A, int n, int ld, double* out) {
  if (n < 0 || n > 12 || ld < n) return -1;
  brute_ctx x;
  memset(&x, 0, sizeof x);
  x.A = A;
  x.ld = ld;
  for_each_permutation(n, visit_complex, &x);
  ld_to_pair(x.re.s, out);
  ld_to_pair(x.im.s, out + 2);
  return 0;
}

/* Unsigned byte entries; out[0..1]: per(A) mod 2^128 as (low, high) words. */
int oracle_brute_int(const uint8_t* B, int n, int ld, uint64_t* out) {
  if (n < 0 || n > 12 || ld < n) return -1;
  brute_ctx x;
  memset(&x, 0, sizeof x);
  x.B = B;
  x.ld = ld;
  for_each_permutation(n, visit_int, &x);
  u128_to_pair(x.acc, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O2 / O3: Ryser over all 2^n subsets in Gray order (Sec. II.A, Eq. ryser)  */
/* ------------------------------------------------------------------------ */

/* Row sums are formed from scratch at the first subset of a thread's range
 * and again every RYSER_REFORM subsets, so long-double round-off in the
 * running sums cannot build up along the walk. */
#define RYSER_REFORM 1024u

typedef struct {
  const double* A;
  const uint8_t* B;
  int n, ld, is_complex;
  uint64_t k0, len;
  long double re, im; /* partial sums (already Kahan-compensated) */
  u128 acc;
} ryser_job;

/* Sum over subsets J = gray(k), k in [k0, k0+len), of (-1)^|J| prod_i sum_{j in J} a_ij. */
static void* ryser_real_worker(void* arg) {
  ryser_job* jb = (ryser_job*)arg;
  const int n = jb->n, ld = jb->ld;
  long double r[ORACLE_MAX_N];
  kahan_ld S = {0.0L, 0.0L};
  for (uint64_t k = jb->k0; k < jb->k0 + jb->len; ++k) {
    uint64_t J = gray(k);
    if (k == jb->k0 || ((k - jb->k0) % RYSER_REFORM) == 0) {
      for (int i = 0; i < n; ++i) {
        r[i] = 0.0L;
        for (int j = 0; j < n; ++j)
          if ((J >> j) & 1) r[i] += (long double)jb->A[i + (size_t)j * ld];
      }
    } else {
      /* gray(k) and gray(k-1) differ in exactly bit ctz(k). */
      int j = __builtin_ctzll(k);
      int added = (int)((J >> j) & 1);
      for (int i = 0; i < n; ++i) {
        long double a = (long double)jb->A[i + (size_t)j * ld];
        r[i] = added ? r[i] + a : r[i] - a;
      }
    }
    long double p = 1.0L;
    for (int i = 0; i < n; ++i) p *= r[i];
    kahan_add(&S, (popcount64(J) & 1) ? -p : p);
  }
  jb->re = S.s;
  return NULL;
}

static void* ryser_complex_worker(void* arg) {
  ryser_job* jb = (ryser_job*)arg;
  const int n = jb->n, ld = jb->ld;
  long double rr[ORACLE_MAX_N], ri[ORACLE_MAX_N];
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (uint64_t k = jb->k0; k < jb->k0 + jb->len; ++k) {
    uint64_t J = gray(k);
    if (k == jb->k0 || ((k - jb->k0) % RYSER_REFORM) == 0) {
      for (int i = 0; i < n; ++i) {
        rr[i] = 0.0L;
        ri[i] = 0.0L;
        for (int j = 0; j < n; ++j)
          if ((J >> j) & 1) {
            size_t o = 2 * (i + (size_t)j * ld);
            rr[i] += (long double)jb->A[o];
            ri[i] += (long double)jb->A[o + 1];
          }
      }
    } else {
      int j = __builtin_ctzll(k);
      int added = (int)((J >> j) & 1);
      for (int i = 0; i < n; ++i) {
        size_t o = 2 * (i + (size_t)j * ld);
        long double ar = jb->A[o], ai = jb->A[o + 1];
        rr[i] = added ? rr[i] + ar : rr[i] - ar;
        ri[i] = added ? ri[i] + ai : ri[i] - ai;
      }
    }
    long double pr = 1.0L, pi = 0.0L;
    for (int i = 0; i < n; ++i) {
      long double nr = pr * rr[i] - pi * ri[i];
      long double ni = pr * ri[i] + pi * rr[i];
      pr = nr;
      pi = ni;
    }
    if (popcount64(J) & 1) {
      pr = -pr;
      pi = -pi;
    }
    kahan_add(&Sr, pr);
    kahan_add(&Si, pi);
  }
  jb->re = Sr.s;
  jb->im = Si.s;
  return NULL;
}

/* Integer entries, arithmetic modulo 2^128 (unsigned wrap-around). */
static void* ryser_int_worker(void* arg) {
  ryser_job* jb = (ryser_job*)arg;
  const int n = jb->n, ld = jb->ld;
  int64_t r[ORACLE_MAX_N];
  u128 S = 0;
  for (uint64_t k = jb->k0; k < jb->k0 + jb->len; ++k) {
    uint64_t J = gray(k);
    if (k == jb->k0) {
      for (int i = 0; i < n; ++i) {
        r[i] = 0;
        for (int j = 0; j < n; ++j)
          if ((J >> j) & 1) r[i] += jb->B[i + (size_t)j * ld];
      }
    } else {
      int j = __builtin_ctzll(k);
      int added = (int)((J >> j) & 1);
      for (int i = 0; i < n; ++i) {
        int64_t a = jb->B[i + (size_t)j * ld];
        r[i] = added ? r[i] + a : r[i] - a;
      }
    }
    u128 p = 1;
    for (int i = 0; i < n; ++i) p *= (u128)(__int128)r[i];
    if (popcount64(J) & 1)
      S -= p;
    else
      S += p;
  }
  jb->acc = S;
  return NULL;
}

static int run_ryser(ryser_job* proto, uint64_t k0, uint64_t count, int nthreads,
                     void* (*worker)(void*), ryser_job* jobs_out, int* used) {
  int T = pick_threads(nthreads, count);
  pthread_t th[ORACLE_MAX_THREADS];
  for (int t = 0; t < T; ++t) {
    jobs_out[t] = *proto;
    uint64_t off, len;
    distribute(count, (uint64_t)T, (uint64_t)t, &off, &len);
    jobs_out[t].k0 = k0 + off;
    jobs_out[t].len = len;
  }
  int started = 0;
  for (int t = 0; t < T; ++t) {
    if (pthread_create(&th[t], NULL, worker, &jobs_out[t]) != 0) break;
    ++started;
  }
  for (int t = started; t < T; ++t) worker(&jobs_out[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  *used = T;
  return 0;
}

/*
 * Partial Ryser sum over subset indices k in [k0, k0+count): the subset is
 * J = gray(k), the term is (-1)^|J| prod_i sum_{j in J} a_ij.  The full
 * permanent is (-1)^n times the sum over k in [0, 2^n).
 * out: real [hi, lo]; complex [re hi, re lo, im hi, im lo].
 */
int oracle_ryser_real_range(const double* A, int n, int ld, uint64_t k0, uint64_t count,
                            int nthreads, double* out) {
  if (n < 1 || n > 62 || ld < n) return -1;
  if (k0 > (1ull << n) || count > (1ull << n) - k0) return -1;
  ryser_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.A = A;
  proto.n = n;
  proto.ld = ld;
  int T = 0;
  run_ryser(&proto, k0, count, nthreads, ryser_real_worker, jobs, &T);
  kahan_ld S = {0.0L, 0.0L};
  for (int t = 0; t < T; ++t) kahan_add(&S, jobs[t].re);
  ld_to_pair(S.s, out);
  return 0;
}

int oracle_ryser_complex_range(const double* A, int n, int ld, uint64_t k0, uint64_t count,
                               int nthreads, double* out) {
  if (n < 1 || n > 62 || ld < n) return -1;
  if (k0 > (1ull << n) || count > (1ull << n) - k0) return -1;
  ryser_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.A = A;
  proto.n = n;
  proto.ld = ld;
  proto.is_complex = 1;
  int T = 0;
  run_ryser(&proto, k0, count, nthreads, ryser_complex_worker, jobs, &T);
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (int t = 0; t < T; ++t) {
    kahan_add(&Sr, jobs[t].re);
    kahan_add(&Si, jobs[t].im);
  }
  ld_to_pair(Sr.s, out);
  ld_to_pair(Si.s, out + 2);
  return 0;
}

/* out: [low, high] words of the partial sum modulo 2^128. */
int oracle_ryser_int_range(const uint8_t* B, int n, int ld, uint64_t k0, uint64_t count,
                           int nthreads, uint64_t* out) {
  if (n < 1 || n > 62 || ld < n) return -1;
  if (k0 > (1ull << n) || count > (1ull << n) - k0) return -1;
  ryser_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.B = B;
  proto.n = n;
  proto.ld = ld;
  int T = 0;
  run_ryser(&proto, k0, count, nthreads, ryser_int_worker, jobs, &T);
  u128 S = 0;
  for (int t = 0; t < T; ++t) S += jobs[t].acc;
  u128_to_pair(S, out);
  return 0;
}

/* per(A) = (-1)^n * sum over all 2^n subsets (Sec. II.A, Eq. ryser). */
int oracle_ryser_real(const double* A, int n, int ld, int nthreads, double* out) {
  if (n == 0) {
    out[0] = 1.0;
    out[1] = 0.0;
    return 0;
  }
  if (n > 40) return -1;
  int rc = oracle_ryser_real_range(A, n, ld, 0, 1ull << n, nthreads, out);
  if (rc == 0 && (n & 1)) {
    out[0] = -out[0];
    out[1] = -out[1];
  }
  return rc;
}

int oracle_ryser_complex(const double* A, int n, int ld, int nthreads, double* out) {
  if (n == 0) {
    out[0] = 1.0;
    out[1] = out[2] = out[3] = 0.0;
    return 0;
  }
  if (n > 40) return -1;
  int rc = oracle_ryser_complex_range(A, n, ld, 0, 1ull << n, nthreads, out);
  if (rc == 0 && (n & 1))
    for (int q = 0; q < 4; ++q) out[q] = -out[q];
  return rc;
}

int oracle_ryser_int(const uint8_t* B, int n, int ld, int nthreads, uint64_t* out) {
  if (n == 0) {
    out[0] = 1;
    out[1] = 0;
    return 0;
  }
  if (n > 40) return -1;
  uint64_t tmp[2];
  int rc = oracle_ryser_int_range(B, n, ld, 0, 1ull << n, nthreads, tmp);
  if (rc != 0) return rc;
  u128 S = ((u128)tmp[1] << 64) | tmp[0];
  if (n & 1) S = (u128)0 - S;
  u128_to_pair(S, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O4: half-range partial sums of App. A, every term formed directly         */
/* ------------------------------------------------------------------------ */

typedef struct {
  const double* A;
  const uint8_t* B;
  int n, ld;
  uint64_t g0, len;
  long double re, im;
  u128 acc;
} chunk_job;

/* Row-sum vector of App. A (subpermanent) for Gray code x:
 *   w_i = a_{i,n} - 1/2 sum_{j=1..n} a_{ij} + sum_{j<n, x_j = 1} a_{ij}
 * (columns and bits 0-based here: bit j of x stands for column j). */
static void* chunk_real_worker(void* arg) {
  chunk_job* jb = (chunk_job*)arg;
  const int n = jb->n, ld = jb->ld;
  kahan_ld S = {0.0L, 0.0L};
  for (uint64_t g = jb->g0; g < jb->g0 + jb->len; ++g) {
    uint64_t x = gray(g);
    long double p = 1.0L;
    for (int i = 0; i < n; ++i) {
      long double half = 0.0L;
      for (int j = 0; j < n; ++j) half += (long double)jb->A[i + (size_t)j * ld];
      long double w = (long double)jb->A[i + (size_t)(n - 1) * ld] - 0.5L * half;
      for (int j = 0; j < n - 1; ++j)
        if ((x >> j) & 1) w += (long double)jb->A[i + (size_t)j * ld];
      p *= w;
    }
    /* term g carries t = (-1)^(g+1) (App. A: nextset negates t before S += t p) */
    kahan_add(&S, (g & 1) ? p : -p);
  }
  jb->re = S.s;
  return NULL;
}

static void* chunk_complex_worker(void* arg) {
  chunk_job* jb = (chunk_job*)arg;
  const int n = jb->n, ld = jb->ld;
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (uint64_t g = jb->g0; g < jb->g0 + jb->len; ++g) {
    uint64_t x = gray(g);
    long double pr = 1.0L, pi = 0.0L;
    for (int i = 0; i < n; ++i) {
      long double hr = 0.0L, hi = 0.0L;
      for (int j = 0; j < n; ++j) {
        size_t o = 2 * (i + (size_t)j * ld);
        hr += (long double)jb->A[o];
        hi += (long double)jb->A[o + 1];
      }
      size_t on = 2 * (i + (size_t)(n - 1) * ld);
      long double wr = (long double)jb->A[on] - 0.5L * hr;
      long double wi = (long double)jb->A[on + 1] - 0.5L * hi;
      for (int j = 0; j < n - 1; ++j)
        if ((x >> j) & 1) {
          size_t o = 2 * (i + (size_t)j * ld);
          wr += (long double)jb->A[o];
          wi += (long double)jb->A[o + 1];
        }
      long double nr = pr * wr - pi * wi;
      long double ni = pr * wi + pi * wr;
      pr = nr;
      pi = ni;
    }
    if (!(g & 1)) {
      pr = -pr;
      pi = -pi;
    }
    kahan_add(&Sr, pr);
    kahan_add(&Si, pi);
  }
  jb->re = Sr.s;
  jb->im = Si.s;
  return NULL;
}

/* Integer form: r_i = 2 w_i is an integer, the sum is kept modulo 2^128.
 * sum_g (-1)^(g+1) prod_i r_i = 2^n * (App. A partial sum). */
static void* chunk_int_worker(void* arg) {
  chunk_job* jb = (chunk_job*)arg;
  const int n = jb->n, ld = jb->ld;
  u128 S = 0;
  for (uint64_t g = jb->g0; g < jb->g0 + jb->len; ++g) {
    uint64_t x = gray(g);
    u128 p = 1;
    for (int i = 0; i < n; ++i) {
      int64_t rowsum = 0;
      for (int j = 0; j < n; ++j) rowsum += jb->B[i + (size_t)j * ld];
      int64_t r = 2 * (int64_t)jb->B[i + (size_t)(n - 1) * ld] - rowsum;
      for (int j = 0; j < n - 1; ++j)
        if ((x >> j) & 1) r += 2 * (int64_t)jb->B[i + (size_t)j * ld];
      p *= (u128)(__int128)r;
    }
    if (g & 1)
      S += p;
    else
      S -= p;
  }
  jb->acc = S;
  return NULL;
}

static int run_chunks(chunk_job* proto, uint64_t g0, uint64_t count, int nthreads,
                      void* (*worker)(void*), chunk_job* jobs, int* used) {
  int T = pick_threads(nthreads, count);
  pthread_t th[ORACLE_MAX_THREADS];
  for (int t = 0; t < T; ++t) {
    jobs[t] = *proto;
    uint64_t off, len;
    distribute(count, (uint64_t)T, (uint64_t)t, &off, &len);
    jobs[t].g0 = g0 + off;
    jobs[t].len = len;
  }
  int started = 0;
  for (int t = 0; t < T; ++t) {
    if (pthread_create(&th[t], NULL, worker, &jobs[t]) != 0) break;
    ++started;
  }
  for (int t = started; t < T; ++t) worker(&jobs[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  *used = T;
  return 0;
}

static int chunk_args_ok(int n, int ld, uint64_t g0, uint64_t count) {
  if (n < 1 || n > ORACLE_MAX_N || ld < n) return 0;
  uint64_t total = (n == 64) ? (1ull << 63) : (1ull << (n - 1));
  if (g0 > total || count > total - g0) return 0;
  return 1;
}

/* App. A partial sum S over Gray indices [g0, g0+count); out [hi, lo]. */
int oracle_chunk_real(const double* A, int n, int ld, uint64_t g0, uint64_t count,
                      int nthreads, double* out) {
  if (!chunk_args_ok(n, ld, g0, count)) return -1;
  chunk_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.A = A;
  proto.n = n;
  proto.ld = ld;
  int T = 0;
  run_chunks(&proto, g0, count, nthreads, chunk_real_worker, jobs, &T);
  kahan_ld S = {0.0L, 0.0L};
  for (int t = 0; t < T; ++t) kahan_add(&S, jobs[t].re);
  ld_to_pair(S.s, out);
  return 0;
}

int oracle_chunk_complex(const double* A, int n, int ld, uint64_t g0, uint64_t count,
                         int nthreads, double* out) {
  if (!chunk_args_ok(n, ld, g0, count)) return -1;
  chunk_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.A = A;
  proto.n = n;
  proto.ld = ld;
  int T = 0;
  run_chunks(&proto, g0, count, nthreads, chunk_complex_worker, jobs, &T);
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (int t = 0; t < T; ++t) {
    kahan_add(&Sr, jobs[t].re);
    kahan_add(&Si, jobs[t].im);
  }
  ld_to_pair(Sr.s, out);
  ld_to_pair(Si.s, out + 2);
  return 0;
}

/* out [low, high] of sum_g (-1)^(g+1) prod_i r_i modulo 2^128, r = 2w. */
int oracle_chunk_int(const uint8_t* B, int n, int ld, uint64_t g0, uint64_t count,
                     int nthreads, uint64_t* out) {
  if (!chunk_args_ok(n, ld, g0, count)) return -1;
  chunk_job proto, jobs[ORACLE_MAX_THREADS];
  memset(&proto, 0, sizeof proto);
  proto.B = B;
  proto.n = n;
  proto.ld = ld;
  int T = 0;
  run_chunks(&proto, g0, count, nthreads, chunk_int_worker, jobs, &T);
  u128 S = 0;
  for (int t = 0; t < T; ++t) S += jobs[t].acc;
  u128_to_pair(S, out);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O5: Ryser's formula with repeated columns (Sec. II.A, Eq. ryser2)         */
/* ------------------------------------------------------------------------ */

/* Binomial coefficients C(m, f), m <= 64, from Pascal's rule in exact 64-bit
 * integers (C(64, 32) < 2^64); long double holds every one of them exactly. */
static uint64_t g_binom[ORACLE_MAX_N + 1][ORACLE_MAX_N + 1];
static pthread_once_t g_binom_once = PTHREAD_ONCE_INIT;

static void binom_init(void) {
  for (int m = 0; m <= ORACLE_MAX_N; ++m) {
    g_binom[m][0] = 1;
    for (int f = 1; f <= m; ++f)
      g_binom[m][f] = g_binom[m - 1][f - 1] + (f <= m - 1 ? g_binom[m - 1][f] : 0);
  }
}

/* Reflected mixed-radix Gray code, digit 0 changing fastest: the sequence for
 * digits j..0 takes digit j through 0, 1, ..., r_j - 1, and under each value v
 * runs the sequence of digits j-1..0, forwards for even v and backwards for
 * odd v.  Q[j] = r_0 r_1 ... r_{j-1} is the length of that lower sequence.
 * Unranking follows the definition from the top digit down. */
static void mixed_gray_unrank(uint64_t g, int R, const uint64_t* Q, int* f) {
  uint64_t pos = g;
  for (int j = R - 1; j >= 0; --j) {
    const uint64_t v = pos / Q[j];
    const uint64_t rem = pos % Q[j];
    f[j] = (int)v;
    pos = (v & 1) ? Q[j] - 1 - rem : rem;
  }
}

/* Counting order: f_k is digit k of g in the mixed radix (m_k + 1). */
static void counting_unrank(uint64_t g, int R, const int* m, int* f) {
  for (int k = 0; k < R; ++k) {
    f[k] = (int)(g % (uint64_t)(m[k] + 1));
    g /= (uint64_t)(m[k] + 1);
  }
}

typedef struct {
  const double* C;
  const int* m;
  const uint64_t* Q;
  int n, R, ld, cplx, gray_order;
  uint64_t g0, len;
  long double re, im;
} rep_job;

static void* ryser2_worker(void* arg) {
  rep_job* jb = (rep_job*)arg;
  const int n = jb->n, R = jb->R, ld = jb->ld;
  int f[ORACLE_MAX_N];
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (uint64_t g = jb->g0; g < jb->g0 + jb->len; ++g) {
    if (jb->gray_order)
      mixed_gray_unrank(g, R, jb->Q, f);
    else
      counting_unrank(g, R, jb->m, f);
    int fsum = 0;
    long double wgt = 1.0L;
    for (int k = 0; k < R; ++k) {
      fsum += f[k];
      wgt *= (long double)g_binom[jb->m[k]][f[k]];
    }
    long double pr = 1.0L, pi = 0.0L;
    for (int i = 0; i < n; ++i) {
      long double sr = 0.0L, si = 0.0L;
      for (int k = 0; k < R; ++k) {
        if (jb->cplx) {
          size_t o = 2 * (i + (size_t)k * ld);
          sr += (long double)f[k] * (long double)jb->C[o];
          si += (long double)f[k] * (long double)jb->C[o + 1];
        } else {
          sr += (long double)f[k] * (long double)jb->C[i + (size_t)k * ld];
        }
      }
      long double nr = pr * sr - pi * si;
      long double ni = pr * si + pi * sr;
      pr = nr;
      pi = ni;
    }
    if (fsum & 1) wgt = -wgt;
    kahan_add(&Sr, wgt * pr);
    kahan_add(&Si, wgt * pi);
  }
  jb->re = Sr.s;
  jb->im = Si.s;
  return NULL;
}

/* Checks the arguments, fills Q and the number of vectors f (T). */
static int ryser2_setup(int n, int R, int ld, const int* m, uint64_t* Q, uint64_t* T) {
  if (n < 1 || n > ORACLE_MAX_N || R < 1 || R > n || ld < n || !m) return 0;
  int total = 0;
  u128 t = 1;
  for (int k = 0; k < R; ++k) {
    if (m[k] < 1) return 0;
    total += m[k];
    Q[k] = (uint64_t)t;
    t *= (u128)(m[k] + 1);
    if (t > ((u128)1 << 63)) return 0;
  }
  if (total != n) return 0;
  *T = (uint64_t)t;
  pthread_once(&g_binom_once, binom_init);
  return 1;
}

static void ryser2_run(rep_job* proto, uint64_t g0, uint64_t count, int nthreads,
                       long double* re, long double* im) {
  rep_job jobs[ORACLE_MAX_THREADS];
  pthread_t th[ORACLE_MAX_THREADS];
  int T = pick_threads(nthreads, count);
  for (int t = 0; t < T; ++t) {
    jobs[t] = *proto;
    uint64_t off, len;
    distribute(count, (uint64_t)T, (uint64_t)t, &off, &len);
    jobs[t].g0 = g0 + off;
    jobs[t].len = len;
  }
  int started = 0;
  for (int t = 0; t < T; ++t) {
    if (pthread_create(&th[t], NULL, ryser2_worker, &jobs[t]) != 0) break;
    ++started;
  }
  for (int t = started; t < T; ++t) ryser2_worker(&jobs[t]);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (int t = 0; t < T; ++t) {
    kahan_add(&Sr, jobs[t].re);
    kahan_add(&Si, jobs[t].im);
  }
  *re = Sr.s;
  *im = Si.s;
}

/* per(A) for the n x n matrix A whose columns are c_k repeated m_k times
 * (k < R, sum m_k = n); C is n x R column-major (complex: interleaved).
 * out: [re hi, re lo, im hi, im lo]. */
int oracle_ryser2(const double* C, int n, int R, int ld, const int* m, int cplx, int nthreads,
                  double* out) {
  uint64_t Q[ORACLE_MAX_N], T;
  if (!ryser2_setup(n, R, ld, m, Q, &T)) return -1;
  rep_job proto;
  memset(&proto, 0, sizeof proto);
  proto.C = C;
  proto.m = m;
  proto.Q = Q;
  proto.n = n;
  proto.R = R;
  proto.ld = ld;
  proto.cplx = cplx;
  long double re, im;
  ryser2_run(&proto, 0, T, nthreads, &re, &im);
  if (n & 1) {
    re = -re;
    im = -im;
  }
  ld_to_pair(re, out);
  ld_to_pair(im, out + 2);
  return 0;
}

/* The raw sum of Eq. ryser2 (without (-1)^n) over Gray indices
 * [g0, g0 + count) of the reflected mixed-radix order. */
int oracle_ryser2_range(const double* C, int n, int R, int ld, const int* m, int cplx,
                        uint64_t g0, uint64_t count, int nthreads, double* out) {
  uint64_t Q[ORACLE_MAX_N], T;
  if (!ryser2_setup(n, R, ld, m, Q, &T)) return -1;
  if (g0 > T || count > T - g0) return -1;
  rep_job proto;
  memset(&proto, 0, sizeof proto);
  proto.C = C;
  proto.m = m;
  proto.Q = Q;
  proto.n = n;
  proto.R = R;
  proto.ld = ld;
  proto.cplx = cplx;
  proto.gray_order = 1;
  long double re, im;
  ryser2_run(&proto, g0, count, nthreads, &re, &im);
  ld_to_pair(re, out);
  ld_to_pair(im, out + 2);
  return 0;
}

/* Digits f_0..f_{R-1} of Gray index g (radices r_k), for tests of the order. */
int oracle_mixed_gray(uint64_t g, int R, const int* radix, int* f) {
  uint64_t Q[ORACLE_MAX_N];
  if (R < 1 || R > ORACLE_MAX_N) return -1;
  u128 t = 1;
  for (int k = 0; k < R; ++k) {
    if (radix[k] < 1) return -1;
    Q[k] = (uint64_t)t;
    t *= (u128)radix[k];
    if (t > ((u128)1 << 63)) return -1;
  }
  if ((u128)g >= t) return -1;
  mixed_gray_unrank(g, R, Q, f);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O6: band transfer matrix (App. C, bandpermanent)                          */
/* ------------------------------------------------------------------------ */

/* The polynomial is stored by its monomials: a monomial is a set of column
 * variables, all from the window of columns [base, base + 2k + 1] that can
 * still be unset (columns below base have been set to 1, columns above the
 * window cannot have appeared yet).  Bit b of a mask stands for column
 * base + b.  Before row i (0-based) base = i - k - 1. */
#define ORACLE_BAND_MAX_K 9

static int band_args_ok(int n, int ld, int k) {
  return n >= 1 && n <= 4096 && ld >= n && k >= 0 && k <= ORACLE_BAND_MAX_K;
}

/* Out-of-band entries must be zero (the algorithm never reads them). */
static int band_zero_outside_real(const double* A, int n, int ld, int k, int cw) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      if (i - j > k || j - i > k)
        for (int c = 0; c < cw; ++c)
          if (A[cw * (i + (size_t)j * ld) + c] != 0.0) return 0;
  return 1;
}

int oracle_band_real(const double* A, int n, int ld, int k, int cplx, double* out) {
  if (!band_args_ok(n, ld, k)) return -1;
  const int cw = cplx ? 2 : 1;
  if (!band_zero_outside_real(A, n, ld, k, cw)) return -1;
  const int W = 2 * k + 2; /* window bits before the shift */
  const size_t S = (size_t)1 << W;
  long double* re = calloc(S, sizeof(long double));
  long double* im = calloc(S, sizeof(long double));
  long double* nre = calloc(S, sizeof(long double));
  long double* nim = calloc(S, sizeof(long double));
  if (!re || !im || !nre || !nim) {
    free(re); free(im); free(nre); free(nim);
    return -2;
  }
  re[0] = 1.0L; /* p := 1 */
  for (int i = 0; i < n; ++i) {
    const int base = i - k - 1;
    /* p := p * C_i, dropping monomials with a squared variable */
    memset(nre, 0, S * sizeof(long double));
    memset(nim, 0, S * sizeof(long double));
    for (size_t m = 0; m < S; ++m) {
      if (re[m] == 0.0L && im[m] == 0.0L) continue;
      for (int j = (i - k > 0 ? i - k : 0); j <= i + k && j < n; ++j) {
        const int b = j - base;
        if ((m >> b) & 1) continue; /* x_j^2 = 0 */
        const size_t o = cw * (i + (size_t)j * ld);
        const long double ar = (long double)A[o];
        const long double ai = cplx ? (long double)A[o + 1] : 0.0L;
        nre[m | ((size_t)1 << b)] += re[m] * ar - im[m] * ai;
        nim[m | ((size_t)1 << b)] += re[m] * ai + im[m] * ar;
      }
    }
    /* set x_{base} = 1 (column i-k-1 leaves the band): merge bit 0 away and
     * move the window up by one column */
    memset(re, 0, S * sizeof(long double));
    memset(im, 0, S * sizeof(long double));
    for (size_t m = 0; m < S; ++m) {
      re[m >> 1] += nre[m];
      im[m >> 1] += nim[m];
    }
  }
  /* set every remaining x_j = 1 */
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  for (size_t m = 0; m < S; ++m) {
    kahan_add(&Sr, re[m]);
    kahan_add(&Si, im[m]);
  }
  ld_to_pair(Sr.s, out);
  ld_to_pair(Si.s, out + 2);
  free(re); free(im); free(nre); free(nim);
  return 0;
}

/* 0/1 band matrices, exact modulo 2^128. */
int oracle_band_int(const uint8_t* B, int n, int ld, int k, uint64_t* out) {
  if (!band_args_ok(n, ld, k)) return -1;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      if ((i - j > k || j - i > k) && B[i + (size_t)j * ld] != 0) return -1;
  const int W = 2 * k + 2;
  const size_t S = (size_t)1 << W;
  u128* c = calloc(S, sizeof(u128));
  u128* nc = calloc(S, sizeof(u128));
  if (!c || !nc) {
    free(c); free(nc);
    return -2;
  }
  c[0] = 1;
  for (int i = 0; i < n; ++i) {
    const int base = i - k - 1;
    memset(nc, 0, S * sizeof(u128));
    for (size_t m = 0; m < S; ++m) {
      if (c[m] == 0) continue;
      for (int j = (i - k > 0 ? i - k : 0); j <= i + k && j < n; ++j) {
        const int b = j - base;
        if ((m >> b) & 1) continue;
        if (B[i + (size_t)j * ld]) nc[m | ((size_t)1 << b)] += c[m] * (u128)B[i + (size_t)j * ld];
      }
    }
    memset(c, 0, S * sizeof(u128));
    for (size_t m = 0; m < S; ++m) c[m >> 1] += nc[m];
  }
  u128 sum = 0;
  for (size_t m = 0; m < S; ++m) sum += c[m];
  u128_to_pair(sum, out);
  free(c); free(nc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O7: sparse matrices (App. B, greedypartition and sparsepermanent)         */
/* ------------------------------------------------------------------------ */

/* Blocks larger than this do not restrict the sum (their columns join T):
 * the enumeration of a block's nonempty subsets is kept to 2^12 - 1 values.
 * Dropping a restriction only adds zero terms. */
#define ORACLE_SPARSE_MAX_BLOCK 12

typedef struct {
  int nblocks;
  int block_first[ORACLE_MAX_N]; /* index into cols[] of block l's first column */
  int block_size[ORACLE_MAX_N];
  int ntail;                     /* |T| */
  int cols[ORACLE_MAX_N];        /* blocks in selection order (columns ascending
                                    inside), then the columns of T ascending */
} sparse_part;

static int entry_nonzero(const double* A, const uint8_t* B, int ld, int cplx, int i, int j) {
  if (B) return B[i + (size_t)j * ld] != 0;
  if (cplx) return A[2 * (i + (size_t)j * ld)] != 0.0 || A[2 * (i + (size_t)j * ld) + 1] != 0.0;
  return A[i + (size_t)j * ld] != 0.0;
}

/* greedypartition (App. B): repeatedly take the remaining row k of least
 * degree (the lowest index among equals), make its column set N_k a block,
 * and drop row k and every remaining row whose column set meets N_k.  The
 * blocks are pairwise disjoint; T is the set of columns in no block. */
static int greedy_partition(const double* A, const uint8_t* B, int n, int ld, int cplx,
                            sparse_part* P) {
  int deg[ORACLE_MAX_N], alive[ORACLE_MAX_N];
  uint64_t nb[ORACLE_MAX_N];
  for (int i = 0; i < n; ++i) {
    nb[i] = 0;
    for (int j = 0; j < n; ++j)
      if (entry_nonzero(A, B, ld, cplx, i, j)) nb[i] |= 1ull << j;
    deg[i] = popcount64(nb[i]);
    if (deg[i] == 0) return 0; /* a zero row: per = 0, no partition */
    alive[i] = 1;
  }
  uint64_t used = 0;
  int nblocks = 0, ncols = 0;
  for (;;) {
    int k = -1;
    for (int i = 0; i < n; ++i)
      if (alive[i] && (k < 0 || deg[i] < deg[k])) k = i;
    if (k < 0) break;
    alive[k] = 0;
    for (int l = 0; l < n; ++l)
      if (alive[l] && (nb[l] & nb[k])) alive[l] = 0;
    if (deg[k] > ORACLE_SPARSE_MAX_BLOCK) continue; /* too large to restrict */
    P->block_first[nblocks] = ncols;
    P->block_size[nblocks] = deg[k];
    for (int j = 0; j < n; ++j)
      if ((nb[k] >> j) & 1) P->cols[ncols++] = j;
    used |= nb[k];
    ++nblocks;
  }
  P->nblocks = nblocks;
  P->ntail = 0;
  for (int j = 0; j < n; ++j)
    if (!((used >> j) & 1)) {
      P->cols[ncols++] = j;
      P->ntail++;
    }
  return 1;
}

/* Digits of the enumeration: one per block (radix 2^s - 1, value v standing
 * for the nonempty subset gray(v + 1) of the block's columns), then one per
 * column of T (radix 2: out or in). */
static int sparse_radices(const sparse_part* P, uint64_t* radix, int* R) {
  int r = 0;
  for (int l = 0; l < P->nblocks; ++l) radix[r++] = (1ull << P->block_size[l]) - 1;
  for (int t = 0; t < P->ntail; ++t) radix[r++] = 2;
  *R = r;
  return r;
}

/* Column set J (bit mask over columns) of digit vector f. */
static uint64_t sparse_set(const sparse_part* P, const int* f) {
  uint64_t J = 0;
  int d = 0;
  for (int l = 0; l < P->nblocks; ++l, ++d) {
    const uint64_t sub = gray((uint64_t)f[d] + 1);
    for (int e = 0; e < P->block_size[l]; ++e)
      if ((sub >> e) & 1) J |= 1ull << P->cols[P->block_first[l] + e];
  }
  const int t0 = P->nblocks ? P->block_first[P->nblocks - 1] + P->block_size[P->nblocks - 1] : 0;
  for (int t = 0; t < P->ntail; ++t, ++d)
    if (f[d]) J |= 1ull << P->cols[t0 + t];
  return J;
}

typedef struct {
  const double* A;
  const uint8_t* B;
  const sparse_part* P;
  const uint64_t* Q;
  int n, ld, cplx, R, gray_order;
  uint64_t g0, len;
  long double re, im;
  u128 acc;
} sparse_job;

static void* sparse_worker(void* arg) {
  sparse_job* jb = (sparse_job*)arg;
  const int n = jb->n, ld = jb->ld;
  int f[ORACLE_MAX_N];
  uint64_t radix[ORACLE_MAX_N];
  int R;
  sparse_radices(jb->P, radix, &R);
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  u128 acc = 0;
  for (uint64_t g = jb->g0; g < jb->g0 + jb->len; ++g) {
    if (jb->gray_order) {
      mixed_gray_unrank(g, R, jb->Q, f);
    } else {
      uint64_t q = g;
      for (int d = 0; d < R; ++d) {
        f[d] = (int)(q % radix[d]);
        q /= radix[d];
      }
    }
    const uint64_t J = sparse_set(jb->P, f);
    const int odd = popcount64(J) & 1;
    if (jb->B) {
      u128 p = 1;
      for (int i = 0; i < n; ++i) {
        int64_t r = 0;
        for (int j = 0; j < n; ++j)
          if ((J >> j) & 1) r += jb->B[i + (size_t)j * ld];
        p *= (u128)r;
      }
      acc = odd ? acc - p : acc + p;
    } else {
      long double pr = 1.0L, pi = 0.0L;
      for (int i = 0; i < n; ++i) {
        long double sr = 0.0L, si = 0.0L;
        for (int j = 0; j < n; ++j)
          if ((J >> j) & 1) {
            if (jb->cplx) {
              sr += (long double)jb->A[2 * (i + (size_t)j * ld)];
              si += (long double)jb->A[2 * (i + (size_t)j * ld) + 1];
            } else {
              sr += (long double)jb->A[i + (size_t)j * ld];
            }
          }
        long double nr = pr * sr - pi * si;
        long double ni = pr * si + pi * sr;
        pr = nr;
        pi = ni;
      }
      kahan_add(&Sr, odd ? -pr : pr);
      kahan_add(&Si, odd ? -pi : pi);
    }
  }
  jb->re = Sr.s;
  jb->im = Si.s;
  jb->acc = acc;
  return NULL;
}

/* Runs the enumeration over [g0, g0 + count) (counting or Gray order);
 * returns -1 on bad arguments, 1 when a row is zero (per = 0), 0 otherwise. */
static int sparse_run(const double* A, const uint8_t* B, int n, int ld, int cplx, int gray_order,
                      uint64_t g0, int64_t count, int nthreads, long double* re, long double* im,
                      u128* acc, uint64_t* total) {
  if (n < 1 || n > ORACLE_MAX_N || ld < n) return -1;
  sparse_part P;
  memset(&P, 0, sizeof P);
  if (!greedy_partition(A, B, n, ld, cplx, &P)) {
    *re = *im = 0.0L;
    *acc = 0;
    *total = 0;
    return 1;
  }
  uint64_t radix[ORACLE_MAX_N], Q[ORACLE_MAX_N];
  int R;
  sparse_radices(&P, radix, &R);
  u128 t = 1;
  for (int d = 0; d < R; ++d) {
    Q[d] = (uint64_t)t;
    t *= radix[d];
    if (t > ((u128)1 << 63)) return -1;
  }
  *total = (uint64_t)t;
  if (count < 0) count = (int64_t)t; /* whole sum */
  if (g0 > (uint64_t)t || (uint64_t)count > (uint64_t)t - g0) return -1;
  sparse_job jobs[ORACLE_MAX_THREADS];
  pthread_t th[ORACLE_MAX_THREADS];
  int T = pick_threads(nthreads, (uint64_t)count);
  for (int k = 0; k < T; ++k) {
    memset(&jobs[k], 0, sizeof jobs[k]);
    jobs[k].A = A;
    jobs[k].B = B;
    jobs[k].P = &P;
    jobs[k].Q = Q;
    jobs[k].n = n;
    jobs[k].ld = ld;
    jobs[k].cplx = cplx;
    jobs[k].R = R;
    jobs[k].gray_order = gray_order;
    uint64_t off, len;
    distribute((uint64_t)count, (uint64_t)T, (uint64_t)k, &off, &len);
    jobs[k].g0 = g0 + off;
    jobs[k].len = len;
  }
  int started = 0;
  for (int k = 0; k < T; ++k) {
    if (pthread_create(&th[k], NULL, sparse_worker, &jobs[k]) != 0) break;
    ++started;
  }
  for (int k = started; k < T; ++k) sparse_worker(&jobs[k]);
  for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
  kahan_ld Sr = {0.0L, 0.0L}, Si = {0.0L, 0.0L};
  u128 a = 0;
  for (int k = 0; k < T; ++k) {
    kahan_add(&Sr, jobs[k].re);
    kahan_add(&Si, jobs[k].im);
    a += jobs[k].acc;
  }
  *re = Sr.s;
  *im = Si.s;
  *acc = a;
  return 0;
}

/* per(A) (sparsepermanent): out [re hi, re lo, im hi, im lo]; terms = the
 * number of column sets enumerated (0 when a row is zero). */
int oracle_sparse_real(const double* A, int n, int ld, int cplx, int nthreads, double* out,
                       uint64_t* terms) {
  long double re, im;
  u128 acc;
  int rc = sparse_run(A, NULL, n, ld, cplx, 0, 0, -1, nthreads, &re, &im, &acc, terms);
  if (rc < 0) return -1;
  if (n & 1) {
    re = -re;
    im = -im;
  }
  ld_to_pair(re, out);
  ld_to_pair(im, out + 2);
  return 0;
}

int oracle_sparse_int(const uint8_t* B, int n, int ld, int nthreads, uint64_t* out,
                      uint64_t* terms) {
  long double re, im;
  u128 acc;
  int rc = sparse_run(NULL, B, n, ld, 0, 0, 0, -1, nthreads, &re, &im, &acc, terms);
  if (rc < 0) return -1;
  if (n & 1) acc = (u128)0 - acc;
  u128_to_pair(acc, out);
  return 0;
}

/* Raw sum (no (-1)^n) over Gray indices [g0, g0 + count) of the mixed-radix
 * order of the digits above. */
int oracle_sparse_range(const double* A, int n, int ld, int cplx, uint64_t g0, uint64_t count,
                        int nthreads, double* out) {
  long double re, im;
  u128 acc;
  uint64_t total;
  if (count > (uint64_t)INT64_MAX) return -1;
  int rc = sparse_run(A, NULL, n, ld, cplx, 1, g0, (int64_t)count, nthreads, &re, &im, &acc,
                      &total);
  if (rc != 0) return -1;
  ld_to_pair(re, out);
  ld_to_pair(im, out + 2);
  return 0;
}

/* 0/1 data: the raw sum (no (-1)^n) over Gray indices [g0, g0 + count) as an
 * integer modulo 2^128 (out[0] low word, out[1] high word). */
int oracle_sparse_range_int(const uint8_t* B, int n, int ld, uint64_t g0, uint64_t count,
                            int nthreads, uint64_t* out) {
  long double re, im;
  u128 acc;
  uint64_t total;
  if (count > (uint64_t)INT64_MAX) return -1;
  int rc = sparse_run(NULL, B, n, ld, 0, 1, g0, (int64_t)count, nthreads, &re, &im, &acc,
                      &total);
  if (rc != 0) return -1;
  u128_to_pair(acc, out);
  return 0;
}

/* The partition: block_of_col[j] = block index (selection order) or -1 for
 * T; returns the number of blocks, or -1 (bad arguments / a zero row). */
int oracle_sparse_partition(const double* A, int n, int ld, int cplx, int* block_of_col) {
  if (n < 1 || n > ORACLE_MAX_N || ld < n) return -1;
  sparse_part P;
  memset(&P, 0, sizeof P);
  if (!greedy_partition(A, NULL, n, ld, cplx, &P)) return -1;
  for (int j = 0; j < n; ++j) block_of_col[j] = -1;
  for (int l = 0; l < P.nblocks; ++l)
    for (int e = 0; e < P.block_size[l]; ++e) block_of_col[P.cols[P.block_first[l] + e]] = l;
  return P.nblocks;
}

/* Column set (bit mask) of Gray index g, for tests of the order. */
int oracle_sparse_set(const double* A, int n, int ld, int cplx, uint64_t g, uint64_t* J) {
  if (n < 1 || n > ORACLE_MAX_N || ld < n) return -1;
  sparse_part P;
  memset(&P, 0, sizeof P);
  if (!greedy_partition(A, NULL, n, ld, cplx, &P)) return -1;
  uint64_t radix[ORACLE_MAX_N], Q[ORACLE_MAX_N];
  int R, f[ORACLE_MAX_N];
  sparse_radices(&P, radix, &R);
  u128 t = 1;
  for (int d = 0; d < R; ++d) {
    Q[d] = (uint64_t)t;
    t *= radix[d];
    if (t > ((u128)1 << 63)) return -1;
  }
  if ((u128)g >= t) return -1;
  mixed_gray_unrank(g, R, Q, f);
  *J = sparse_set(&P, f);
  return 0;
}

/* Number of worker threads a call with nthreads <= 0 would use. */
int oracle_default_threads(void) { return pick_threads(0, ~0ull); }
