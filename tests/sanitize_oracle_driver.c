/*
 * Test driver for the oracle under AddressSanitizer/UBSan or ThreadSanitizer
 * (built and run by tests/test_oracle_sanitizers.py; CPU only).  It calls every
 * route of the oracle on small random inputs, with several threads, and checks
 * that the routes agree: exactly for 0/1 matrices (all integer routes modulo
 * 2^128), to 1e-9 relative for real and complex ones.  Exit status 0 = pass.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

int oracle_brute_real(const double* A, int n, int ld, double* out);
int oracle_brute_complex(const double* A, int n, int ld, double* out);
int oracle_brute_int(const uint8_t* B, int n, int ld, uint64_t* out);
int oracle_ryser_real(const double* A, int n, int ld, int nthreads, double* out);
int oracle_ryser_complex(const double* A, int n, int ld, int nthreads, double* out);
int oracle_ryser_int(const uint8_t* B, int n, int ld, int nthreads, uint64_t* out);
int oracle_chunk_int(const uint8_t* B, int n, int ld, uint64_t g0, uint64_t count, int nthreads,
                     uint64_t* out);
int oracle_chunk_real(const double* A, int n, int ld, uint64_t g0, uint64_t count, int nthreads,
                      double* out);
int oracle_sparse_int(const uint8_t* B, int n, int ld, int nthreads, uint64_t* out,
                      uint64_t* terms);
int oracle_sparse_range_int(const uint8_t* B, int n, int ld, uint64_t g0, uint64_t count,
                            int nthreads, uint64_t* out);
int oracle_band_int(const uint8_t* B, int n, int ld, int k, uint64_t* out);
int oracle_band_real(const double* A, int n, int ld, int k, int cplx, double* out);
int oracle_ryser2(const double* C, int n, int R, int ld, const int* m, int cplx, int nthreads,
                  double* out);

static uint64_t state = 20190409u;
static uint64_t next_u64(void) {  /* splitmix64 */
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static u128 words(const uint64_t* w) { return ((u128)w[1] << 64) | w[0]; }

static int fails = 0;
static void check(int ok, const char* what, int n) {
  if (!ok) {
    fprintf(stderr, "FAIL %s at n = %d\n", what, n);
    ++fails;
  }
}

static int close_rel(double a, double b) { return fabs(a - b) <= 1e-9 * fmax(1.0, fabs(b)); }

int main(void) {
  enum { T = 4 };  /* threads for the threaded routes */
  for (int n = 1; n <= 9; ++n) {
    uint8_t B[81];
    double A[81], Z[162];
    for (int t = 0; t < n * n; ++t) {
      B[t] = next_u64() % 3 != 0;
      A[t] = 2.0 * uniform() - 1.0;
      Z[2 * t] = 2.0 * uniform() - 1.0;
      Z[2 * t + 1] = 2.0 * uniform() - 1.0;
    }
    uint64_t w[2], v[2], terms = 0;
    /* 0/1: every integer route, exactly */
    if (oracle_brute_int(B, n, n, w)) return 2;
    const u128 per = words(w);
    if (oracle_ryser_int(B, n, n, T, v)) return 2;
    check(words(v) == per, "ryser_int vs brute_int", n);
    if (oracle_chunk_int(B, n, n, 0, 1ull << (n - 1), T, v)) return 2;
    {  /* sum_g (-1)^(g+1) prod r_i = (-1)^n 2^(n-1) per */
      u128 want = per << (n - 1);
      if (n & 1) want = (u128)0 - want;
      check(words(v) == want, "chunk_int vs brute_int", n);
    }
    if (oracle_sparse_int(B, n, n, T, v, &terms) == 0)
      check(words(v) == per, "sparse_int vs brute_int", n);
    if (terms > 0 && oracle_sparse_range_int(B, n, n, 0, terms, T, v) == 0) {
      u128 want = (n & 1) ? (u128)0 - per : per;
      check(words(v) == want, "sparse_range_int vs brute_int", n);
    }
    if (oracle_band_int(B, n, n, n - 1 < 9 ? n - 1 : 9, v)) return 2;
    check(words(v) == per, "band_int (full band) vs brute_int", n);
    /* real and complex: brute force against Ryser and the other routes */
    double r1[4], r2[4];
    if (oracle_brute_real(A, n, n, r1) || oracle_ryser_real(A, n, n, T, r2)) return 2;
    check(close_rel(r1[0] + r1[1], r2[0] + r2[1]), "ryser_real vs brute_real", n);
    if (oracle_chunk_real(A, n, n, 0, 1ull << (n - 1), T, r2)) return 2;
    check(close_rel(2.0 * ((n & 1) ? -1.0 : 1.0) * (r2[0] + r2[1]), r1[0] + r1[1]),
          "chunk_real vs brute_real", n);
    if (oracle_band_real(A, n, n, n - 1 < 9 ? n - 1 : 9, 0, r2)) return 2;
    check(close_rel(r2[0] + r2[1], r1[0] + r1[1]), "band_real vs brute_real", n);
    if (oracle_brute_complex(Z, n, n, r1) || oracle_ryser_complex(Z, n, n, T, r2)) return 2;
    check(close_rel(r1[0] + r1[1], r2[0] + r2[1]) && close_rel(r1[2] + r1[3], r2[2] + r2[3]),
          "ryser_complex vs brute_complex", n);
    /* Eq. ryser2 with every multiplicity 1 is plain Ryser */
    {
      int m[9];
      for (int k = 0; k < n; ++k) m[k] = 1;
      if (oracle_ryser2(A, n, n, n, m, 0, T, r2)) return 2;
      if (oracle_brute_real(A, n, n, r1)) return 2;
      check(close_rel(r2[0] + r2[1], r1[0] + r1[1]), "ryser2 (m = 1) vs brute_real", n);
    }
  }
  if (fails) return 1;
  puts("oracle sanitizer driver: all routes agree");
  return 0;
}
