// Chunk walks of the half-range Gray-code sum (App. A, subpermanent),
// shared by the single-matrix kernels and the batched persistent kernel.
//
// One lane walks one chunk of L = 2^b consecutive Gray terms starting at
// G*L.  Terms are taken in pairs: term 2t has sign -1 and term 2t+1 sign +1
// (App. A: term g carries (-1)^(g+1), and g has the parity of the step
// because chunks start at multiples of L), and the flip between them is
// always column 0.  The last pair has no flip after it (a flip past the end
// of the chunk would be wasted).  Chunks of one term (b = 0) use the
// single_term functions instead.
//
// MODE 0: FP64 products, double-double lane sum (default)
// MODE 1: FP64 products, plain FP64 lane sum
// MODE 2: FP32 products of the FP64 row sums, double-double lane sum
#pragma once

#include "perm_device.hpp"

namespace perm {

template <int N, int MODE>
__device__ __forceinline__ double term_prod_real(const double (&w)[N]) {
  if constexpr (MODE == 2)
    return prod_f32<N>(w);
  else
    return prod_f64<N>(w);
}

template <int N>
__device__ __forceinline__ void add_col_real(double (&w)[N], const double* __restrict__ staged,
                                        uint32_t sub, int j) {
  cdptr col = as_const(staged + sub * (N * N) + j * N);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] += col[i];
}

template <int MODE>
__device__ __forceinline__ void lane_acc(dd& acc, double q) {
  if constexpr (MODE == 1)
    acc.hi += q;
  else
    dd_acc(acc, q);
}

// The single term g, with its sign (-1)^(g+1).  Kept apart from the chunk
// walk: sharing its first product with the pair loop lets the compiler hoist
// it and keep two copies of the row sums live.
template <int N, int MODE>
__device__ __forceinline__ dd single_term_real(const double* __restrict__ staged, uint64_t g) {
  staged = opaque(staged);
  double w[N];
  form_w_real<N>(staged, g, w);
  const double p = term_prod_real<N, MODE>(w);
  return dd{(g & 1) ? p : -p, 0.0};
}

// Signed sum of the 2^b terms of an aligned chunk whose start row sums are w
// (b >= 1); w ends as the row sums of the chunk's last term.
template <int N, int MODE>
__device__ __forceinline__ dd walk_pairs_real(const double* __restrict__ staged, double (&w)[N],
                                              int b, uint32_t gpar) {
  dd acc{0.0, 0.0};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  // All pairs but the last: both flips (column 0, then column ctz(2t+2)).
  for (; t + 1 < half; ++t) {
    const double p0 = term_prod_real<N, MODE>(w);
    add_col_real<N>(w, staged, t & 1u, 0);
    const double p1 = term_prod_real<N, MODE>(w);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    add_col_real<N>(w, staged, flip_subtracts(s1, j, b, gpar), j);
    lane_acc<MODE>(acc, p1 - p0);
  }
  // Last pair: no flip after the chunk's last term.
  {
    const double p0 = term_prod_real<N, MODE>(w);
    add_col_real<N>(w, staged, (b >= 2) ? (t & 1u) : gpar, 0);
    const double p1 = term_prod_real<N, MODE>(w);
    lane_acc<MODE>(acc, p1 - p0);
  }
  return acc;
}

// Signed sum of the terms of chunk G (Gray indices [G*L, (G+1)*L)), b >= 1.
template <int N, int MODE, bool DRIFT>
__device__ __forceinline__ dd walk_chunk_real(const double* __restrict__ staged,
                                         const double* __restrict__ rowabs, uint64_t G, int b,
                                         uint32_t gpar, double& drift) {
  staged = opaque(staged);
  double w[N];
  form_w_real<N>(staged, G << b, w);
  const dd acc = walk_pairs_real<N, MODE>(staged, w, b, gpar);
  if constexpr (DRIFT) {
    double f[N];
    form_w_real<N>(staged, ((G + 1) << b) - 1, f);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double s = rowabs[i];
      if (s > 0.0) drift = fmax(drift, fabs(w[i] - f[i]) / s);
    }
  }
  return acc;
}

template <int N, int MODE>
__device__ __forceinline__ void term_prod_complex(const double (&wr)[N], const double (&wi)[N],
                                          double& pr, double& pi) {
  if constexpr (MODE == 2)
    prod_c32<N>(wr, wi, pr, pi);
  else
    prod_c64<N>(wr, wi, pr, pi);
}

// Columns of this many rows or more are read in blocks of kColRows rows,
// block k only after block k-2 has been added (at most two blocks, 64 SGPRs,
// in flight).
constexpr int kColBlockedFrom = 49;
constexpr int kColRows = 8;

// Adds rows [0, ROWS) of column j (of +A or -A, by sub) of the staged n x n
// complex copy to the row sums.
template <int N, int ROWS>
__device__ __forceinline__ void add_col_complex(double (&wr)[ROWS], double (&wi)[ROWS],
                                        const double* __restrict__ staged, uint32_t sub, int j) {
  const double* base = staged + sub * (2 * N * N) + 2 * j * N;
  if constexpr (ROWS < kColBlockedFrom) {
    cdptr col = as_const(base);
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      wr[i] += col[2 * i];
      wi[i] += col[2 * i + 1];
    }
  } else {
#pragma unroll
    for (int r0 = 0; r0 < ROWS; r0 += kColRows) {
      const double* p = base + 2 * r0;
      if (r0 >= 2 * kColRows) p = after(p, wi[r0 - kColRows - 1]);
      cdptr col = as_const(p);
#pragma unroll
      for (int i = r0; i < r0 + kColRows && i < ROWS; ++i) {
        wr[i] += col[2 * (i - r0)];
        wi[i] += col[2 * (i - r0) + 1];
      }
    }
  }
}

struct cdd {
  dd re, im;
};

template <int N, int MODE>
__device__ __forceinline__ cdd single_term_complex(const double* __restrict__ staged, uint64_t g) {
  staged = opaque(staged);
  double wr[N], wi[N];
  form_w_complex<N>(staged, g, wr, wi);
  double pr, pi;
  term_prod_complex<N, MODE>(wr, wi, pr, pi);
  const bool pos = (g & 1) != 0;
  return cdd{{pos ? pr : -pr, 0.0}, {pos ? pi : -pi, 0.0}};
}

// Signed sums of the 2^b terms of an aligned chunk whose start row sums are
// (wr, wi) (b >= 1); they end as the row sums of the chunk's last term.
template <int N, int MODE>
__device__ __forceinline__ cdd walk_pairs_complex(const double* __restrict__ staged,
                                                  double (&wr)[N], double (&wi)[N], int b,
                                                  uint32_t gpar) {
  cdd acc{{0.0, 0.0}, {0.0, 0.0}};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    double p0r, p0i, p1r, p1i;
    term_prod_complex<N, MODE>(wr, wi, p0r, p0i);
    add_col_complex<N>(wr, wi, staged, t & 1u, 0);
    term_prod_complex<N, MODE>(wr, wi, p1r, p1i);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    add_col_complex<N>(wr, wi, staged, flip_subtracts(s1, j, b, gpar), j);
    lane_acc<MODE>(acc.re, p1r - p0r);
    lane_acc<MODE>(acc.im, p1i - p0i);
  }
  {
    double p0r, p0i, p1r, p1i;
    term_prod_complex<N, MODE>(wr, wi, p0r, p0i);
    add_col_complex<N>(wr, wi, staged, (b >= 2) ? (t & 1u) : gpar, 0);
    term_prod_complex<N, MODE>(wr, wi, p1r, p1i);
    lane_acc<MODE>(acc.re, p1r - p0r);
    lane_acc<MODE>(acc.im, p1i - p0i);
  }
  return acc;
}

// Signed sums of chunk G's terms, b >= 1.
template <int N, int MODE, bool DRIFT>
__device__ __forceinline__ cdd walk_chunk_complex(const double* __restrict__ staged,
                                          const double* __restrict__ rowabs, uint64_t G, int b,
                                          uint32_t gpar, double& drift) {
  staged = opaque(staged);
  double wr[N], wi[N];
  form_w_complex<N>(staged, G << b, wr, wi);
  const cdd acc = walk_pairs_complex<N, MODE>(staged, wr, wi, b, gpar);
  if constexpr (DRIFT) {
    double fr[N], fi[N];
    form_w_complex<N>(staged, ((G + 1) << b) - 1, fr, fi);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double s = rowabs[i];
      if (s > 0.0) drift = fmax(drift, hypot(wr[i] - fr[i], wi[i] - fi[i]) / s);
    }
  }
  return acc;
}

// Two aligned chunks Ga and Gb of 2^b terms with the same parity (gpar)
// walked in lockstep: they flip the same column in the same direction at
// every step, so every column read serves both.  Returns their sums apart.
template <int N, int MODE>
__device__ __forceinline__ void walk_chunks_complex_twin(const double* __restrict__ staged,
                                                        uint64_t Ga, uint64_t Gb, int b,
                                                        uint32_t gpar, cdd& acc_a, cdd& acc_b) {
  staged = opaque(staged);
  double ar[N], ai[N], br[N], bi[N];
  form_w_complex<N>(staged, Ga << b, ar, ai);
  form_w_complex<N>(opaque(staged), Gb << b, br, bi);
  acc_a = cdd{{0.0, 0.0}, {0.0, 0.0}};
  acc_b = cdd{{0.0, 0.0}, {0.0, 0.0}};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    double pa0r, pa0i, pa1r, pa1i, pb0r, pb0i, pb1r, pb1i;
    term_prod_complex<N, MODE>(ar, ai, pa0r, pa0i);
    term_prod_complex<N, MODE>(br, bi, pb0r, pb0i);
    add_col_complex<N>(ar, ai, staged, t & 1u, 0);
    add_col_complex<N>(br, bi, staged, t & 1u, 0);
    term_prod_complex<N, MODE>(ar, ai, pa1r, pa1i);
    term_prod_complex<N, MODE>(br, bi, pb1r, pb1i);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    const uint32_t sub = flip_subtracts(s1, j, b, gpar);
    add_col_complex<N>(ar, ai, staged, sub, j);
    add_col_complex<N>(br, bi, staged, sub, j);
    lane_acc<MODE>(acc_a.re, pa1r - pa0r);
    lane_acc<MODE>(acc_a.im, pa1i - pa0i);
    lane_acc<MODE>(acc_b.re, pb1r - pb0r);
    lane_acc<MODE>(acc_b.im, pb1i - pb0i);
  }
  {
    const uint32_t sub0 = (b >= 2) ? (t & 1u) : gpar;
    double pa0r, pa0i, pa1r, pa1i, pb0r, pb0i, pb1r, pb1i;
    term_prod_complex<N, MODE>(ar, ai, pa0r, pa0i);
    term_prod_complex<N, MODE>(br, bi, pb0r, pb0i);
    add_col_complex<N>(ar, ai, staged, sub0, 0);
    add_col_complex<N>(br, bi, staged, sub0, 0);
    term_prod_complex<N, MODE>(ar, ai, pa1r, pa1i);
    term_prod_complex<N, MODE>(br, bi, pb1r, pb1i);
    lane_acc<MODE>(acc_a.re, pa1r - pa0r);
    lane_acc<MODE>(acc_a.im, pa1i - pa0i);
    lane_acc<MODE>(acc_b.re, pb1r - pb0r);
    lane_acc<MODE>(acc_b.im, pb1i - pb0i);
  }
}

// ------------------------------------------------- rows kept in LDS ----
// Above n = 48 the complex row sums alone (4n VGPRs) leave room for one wave
// per SIMD, which cannot hide the latency of the scalar column loads and of
// the FP64 chains.  The split walk keeps rows [0, R) in VGPRs and rows
// [R, n) in LDS: one 16-byte slot per row and lane, row r of a wave's 64
// lanes 1 KB contiguous (conflict-free).  In each pair an LDS row is read
// once, multiplied into the products of both terms (before and after the
// column-0 flip), takes the second flip and is written back: two LDS
// accesses per LDS row and pair, each row's read issued while the row before
// it is being used.  The VALU work is the same as in the register walk (the
// two terms' products are split into the register rows' and the LDS rows'
// and joined by one complex multiply each), the register rows' columns are
// read as whole columns are up to n = 48, and the kernel runs two waves per
// SIMD.  46 register rows measured faster than fewer; at n = 49..52 the
// optimiser keeps the few LDS rows in VGPRs across the pair loop, which also
// measured faster than forcing their LDS accesses.
constexpr int kSplitFrom = kColBlockedFrom;
constexpr int kSplitRegRows = 46;

template <int N>
struct SplitRows {
  static constexpr int R = N >= kSplitFrom ? kSplitRegRows : N;  // rows in VGPRs
  static constexpr int L = N - R;                                // rows in LDS
};

// This lane's LDS slots: row r at [r * kWave].
template <int L>
__device__ __forceinline__ double2* lane_rows() {
  __shared__ double2 s_rows[kWavesPerBlock * L * kWave];
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  return s_rows + wave * L * kWave + lane;
}

// (pr, pi) *= (xr, xi) in the product precision of MODE.
template <int MODE>
__device__ __forceinline__ void cmul_acc(double& pr, double& pi, double xr, double xi) {
  if constexpr (MODE == 2) {
    const float ar = (float)pr, ai = (float)pi, br = (float)xr, bi = (float)xi;
    const float t = ai * bi, u = ai * br;
    pr = (double)fmaf(ar, br, -t);
    pi = (double)fmaf(ar, bi, u);
  } else {
    const double t = pi * xi, u = pi * xr;
    const double nr = fma(pr, xr, -t);
    const double ni = fma(pr, xi, u);
    pr = nr;
    pi = ni;
  }
}

// Chunk start of the split walk: rows [0, R) into registers, rows [R, N)
// into the lane's LDS slots (App. A, subpermanent, as form_w_complex).
template <int N, int R>
__device__ __forceinline__ void form_w_complex_split(const double* __restrict__ staged, uint64_t g,
                                                     double (&wr)[R], double (&wi)[R],
                                                     double2* __restrict__ rows) {
  const uint64_t x = gray(g);
  {
    cdptr last = as_const(staged + 2 * (N - 1) * N);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      wr[i] = last[2 * i];
      wi[i] = last[2 * i + 1];
    }
#pragma unroll 1
    for (int j = 0; j < N - 1; ++j) {
      const double d = ((x >> j) & 1) ? 1.0 : -1.0;
      cdptr col = as_const(staged + 2 * j * N);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        wr[i] = fma(d, col[2 * i], wr[i]);
        wi[i] = fma(d, col[2 * i + 1], wi[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      wr[i] *= 0.5;
      wi[i] *= 0.5;
    }
  }
  constexpr int kB = 4;
#pragma unroll
  for (int r0 = R; r0 < N; r0 += kB) {
    const double* base = opaque(staged);
    double vr[kB], vi[kB];
    cdptr last = as_const(base + 2 * (N - 1) * N + 2 * r0);
#pragma unroll
    for (int k = 0; k < kB; ++k)
      if (r0 + k < N) {
        vr[k] = last[2 * k];
        vi[k] = last[2 * k + 1];
      }
#pragma unroll 1
    for (int j = 0; j < N - 1; ++j) {
      const double d = ((x >> j) & 1) ? 1.0 : -1.0;
      cdptr col = as_const(base + 2 * j * N + 2 * r0);
#pragma unroll
      for (int k = 0; k < kB; ++k)
        if (r0 + k < N) {
          vr[k] = fma(d, col[2 * k], vr[k]);
          vi[k] = fma(d, col[2 * k + 1], vi[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < kB; ++k)
      if (r0 + k < N) rows[(r0 - R + k) * kWave] = double2{0.5 * vr[k], 0.5 * vi[k]};
  }
}

// The LDS rows' share of one pair: q0 = product of the rows before the first
// flip (the column at c0), q1 = after it; with UPDATE the rows then take the
// second flip (the column at c1) and are stored back.  c0 and c1 point at row
// R of their (interleaved complex) columns; c1 is not read without UPDATE.
template <int N, int R, int MODE, bool UPDATE>
__device__ __forceinline__ void lds_rows_pair(double2* __restrict__ rows,
                                              const double* __restrict__ c0,
                                              const double* __restrict__ c1, double& q0r,
                                              double& q0i, double& q1r, double& q1i) {
  constexpr int L = N - R;
  double tie[L];
  double2 next = rows[0];  // each row's read is issued one row ahead
#pragma unroll
  for (int r0 = 0; r0 < L; r0 += kColRows) {
    const double* p0 = c0 + 2 * r0;
    const double* p1 = c1 + 2 * r0;
    if (r0 >= 2 * kColRows) {
      p0 = after(p0, tie[r0 - kColRows - 1]);
      p1 = after(p1, tie[r0 - kColRows - 1]);
    }
    cdptr a0 = as_const(p0);
    cdptr a1 = as_const(p1);
#pragma unroll
    for (int r = r0; r < r0 + kColRows && r < L; ++r) {
      double2 v = next;
      if (r + 1 < L) next = rows[(r + 1) * kWave];
      if (r == 0) {
        q0r = v.x;
        q0i = v.y;
      } else {
        cmul_acc<MODE>(q0r, q0i, v.x, v.y);
      }
      v.x += a0[2 * (r - r0)];
      v.y += a0[2 * (r - r0) + 1];
      if (r == 0) {
        q1r = v.x;
        q1i = v.y;
      } else {
        cmul_acc<MODE>(q1r, q1i, v.x, v.y);
      }
      if constexpr (UPDATE) {
        v.x += a1[2 * (r - r0)];
        v.y += a1[2 * (r - r0) + 1];
        rows[r * kWave] = v;
      }
      tie[r] = v.y;
    }
  }
}

// Signed sums of chunk G's terms with rows [R, N) in LDS (b >= 1).
template <int N, int MODE>
__device__ __forceinline__ cdd walk_chunk_complex_split(const double* __restrict__ staged,
                                                        uint64_t G, int b, uint32_t gpar,
                                                        double2* __restrict__ rows) {
  constexpr int R = SplitRows<N>::R;
  staged = opaque(staged);
  double wr[R], wi[R];
  form_w_complex_split<N, R>(staged, G << b, wr, wi, rows);
  cdd acc{{0.0, 0.0}, {0.0, 0.0}};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    const uint32_t subj = flip_subtracts(s1, j, b, gpar);
    double q0r, q0i, q1r, q1i, p0r, p0i, p1r, p1i;
    lds_rows_pair<N, R, MODE, true>(rows, staged + (t & 1u) * (2 * N * N) + 2 * R,
                                    staged + subj * (2 * N * N) + 2 * j * N + 2 * R, q0r, q0i,
                                    q1r, q1i);
    term_prod_complex<R, MODE>(wr, wi, p0r, p0i);
    add_col_complex<N>(wr, wi, staged, t & 1u, 0);
    term_prod_complex<R, MODE>(wr, wi, p1r, p1i);
    add_col_complex<N>(wr, wi, staged, subj, j);
    cmul_acc<MODE>(p0r, p0i, q0r, q0i);
    cmul_acc<MODE>(p1r, p1i, q1r, q1i);
    lane_acc<MODE>(acc.re, p1r - p0r);
    lane_acc<MODE>(acc.im, p1i - p0i);
  }
  {
    const uint32_t sub0 = (b >= 2) ? (t & 1u) : gpar;
    double q0r, q0i, q1r, q1i, p0r, p0i, p1r, p1i;
    const double* c0 = staged + sub0 * (2 * N * N) + 2 * R;
    lds_rows_pair<N, R, MODE, false>(rows, c0, c0, q0r, q0i, q1r, q1i);
    term_prod_complex<R, MODE>(wr, wi, p0r, p0i);
    add_col_complex<N>(wr, wi, staged, sub0, 0);
    term_prod_complex<R, MODE>(wr, wi, p1r, p1i);
    cmul_acc<MODE>(p0r, p0i, q0r, q0i);
    cmul_acc<MODE>(p1r, p1i, q1r, q1i);
    lane_acc<MODE>(acc.re, p1r - p0r);
    lane_acc<MODE>(acc.im, p1i - p0i);
  }
  return acc;
}

}  // namespace perm
