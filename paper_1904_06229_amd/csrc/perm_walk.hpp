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

// Signed sum of the terms of chunk G (Gray indices [G*L, (G+1)*L)), b >= 1.
template <int N, int MODE, bool DRIFT>
__device__ __forceinline__ dd walk_chunk_real(const double* __restrict__ staged,
                                         const double* __restrict__ rowabs, uint64_t G, int b,
                                         uint32_t gpar, double& drift) {
  staged = opaque(staged);
  double w[N];
  form_w_real<N>(staged, G << b, w);
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

// Sizes above this read a complex column in blocks of kColRows rows, block k
// only after block k-2 has been added (at most two blocks, 64 SGPRs, in flight).
constexpr int kColBlockedFrom = 49;
constexpr int kColRows = 8;

template <int N>
__device__ __forceinline__ void add_col_complex(double (&wr)[N], double (&wi)[N],
                                        const double* __restrict__ staged, uint32_t sub, int j) {
  const double* base = staged + sub * (2 * N * N) + 2 * j * N;
  if constexpr (N < kColBlockedFrom) {
    cdptr col = as_const(base);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      wr[i] += col[2 * i];
      wi[i] += col[2 * i + 1];
    }
  } else {
#pragma unroll
    for (int r0 = 0; r0 < N; r0 += kColRows) {
      const double* p = base + 2 * r0;
      if (r0 >= 2 * kColRows) p = after(p, wi[r0 - kColRows - 1]);
      cdptr col = as_const(p);
#pragma unroll
      for (int i = r0; i < r0 + kColRows && i < N; ++i) {
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

// Signed sums of chunk G's terms, b >= 1.
template <int N, int MODE, bool DRIFT>
__device__ __forceinline__ cdd walk_chunk_complex(const double* __restrict__ staged,
                                          const double* __restrict__ rowabs, uint64_t G, int b,
                                          uint32_t gpar, double& drift) {
  staged = opaque(staged);
  double wr[N], wi[N];
  form_w_complex<N>(staged, G << b, wr, wi);
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

}  // namespace perm
