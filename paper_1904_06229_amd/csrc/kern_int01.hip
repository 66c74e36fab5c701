// Exact Gray-code walk for 0/1 matrices.
//
// The walk keeps r_i = 2 w_i (App. A, subpermanent), which for a 0/1 matrix
// is an integer with |r_i| <= d_i <= n (d_i = row sum), and accumulates
// sum_g (-1)^(g+1) prod_i r_i = (-1)^n 2^(n-1) per(A) exactly modulo 2^128.
//
// Exact arithmetic on a VALU whose fast integer multiplier is 24 bits wide:
//   * r_i are carried in FP64 registers (exact: small integers); the update
//     r += (+/-)2 a_ij is a v_add_f64 with an SGPR operand, as in the real walk.
//   * Rows are multiplied in groups of k = int01_group_rows(n) rows with
//     n^k < 2^50, so every group product G is an exact FP64 integer.
//   * Group products are combined with error-free transformations: TwoProduct
//     (h = G1*G2, l = fma(G1, G2, -h), G1*G2 = h + l exactly) and an exact
//     split at 2^51 (q = h + 1.5*2^103 rounds h to a multiple of 2^51; then
//     h - (q - 1.5*2^103) is exact, and the bit pattern of q minus that of
//     1.5*2^103 is h's high part as an integer).  The product is carried as
//     integer limbs of weight 1, 2^51, 2^102 held in doubles.
//   * Limbs land in three 64-bit integer bins through their bit patterns:
//     for |y| <= 2^51, bits(y + 1.5*2^52) - bits(1.5*2^52) = y.  The two terms
//     of a pair enter with opposite signs, so the constant offsets cancel and
//     only add/sub of bit patterns remains in the loop.
//   * Bins are folded into a 128-bit sum at the end of every chunk (chunks are
//     at most 2^10 terms, so the weight-1 and weight-2^51 bins cannot wrap).
#include "perm_device.hpp"
#include "perm_exact.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

using namespace exact;

template <int N>
__device__ __forceinline__ void add_col(double (&w)[N], const double* __restrict__ staged,
                                        uint32_t sub, int j) {
  cdptr col = as_const(staged + sub * (N * N) + j * N);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] += col[i];
}

// Integer form of the single term g, (-1)^(g+1) prod_i r_i, modulo 2^128.
// Kept apart from the chunk walk (see single_term_real).
template <int N>
__device__ __forceinline__ u128 single_term(const double* __restrict__ staged, uint64_t g) {
  staged = opaque(staged);
  double r[N];
  form_w_real<N>(staged, g, r);
  Bins B{0, 0, 0};
  const Bins off = term_offsets<N>();
  if (g & 1) {
    term_bins<N, true>(r, B);
    B.b0 -= off.b0;
    B.b1 -= off.b1;
    B.b2 -= off.b2;
  } else {
    term_bins<N, false>(r, B);
    B.b0 += off.b0;
    B.b1 += off.b1;
    B.b2 += off.b2;
  }
  return fold(B);
}

// Integer-form sum of chunk G's terms (b >= 1), modulo 2^128.
template <int N, bool DRIFT>
__device__ __forceinline__ u128 walk_chunk(const double* __restrict__ staged, uint64_t G, int b,
                                           uint32_t gpar, double& drift) {
  staged = opaque(staged);
  double r[N];
  form_w_real<N>(staged, G << b, r);  // staged holds +2A/-2A, so this is r = 2w
  Bins B{0, 0, 0};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    term_bins<N, false>(r, B);
    add_col<N>(r, staged, t & 1u, 0);
    term_bins<N, true>(r, B);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    add_col<N>(r, staged, flip_subtracts(s1, j, b, gpar), j);
  }
  term_bins<N, false>(r, B);
  add_col<N>(r, staged, (b >= 2) ? (t & 1u) : gpar, 0);
  term_bins<N, true>(r, B);
  if constexpr (DRIFT) {
    // The integer walk cannot drift; the check confirms it.
    double f[N];
    form_w_real<N>(staged, ((G + 1) << b) - 1, f);
#pragma unroll
    for (int i = 0; i < N; ++i) drift = fmax(drift, fabs(r[i] - f[i]));
  }
  return fold(B);
}

// ----------------------------------------------------------- pair-shared ----
// For a 0/1 matrix staged with its sparsest column first (column 0, the one
// flipped between the two terms of every pair) and that column's m nonzero
// rows on top, rows M..N-1 (M = N/3 >= m) do not change between the terms of
// a pair.  With S their product and D0, D1 the products of rows 0..M-1 before
// and after the flip, the pair contributes P1 - P0 = S (D1 - D0): S and the
// exact combination are formed once per pair instead of twice, and the
// column-0 update touches M rows instead of N.  The staging kernel checks
// that m <= M and that the degrees of rows 0..M-1 multiply to less than 2^50
// (so D0, D1 and D1 - D0 are exact); otherwise this variant does nothing and
// the plain walk runs.
template <int N>
constexpr int pair_rows() {
  return N / 3;
}

template <int N, int M, int KS>
__device__ __forceinline__ void pair_bins(double (&r)[N], const double* __restrict__ staged,
                                          uint32_t sub0, Bins& B) {
  constexpr int k = int01_group_rows(N);
  double G[KS + 1];
#pragma unroll
  for (int g = 0; g < KS; ++g) {
    const int lo = M + g * k;
    double p = r[lo];
#pragma unroll
    for (int i = lo + 1; i < lo + k && i < N; ++i) p *= r[i];
    G[g] = p;
  }
  const double D0 = rows_prod<N, 0, M>(r);
  cdptr col = as_const(staged + sub0 * (N * N));  // column 0; zero below row M
#pragma unroll
  for (int i = 0; i < M; ++i) r[i] += col[i];
  const double D1 = rows_prod<N, 0, M>(r);
  G[KS] = D1 - D0;
  product_bins<KS + 1, true>(G, B);
}

template <int N>
__device__ __forceinline__ u128 walk_chunk_pairs(const double* __restrict__ staged, uint64_t G,
                                                 int b, uint32_t gpar) {
  constexpr int M = pair_rows<N>();
  constexpr int k = int01_group_rows(N);
  constexpr int KS = (N - M + k - 1) / k;
  staged = opaque(staged);
  double r[N];
  form_w_real<N>(staged, G << b, r);
  Bins B{0, 0, 0};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    pair_bins<N, M, KS>(r, staged, t & 1u, B);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    add_col<N>(r, staged, flip_subtracts(s1, j, b, gpar), j);
  }
  pair_bins<N, M, KS>(r, staged, (b >= 2) ? (t & 1u) : gpar, B);
  // every pair entered its bit patterns with a + sign: remove the offsets
  const Bins off = product_offsets<KS + 1>();
  B.b0 -= (uint64_t)half * off.b0;
  B.b1 -= (uint64_t)half * off.b1;
  B.b2 -= (uint64_t)half * off.b2;
  return fold(B);
}

// ---------------------------------------------------------- banded ----
// Column 1 is flipped after every other pair (the flip after pair t is column
// ctz(2t + 2)).  The staging kernel places after group D (rows 0..M-1) the
// rows with a one in column 1 and pads them to E = (N - M) / 2 rows (group
// E); the remaining rows S' have zeros in columns 0 and 1.  In a quad of
// pairs (2u, 2u + 1) S' is therefore unchanged: its product is formed once per
// quad, and the column-1 flip between the two pairs touches rows 0..M+E-1
// only.  Each pair contributes S' E (D1 - D0), the three factors exact below
// 2^50 (the staging kernel checks the degree products of E and S') and
// combined into the bins as in the pair-shared walk.
template <int N>
constexpr int band_rows() {
  return (N - pair_rows<N>()) / 2;
}

template <int N, int M, int E>
__device__ __forceinline__ void band_pair(double (&r)[N], const double* __restrict__ staged,
                                          uint32_t sub0, double gs, Bins& B) {
  double G[3];
  G[0] = gs;
  G[1] = rows_prod<N, M, M + E>(r);
  const double D0 = rows_prod<N, 0, M>(r);
  cdptr col = as_const(staged + sub0 * (N * N));  // column 0; zero below row M
#pragma unroll
  for (int i = 0; i < M; ++i) r[i] += col[i];
  const double D1 = rows_prod<N, 0, M>(r);
  G[2] = D1 - D0;
  product_bins<3, true>(G, B);
}

// Rows 0..ROWS-1 of column j (the rows below have zeros there).
template <int N, int ROWS>
__device__ __forceinline__ void add_col_rows(double (&r)[N], const double* __restrict__ staged,
                                             uint32_t sub, int j) {
  cdptr col = as_const(staged + sub * (N * N) + j * N);
#pragma unroll
  for (int i = 0; i < ROWS; ++i) r[i] += col[i];
}

// Chunk G (b >= 2: whole quads; in a quad the column-0 flip of the first pair
// adds the column and that of the second subtracts it, as t & 1 says for
// pairs t = 2u and 2u + 1).
template <int N>
__device__ __forceinline__ u128 walk_chunk_band(const double* __restrict__ staged, uint64_t G,
                                                int b, uint32_t gpar) {
  constexpr int M = pair_rows<N>();
  constexpr int E = band_rows<N>();
  constexpr int S0 = M + E;
  staged = opaque(staged);
  double r[N];
  form_w_real<N>(staged, G << b, r);
  Bins B{0, 0, 0};
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 2 < half; t += 2) {
    const double gs = rows_prod<N, S0, N>(r);
    band_pair<N, M, E>(r, staged, 0u, gs, B);
    add_col_rows<N, S0>(r, staged, flip_subtracts(2 * t + 2, 1, b, gpar), 1);
    band_pair<N, M, E>(r, staged, 1u, gs, B);
    const uint32_t s1 = 2 * t + 4;
    const int j = __builtin_ctz(s1);
    add_col<N>(r, staged, flip_subtracts(s1, j, b, gpar), j);
  }
  {  // last quad: no flip after it
    const double gs = rows_prod<N, S0, N>(r);
    band_pair<N, M, E>(r, staged, 0u, gs, B);
    add_col_rows<N, S0>(r, staged, flip_subtracts(2 * t + 2, 1, b, gpar), 1);
    band_pair<N, M, E>(r, staged, 1u, gs, B);
  }
  // every pair entered its bit patterns with a + sign: remove the offsets
  const Bins off = product_offsets<3>();
  B.b0 -= (uint64_t)half * off.b0;
  B.b1 -= (uint64_t)half * off.b1;
  B.b2 -= (uint64_t)half * off.b2;
  return fold(B);
}

// VARIANT 0: plain walk; VARIANT 1: by status[1] (set by the staging
// kernel), the banded walk (2, chunks of at least 4 terms), the pair-shared
// walk (1, or 2 with 2-term chunks) or the plain walk -- one launch,
// wave-uniform branches.
template <int N, bool DRIFT, bool SINGLE, int VARIANT>
__global__ __launch_bounds__(kBlock) void walk_int01_kernel(WalkArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  u128 acc{0, 0};
  double drift = 0.0;
  if (a.status[0] == kStOk) {
    const int pv = VARIANT == 1 ? a.status[1] : 0;
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      const uint32_t gpar = (uint32_t)((a.first + (task & 1)) & 1);
      double dr = 0.0;
      u128 part;
      if constexpr (SINGLE) {
        part = single_term<N>(a.staged, a.first + c);
      } else if constexpr (VARIANT == 1) {
        if (pv == 2 && a.b >= 2)
          part = walk_chunk_band<N>(a.staged, a.first + c, a.b, gpar);
        else if (pv >= 1)
          part = walk_chunk_pairs<N>(a.staged, a.first + c, a.b, gpar);
        else
          part = walk_chunk<N, DRIFT>(a.staged, a.first + c, a.b, gpar, dr);
      } else {
        part = walk_chunk<N, DRIFT>(a.staged, a.first + c, a.b, gpar, dr);
      }
      if (c < a.nchunks) {
        acc = u128_add(acc, part);
        drift = fmax(drift, dr);
      }
    }
  }
  const u128 v = wave_sum(acc);
  const u128 blk = block_sum(v, u128_add);
  uint64_t* out = (uint64_t*)a.partials;
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = blk.lo;
    out[2 * blockIdx.x + 1] = blk.hi;
  }
  // drift-checked calls: every launch writes its slot (the single-term launches
  // of unaligned range ends, which cannot drift, write 0)
  if (DRIFT || a.drift) {
    const double m = wave_max(drift);
    const double bm = block_sum(m, [](double x, double y) { return fmax(x, y); });
    if (threadIdx.x == 0) a.drift_part[blockIdx.x] = bm;
  }
}

template <int N>
hipError_t dispatch(bool drift, int variant, const WalkArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), blk(kBlock);
  if (variant == 1) {
    if constexpr (pair_rows<N>() >= kInt01PairMinRows) {
      if (a.b == 0 || drift) return hipErrorInvalidValue;
      hipLaunchKernelGGL((walk_int01_kernel<N, false, false, 1>), g, blk, 0, s, a);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (a.b == 0) {
    hipLaunchKernelGGL((walk_int01_kernel<N, false, true, 0>), g, blk, 0, s, a);
  } else if (drift) {
    hipLaunchKernelGGL((walk_int01_kernel<N, true, false, 0>), g, blk, 0, s, a);
  } else {
    hipLaunchKernelGGL((walk_int01_kernel<N, false, false, 0>), g, blk, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

#define PERM_CASE(N) \
  case N:            \
    return dispatch<N>(drift, variant, a, grid, s);

// Compiled twice: PERM_HALF = 0 instantiates n = 1..32, PERM_HALF = 1 n = 33..64
// (two translation units that build in parallel).
#if PERM_HALF == 0
#define PERM_LAUNCH launch_walk_int01_lo
#define PERM_CASES "perm_cases_lo.inc"
#else
#define PERM_LAUNCH launch_walk_int01_hi
#define PERM_CASES "perm_cases_hi.inc"
#endif

hipError_t PERM_LAUNCH(int n, bool drift, int variant, const WalkArgs& a, int grid,
                             hipStream_t s) {
  switch (n) {
#include PERM_CASES
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace perm
