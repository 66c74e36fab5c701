// Mixed-radix walk of Ryser-type sums: repeated columns (Sec. II.A,
// Eq. ryser2) and the restricted column sets of sparse matrices (App. B).
//
// Term of the digit vector f: prod_k omega_k(f_k) * prod_i w_i, where w_i is
// row i's sum over the term's columns (kind 0 digit: f_k copies of column
// c_k; kind 1 digit: the nonempty subset gray(f_k + 1) of its block) and
// omega_k(f_k) the digit value's signed weight ((-1)^f C(m, f), or
// (-1)^|subset|).  The vectors are taken in reflected mixed-radix Gray order,
// so from one term to the next one digit moves by one and w changes by one
// column: n additions per term, as in the binary walk of App. A.  One lane
// walks one chunk (a full run of the inner digits, L terms); the column added
// at step s and the inner weight come from the staged tables (wave-uniform:
// all chunks of a wave have the same parity), and the column is read with
// scalar loads.  The outer digits are formed afresh from the chunk index at
// every chunk start, so the walk's rounding does not carry over from chunk to
// chunk; their weight multiplies the chunk sum.
//
// Per term: n FP64 additions (complex 2n), the product of the row sums, one
// multiply by the inner weight, and a double-double lane sum per pair of terms.
//
// Exact variant (0/1 data of the sparse enumeration, whose digit weights are
// all +-1): the row sums are integers, every product is formed exactly in
// row groups and entered into 51-bit integer bins (perm_exact.hpp), and a
// chunk's bins fold into a 128-bit integer.  There the signs alternate from
// step to step, so a pair of terms enters as P_s - P_{s+1} and the chunk sum
// is multiplied by the sign of its first term at the end.
#include "perm_device.hpp"
#if PERM_CPLX
#include "perm_walk.hpp"
#else
#include "perm_exact.hpp"
#endif

namespace perm {
namespace {

typedef const __attribute__((address_space(4))) int32_t* ciptr;

#if PERM_CPLX
constexpr int kCw = 2;
#else
constexpr int kCw = 1;
#endif

struct Acc {
  dd re, im;
};

// Row sums of one term or chunk start.
template <int N>
struct Rows {
  double r[N];
#if PERM_CPLX
  double i[N];
#endif
};

template <int N>
__device__ __forceinline__ void add_col(Rows<N>& w, const double* staged, int32_t off) {
  cdptr col = as_const(staged + off);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    w.r[i] += col[kCw * i];
#if PERM_CPLX
    w.i[i] += col[kCw * i + 1];
#endif
  }
}

template <int N>
__device__ __forceinline__ void add_col_times(Rows<N>& w, const double* staged, int k,
                                              double f) {
  cdptr col = as_const(staged + kCw * k * N);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    w.r[i] = fma(f, col[kCw * i], w.r[i]);
#if PERM_CPLX
    w.i[i] = fma(f, col[kCw * i + 1], w.i[i]);
#endif
  }
}

template <int N>
__device__ __forceinline__ void product(const Rows<N>& w, double& pr, double& pi) {
#if PERM_CPLX
  prod_c64<N>(w.r, w.i, pr, pi);
#else
  pr = prod_f64<N>(w.r);
  pi = 0.0;
#endif
}

typedef const __attribute__((address_space(4))) uint64_t* cu64ptr;

// Columns c0 .. ncols-1 of the term with Gray index g (c0 = 0: all digits;
// c0 = the first column of digit b: the outer digits of a chunk starting at
// g): f_k = a_k or r_k - 1 - a_k by the parity of floor(g / Q_{k+1}) (a_k the
// counting digit), then each column adds its coefficient times itself to the
// row sums (kind 0: f copies; kind 1: bit e of gray(f + 1)) and the digit's
// first column multiplies the weight by omega_k(f_k).  One flat loop over
// columns keeps a single copy of the row sums live.  column_coef gives the
// coefficient of staged column c (and updates the weight).
__device__ __forceinline__ double column_coef(const MixArgs& a, uint64_t g, int c, double& W) {
  ciptr dig = (ciptr)a.dig;
  cu64ptr qabs = (cu64ptr)a.qabs;
  const int k = dig[kDigColDigit * kMaxN + c];
  const int e = dig[kDigColBit * kMaxN + c];
  const uint32_t r = (uint32_t)dig[kDigRadix * kMaxN + k];
  const uint64_t x = g / qabs[k];
  const uint64_t hi = x / r;
  const uint32_t dgt = (uint32_t)(x - hi * r);
  const uint32_t f = (hi & 1) ? r - 1u - dgt : dgt;
  if (e == 0) W *= a.omega[dig[kDigWofs * kMaxN + k] + f];
  const uint32_t sub = (f + 1u) ^ ((f + 1u) >> 1);
  return dig[kDigKind * kMaxN + k] == 0 ? (double)f : (double)((sub >> e) & 1u);
}

template <int N>
__device__ __forceinline__ void outer_digits(const MixArgs& a, const double* staged, uint64_t g,
                                             int c0, Rows<N>& w, double& W) {
#pragma unroll 1
  for (int c = c0; c < a.ncols; ++c) add_col_times<N>(w, staged, c, column_coef(a, g, c, W));
}

// Exact product of a double-double by a double (TwoProduct on the high part).
__device__ __forceinline__ dd dd_scale(dd x, double s) {
  const double h = x.hi * s;
  const double e = fma(x.hi, s, -h);
  return dd{h, fma(x.lo, s, e)};
}

template <int N>
__device__ __forceinline__ Acc single_term(const MixArgs& a, uint64_t g) {
  const double* staged = opaque(a.staged);
  Rows<N> w;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    w.r[i] = 0.0;
#if PERM_CPLX
    w.i[i] = 0.0;
#endif
  }
  double W = 1.0;
  outer_digits<N>(a, staged, g, 0, w, W);
  double pr, pi;
  product<N>(w, pr, pi);
  const double hr = W * pr, hi = W * pi;
  return Acc{{hr, fma(W, pr, -hr)}, {hi, fma(W, pi, -hi)}};
}

template <int N>
__device__ __forceinline__ Acc walk_chunk(const MixArgs& a, uint64_t c, uint32_t par) {
  const double* staged = opaque(a.staged);
  Rows<N> w;
  {
    cdptr st = as_const(staged + kCw * (2 * (a.ncols + 1) + (int)par) * N);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      w.r[i] = st[kCw * i];
#if PERM_CPLX
      w.i[i] = st[kCw * i + 1];
#endif
    }
  }
  double W = 1.0;
  outer_digits<N>(a, staged, c * (uint64_t)a.L, a.outer_col, w, W);
  cdptr tin = as_const(a.tin + par * (uint32_t)a.L);
  ciptr toff = (ciptr)(a.toff + par * (uint32_t)a.L);
  Acc acc{{0.0, 0.0}, {0.0, 0.0}};
  const int L = a.L;
  int s = 0;
  for (; s + 1 < L; s += 2) {
    const double t0 = tin[s], t1 = tin[s + 1];
    const int32_t o0 = toff[s], o1 = toff[s + 1];
    double p0r, p0i, p1r, p1i;
    product<N>(w, p0r, p0i);
    add_col<N>(w, staged, o0);
    // keep the next column's scalar loads behind this one's adds: two columns
    // in SGPRs at once would spill
    __builtin_amdgcn_sched_barrier(0);
    product<N>(w, p1r, p1i);
    add_col<N>(w, staged, o1);
    __builtin_amdgcn_sched_barrier(0);
    dd_acc(acc.re, fma(t1, p1r, t0 * p0r));
#if PERM_CPLX
    dd_acc(acc.im, fma(t1, p1i, t0 * p0i));
#endif
  }
  if (s < L) {  // odd L: the last term has no partner
    double pr, pi;
    product<N>(w, pr, pi);
    dd_acc(acc.re, tin[s] * pr);
#if PERM_CPLX
    dd_acc(acc.im, tin[s] * pi);
#endif
  }
  return Acc{dd_scale(acc.re, W), dd_scale(acc.im, W)};
}

#if PERM_CPLX
// ------------------------------------------------- rows kept in LDS ----
// From n = kSplitFrom the complex chunk walk keeps rows [R, n) of each lane's
// row sums in LDS, as the dense complex walk does (perm_walk.hpp): the rows
// in VGPRs then leave room for two waves per SIMD instead of one.  At the
// chunk start every outer column updates the LDS rows in place (its
// coefficient is formed once per column, as in outer_digits); in the walk each
// LDS row is read once per pair of terms, multiplied into both terms'
// products and written back after the pair's second column.
template <int R>
__device__ __forceinline__ void add_col_rows(double (&wr)[R], double (&wi)[R], const double* col) {
  cdptr c = as_const(col);
#pragma unroll
  for (int i = 0; i < R; ++i) {
    wr[i] += c[2 * i];
    wi[i] += c[2 * i + 1];
  }
}

template <int N>
__device__ __forceinline__ Acc walk_chunk_split(const MixArgs& a, uint64_t c, uint32_t par,
                                                double2* __restrict__ rows) {
  constexpr int R = SplitRows<N>::R, L = SplitRows<N>::L;
  const double* staged = opaque(a.staged);
  const uint64_t g = c * (uint64_t)a.L;
  double wr[R], wi[R];
  {
    cdptr st = as_const(staged + kCw * (2 * (a.ncols + 1) + (int)par) * N);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      wr[i] = st[2 * i];
      wi[i] = st[2 * i + 1];
    }
#pragma unroll
    for (int r = 0; r < L; ++r) rows[r * kWave] = double2{st[2 * (R + r)], st[2 * (R + r) + 1]};
  }
  double W = 1.0;
#pragma unroll 1
  for (int k = a.outer_col; k < a.ncols; ++k) {
    const double f = column_coef(a, g, k, W);
    cdptr col = as_const(staged + kCw * k * N);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      wr[i] = fma(f, col[2 * i], wr[i]);
      wi[i] = fma(f, col[2 * i + 1], wi[i]);
    }
#pragma unroll
    for (int r = 0; r < L; ++r) {
      double2 v = rows[r * kWave];
      v.x = fma(f, col[2 * (R + r)], v.x);
      v.y = fma(f, col[2 * (R + r) + 1], v.y);
      rows[r * kWave] = v;
    }
  }
  cdptr tin = as_const(a.tin + par * (uint32_t)a.L);
  ciptr toff = (ciptr)(a.toff + par * (uint32_t)a.L);
  Acc acc{{0.0, 0.0}, {0.0, 0.0}};
  const int Lc = a.L;
  int s = 0;
  for (; s + 1 < Lc; s += 2) {
    const double t0 = tin[s], t1 = tin[s + 1];
    const int32_t o0 = toff[s], o1 = toff[s + 1];
    double q0r, q0i, q1r, q1i, p0r, p0i, p1r, p1i;
    lds_rows_pair<N, R, 0, true>(rows, staged + o0 + 2 * R, staged + o1 + 2 * R, q0r, q0i, q1r,
                                 q1i);
    prod_c64<R>(wr, wi, p0r, p0i);
    add_col_rows<R>(wr, wi, staged + o0);
    // as in walk_chunk: one column's scalar loads at a time
    __builtin_amdgcn_sched_barrier(0);
    prod_c64<R>(wr, wi, p1r, p1i);
    add_col_rows<R>(wr, wi, staged + o1);
    __builtin_amdgcn_sched_barrier(0);
    cmul_acc<0>(p0r, p0i, q0r, q0i);
    cmul_acc<0>(p1r, p1i, q1r, q1i);
    dd_acc(acc.re, fma(t1, p1r, t0 * p0r));
    dd_acc(acc.im, fma(t1, p1i, t0 * p0i));
  }
  if (s < Lc) {  // odd L: the last term has no partner (only its product is used)
    const double* cz = staged + toff[s] + 2 * R;
    double q0r, q0i, q1r, q1i, pr, pi;
    lds_rows_pair<N, R, 0, false>(rows, cz, cz, q0r, q0i, q1r, q1i);
    prod_c64<R>(wr, wi, pr, pi);
    cmul_acc<0>(pr, pi, q0r, q0i);
    dd_acc(acc.re, tin[s] * pr);
    dd_acc(acc.im, tin[s] * pi);
  }
  return Acc{dd_scale(acc.re, W), dd_scale(acc.im, W)};
}

template <int N, bool SINGLE>
constexpr bool mix_split() {
  return N >= kSplitFrom && !SINGLE;
}
#else
template <int N, bool SINGLE>
constexpr bool mix_split() {
  return false;
}
#endif

#if !PERM_CPLX
__device__ __forceinline__ u128 u128_neg(u128 v) {
  const uint64_t lo = ~v.lo + 1u;
  return u128{lo, ~v.hi + (lo == 0 ? 1u : 0u)};
}

// Exact integer form of the single term g.
template <int N>
__device__ __forceinline__ u128 exact_single(const MixArgs& a, uint64_t g) {
  const double* staged = opaque(a.staged);
  Rows<N> w;
#pragma unroll
  for (int i = 0; i < N; ++i) w.r[i] = 0.0;
  double W = 1.0;
  outer_digits<N>(a, staged, g, 0, w, W);
  exact::Bins B{0, 0, 0};
  const exact::Bins off = exact::term_offsets<N>();
  if (W > 0.0) {
    exact::term_bins<N, true>(w.r, B);
    B.b0 -= off.b0;
    B.b1 -= off.b1;
    B.b2 -= off.b2;
  } else {
    exact::term_bins<N, false>(w.r, B);
    B.b0 += off.b0;
    B.b1 += off.b1;
    B.b2 += off.b2;
  }
  return exact::fold(B);
}

// Exact product of the row sums into the bins.  KG = 0: groups of
// int01_group_rows(N) rows (any 0/1 matrix).  KG >= 1: KG equal groups of
// staged rows, each product formed by two interleaved chains; the caller has
// ordered the rows so that every group's product of row degrees, which bounds
// every partial product of the group, is below 2^50.
template <int N, int KG, bool ADD>
__device__ __forceinline__ void group_bins(const double (&r)[N], exact::Bins& B) {
  if constexpr (KG == 0) {
    exact::term_bins<N, ADD>(r, B);
  } else {
    constexpr int GS = (N + KG - 1) / KG;
    double G[KG];
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int lo = g * GS, hi = (g + 1) * GS < N ? (g + 1) * GS : N;
      double p0 = r[lo], p1 = lo + 1 < hi ? r[lo + 1] : 1.0;
#pragma unroll
      for (int i = lo + 2; i < hi; i += 2) {
        p0 *= r[i];
        if (i + 1 < hi) p1 *= r[i + 1];
      }
      G[g] = p0 * p1;
    }
    exact::product_bins<KG, ADD>(G, B);
  }
}

template <int N, int KG>
__device__ __forceinline__ exact::Bins group_offsets() {
  if constexpr (KG == 0)
    return exact::term_offsets<N>();
  else
    return exact::product_offsets<KG>();
}

// Exact integer sum of chunk c (L <= 2^10 terms, weights +-1 alternating).
template <int N, int KG>
__device__ __forceinline__ u128 exact_chunk(const MixArgs& a, uint64_t c, uint32_t par) {
  const double* staged = opaque(a.staged);
  Rows<N> w;
  {
    cdptr st = as_const(staged + (2 * (a.ncols + 1) + (int)par) * N);
#pragma unroll
    for (int i = 0; i < N; ++i) w.r[i] = st[i];
  }
  double W = 1.0;
  outer_digits<N>(a, staged, c * (uint64_t)a.L, a.outer_col, w, W);
  cdptr tin = as_const(a.tin + par * (uint32_t)a.L);
  ciptr toff = (ciptr)(a.toff + par * (uint32_t)a.L);
  exact::Bins B{0, 0, 0};
  const int L = a.L;
  int s = 0;
  for (; s + 1 < L; s += 2) {
    const int32_t o0 = toff[s], o1 = toff[s + 1];
    group_bins<N, KG, true>(w.r, B);   // + P_s
    add_col<N>(w, staged, o0);
    group_bins<N, KG, false>(w.r, B);  // - P_{s+1}
    add_col<N>(w, staged, o1);
  }
  if (s < L) {  // odd L: an unpaired + P_{L-1}
    group_bins<N, KG, true>(w.r, B);
    const exact::Bins off = group_offsets<N, KG>();
    B.b0 -= off.b0;
    B.b1 -= off.b1;
    B.b2 -= off.b2;
  }
  const u128 v = exact::fold(B);  // sum_s (-1)^s P_s
  return ((tin[0] < 0.0) != (W < 0.0)) ? u128_neg(v) : v;
}

template <int N, bool SINGLE, int KG>
__global__ __launch_bounds__(kBlock) void mix_exact_kernel(MixArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  u128 acc{0, 0};
  if (a.status[0] == kStOk) {
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      u128 part;
      if constexpr (SINGLE) {
        part = exact_single<N>(a, a.first + c);
      } else {
        const uint32_t par = (uint32_t)((a.first + (task & 1)) & 1);
        part = exact_chunk<N, KG>(a, a.first + c, par);
      }
      if (c < a.nchunks) acc = u128_add(acc, part);
    }
  }
  const u128 bs = block_sum(wave_sum(acc), u128_add);
  if (threadIdx.x == 0) {
    uint64_t* out = (uint64_t*)a.partials;
    out[2 * blockIdx.x] = bs.lo;
    out[2 * blockIdx.x + 1] = bs.hi;
  }
}
#endif

template <int N, bool SINGLE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(mix_split<N, SINGLE>() ? 2 : 1)))
void mix_walk_kernel(MixArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  dd re{0.0, 0.0}, im{0.0, 0.0};
#if PERM_CPLX
  double2* rows = nullptr;
  if constexpr (mix_split<N, SINGLE>()) rows = lane_rows<SplitRows<N>::L>();
#endif
  if (a.status[0] == kStOk) {
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      Acc part;
      if constexpr (SINGLE) {
        part = single_term<N>(a, a.first + c);
      } else {
        const uint32_t par = (uint32_t)((a.first + (task & 1)) & 1);
#if PERM_CPLX
        if constexpr (mix_split<N, SINGLE>())
          part = walk_chunk_split<N>(a, a.first + c, par, rows);
        else
#endif
          part = walk_chunk<N>(a, a.first + c, par);
      }
      if (c < a.nchunks) {
        re = dd_add(re, part.re);
#if PERM_CPLX
        im = dd_add(im, part.im);
#endif
      }
    }
  }
  const dd br = block_sum(wave_sum(re), dd_add);
  double* out = (double*)a.partials;
#if PERM_CPLX
  __syncthreads();
  const dd bi = block_sum(wave_sum(im), dd_add);
  if (threadIdx.x == 0) {
    out[4 * blockIdx.x] = br.hi;
    out[4 * blockIdx.x + 1] = br.lo;
    out[4 * blockIdx.x + 2] = bi.hi;
    out[4 * blockIdx.x + 3] = bi.lo;
  }
#else
  (void)im;
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = br.hi;
    out[2 * blockIdx.x + 1] = br.lo;
  }
#endif
}

#if !PERM_CPLX
// Row groups of the default exact product at size N.
template <int N>
constexpr int default_groups() {
  return (N + int01_group_rows(N) - 1) / int01_group_rows(N);
}

// The exact chunk walk with KG row groups; only KG below the default count
// is instantiated (others fall back to the default grouping, always valid).
template <int N, int KG>
void launch_exact_groups(const MixArgs& a, int grid, hipStream_t s) {
  if constexpr (KG < default_groups<N>())
    hipLaunchKernelGGL((mix_exact_kernel<N, false, KG>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((mix_exact_kernel<N, false, 0>), dim3(grid), dim3(kBlock), 0, s, a);
}
#endif

template <int N>
hipError_t dispatch(bool single, bool exact, int groups, const MixArgs& a, int grid,
                    hipStream_t s) {
  if (exact) {
#if PERM_CPLX
    (void)groups;
    return hipErrorInvalidValue;
#else
    static_assert(kMixMaxRowGroups == 4, "one case per group count");
    if (single) {
      hipLaunchKernelGGL((mix_exact_kernel<N, true, 0>), dim3(grid), dim3(kBlock), 0, s, a);
    } else {
      switch (groups) {
        case 1: launch_exact_groups<N, 1>(a, grid, s); break;
        case 2: launch_exact_groups<N, 2>(a, grid, s); break;
        case 3: launch_exact_groups<N, 3>(a, grid, s); break;
        case 4: launch_exact_groups<N, 4>(a, grid, s); break;
        default: launch_exact_groups<N, 0>(a, grid, s); break;
      }
    }
    return hipGetLastError();
#endif
  }
  if (single)
    hipLaunchKernelGGL((mix_walk_kernel<N, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((mix_walk_kernel<N, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

#define PERM_CASE(N) \
  case N:            \
    return dispatch<N>(single, exact, groups, a, grid, s);

// Built four times: PERM_CPLX selects real or complex, PERM_HALF the sizes
// n = 1..32 or n = 33..64.
#if PERM_CPLX
#if PERM_HALF == 0
#define PERM_LAUNCH launch_mix_walk_complex_lo
#else
#define PERM_LAUNCH launch_mix_walk_complex_hi
#endif
#else
#if PERM_HALF == 0
#define PERM_LAUNCH launch_mix_walk_real_lo
#else
#define PERM_LAUNCH launch_mix_walk_real_hi
#endif
#endif
#if PERM_HALF == 0
#define PERM_CASES "perm_cases_lo.inc"
#else
#define PERM_CASES "perm_cases_hi.inc"
#endif

hipError_t PERM_LAUNCH(int n, bool single, bool exact, int groups, const MixArgs& a, int grid,
                       hipStream_t s) {
  switch (n) {
#include PERM_CASES
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace perm
