// Band transfer matrix (App. C, bandpermanent) for matrices with a_ij = 0
// when |i - j| > k.
//
// per(A) is the coefficient sum of prod_i C_i, C_i = sum_j a_ij x_j, taken
// with x_j^2 = 0 (each column used once).  After row i the variable of
// column i-k-1 is set to 1: no later row reaches that column.  The polynomial
// then lives on the W = 2k+1 columns [i-k, i+k]; bit b of a mask stands for
// column i-k+b.
//
// Only one popcount class of masks can carry a term that survives to the
// end.  After row i, rows 0..i have used i+1 columns, and every column below
// i-k must be among them (no later row reaches it); so a surviving monomial
// holds exactly p_i = min(i+1, k+1) columns of the window.  A monomial with
// fewer columns never arises, and one with more has skipped a column for good:
// all its descendants die by x_j^2 = 0 before the last row (pigeonhole), and
// it never feeds a mask of the surviving class.  The kernel therefore keeps
// the p_i-class only, binom(W, p_i) <= binom(2k+1, k+1) coefficients, stored
// densely by the mask's rank in its class.  Ascending numeric order of the
// masks of one popcount is colex order, so rank(M) = sum_j binom(b_j, j) over
// the set bits b_1 < b_2 < ... of M (the combinatorial number system).
//
// One row, for a mask M of the new class: with b0 = 1 when column i-k-1
// exists (it must then be in the term) and Q = 2M + b0 over the columns
// [i-k-1, i+k], new[M] = sum over the band columns j in Q of old[Q \ j] a_ij.
// Column i+k is new in this row, so a Q holding it has the single term
// j = i+k; otherwise the sum runs over the p_i columns of M.
//
// For the interior rows (i > k: b0 = 1, p = k+1 before and after) the sources
// of a mask do not depend on i.  The class's masks without column i+k come
// first in rank order (they are the smaller numbers); lane l owns the masks
// l, l+64, ... of each kind (k+1 sources for the first kind, one for the
// second) and keeps their source ranks and columns in registers for the whole
// launch.  A term whose column is the same in every lane (column i+k, and the
// high columns of the later colex slots) takes the row's entry from a scalar
// register instead of LDS.  The first k+1 rows, where the class grows, look
// the ranks up in LDS.
//
// One wavefront per matrix, four per workgroup, each with its own pair of
// coefficient buffers and its own row slot; the rank tables are shared.  A row
// then needs no barrier: a wave's LDS accesses are served in order, so a
// compiler fence between rows suffices.  Lane c loads entry c of the next row
// (vector loads) while the current row is computed.  Powers of two keep long
// products in range, exactly: each row's entries are scaled into [1/2, 1); and
// every 4 rows the wave takes the largest binary exponent of the coefficients
// it wrote, which the next row applies to the values it produces (one row
// late, off the row's critical path).  Both maxima are taken over frexp
// exponents with DPP lane permutes and lane reads, which keeps LDS round trips
// off the row.  The exponents are restored at the end.  The final coefficient
// sum is a fixed-order double-double reduction.
#include <type_traits>
#include <utility>

#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

__host__ __device__ constexpr int binom_c(int n, int r) {
  if (r < 0 || r > n) return 0;
  int v = 1;
  for (int t = 1; t <= r; ++t) v = v * (n - r + t) / t;
  return v;
}

// Binary exponent of x (frexp: x = f 2^e, 1/2 <= |f| < 1), or kNoExp for 0.
// The exponent of the largest magnitude is the largest exponent.
constexpr int kNoExp = INT32_MIN;
__device__ __forceinline__ int exponent(double x) {
  int e = 0;
  frexp(x, &e);
  return x != 0.0 ? e : kNoExp;
}

// Maximum over the 16 lanes of each row of the wave, by DPP lane permutes
// (VALU only, no LDS round trip): quad swaps, then the half-row and row mirrors.
__device__ __forceinline__ int row16_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
  return v;
}

// Maximum over the wave (uniform): the four rows' maxima read from lanes 0, 16, 32, 48.
__device__ __forceinline__ int wave_max_int(int v) {
  v = row16_max(v);
  const int a = max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
  const int b = max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
  return max(a, b);
}

template <bool CPLX>
struct Coef;
template <>
struct alignas(16) Coef<true> {
  double re, im;
};
template <>
struct Coef<false> {
  double re;
};

// The mask of colex rank r among the p-subsets of the bits 0, 1, 2, ...: its
// set bits b_p > ... > b_1 are, in turn, the largest b with binom(b, j) not
// above what is left of r (the combinatorial number system read backwards).
__host__ __device__ constexpr int unrank_colex(int r, int p) {
  int m = 0;
  for (int j = p; j >= 1; --j) {
    int b = j - 1;
    while (binom_c(b + 1, j) <= r) ++b;
    m |= 1 << b;
    r -= binom_c(b, j);
  }
  return m;
}

// Position of the t-th lowest set bit of m (t = 0: the lowest), or -1.
__host__ __device__ constexpr int nth_bit(int m, int t) {
  for (int b = 0; b < 31; ++b) {
    if ((m >> b) & 1) {
      if (t == 0) return b;
      --t;
    }
  }
  return -1;
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>), in order.
template <class F, int... J>
__device__ __forceinline__ void for_each_index_impl(F&& f, std::integer_sequence<int, J...>) {
  (f(std::integral_constant<int, J>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void for_each_index(F&& f) {
  for_each_index_impl(f, std::make_integer_sequence<int, N>{});
}

// Lane `lane`'s value of a wave-uniform read of v (a scalar register).
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sizes of the live class for half-width K.
template <int K>
struct Shape {
  static constexpr int W = 2 * K + 1;              // window columns
  static constexpr int S = 1 << W;                 // masks
  static constexpr int TOP = W;                    // bit of column i+k in Q
  static constexpr int NC = binom_c(W, K + 1);     // largest class
  static constexpr int NT = binom_c(W - 1, K + 1); // interior masks without column i+k
  static constexpr int NTOP = NC - NT;             // interior masks with it
  // of the first kind per lane (at least one slot: k = 0 has none)
  static constexpr int JN = NT > 0 ? (NT + kWave - 1) / kWave : 1;
  static constexpr int JT = (NTOP + kWave - 1) / kWave;  // of the second kind per lane
  // The column of term t (the t-th set column of Q above bit 0) of every
  // mask in slot jj of the first kind (ranks 64 jj .. 64 jj + 63), when it is
  // the same for all of them, else -1.  Ranks are colex, so the high columns
  // agree within the later slots.  Such a term takes the row's entry from a
  // scalar register instead of LDS.
  static constexpr int uniform_col(int jj, int t) {
    int c = -1;
    for (int r = kWave * jj; r < NT && r < kWave * (jj + 1); ++r) {
      const int cr = nth_bit(unrank_colex(r, K + 1), t) + 1;
      if (c == -1)
        c = cr;
      else if (c != cr)
        return -1;
    }
    return c;
  }
};

// One interior row (i > k: b0 = 1, class k+1 before and after) for the
// lane's masks.  Coefficients come from buffer P of the wave's pair (P = i
// mod 2, fixed at compile time so that every LDS address is a loop-invariant
// register plus a constant); the results go to buffer P ^ 1, scaled by
// 2^-ex.  When pub is set, returns the largest exponent written.
//
// One term of a first-kind mask of slot JJ: coefficient times row entry, the
// entry from the scalar copy au when its column is the same in every lane.
template <int K, bool CPLX, int JJ, int T>
__device__ __forceinline__ void nt_term(double& xr_acc, double& xi_acc, const Coef<CPLX>* old,
                                        const Coef<CPLX>* ar, const Coef<CPLX> (&au)[2 * K + 2],
                                        uint32_t src) {
  constexpr int cu = Shape<K>::uniform_col(JJ, T);
  const Coef<CPLX> x = old[src & 0xffff];
  Coef<CPLX> av;
  if constexpr (cu >= 0)
    av = au[cu];
  else
    av = ar[src >> 16];
  xr_acc = fma(x.re, av.re, xr_acc);
  if constexpr (CPLX) {
    xr_acc = fma(-x.im, av.im, xr_acc);
    xi_acc = fma(x.re, av.im, fma(x.im, av.re, xi_acc));
  }
}

template <int K, bool CPLX, int JJ, int... T>
__device__ __forceinline__ void nt_terms(double& xr_acc, double& xi_acc, const Coef<CPLX>* old,
                                         const Coef<CPLX>* ar, const Coef<CPLX> (&au)[2 * K + 2],
                                         const uint32_t (&src)[K + 1],
                                         std::integer_sequence<int, T...>) {
  (nt_term<K, CPLX, JJ, T>(xr_acc, xi_acc, old, ar, au, src[T]), ...);  // t = 0, 1, ..., K
}

template <int K, bool CPLX, int P>
__device__ __forceinline__ int interior_row(Coef<CPLX> (*sc)[Shape<K>::NC],
                                            const Coef<CPLX>* ar,
                                            const Coef<CPLX> (&au)[2 * K + 2],
                                            const uint32_t (&src_nt)[Shape<K>::JN][K + 1],
                                            const uint32_t (&src_top)[Shape<K>::JT], int lane,
                                            int ex, bool pub) {
  using Sh = Shape<K>;
  using C = Coef<CPLX>;
  const C* old = sc[P];
  C* nw = sc[P ^ 1];
  int lm = kNoExp;
  auto put = [&](int r, double xr, double xi) {
    C v;
    v.re = xr;
    if constexpr (CPLX) v.im = xi;
    if (ex != 0) {  // uniform: the renormalisation row
      v.re = ldexp(v.re, -ex);
      if constexpr (CPLX) v.im = ldexp(v.im, -ex);
    }
    if (pub) {  // uniform: the row that publishes the class's exponent
      lm = max(lm, exponent(v.re));
      if constexpr (CPLX) lm = max(lm, exponent(v.im));
    }
    nw[r] = v;
  };
  for_each_index<Sh::JN>([&](auto jjc) {
    constexpr int JJ = decltype(jjc)::value;
    const int r = lane + kWave * JJ;
    if (r < Sh::NT) {
      double xr_acc = 0.0, xi_acc = 0.0;
      nt_terms<K, CPLX, JJ>(xr_acc, xi_acc, old, ar, au, src_nt[JJ],
                            std::make_integer_sequence<int, K + 1>{});
      put(r, xr_acc, xi_acc);
    }
  });
  const C at = au[Sh::TOP];  // column i+k: the same for every mask of the second kind
#pragma unroll
  for (int jj = 0; jj < Sh::JT; ++jj) {
    const int r = lane + kWave * jj;
    if (r < Sh::NTOP) {
      const C x = old[src_top[jj]];
      double xr_acc = x.re * at.re, xi_acc = 0.0;
      if constexpr (CPLX) {
        xr_acc = fma(-x.im, at.im, xr_acc);
        xi_acc = fma(x.re, at.im, x.im * at.re);
      }
      put(Sh::NT + r, xr_acc, xi_acc);
    }
  }
  return lm;
}

// A wave's LDS writes are visible to its own later LDS reads (the LDS serves a
// wave's instructions in order); this keeps the compiler from moving reads of
// one row above the writes of the previous one.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int K, bool CPLX>
__global__ __launch_bounds__(kBlock) void band_kernel(BandArgs a) {
  using Sh = Shape<K>;
  constexpr int W = Sh::W, S = Sh::S, TOP = Sh::TOP, NC = Sh::NC, NT = Sh::NT;
  constexpr int NTOP = Sh::NTOP, JN = Sh::JN, JT = Sh::JT;
  static_assert(NC < 65536 && NC * 16 < 65536, "ranks are 16-bit");
  static_assert(TOP < 16, "a row's entries sit in the first 16 lanes of the wave");
  constexpr int cw = CPLX ? 2 : 1;
  using C = Coef<CPLX>;
  __shared__ C s_c[kWavesPerBlock][2][NC];     // per wave: the live class, by rank
  __shared__ C s_a[kWavesPerBlock][TOP + 1];   // per wave: scaled band entries of the row
  __shared__ uint16_t s_rank[S];               // rank of a mask in its popcount class
  __shared__ uint16_t s_cls[S];                // masks grouped by popcount, ascending
  __shared__ int cstart[W + 2];                // first index of each class in s_cls
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  typedef const __attribute__((address_space(4))) int32_t* ci32;
  typedef const __attribute__((address_space(4))) int64_t* ci64;

  if (tid < W + 2) {
    int v = 0;
    for (int p = 0; p < tid; ++p) v += binom_c(W, p);
    cstart[tid] = v;
  }
  __syncthreads();
  for (int M = tid; M < S; M += kBlock) {
    int r = 0, j = 0;
    for (int q = M; q; q &= q - 1) r += binom_c(__ffs(q) - 1, ++j);
    s_rank[M] = (uint16_t)r;
    s_cls[cstart[j] + r] = (uint16_t)M;
  }
  __syncthreads();
  // interior sources of the lane's masks: rank | column << 16
  uint32_t src_nt[JN][K + 1];
  uint32_t src_top[JT];
#pragma unroll
  for (int jj = 0; jj < JN; ++jj) {
    const int r = lane + kWave * jj;
    const int M = r < NT ? s_cls[cstart[K + 1] + r] : 0;
    const int Q = (M << 1) | 1;
    int q = Q & ~1;
#pragma unroll
    for (int t = 0; t <= K; ++t) {  // the t-th set column of Q above bit 0
      const int c = q ? __ffs(q) - 1 : 0;
      src_nt[jj][t] = q ? (s_rank[Q ^ (1 << c)] | ((uint32_t)c << 16)) : 0u;
      q &= q - 1;
    }
  }
#pragma unroll
  for (int jj = 0; jj < JT; ++jj) {
    const int r = lane + kWave * jj;
    const int M = r < NTOP ? s_cls[cstart[K + 1] + NT + r] : 0;
    const int Q = (M << 1) | 1;
    src_top[jj] = r < NTOP ? s_rank[Q ^ (1 << TOP)] : 0u;
  }

  C (*sc)[NC] = s_c[wave];  // this wave's pair of coefficient buffers
  C* sa = s_a[wave];
  C au[TOP + 1];            // the row's scaled entries as wave-uniform (scalar) values
  for (int m = blockIdx.x * kWavesPerBlock + wave; m < a.count;
       m += gridDim.x * kWavesPerBlock) {
    const int n = ((ci32)a.n)[m];  // uniform: scalar loads
    const double* A = a.A + ((ci64)a.off)[m];
    if (lane == 0) {  // p = 0 class: the empty monomial, coefficient 1
      sc[0][0].re = 1.0;
      if constexpr (CPLX) sc[0][0].im = 0.0;
    }
    int esum = 0, epub = 0;
    bool bad = false;
    // Lane c holds the entry of column i-k-1+c (c = 1..2k+1) of row i.
    double vr = 0.0, vi = 0.0;
    auto load_entry = [&](int i) {
      const int j = i - K - 1 + lane;
      vr = 0.0;
      vi = 0.0;
      if (lane >= 1 && lane <= TOP && j >= 0 && j < n) {
        const double* p = A + (size_t)cw * ((size_t)i + (size_t)j * n);
        vr = p[0];
        if constexpr (CPLX) vi = p[1];
      }
    };
    load_entry(0);
    // Start of row i: the row's entries, scaled, into the wave's slot; row
    // i+1's loads issued; then the class exponent published by row i-1 (on
    // renormalisation rows).
    auto head = [&](int i) -> int {
      const bool nf = !isfinite(vr) || !isfinite(vi);
      bad = bad || __ballot(nf) != 0;
      // the exponent of the row's largest entry, from lanes 0..15
      const int emx = __builtin_amdgcn_readfirstlane(
          row16_max(max(exponent(vr), exponent(vi))));
      const int e = (emx != kNoExp && !bad) ? emx : 0;  // scale the row by 2^-e
      esum += e;
      const double sr = ldexp(vr, -e), si = ldexp(vi, -e);
      if (lane <= TOP) {
        sa[lane].re = sr;
        if constexpr (CPLX) sa[lane].im = si;
      }
      // scalar copies (the interior rows use those of the columns that are the
      // same in every lane; the other reads are dead and dropped)
#pragma unroll
      for (int c = 1; c <= TOP; ++c) {
        au[c].re = readlane_d(sr, c);
        if constexpr (CPLX) au[c].im = readlane_d(si, c);
      }
      if (i + 1 < n) load_entry(i + 1);  // in flight during row i
      wave_lds_order();
      int ex = 0;
      if (i > 0 && (i & 3) == 0) {
        ex = epub != kNoExp ? epub : 0;
        esum += ex;
      }
      return ex;
    };
    // End of row i: every 4 rows, the class's largest exponent for row i+1.
    auto tail = [&](int i, int lm) {
      if ((i & 3) == 3) epub = wave_max_int(lm);
      wave_lds_order();
    };
    // rows 0..k: class i+1 over b0 = 0, sources in class i (ranks from the table)
    const int ng = n < K + 1 ? n : K + 1;
    for (int i = 0; i < ng; ++i) {
      const int ex = head(i);
      const C* old = sc[i & 1];
      C* nw = sc[(i & 1) ^ 1];
      int lm = kNoExp;
      const int c0 = cstart[i + 1], c1 = cstart[i + 2];
      for (int r = c0 + lane; r < c1; r += kWave) {
        const int Q = s_cls[r] << 1;
        double xr_acc = 0.0, xi_acc = 0.0;
        for (int q = (Q >> TOP) & 1 ? (1 << TOP) : Q; q; q &= q - 1) {
          const int c = __ffs(q) - 1;
          const C x = old[s_rank[Q ^ (1 << c)]];
          const C av = sa[c];
          xr_acc = fma(x.re, av.re, xr_acc);
          if constexpr (CPLX) {
            xr_acc = fma(-x.im, av.im, xr_acc);
            xi_acc = fma(x.re, av.im, fma(x.im, av.re, xi_acc));
          }
        }
        C v;
        v.re = ldexp(xr_acc, -ex);
        lm = max(lm, exponent(v.re));
        if constexpr (CPLX) {
          v.im = ldexp(xi_acc, -ex);
          lm = max(lm, exponent(v.im));
        }
        nw[r - c0] = v;
      }
      tail(i, lm);
    }
    // interior rows, two at a time so that the buffer parity is a constant
    constexpr int P0 = (K + 1) & 1;
    int i = K + 1;
    for (; i + 1 < n; i += 2) {
      int ex = head(i);
      tail(i, interior_row<K, CPLX, P0>(sc, sa, au, src_nt, src_top, lane, ex, (i & 3) == 3));
      ex = head(i + 1);
      tail(i + 1, interior_row<K, CPLX, P0 ^ 1>(sc, sa, au, src_nt, src_top, lane, ex,
                                                 ((i + 1) & 3) == 3));
    }
    if (i < n) {
      const int ex = head(i);
      tail(i, interior_row<K, CPLX, P0>(sc, sa, au, src_nt, src_top, lane, ex, (i & 3) == 3));
    }
    // set every remaining x_j = 1: the sum of the class's coefficients, fixed order
    const C* fin = sc[n & 1];  // the buffer row n-1 wrote
    const int pl = n < K + 1 ? n : K + 1;
    const int cnt = cstart[pl + 1] - cstart[pl];
    dd r{0.0, 0.0}, q{0.0, 0.0};
    for (int t = lane; t < cnt; t += kWave) {
      dd_acc(r, fin[t].re);
      if constexpr (CPLX) dd_acc(q, fin[t].im);
    }
    r = wave_sum(r);
    if constexpr (CPLX) q = wave_sum(q);
    if (lane == 0) {
      double* o = a.out + 4 * (size_t)m;
      o[0] = bad ? 0.0 : ldexp(r.hi, esum);
      o[1] = bad ? 0.0 : ldexp(r.lo, esum);
      o[2] = bad ? 0.0 : (CPLX ? ldexp(q.hi, esum) : 0.0);
      o[3] = bad ? 0.0 : (CPLX ? ldexp(q.lo, esum) : 0.0);
      if (a.status) a.status[m] = bad ? kStNonFinite : kStOk;
    }
    wave_lds_order();
  }
}

template <int K>
hipError_t launch_k(bool cplx, const BandArgs& a, int grid, hipStream_t s) {
  if (cplx)
    hipLaunchKernelGGL((band_kernel<K, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((band_kernel<K, false>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int K>
int blocks_k(bool cplx) {
  int nb = 0;
  hipError_t e = cplx ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, band_kernel<K, true>, kBlock, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, band_kernel<K, false>, kBlock, 0);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

}  // namespace

hipError_t launch_band(bool cplx, int k, const BandArgs& a, int grid, hipStream_t s) {
  switch (k) {
    case 0: return launch_k<0>(cplx, a, grid, s);
    case 1: return launch_k<1>(cplx, a, grid, s);
    case 2: return launch_k<2>(cplx, a, grid, s);
    case 3: return launch_k<3>(cplx, a, grid, s);
    case 4: return launch_k<4>(cplx, a, grid, s);
    case 5: return launch_k<5>(cplx, a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

int band_blocks_per_cu(bool cplx, int k) {
  switch (k) {
    case 0: return blocks_k<0>(cplx);
    case 1: return blocks_k<1>(cplx);
    case 2: return blocks_k<2>(cplx);
    case 3: return blocks_k<3>(cplx);
    case 4: return blocks_k<4>(cplx);
    case 5: return blocks_k<5>(cplx);
    default: return 1;
  }
}

}  // namespace perm
