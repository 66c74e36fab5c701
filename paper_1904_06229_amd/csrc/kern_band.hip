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
// first in rank order (they are the smaller numbers); thread t owns the t-th
// of them (k+1 sources) and the t-th of the others (one source), and keeps
// their source ranks and columns in registers for the whole launch.  The
// first k+1 rows, where the class grows, look the ranks up in LDS.
//
// One workgroup per matrix (grid-stride over the batch).  Wave 0 loads the
// next row's 2k+1 band entries (one per lane, vector loads) while the current
// row is computed; the rows' entries alternate between two LDS slots, so one
// barrier per row suffices.  Powers of two keep long products in range,
// exactly: each row's entries are scaled into [1/2, 1); and every 4 rows the
// threads publish the largest binary exponent of the coefficients they wrote,
// which the next row applies to the values it produces (one row late, no
// barrier of its own).  Both maxima are taken over frexp exponents with DPP
// lane permutes and lane reads, which keeps LDS round trips off the row's
// critical path.  The exponents are restored at the end.  The
// final coefficient sum is a fixed-order double-double reduction.
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

// One interior row (i > k: b0 = 1, class k+1 before and after) for the
// thread's two masks.  Coefficients come from buffer P and the row's entries
// from slot P (P = i mod 2, fixed at compile time so that every LDS address is
// a loop-invariant register plus a constant); the results go to buffer P ^ 1,
// scaled by 2^-ex.  When pub is set, returns the largest exponent written.
template <int K, bool CPLX, int P>
__device__ __forceinline__ int interior_row(Coef<CPLX> (*s_c)[binom_c(2 * K + 1, K + 1)],
                                            const Coef<CPLX> (*s_a)[2 * K + 2],
                                            const uint32_t (&src_nt)[K + 1], uint32_t src_top,
                                            int tid, int ex, bool pub) {
  constexpr int W = 2 * K + 1;
  constexpr int TOP = W;
  constexpr int NC = binom_c(W, K + 1);
  constexpr int NT = binom_c(W - 1, K + 1);
  constexpr int NTOP = NC - NT;
  using C = Coef<CPLX>;
  const C* old = s_c[P];
  C* nw = s_c[P ^ 1];
  const C* ar = s_a[P];
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
  if (tid < NT) {
    double xr_acc = 0.0, xi_acc = 0.0;
#pragma unroll
    for (int t = 0; t <= K; ++t) {
      const C x = old[src_nt[t] & 0xffff];
      const C av = ar[src_nt[t] >> 16];
      xr_acc = fma(x.re, av.re, xr_acc);
      if constexpr (CPLX) {
        xr_acc = fma(-x.im, av.im, xr_acc);
        xi_acc = fma(x.re, av.im, fma(x.im, av.re, xi_acc));
      }
    }
    put(tid, xr_acc, xi_acc);
  }
  if (tid < NTOP) {
    const C x = old[src_top];
    const C av = ar[TOP];
    double xr_acc = x.re * av.re, xi_acc = 0.0;
    if constexpr (CPLX) {
      xr_acc = fma(-x.im, av.im, xr_acc);
      xi_acc = fma(x.re, av.im, x.im * av.re);
    }
    put(NT + tid, xr_acc, xi_acc);
  }
  return lm;
}

template <int K, bool CPLX>
__global__ __launch_bounds__(kBlock) void band_kernel(BandArgs a) {
  constexpr int W = 2 * K + 1;              // window columns
  constexpr int S = 1 << W;                 // masks
  constexpr int TOP = W;                    // bit of column i+k in Q
  constexpr int NC = binom_c(W, K + 1);     // largest class
  constexpr int NT = binom_c(W - 1, K + 1); // interior masks without column i+k
  constexpr int NTOP = NC - NT;             // interior masks with it
  static_assert(NT <= kBlock && NTOP <= kBlock, "one mask of each kind per thread");
  static_assert(NC < 65536, "ranks are 16-bit");
  static_assert(TOP < 16, "a row's entries sit in the first 16 lanes of wave 0");
  constexpr int cw = CPLX ? 2 : 1;
  using C = Coef<CPLX>;
  __shared__ C s_c[2][NC];           // coefficients of the live class, by rank
  __shared__ uint16_t s_rank[S];     // rank of a mask in its popcount class
  __shared__ uint16_t s_cls[S];      // masks grouped by popcount, ascending in a group
  __shared__ C s_a[2][TOP + 1];      // scaled band entries of a row, by row parity
  __shared__ int s_mx[kWavesPerBlock];  // largest coefficient exponent per wave
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  typedef const __attribute__((address_space(4))) int32_t* ci32;
  typedef const __attribute__((address_space(4))) int64_t* ci64;

  __shared__ int cstart[W + 2];      // first index of each popcount class in s_cls
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
  // interior sources: rank | column << 16
  uint32_t src_nt[K + 1];
  uint32_t src_top = 0;
  {
    const int M = tid < NT ? s_cls[cstart[K + 1] + tid] : 0;
    const int Q = (M << 1) | 1;
    int q = Q & ~1;
#pragma unroll
    for (int t = 0; t <= K; ++t) {  // the t-th set column of Q above bit 0
      const int c = q ? __ffs(q) - 1 : 0;
      src_nt[t] = q ? (s_rank[Q ^ (1 << c)] | ((uint32_t)c << 16)) : 0u;
      q &= q - 1;
    }
  }
  if (tid < NTOP) {
    const int M = s_cls[cstart[K + 1] + NT + tid];
    const int Q = (M << 1) | 1;
    src_top = s_rank[Q ^ (1 << TOP)];
  }

  for (int m = blockIdx.x; m < a.count; m += gridDim.x) {
    const int n = ((ci32)a.n)[m];  // uniform: scalar loads
    const double* A = a.A + ((ci64)a.off)[m];
    if (tid == 0) {  // p = 0 class: the empty monomial, coefficient 1
      s_c[0][0].re = 1.0;
      if constexpr (CPLX) s_c[0][0].im = 0.0;
    }
    int esum = 0;
    bool bad = false;
    // Lane c of wave 0 holds the entry of column i-k-1+c (c = 1..2k+1) of row i.
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
    if (wave == 0) load_entry(0);
    // Start of row i: wave 0 scales the row's entries into slot i mod 2 and
    // loads row i+1's; the barrier; then the class exponent published by row
    // i-1 (on renormalisation rows), uniform.
    auto head = [&](int i) -> int {
      if (wave == 0) {
        const bool nf = !isfinite(vr) || !isfinite(vi);
        bad = bad || __ballot(nf) != 0;
        // the exponent of the row's largest entry, from lanes 0..15
        const int emx = __builtin_amdgcn_readfirstlane(
            row16_max(max(exponent(vr), exponent(vi))));
        const int e = (emx != kNoExp && !bad) ? emx : 0;  // scale the row by 2^-e
        esum += e;
        if (lane <= TOP) {
          s_a[i & 1][lane].re = ldexp(vr, -e);
          if constexpr (CPLX) s_a[i & 1][lane].im = ldexp(vi, -e);
        }
        if (i + 1 < n) load_entry(i + 1);  // in flight during row i
      }
      // one barrier: row i's entries, and row i-1's coefficients, are in LDS
      __syncthreads();
      int ex = 0;
      if (i > 0 && (i & 3) == 0) {
        int Mx = s_mx[0];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) Mx = max(Mx, s_mx[w]);
        ex = Mx != kNoExp ? Mx : 0;
        esum += ex;
      }
      return __builtin_amdgcn_readfirstlane(ex);
    };
    // End of row i: every 4 rows, publish the class's largest exponent for row i+1.
    auto tail = [&](int i, int lm) {
      if ((i & 3) == 3) {
        lm = wave_max_int(lm);
        if (lane == 0) s_mx[wave] = lm;
      }
    };
    // rows 0..k: class i+1 over b0 = 0, sources in class i (ranks from the table)
    const int ng = n < K + 1 ? n : K + 1;
    for (int i = 0; i < ng; ++i) {
      const int ex = head(i);
      const C* old = s_c[i & 1];
      C* nw = s_c[(i & 1) ^ 1];
      const C* ar = s_a[i & 1];
      int lm = kNoExp;
      const int c0 = cstart[i + 1], c1 = cstart[i + 2];
      for (int r = c0 + tid; r < c1; r += kBlock) {
        const int Q = s_cls[r] << 1;
        double xr_acc = 0.0, xi_acc = 0.0;
        for (int q = (Q >> TOP) & 1 ? (1 << TOP) : Q; q; q &= q - 1) {
          const int c = __ffs(q) - 1;
          const C x = old[s_rank[Q ^ (1 << c)]];
          const C av = ar[c];
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
      tail(i, interior_row<K, CPLX, P0>(s_c, s_a, src_nt, src_top, tid, ex, (i & 3) == 3));
      ex = head(i + 1);
      tail(i + 1, interior_row<K, CPLX, P0 ^ 1>(s_c, s_a, src_nt, src_top, tid, ex,
                                                 ((i + 1) & 3) == 3));
    }
    if (i < n) {
      const int ex = head(i);
      tail(i, interior_row<K, CPLX, P0>(s_c, s_a, src_nt, src_top, tid, ex, (i & 3) == 3));
    }
    const int cur = n & 1;  // the buffer row n-1 wrote
    __syncthreads();
    // set every remaining x_j = 1: the sum of the class's coefficients, fixed order
    const int pl = n < K + 1 ? n : K + 1;
    const int cnt = cstart[pl + 1] - cstart[pl];
    dd r{0.0, 0.0}, q{0.0, 0.0};
    for (int t = tid; t < cnt; t += kBlock) {
      dd_acc(r, s_c[cur][t].re);
      if constexpr (CPLX) dd_acc(q, s_c[cur][t].im);
    }
    r = wave_sum(r);
    if constexpr (CPLX) q = wave_sum(q);
    const dd R = block_sum(r, dd_add);
    dd I{0.0, 0.0};
    if constexpr (CPLX) {
      __syncthreads();  // the two sums share block_sum's slots
      I = block_sum(q, dd_add);
    }
    if (tid == 0) {
      double* o = a.out + 4 * (size_t)m;
      o[0] = bad ? 0.0 : ldexp(R.hi, esum);
      o[1] = bad ? 0.0 : ldexp(R.lo, esum);
      o[2] = bad ? 0.0 : ldexp(I.hi, esum);
      o[3] = bad ? 0.0 : ldexp(I.lo, esum);
      if (a.status) a.status[m] = bad ? kStNonFinite : kStOk;
    }
    __syncthreads();
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
