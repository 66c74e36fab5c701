// Band transfer matrix (App. C, bandpermanent) for matrices with a_ij = 0
// when |i - j| > k.
//
// per(A) is the coefficient sum of prod_i C_i, C_i = sum_j a_ij x_j, taken
// with x_j^2 = 0 (each column used once).  After row i the variable of
// column i-k-1 is set to 1: no later row reaches that column.  The polynomial
// then lives on the 2k+1 columns [i-k, i+k]; bit b of a mask stands for
// column i-k+b.
//
// Only one popcount class of masks can carry a term that survives to the
// end.  After row i, rows 0..i have used i+1 columns, and every column below
// i-k must be among them (no later row reaches it); so a surviving monomial
// holds exactly p_i = min(i+1, k+1) columns of the window.  A monomial with
// fewer columns never arises, and one with more has skipped a column for good:
// all its descendants die by x_j^2 = 0 before the last row (pigeonhole), and
// it never feeds a mask of the surviving class.  The kernel therefore computes
// the p_i-class only.  Those coefficients are the same numbers the full
// polynomial holds (the other classes would only add exact zeros to them),
// and the final coefficient sum needs only them.
//
// One row, for a mask M of the new class: with b0 = 1 when column i-k-1
// exists (it must then be in the term) and Q = 2M + b0 over the columns
// [i-k-1, i+k], new[M] = sum over the band columns j in Q of old[Q \ j] a_ij.
// Column i+k is new in this row, so a Q holding it has the single term
// j = i+k; otherwise the sum runs over the p_i columns of M.  Each lane owns
// masks of one class (sorted by value, so a wave rarely mixes the two cases)
// and walks their set bits; the row's band entries sit in LDS.
//
// One workgroup per matrix (grid-stride over the batch).  The next row's band
// entries are loaded (as wave-uniform scalars) while the current row is
// computed, and the rows' entries alternate between two LDS slots, so one
// barrier per row suffices.  Powers of two keep long products in range,
// exactly: each row's entries are scaled into [1/2, 1), and every 4 rows the
// class's coefficients are scaled by the power of two of their largest
// magnitude; the exponents are restored at the end.
// The final coefficient sum is a fixed-order double-double tree.
#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

template <int K, bool CPLX>
__global__ __launch_bounds__(kBlock) void band_kernel(BandArgs a) {
  constexpr int W = 2 * K + 1;   // window columns
  constexpr int S = 1 << W;      // masks
  constexpr int TOP = W;         // bit of column i+k in Q
  constexpr int cw = CPLX ? 2 : 1;
  __shared__ double s_re[2][S];
  __shared__ double s_im[CPLX ? 2 : 1][CPLX ? S : 1];
  __shared__ uint16_t s_cls[S];          // masks grouped by popcount, ascending in a group
  __shared__ int32_t s_cls_start[W + 2];
  __shared__ double s_ar[2][W + 1], s_ai[2][CPLX ? W + 1 : 1];
  __shared__ dd s_red[kBlock], s_red_i[CPLX ? kBlock : 1];
  __shared__ double s_mx[kWavesPerBlock];
  typedef const __attribute__((address_space(4))) int32_t* ci32;
  typedef const __attribute__((address_space(4))) int64_t* ci64;
  const int tid = threadIdx.x;
  if (tid == 0) {  // counting sort of the masks by popcount
    int cnt[W + 2];
    for (int p = 0; p <= W + 1; ++p) cnt[p] = 0;
    for (int t = 0; t < S; ++t) ++cnt[__popc(t) + 1];
    s_cls_start[0] = 0;
    for (int p = 1; p <= W + 1; ++p) s_cls_start[p] = s_cls_start[p - 1] + cnt[p];
    for (int p = 0; p <= W; ++p) cnt[p] = s_cls_start[p];
    for (int t = 0; t < S; ++t) s_cls[cnt[__popc(t)]++] = (uint16_t)t;
  }
  __syncthreads();
  for (int m = blockIdx.x; m < a.count; m += gridDim.x) {
    const int n = ((ci32)a.n)[m];  // uniform: scalar loads
    const double* A = a.A + ((ci64)a.off)[m];
    if (tid == 0) {  // p = 0 class: the empty monomial, coefficient 1
      s_re[0][0] = 1.0;
      if constexpr (CPLX) s_im[0][0] = 0.0;
    }
    int cur = 0, esum = 0;
    bool bad = false;
    // Band entries of row i, c = 1..2k+1 <-> column j = i-k-1+c, as wave-uniform
    // values; the next row's are loaded while the current row is computed.
    double vr[TOP + 1], vi[TOP + 1];
    auto load_row = [&](int i) {
#pragma unroll
      for (int c = 1; c <= TOP; ++c) {
        const int j = i - K - 1 + c;
        const bool in = j >= 0 && j < n;
        cdptr p = as_const(A + (size_t)cw * ((size_t)i + (size_t)(in ? j : 0) * n));
        vr[c] = in ? p[0] : 0.0;
        vi[c] = (CPLX && in) ? p[1] : 0.0;
      }
    };
    load_row(0);
    for (int i = 0; i < n; ++i) {
      // row i's scale, and its entries into this row's LDS slot
      double mx = 0.0;
#pragma unroll
      for (int c = 1; c <= TOP; ++c) {
        if (!isfinite(vr[c]) || !isfinite(vi[c])) bad = true;
        mx = fmax(mx, fmax(fabs(vr[c]), fabs(vi[c])));
      }
      int e = 0;
      if (mx > 0.0 && !bad) frexp(mx, &e);  // scale the row by 2^-e
      esum += e;
      const int ab = i & 1;
#pragma unroll
      for (int c = 1; c <= TOP; ++c)
        if (tid == c) {
          s_ar[ab][c] = ldexp(vr[c], -e);
          if constexpr (CPLX) s_ai[ab][c] = ldexp(vi[c], -e);
        }
      if (i + 1 < n) load_row(i + 1);  // in flight during row i
      // one barrier: row i's entries, and row i-1's coefficients, are in LDS
      __syncthreads();
      const double* ar = s_ar[ab];
      const double* ai = s_ai[CPLX ? ab : 0];
      const int pcls = i + 1 < K + 1 ? i + 1 : K + 1;
      const int b0 = (i - K - 1 >= 0) ? 1 : 0;
      const int c0 = s_cls_start[pcls], c1 = s_cls_start[pcls + 1];
      const double* ore = s_re[cur];
      const double* oim = CPLX ? s_im[cur] : nullptr;
      double* nre = s_re[cur ^ 1];
      double* nim = CPLX ? s_im[cur ^ 1] : nullptr;
      for (int r = c0 + tid; r < c1; r += kBlock) {
        const int M = s_cls[r];
        const int Q = (M << 1) | b0;
        double xr_acc = 0.0, xi_acc = 0.0;
        if ((Q >> TOP) & 1) {
          const int o = Q ^ (1 << TOP);
          const double xr = ore[o];
          xr_acc = xr * ar[TOP];
          if constexpr (CPLX) {
            const double xi = oim[o];
            xr_acc = fma(-xi, ai[TOP], xr_acc);
            xi_acc = fma(xr, ai[TOP], xi * ar[TOP]);
          }
        } else {
          for (int q = Q & ~1; q; q &= q - 1) {
            const int c = __ffs(q) - 1;
            const int o = Q ^ (1 << c);
            const double xr = ore[o], arc = ar[c];
            xr_acc = fma(xr, arc, xr_acc);
            if constexpr (CPLX) {
              const double xi = oim[o], aic = ai[c];
              xr_acc = fma(-xi, aic, xr_acc);
              xi_acc = fma(xr, aic, fma(xi, arc, xi_acc));
            }
          }
        }
        nre[M] = xr_acc;
        if constexpr (CPLX) nim[M] = xi_acc;
      }
      cur ^= 1;
      if ((i & 3) == 3 || i == n - 1) {  // renormalise the class by a power of two
        __syncthreads();
        double lm = 0.0;
        for (int r = c0 + tid; r < c1; r += kBlock) {
          const int M = s_cls[r];
          lm = fmax(lm, fabs(s_re[cur][M]));
          if constexpr (CPLX) lm = fmax(lm, fabs(s_im[cur][M]));
        }
        lm = wave_max(lm);
        if ((tid & (kWave - 1)) == 0) s_mx[tid / kWave] = lm;
        __syncthreads();
        double Mx = s_mx[0];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) Mx = fmax(Mx, s_mx[w]);
        int ex = 0;
        if (Mx > 0.0 && isfinite(Mx)) frexp(Mx, &ex);
        if (ex != 0) {
          for (int r = c0 + tid; r < c1; r += kBlock) {
            const int M = s_cls[r];
            s_re[cur][M] = ldexp(s_re[cur][M], -ex);
            if constexpr (CPLX) s_im[cur][M] = ldexp(s_im[cur][M], -ex);
          }
        }
        esum += ex;
      }
    }
    __syncthreads();
    // set every remaining x_j = 1: the sum of the class's coefficients, fixed order
    const int pl = n < K + 1 ? n : K + 1;
    dd r{0.0, 0.0}, q{0.0, 0.0};
    for (int t = s_cls_start[pl] + tid; t < s_cls_start[pl + 1]; t += kBlock) {
      dd_acc(r, s_re[cur][s_cls[t]]);
      if constexpr (CPLX) dd_acc(q, s_im[cur][s_cls[t]]);
    }
    s_red[tid] = r;
    if constexpr (CPLX) s_red_i[tid] = q;
    __syncthreads();
    for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
      if (tid < stride) {
        s_red[tid] = dd_add(s_red[tid], s_red[tid + stride]);
        if constexpr (CPLX) s_red_i[tid] = dd_add(s_red_i[tid], s_red_i[tid + stride]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      double* o = a.out + 4 * (size_t)m;
      const dd R = s_red[0];
      const dd I = CPLX ? s_red_i[0] : dd{0.0, 0.0};
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

}  // namespace perm
