// Band transfer matrix (App. C, bandpermanent) for matrices with a_ij = 0
// when |i - j| > k.
//
// per(A) is the coefficient sum of prod_i C_i, C_i = sum_j a_ij x_j, taken
// with x_j^2 = 0 (each column used once).  After row i the variable of
// column i-k-1 is set to 1: no later row reaches that column.  The live
// polynomial therefore has monomials over the 2k+1 columns [i-k, i+k] only:
// 2^(2k+1) coefficients, kept in LDS, bit b of a mask standing for column
// i-k+b.
//
// One row in gather form: the new coefficient of mask M (window after the
// row) is the sum over the state of column i-k-1 (bit 0 of Q = 2M + b0, the
// column dropped by the shift) of P[Q], and P[Q] = sum over the band columns
// j in Q of old[Q without j] * a_ij.  Column i+k is new in this row, so a Q
// holding it can only come from j = i+k.  Each thread owns masks t, t+256, ...
// and reads the old coefficients from the other LDS buffer.
//
// One workgroup per matrix (grid-stride over the batch).  Row entries are
// wave-uniform and read with scalar loads.  Powers of two keep long products
// in range, exactly: each row's entries are scaled into [1/2, 1), and every
// 4 rows the coefficients are scaled by the power of two of their largest
// magnitude (a workgroup max); the exponents are added up and restored at the
// end.  The final coefficient sum is a fixed-order double-double tree.
#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

template <int K, bool CPLX>
__global__ __launch_bounds__(kBlock) void band_kernel(BandArgs a) {
  constexpr int S = 1 << (2 * K + 1);   // coefficients after a row
  constexpr int TOP = 2 * K + 1;        // bit of column i+k in Q
  constexpr int cw = CPLX ? 2 : 1;
  __shared__ double s_re[2][S];
  __shared__ double s_im[CPLX ? 2 : 1][CPLX ? S : 1];
  __shared__ dd s_red[kBlock], s_red_i[CPLX ? kBlock : 1];
  __shared__ double s_mx[kWavesPerBlock];
  const int tid = threadIdx.x;
  typedef const __attribute__((address_space(4))) int32_t* ci32;
  typedef const __attribute__((address_space(4))) int64_t* ci64;
  for (int m = blockIdx.x; m < a.count; m += gridDim.x) {
    const int n = ((ci32)a.n)[m];  // uniform: scalar loads
    const double* A = a.A + ((ci64)a.off)[m];
    for (int t = tid; t < S; t += kBlock) {
      s_re[0][t] = t == 0 ? 1.0 : 0.0;
      if constexpr (CPLX) s_im[0][t] = 0.0;
    }
    int cur = 0, esum = 0;
    bool bad = false;
    __syncthreads();
    for (int i = 0; i < n; ++i) {
      // band entries of row i: c = 1..2k+1 <-> column j = i-k-1+c
      double ar[TOP + 1], ai[TOP + 1];
      double mx = 0.0;
#pragma unroll
      for (int c = 1; c <= TOP; ++c) {
        const int j = i - K - 1 + c;
        const bool in = j >= 0 && j < n;
        cdptr p = as_const(A + (size_t)cw * ((size_t)i + (size_t)(in ? j : 0) * n));
        ar[c] = in ? p[0] : 0.0;
        ai[c] = (CPLX && in) ? p[1] : 0.0;
        if (!isfinite(ar[c]) || !isfinite(ai[c])) bad = true;
        mx = fmax(mx, fmax(fabs(ar[c]), fabs(ai[c])));
      }
      int e = 0;
      if (mx > 0.0 && !bad) {
        frexp(mx, &e);  // mx in [2^(e-1), 2^e): scale the row by 2^-e
#pragma unroll
        for (int c = 1; c <= TOP; ++c) {
          ar[c] = ldexp(ar[c], -e);
          ai[c] = ldexp(ai[c], -e);
        }
      }
      esum += e;
      const double* ore = s_re[cur];
      const double* oim = CPLX ? s_im[cur] : nullptr;
      double* nre = s_re[cur ^ 1];
      double* nim = CPLX ? s_im[cur ^ 1] : nullptr;
      for (int t = tid; t < S; t += kBlock) {
        double vr = 0.0, vi = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < 2; ++b0) {
          const int Q = (t << 1) | b0;
          if ((Q >> TOP) & 1) {
            const int o = Q ^ (1 << TOP);
            const double xr = ore[o];
            vr = fma(xr, ar[TOP], vr);
            if constexpr (CPLX) {
              const double xi = oim[o];
              vr = fma(-xi, ai[TOP], vr);
              vi = fma(xr, ai[TOP], fma(xi, ar[TOP], vi));
            }
          } else {
#pragma unroll
            for (int c = 1; c < TOP; ++c) {
              if ((Q >> c) & 1) {
                const int o = Q ^ (1 << c);
                const double xr = ore[o];
                vr = fma(xr, ar[c], vr);
                if constexpr (CPLX) {
                  const double xi = oim[o];
                  vr = fma(-xi, ai[c], vr);
                  vi = fma(xr, ai[c], fma(xi, ar[c], vi));
                }
              }
            }
          }
        }
        nre[t] = vr;
        if constexpr (CPLX) nim[t] = vi;
      }
      cur ^= 1;
      __syncthreads();
      if ((i & 3) == 3 || i == n - 1) {  // renormalise by a power of two
        double lm = 0.0;
        for (int t = tid; t < S; t += kBlock) {
          lm = fmax(lm, fabs(s_re[cur][t]));
          if constexpr (CPLX) lm = fmax(lm, fabs(s_im[cur][t]));
        }
        lm = wave_max(lm);
        if ((tid & (kWave - 1)) == 0) s_mx[tid / kWave] = lm;
        __syncthreads();
        double M = s_mx[0];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) M = fmax(M, s_mx[w]);
        int ex = 0;
        if (M > 0.0 && isfinite(M)) frexp(M, &ex);
        if (ex != 0) {
          for (int t = tid; t < S; t += kBlock) {
            s_re[cur][t] = ldexp(s_re[cur][t], -ex);
            if constexpr (CPLX) s_im[cur][t] = ldexp(s_im[cur][t], -ex);
          }
        }
        esum += ex;
        __syncthreads();
      }
    }
    // set every remaining x_j = 1: the sum of the coefficients, fixed order
    dd r{0.0, 0.0}, q{0.0, 0.0};
    for (int t = tid; t < S; t += kBlock) {
      dd_acc(r, s_re[cur][t]);
      if constexpr (CPLX) dd_acc(q, s_im[cur][t]);
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
