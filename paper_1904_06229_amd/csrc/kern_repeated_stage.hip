// Staging for the repeated-column walk (Sec. II.A, Eq. ryser2).
//
// One workgroup.  Checks C for NaN/infinity, picks power-of-two row scales
// (row i of C scales row i of the expanded matrix, so per(DA) = prod_i d_i
// per(A) as for the dense path), and writes
//   staged : [+C | 0] [-C | 0]  (n x (R+1) each, column-major, ld = n), then
//            the two start columns sum_{k<b} f_k(start) c_k (chunk parity 0, 1)
//   binom  : C(m_k, f) for every digit k, from Pascal's rule in exact 64-bit
//            integers (C(64, 32) < 2^64), each rounded once to double
//   radix  : m_k + 1
//   tin    : signed weight (-1)^(f_0+...+f_{b-1}) prod_{k<b} C(m_k, f_k) of the
//            inner digits at step s of a chunk of parity 0 or 1
//   toff   : offset of the column added after step s (+c_j or -c_j for the
//            changed digit j; the zero column after the chunk's last step).
//
// Reflected mixed-radix Gray order, digit 0 fastest: with Q_k = r_0...r_{k-1}
// and counting digit a_k = floor(g / Q_k) mod r_k, the Gray digit is
// f_k = a_k when floor(g / Q_{k+1}) is even and r_k - 1 - a_k when it is odd.
// Inside a chunk (g = c L + s, L = Q_b) the parity of floor(g / Q_{k+1}) for
// k < b is that of c (L / Q_{k+1}) + floor(s / Q_{k+1}), so the inner digits
// depend only on s and the parity of c.  Going from s to s + 1 changes the
// digit j = max{ j : Q_j divides s + 1 } by one.
#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

__device__ __forceinline__ uint32_t inner_digit(uint32_t s, int k, uint32_t par, uint32_t L,
                                                const uint32_t* Q, const int32_t* r) {
  const uint32_t a = (s / Q[k]) % (uint32_t)r[k];
  const uint32_t hi = par * (L / Q[k + 1]) + s / Q[k + 1];
  return (hi & 1u) ? (uint32_t)r[k] - 1u - a : a;
}

__global__ __launch_bounds__(kBlock) void stage_rep_kernel(const double* __restrict__ C, int n,
                                                           int R, int ld, int is_complex,
                                                           RepMult mult, int b, int L,
                                                           int row_scaling, double* staged,
                                                           double* binom, double* tin,
                                                           int32_t* toff, int32_t* radix,
                                                           int32_t* rowexp, int32_t* status) {
  __shared__ uint64_t s_pascal[kMaxN + 1][kMaxN + 1];
  __shared__ int32_t s_exp[kMaxN], s_r[kMaxN];
  __shared__ uint32_t s_Q[kMaxN + 1];
  __shared__ int32_t s_bad;
  const int tid = threadIdx.x;
  const int cw = is_complex ? 2 : 1;
  if (tid == 0) s_bad = 0;
  if (tid < R) s_r[tid] = mult.m[tid] + 1;
  // Pascal's triangle, one row per step
  if (tid <= kMaxN) s_pascal[0][tid] = tid == 0 ? 1 : 0;
  __syncthreads();
  for (int m = 1; m <= kMaxN; ++m) {
    if (tid <= kMaxN) s_pascal[m][tid] = (tid == 0 ? 0 : s_pascal[m - 1][tid - 1]) + s_pascal[m - 1][tid];
    __syncthreads();
  }
  if (tid == 0) {
    s_Q[0] = 1;
    for (int k = 0; k < b; ++k) s_Q[k + 1] = s_Q[k] * (uint32_t)s_r[k];
  }
  if (tid < n) {
    const int i = tid;
    double mx = 0.0;
    bool bad = false;
    for (int k = 0; k < R; ++k)
      for (int c = 0; c < cw; ++c) {
        const double v = C[cw * ((size_t)i + (size_t)k * ld) + c];
        if (!isfinite(v)) bad = true;
        mx = fmax(mx, fabs(v));
      }
    int e = 0;
    if (!bad && row_scaling && mx > 0.0) {
      double ss = 0.0;  // squared 2-norm of row i of the expanded matrix, over mx^2
      for (int k = 0; k < R; ++k)
        for (int c = 0; c < cw; ++c) {
          const double v = C[cw * ((size_t)i + (size_t)k * ld) + c] / mx;
          ss += (double)mult.m[k] * v * v;
        }
      int q;
      frexp(mx * sqrt(ss), &q);
      e = 2 - q;
      e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
    }
    s_exp[i] = e;
    rowexp[i] = e;
    if (bad) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  const int cols = (R + 1) * n;  // entries of [+C | 0]
  for (int idx = tid; idx < cols; idx += kBlock) {
    const int i = idx % n, k = idx / n;
    for (int c = 0; c < cw; ++c) {
      const double v = k < R ? ldexp(C[cw * ((size_t)i + (size_t)k * ld) + c], s_exp[i]) : 0.0;
      staged[cw * idx + c] = v;
      staged[cw * (cols + idx) + c] = k < R ? -v : 0.0;
    }
  }
  for (int idx = tid; idx < R * kRepBinomStride; idx += kBlock) {
    const int k = idx / kRepBinomStride, f = idx % kRepBinomStride;
    binom[idx] = f <= mult.m[k] ? (double)s_pascal[mult.m[k]][f] : 0.0;
  }
  if (tid < R) radix[tid] = s_r[tid];
  const uint32_t uL = (uint32_t)L;
  for (int t = tid; t < 2 * L; t += kBlock) {
    const uint32_t par = (uint32_t)(t / L), s = (uint32_t)(t % L);
    double wgt = 1.0;
    uint32_t odd = 0;
    for (int k = 0; k < b; ++k) {
      const uint32_t f = inner_digit(s, k, par, uL, s_Q, s_r);
      odd ^= f & 1u;
      wgt *= (double)s_pascal[mult.m[k]][f];
    }
    tin[t] = odd ? -wgt : wgt;
    int32_t off = R * n * cw;  // zero column
    if (s + 1 < uL) {
      int j = b - 1;
      while (j > 0 && (s + 1) % s_Q[j] != 0) --j;
      const uint32_t f0 = inner_digit(s, j, par, uL, s_Q, s_r);
      const uint32_t f1 = inner_digit(s + 1, j, par, uL, s_Q, s_r);
      off = ((f1 > f0) ? j : (R + 1) + j) * n * cw;
    }
    toff[t] = off;
  }
  __syncthreads();  // staged +C is complete
  for (int t = tid; t < 2 * n; t += kBlock) {
    const uint32_t par = (uint32_t)(t / n);
    const int i = t % n;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < b; ++k) {
      const uint32_t f = inner_digit(0, k, par, uL, s_Q, s_r);
      sr = fma((double)f, staged[cw * (i + k * n)], sr);
      if (cw == 2) si = fma((double)f, staged[cw * (i + k * n) + 1], si);
    }
    const int o = cw * (2 * cols + t);
    staged[o] = sr;
    if (cw == 2) staged[o + 1] = si;
  }
  if (tid == 0) status[0] = s_bad ? kStNonFinite : kStOk;
}

}  // namespace

hipError_t launch_rep_stage(int is_complex, const double* C, int n, int R, int ld,
                            const RepMult& mult, int b, int L, int row_scaling, double* staged,
                            double* binom, double* tin, int32_t* toff, int32_t* radix,
                            int32_t* rowexp, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(stage_rep_kernel, dim3(1), dim3(kBlock), 0, s, C, n, R, ld, is_complex, mult,
                     b, L, row_scaling, staged, binom, tin, toff, radix, rowexp, status);
  return hipGetLastError();
}

}  // namespace perm
