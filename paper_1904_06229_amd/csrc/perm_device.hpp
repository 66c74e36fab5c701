// Device helpers shared by the Gray-walk kernels (gfx950, wave64).
//
// Layout of a staged matrix (written by the staging kernels): the n x n
// matrix, column-major with ld = n, followed by its negation.  Column j of
// +A starts at staged + j*n, column j of -A at staged + n*n + j*n (complex:
// interleaved pairs, offsets doubled).  Every lane of a wave flips the same
// column in the same direction at the same step, so a column is read with
// scalar loads into SGPRs and fed to v_add_f64 as a scalar operand: the
// matrix never occupies LDS or VGPRs and costs no VALU issue slots.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "perm_internal.hpp"

namespace perm {

// Read-only view of device memory in the constant address space: uniform
// reads through it become scalar (s_load) reads.
typedef const __attribute__((address_space(4))) double* cdptr;

__device__ __forceinline__ cdptr as_const(const double* p) { return (cdptr)(p); }

// The same (uniform) pointer, hidden from the optimiser.  Without this the
// column reads of a chunk start are loop-invariant across chunks, get hoisted
// out of the chunk loop and stay resident -- the whole matrix in VGPRs, which
// costs occupancy.  The empty asm emits no instruction.
__device__ __forceinline__ const double* opaque(const double* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// The (uniform) pointer p, released only once v has been computed.  A column
// of a large complex matrix is more data than the scalar registers hold, so
// its reads are split into blocks, and each block's reads are tied to the
// update of an earlier block: the loads in flight then never exceed what the
// SGPRs hold (otherwise the compiler issues them all at once and spills the
// SGPRs into VGPR lanes, which costs VALU instructions in the walk).  The
// empty asm emits no instruction.
__device__ __forceinline__ const double* after(const double* p, double v) {
  asm volatile("" : "+s"(p) : "v"(v));
  return p;
}

// ---------------------------------------------------------------- gray ----

__device__ __forceinline__ uint64_t gray(uint64_t k) { return k ^ (k >> 1); }

// ------------------------------------------------------- double-double ----
// Error-free transformations (Knuth's TwoSum, Dekker's FastTwoSum,
// TwoProduct with fma).  Every file including this header is compiled with
// -ffp-contract=off and without fast-math, so none of these is fused or
// re-associated.

struct dd {
  double hi, lo;
};

// a += b for a double b: TwoSum into hi, the rounding error into lo.  lo is
// not renormalised on every add; it only collects errors (each below half an
// ulp of hi), so its own rounding is negligible for the chunk lengths used.
__device__ __forceinline__ void dd_acc(dd& a, double b) {
  double s = a.hi + b;
  double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (b - bb);
  a.hi = s;
  a.lo += e;
}

__device__ __forceinline__ dd dd_norm(dd a) {
  double s = a.hi + a.lo;
  return dd{s, a.lo - (s - a.hi)};
}

// Accurate double-double sum (two TwoSums and two renormalisations).
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double s = a.hi + b.hi;
  double bs = s - a.hi;
  double e = (a.hi - (s - bs)) + (b.hi - bs);
  double t = a.lo + b.lo;
  double bt = t - a.lo;
  double f = (a.lo - (t - bt)) + (b.lo - bt);
  e += t;
  double s2 = s + e;
  e = e - (s2 - s);
  e += f;
  double s3 = s2 + e;
  e = e - (s3 - s2);
  return dd{s3, e};
}

// ------------------------------------------------------ wave reductions ----

__device__ __forceinline__ dd wave_sum(dd v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    dd o{__shfl_xor(v.hi, off), __shfl_xor(v.lo, off)};
    v = dd_add(v, o);
  }
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

struct u128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ u128 u128_add(u128 a, u128 b) {
  uint64_t lo = a.lo + b.lo;
  uint64_t c = lo < a.lo ? 1u : 0u;
  return u128{lo, a.hi + b.hi + c};
}

__device__ __forceinline__ u128 wave_sum(u128 v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    u128 o{(uint64_t)__shfl_xor((unsigned long long)v.lo, off),
           (uint64_t)__shfl_xor((unsigned long long)v.hi, off)};
    v = u128_add(v, o);
  }
  return v;
}

// Sum one value per wave of the workgroup in wave order; thread 0 gets it.
template <class T, class Add>
__device__ __forceinline__ T block_sum(T v, Add add) {
  __shared__ T slots[kWavesPerBlock];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  if (lane == 0) slots[wave] = v;
  __syncthreads();
  T r = slots[0];
  if (threadIdx.x == 0)
    for (int w = 1; w < kWavesPerBlock; ++w) r = add(r, slots[w]);
  return r;
}

// ------------------------------------------------------------ products ----
// Products of the row sums.  kChains independent multiply chains give the
// VALU independent work; the chains are then multiplied together.

template <int N>
struct Chains {
  static constexpr int value = N >= 16 ? 4 : (N >= 6 ? 2 : 1);
};

template <int N>
__device__ __forceinline__ double prod_f64(const double (&w)[N]) {
  constexpr int C = Chains<N>::value;
  double c[C];
#pragma unroll
  for (int k = 0; k < C; ++k) c[k] = w[k];
#pragma unroll
  for (int i = C; i < N; ++i) c[i % C] *= w[i];
  double p = c[0];
#pragma unroll
  for (int k = 1; k < C; ++k) p *= c[k];
  return p;
}

// FP32 product of FP64 row sums (the split-precision walk).
template <int N>
__device__ __forceinline__ double prod_f32(const double (&w)[N]) {
  constexpr int C = Chains<N>::value;
  float c[C];
#pragma unroll
  for (int k = 0; k < C; ++k) c[k] = (float)w[k];
#pragma unroll
  for (int i = C; i < N; ++i) c[i % C] *= (float)w[i];
  float p = c[0];
#pragma unroll
  for (int k = 1; k < C; ++k) p *= c[k];
  return (double)p;
}

// Complex product (4 VALU ops per complex multiply: mul, fma, mul, fma).
template <int N>
__device__ __forceinline__ void prod_c64(const double (&wr)[N], const double (&wi)[N],
                                         double& pr, double& pi) {
  constexpr int C = Chains<N>::value;
  double cr[C], ci[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    cr[k] = wr[k];
    ci[k] = wi[k];
  }
#pragma unroll
  for (int i = C; i < N; ++i) {
    const int k = i % C;
    double t = ci[k] * wi[i];
    double u = ci[k] * wr[i];
    double nr = fma(cr[k], wr[i], -t);
    double ni = fma(cr[k], wi[i], u);
    cr[k] = nr;
    ci[k] = ni;
  }
  pr = cr[0];
  pi = ci[0];
#pragma unroll
  for (int k = 1; k < C; ++k) {
    double t = pi * ci[k];
    double u = pi * cr[k];
    double nr = fma(pr, cr[k], -t);
    double ni = fma(pr, ci[k], u);
    pr = nr;
    pi = ni;
  }
}

template <int N>
__device__ __forceinline__ void prod_c32(const double (&wr)[N], const double (&wi)[N],
                                         double& pr, double& pi) {
  constexpr int C = Chains<N>::value;
  float cr[C], ci[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    cr[k] = (float)wr[k];
    ci[k] = (float)wi[k];
  }
#pragma unroll
  for (int i = C; i < N; ++i) {
    const int k = i % C;
    float xr = (float)wr[i], xi = (float)wi[i];
    float t = ci[k] * xi;
    float u = ci[k] * xr;
    float nr = fmaf(cr[k], xr, -t);
    float ni = fmaf(cr[k], xi, u);
    cr[k] = nr;
    ci[k] = ni;
  }
  float r = cr[0], m = ci[0];
#pragma unroll
  for (int k = 1; k < C; ++k) {
    float t = m * ci[k];
    float u = m * cr[k];
    float nr = fmaf(r, cr[k], -t);
    float ni = fmaf(r, ci[k], u);
    r = nr;
    m = ni;
  }
  pr = (double)r;
  pi = (double)m;
}

// ------------------------------------------------------------ row sums ----
// Start vector of a chunk (App. A, subpermanent, written as
// w_i = 1/2 (a_{i,n} + sum_{j<n} delta_j a_ij), delta_j = 2 x_j - 1), formed
// directly from the staged +A for the Gray code of term index g.

template <int N>
__device__ __forceinline__ void form_w_real(const double* __restrict__ staged, uint64_t g,
                                            double (&w)[N]) {
  const uint64_t x = gray(g);
  cdptr last = as_const(staged + (N - 1) * N);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = last[i];
#pragma unroll 1
  for (int j = 0; j < N - 1; ++j) {
    const double d = ((x >> j) & 1) ? 1.0 : -1.0;
    cdptr col = as_const(staged + j * N);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = fma(d, col[i], w[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] *= 0.5;
}

template <int N>
__device__ __forceinline__ void form_w_complex(const double* __restrict__ staged, uint64_t g,
                                               double (&wr)[N], double (&wi)[N]) {
  const uint64_t x = gray(g);
  cdptr last = as_const(staged + 2 * (N - 1) * N);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wr[i] = last[2 * i];
    wi[i] = last[2 * i + 1];
  }
#pragma unroll 1
  for (int j = 0; j < N - 1; ++j) {
    const double d = ((x >> j) & 1) ? 1.0 : -1.0;
    cdptr col = as_const(staged + 2 * j * N);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      wr[i] = fma(d, col[2 * i], wr[i]);
      wi[i] = fma(d, col[2 * i + 1], wi[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wr[i] *= 0.5;
    wi[i] *= 0.5;
  }
}

// Direction of the flip between term g and g+1 of an aligned chunk.
// Within a chunk of L = 2^b terms starting at G*L, going from step s to
// s+1 flips bit j = ctz(s+1) of the Gray code (App. A, nextset); the bit
// becomes 1 (column added) unless bit j+1 of g+1 is set.  For j+1 < b that
// bit lies inside the chunk and is the same for every lane; for j+1 = b it
// is bit 0 of the chunk index G, which the lane mapping keeps uniform per
// wave (gpar).  Returns 1 when the column is subtracted.  Integer flags (not
// bool) keep the value in SGPRs instead of a lane mask.
__device__ __forceinline__ uint32_t flip_subtracts(uint32_t s1, int j, int b, uint32_t gpar) {
  return (j + 1 < b) ? ((s1 >> (j + 1)) & 1u) : gpar;
}

// Index of the calling wave in the grid, as a wave-uniform (SGPR) value.
__device__ __forceinline__ uint64_t wave_id() {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  return (uint64_t)blockIdx.x * kWavesPerBlock + w;
}

// Lane -> chunk mapping.  Wave task v covers chunks 2*(64*(v>>1) + lane) +
// (v & 1) of the body: all 64 chunks of a task share the parity of their
// index, so the mid-chunk flip direction above is wave-uniform.
__device__ __forceinline__ uint64_t task_chunk(uint64_t task, int lane) {
  return 2 * (uint64_t(kWave) * (task >> 1) + (uint64_t)lane) + (task & 1);
}

}  // namespace perm
