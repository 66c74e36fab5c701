// Gray-code walk for complex matrices (App. A, subpermanent; Sec. II.B).
//
// Same structure as the real walk (kern_real.hip): one lane per chunk of
// 2^b terms, terms taken in pairs (signs -1, +1), the column of each flip
// read through scalar loads.  Per term: the complex product of the n row
// sums (n-1 complex multiplies of 4 VALU ops: mul, fma, mul, fma), the
// signed accumulation of real and imaginary parts, and 2n v_add_f64 for the
// update of real and imaginary row sums.
//
// MODE 0: FP64 products, double-double lane sums (default)
// MODE 1: FP64 products, plain FP64 lane sums
// MODE 2: FP32 products of the FP64 row sums, double-double lane sums
#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

template <int N, int MODE>
__device__ __forceinline__ void term_prod(const double (&wr)[N], const double (&wi)[N],
                                          double& pr, double& pi) {
  if constexpr (MODE == 2)
    prod_c32<N>(wr, wi, pr, pi);
  else
    prod_c64<N>(wr, wi, pr, pi);
}

template <int N>
__device__ __forceinline__ void add_col(double (&wr)[N], double (&wi)[N],
                                        const double* __restrict__ staged, uint32_t sub, int j) {
  cdptr col = as_const(staged + sub * (2 * N * N) + 2 * j * N);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wr[i] += col[2 * i];
    wi[i] += col[2 * i + 1];
  }
}

template <int MODE>
__device__ __forceinline__ void lane_acc(dd& acc, double q) {
  if constexpr (MODE == 1)
    acc.hi += q;
  else
    dd_acc(acc, q);
}

struct cdd {
  dd re, im;
};

template <int N, int MODE, bool DRIFT>
__device__ __forceinline__ cdd walk_chunk(const double* __restrict__ staged,
                                          const double* __restrict__ rowabs, uint64_t G, int b,
                                          uint32_t gpar, double& drift) {
  double wr[N], wi[N];
  form_w_complex<N>(staged, G << b, wr, wi);
  cdd acc{{0.0, 0.0}, {0.0, 0.0}};
  if (b == 0) {
    double pr, pi;
    term_prod<N, MODE>(wr, wi, pr, pi);
    const bool pos = (G & 1) != 0;
    acc.re.hi = pos ? pr : -pr;
    acc.im.hi = pos ? pi : -pi;
    return acc;
  }
  const uint32_t half = 1u << (b - 1);
  uint32_t t = 0;
  for (; t + 1 < half; ++t) {
    double p0r, p0i, p1r, p1i;
    term_prod<N, MODE>(wr, wi, p0r, p0i);
    add_col<N>(wr, wi, staged, t & 1u, 0);
    term_prod<N, MODE>(wr, wi, p1r, p1i);
    const uint32_t s1 = 2 * t + 2;
    const int j = __builtin_ctz(s1);
    add_col<N>(wr, wi, staged, flip_subtracts(s1, j, b, gpar), j);
    lane_acc<MODE>(acc.re, p1r - p0r);
    lane_acc<MODE>(acc.im, p1i - p0i);
  }
  {
    double p0r, p0i, p1r, p1i;
    term_prod<N, MODE>(wr, wi, p0r, p0i);
    add_col<N>(wr, wi, staged, (b >= 2) ? (t & 1u) : gpar, 0);
    term_prod<N, MODE>(wr, wi, p1r, p1i);
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

template <int N, int MODE, bool DRIFT>
__global__ __launch_bounds__(kBlock) void walk_complex_kernel(WalkArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  dd re{0.0, 0.0}, im{0.0, 0.0};
  double drift = 0.0;
  if (a.status[0] == kStOk) {
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      const uint32_t gpar = (uint32_t)((a.first + (task & 1)) & 1);
      double dr = 0.0;
      const cdd part =
          walk_chunk<N, MODE, DRIFT>(a.staged, a.rowabs, a.first + c, a.b, gpar, dr);
      if (c < a.nchunks) {
        re = dd_add(re, part.re);
        im = dd_add(im, part.im);
        drift = fmax(drift, dr);
      }
    }
  }
  const dd vr = wave_sum(re);
  const dd vi = wave_sum(im);
  const dd br = block_sum(vr, dd_add);
  __syncthreads();
  const dd bi = block_sum(vi, dd_add);
  double* out = (double*)a.partials;
  if (threadIdx.x == 0) {
    out[4 * blockIdx.x] = br.hi;
    out[4 * blockIdx.x + 1] = br.lo;
    out[4 * blockIdx.x + 2] = bi.hi;
    out[4 * blockIdx.x + 3] = bi.lo;
  }
  if (DRIFT) {
    __syncthreads();
    const double m = wave_max(drift);
    const double bm = block_sum(m, [](double x, double y) { return fmax(x, y); });
    if (threadIdx.x == 0) a.drift_part[blockIdx.x] = bm;
  }
}

template <int N>
hipError_t dispatch(int mode, bool drift, const WalkArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), blk(kBlock);
  if (drift) {
    switch (mode) {
      case 0: hipLaunchKernelGGL((walk_complex_kernel<N, 0, true>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((walk_complex_kernel<N, 1, true>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((walk_complex_kernel<N, 2, true>), g, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (mode) {
      case 0: hipLaunchKernelGGL((walk_complex_kernel<N, 0, false>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((walk_complex_kernel<N, 1, false>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((walk_complex_kernel<N, 2, false>), g, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

#define PERM_CASE(N) \
  case N:            \
    return dispatch<N>(mode, drift, a, grid, s);

hipError_t launch_walk_complex(int n, int mode, bool drift, const WalkArgs& a, int grid,
                               hipStream_t s) {
  switch (n) {
#include "perm_cases.inc"
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace perm
