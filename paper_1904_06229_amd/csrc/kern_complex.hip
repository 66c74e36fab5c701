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
#include "perm_walk.hpp"

namespace perm {
namespace {

// Sizes from kSplitFrom on keep rows [R, n) of the row sums in LDS (the
// plain chunk walk; drift-checked and single-term launches keep every row in
// registers) and run two waves per SIMD.
template <int N, bool DRIFT, bool SINGLE>
constexpr bool split_rows() {
  return N >= kSplitFrom && !DRIFT && !SINGLE;
}

template <int N, int MODE, bool DRIFT, bool SINGLE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(split_rows<N, DRIFT, SINGLE>() ? 2 : 1)))
void walk_complex_kernel(WalkArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  dd re{0.0, 0.0}, im{0.0, 0.0};
  double drift = 0.0;
  double2* rows = nullptr;
  if constexpr (split_rows<N, DRIFT, SINGLE>()) rows = lane_rows<SplitRows<N>::L>();
  if (a.status[0] == kStOk) {
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      const uint32_t gpar = (uint32_t)((a.first + (task & 1)) & 1);
      double dr = 0.0;
      cdd part;
      if constexpr (SINGLE)
        part = single_term_complex<N, MODE>(a.staged, a.first + c);
      else if constexpr (split_rows<N, DRIFT, SINGLE>())
        part = walk_chunk_complex_split<N, MODE>(a.staged, a.first + c, a.b, gpar, rows);
      else
        part = walk_chunk_complex<N, MODE, DRIFT>(a.staged, a.rowabs, a.first + c, a.b, gpar, dr);
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
  // drift-checked calls: every launch writes its slot (the single-term launches
  // of unaligned range ends, which cannot drift, write 0)
  if (DRIFT || a.drift) {
    __syncthreads();
    const double m = wave_max(drift);
    const double bm = block_sum(m, [](double x, double y) { return fmax(x, y); });
    if (threadIdx.x == 0) a.drift_part[blockIdx.x] = bm;
  }
}

template <int N>
hipError_t dispatch(int mode, bool drift, const WalkArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), blk(kBlock);
  if (a.b == 0) {  // single-term chunks (unaligned range ends); no drift to check
    switch (mode) {
      case 0: hipLaunchKernelGGL((walk_complex_kernel<N, 0, false, true>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((walk_complex_kernel<N, 1, false, true>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((walk_complex_kernel<N, 2, false, true>), g, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else if (drift) {
    switch (mode) {
      case 0: hipLaunchKernelGGL((walk_complex_kernel<N, 0, true, false>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((walk_complex_kernel<N, 1, true, false>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((walk_complex_kernel<N, 2, true, false>), g, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (mode) {
      case 0: hipLaunchKernelGGL((walk_complex_kernel<N, 0, false, false>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((walk_complex_kernel<N, 1, false, false>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((walk_complex_kernel<N, 2, false, false>), g, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

#define PERM_CASE(N) \
  case N:            \
    return dispatch<N>(mode, drift, a, grid, s);

// Compiled twice: PERM_HALF = 0 instantiates n = 1..32, PERM_HALF = 1 n = 33..64
// (two translation units that build in parallel).
#if PERM_HALF == 0
#define PERM_LAUNCH launch_walk_complex_lo
#define PERM_CASES "perm_cases_lo.inc"
#else
#define PERM_LAUNCH launch_walk_complex_hi
#define PERM_CASES "perm_cases_hi.inc"
#endif

hipError_t PERM_LAUNCH(int n, int mode, bool drift, const WalkArgs& a, int grid,
                               hipStream_t s) {
  switch (n) {
#include PERM_CASES
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace perm
