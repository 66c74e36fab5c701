// One-launch permanent of a small real or complex matrix (App. A,
// subpermanent and permanent over the whole range [0, 2^(n-1))).
//
// For small n the walk itself takes a few microseconds, and the separate
// staging and finishing launches (with the gaps between dependent launches)
// would cost more than it.  Here one launch does all three steps:
//
//   1. every workgroup stages its own copy of the matrix: the entries go to
//      LDS, each row gets its power-of-two scale (as stage_float_kernel:
//      row 2-norm in [2, 4), exact, undone by the host), and +A / -A are
//      written to the workgroup's own slot of device memory, from where the
//      walk reads its columns with scalar loads.  The slot is written and
//      read by this workgroup only; the stores are waited for before the
//      barrier, so the scalar loads (which go to L2) find them;
//   2. the waves walk their chunks as walk_real_kernel / walk_complex_kernel
//      do (same lane -> chunk map, same pair loop); only the chunk starts are
//      formed differently, the columns shared by a wave's lanes from LDS (see
//      fused_chunk_start), so the last bits can differ from those paths;
//   3. each workgroup writes its double-double partial, and the workgroup
//      that finishes last (a device-wide completion counter) adds all
//      partials in a fixed order (one wave: strided lane sums, then the
//      shuffle butterfly), writes the result record and sets the counter back
//      to zero for the next call.  The order of the sum does not depend on
//      which workgroup finishes last, so results are bit-reproducible.
//      The record also carries the launch's duration in wall-clock ticks:
//      from the earliest workgroup start (an atomic minimum) to the end.
//
// MODE 0: FP64 products, double-double lane sums (default)
// MODE 1: FP64 products, plain FP64 lane sums
// MODE 2: FP32 products of the FP64 row sums, double-double lane sums
#include "perm_walk.hpp"

namespace perm {
namespace {

// Threads that share one row in the row statistics (a power of two that
// divides the wave, kFusedMaxN * kRowThreads <= kBlock).
constexpr int kRowThreads = 8;
static_assert(kFusedMaxN * kRowThreads <= kBlock, "row statistics need a thread group per row");

// Lane moves inside groups of kRowThreads = 8 lanes (DPP, no LDS round trip):
// swap neighbours, swap pairs, then mirror the group (lane i <-> 7 - i).  The
// three steps give every lane of the group the combination of all eight.
constexpr int kDppXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppMirror8 = 0x141;  // row_half_mirror
static_assert(kRowThreads == 8, "the DPP steps combine groups of 8 lanes");

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <int N, bool CPLX>
__device__ __forceinline__ void fused_stage(const FusedArgs& a, double* slot, int32_t* s_exp,
                                            int32_t* s_bad, double* s_a) {
  constexpr int CW = CPLX ? 2 : 1;
  constexpr int TOT = CW * N * N;
  constexpr int LOADS = (TOT + kBlock - 1) / kBlock;
  const int tid = threadIdx.x;
  {
    double v[LOADS];
#pragma unroll
    for (int u = 0; u < LOADS; ++u) {
      const int t = tid + u * kBlock;
      const int idx = t / CW, c = t - CW * (t / CW);
      const int i = idx % N, j = idx / N;
      v[u] = t < TOT ? a.A[CW * ((size_t)i + (size_t)j * a.ld) + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LOADS; ++u) {
      const int t = tid + u * kBlock;
      if (t < TOT) s_a[t] = v[u];
    }
  }
  __syncthreads();
  // row statistics: kRowThreads threads per row, each over every
  // kRowThreads-th column, combined by DPP lane moves inside the group (fixed order)
  {
    const int i = tid / kRowThreads, sub = tid % kRowThreads;
    double mx = 0.0;
    int bad = 0;
    if (i < N) {
      for (int j = sub; j < N; j += kRowThreads)
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          const double x = s_a[CW * (i + j * N) + c];
          bad |= !isfinite(x);
          mx = fmax(mx, fabs(x));
        }
    }
    mx = fmax(mx, dpp_f64<kDppXor1>(mx));
    bad |= __builtin_amdgcn_mov_dpp(bad, kDppXor1, 0xF, 0xF, false);
    mx = fmax(mx, dpp_f64<kDppXor2>(mx));
    bad |= __builtin_amdgcn_mov_dpp(bad, kDppXor2, 0xF, 0xF, false);
    mx = fmax(mx, dpp_f64<kDppMirror8>(mx));
    bad |= __builtin_amdgcn_mov_dpp(bad, kDppMirror8, 0xF, 0xF, false);
    // the row scaled by 2^-k1 (mx = f 2^k1, f in [1/2, 1)): exact, no division,
    // every entry at most 1 in magnitude
    int k1 = 0;
    (void)frexp(mx, &k1);
    double ss = 0.0;
    if (i < N && !bad && mx > 0.0) {
      for (int j = sub; j < N; j += kRowThreads)
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          const double x = ldexp(s_a[CW * (i + j * N) + c], -k1);
          ss += x * x;
        }
    }
    ss += dpp_f64<kDppXor1>(ss);
    ss += dpp_f64<kDppXor2>(ss);
    ss += dpp_f64<kDppMirror8>(ss);
    if (i < N && sub == 0) {
      int e = 0;
      if (!bad && a.row_scaling && mx > 0.0) {
        // norm = 2^k1 sqrt(ss) in [2^(k-1), 2^k) with k = k1 + k2, sqrt(ss) =
        // g 2^k2, g in [1/2, 1)
        int k2;
        (void)frexp(sqrt(ss), &k2);
        const int k = k1 + k2;
        e = 2 - k;
        e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
      }
      s_exp[i] = e;
      if (bad) atomicOr(s_bad, 1);
    }
  }
  __syncthreads();
  for (int t = tid; t < TOT; t += kBlock) {
    const int i = (t / CW) % N;
    const double v = ldexp(s_a[t], s_exp[i]);
    s_a[t] = v;  // the chunk starts read the scaled entries from here
    slot[t] = v;
    slot[TOT + t] = -v;
  }
  // The walk reads the slot with scalar loads, which go to L2: wait until
  // this thread's stores have completed there, then meet the other waves.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

// Row sums at the start of chunk G (App. A: w = (1/2) sum_j delta_j a_j with
// delta_{n-1} = +1 and delta_j = 2 x_j - 1, x = gray(G 2^b)), from the scaled
// entries in LDS (s_a, column-major, CW doubles per entry) and the staged copy
// in device memory (slot).
//
// Every column read by a chunk start on the scalar path costs one scalar-load
// round trip, and with one wave per SIMD nothing hides it.  Under the lane ->
// chunk map the 64 lanes of a wave differ only in bits 1..6 of the chunk index,
// so only the Gray bits of columns b..b+6 differ between them.  The part of w
// from the other columns is the same for the whole wave: lane k sums component
// k (row k / CW) over them from LDS, all reads in flight at once, and leaves it
// in the wave's row of s_u, from where every lane reads the whole vector.  Each
// lane then adds its own columns b..b+6 on the scalar path.  A wave whose lanes
// disagree outside b..b+6 forms every column per lane instead.
template <int N, bool CPLX>
__device__ __forceinline__ void fused_chunk_start(const double* s_a, double* s_u,
                                                  const double* slot, uint64_t G, int b,
                                                  double (&wr)[N], double (&wi)[N]) {
  constexpr int CW = CPLX ? 2 : 1;
  const uint64_t x = gray(G << b);
  const uint64_t xu = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
                      __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint64_t lane_cols = 0x7Full << b;
  const uint64_t cols = (1ull << (N - 1)) - 1;  // columns 0..N-2
  const uint64_t shared = cols & ~lane_cols;
  if (__builtin_amdgcn_ballot_w64(((x ^ xu) & shared) != 0) != 0) {
    if constexpr (CPLX)
      form_w_complex<N>(slot, G << b, wr, wi);
    else
      form_w_real<N>(slot, G << b, wr);
    return;
  }
  const int k = threadIdx.x & (kWave - 1);
  if (k < CW * N) {
    const int r = k / CW, c = k - CW * (k / CW);
    double e[N];
#pragma unroll
    for (int j = 0; j < N; ++j) e[j] = s_a[CW * (r + j * N) + c];
    double u = e[N - 1];
#pragma unroll
    for (int j = 0; j < N - 1; ++j) {
      // +1 / -1 by the shared Gray bit; 0 for the lanes' own columns
      const double d = ((shared >> j) & 1) ? (((xu >> j) & 1) ? 1.0 : -1.0) : 0.0;
      u = fma(d, e[j], u);
    }
    s_u[k] = u;
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wr[i] = s_u[CW * i];
    if constexpr (CPLX) wi[i] = s_u[CW * i + 1];
  }
  __builtin_amdgcn_wave_barrier();
  const int jend = b + 7 < N - 1 ? b + 7 : N - 1;
#pragma unroll 1
  for (int j = b; j < jend; ++j) {
    const double d = ((x >> j) & 1) ? 1.0 : -1.0;
    cdptr col = as_const(slot + CW * j * N);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      wr[i] = fma(d, col[CW * i], wr[i]);
      if constexpr (CPLX) wi[i] = fma(d, col[CW * i + 1], wi[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    wr[i] *= 0.5;
    if constexpr (CPLX) wi[i] *= 0.5;
  }
}

constexpr int kDppMirror16 = 0x140;  // row_mirror: lane i <-> 15 - i in each row of 16

template <int CTRL>
__device__ __forceinline__ void wave_step_dpp(cdd& v) {
  const dd o_re{dpp_f64<CTRL>(v.re.hi), dpp_f64<CTRL>(v.re.lo)};
  const dd o_im{dpp_f64<CTRL>(v.im.hi), dpp_f64<CTRL>(v.im.lo)};
  v.re = dd_add(v.re, o_re);
  v.im = dd_add(v.im, o_im);
}

// Both parts of a complex partial summed over the wave, side by side (the two
// chains are independent, so each hides the other's latency), in a fixed
// order: within groups of 2, 4, 8 and 16 lanes by DPP lane moves (no LDS round
// trip), then across the rows of 16 by shuffles.  Every lane ends with the
// wave's sum.
__device__ __forceinline__ cdd wave_sum_c(cdd v) {
  wave_step_dpp<kDppXor1>(v);
  wave_step_dpp<kDppXor2>(v);
  wave_step_dpp<kDppMirror8>(v);
  wave_step_dpp<kDppMirror16>(v);
#pragma unroll
  for (int off = 16; off < kWave; off <<= 1) {
    const dd o_re{__shfl_xor(v.re.hi, off), __shfl_xor(v.re.lo, off)};
    const dd o_im{__shfl_xor(v.im.hi, off), __shfl_xor(v.im.lo, off)};
    v.re = dd_add(v.re, o_re);
    v.im = dd_add(v.im, o_im);
  }
  return v;
}

template <int N, bool CPLX, int MODE>
__global__ __launch_bounds__(kBlock) void fused_kernel(FusedArgs a) {
  constexpr int CW = CPLX ? 2 : 1;
  __shared__ double s_a[CW * N * N];
  __shared__ double s_u[kWavesPerBlock][CW * N];
  __shared__ int32_t s_exp[N];
  __shared__ int32_t s_bad;
  __shared__ int32_t s_last;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_bad = 0;
    atomicMin((unsigned long long*)a.t0, (unsigned long long)wall_clock64());
  }
  double* slot = a.slots + (size_t)blockIdx.x * a.slot_stride;
  fused_stage<N, CPLX>(a, slot, s_exp, &s_bad, s_a);
  const bool ok = s_bad == 0;

  const int lane = tid & (kWave - 1);
  const int wave_in_block = tid / kWave;
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  dd re{0.0, 0.0}, im{0.0, 0.0};
  if (ok) {
    for (uint64_t task = wave; task < a.ntasks; task += nwaves) {
      const uint64_t c = task_chunk(task, lane);
      const uint32_t gpar = (uint32_t)(task & 1);
      const double* staged = opaque(slot);
      double wr[N], wi[N];
      fused_chunk_start<N, CPLX>(s_a, s_u[wave_in_block], staged, c, a.b, wr, wi);
      if constexpr (CPLX) {
        const cdd part = walk_pairs_complex<N, MODE>(staged, wr, wi, a.b, gpar);
        if (c < a.nchunks) {
          re = dd_add(re, part.re);
          im = dd_add(im, part.im);
        }
      } else {
        const dd part = walk_pairs_real<N, MODE>(staged, wr, a.b, gpar);
        if (c < a.nchunks) re = dd_add(re, part);
      }
    }
  }
  // this workgroup's partial (the walk kernels' reduction; the complex wave sum has
  // its own fixed order)
  dd br, bi{0.0, 0.0};
  if constexpr (CPLX) {
    const cdd v = wave_sum_c(cdd{re, im});
    const cdd blk = block_sum(v, [](cdd x, cdd y) { return cdd{dd_add(x.re, y.re), dd_add(x.im, y.im)}; });
    br = blk.re;
    bi = blk.im;
  } else {
    br = block_sum(wave_sum(re), dd_add);
  }
  if (tid == 0) {
    double* p = a.partials + 4 * (size_t)blockIdx.x;
    p[0] = br.hi;
    p[1] = br.lo;
    p[2] = bi.hi;
    p[3] = bi.lo;
    // release: the partial is visible device-wide before the count that
    // announces it (the counter's read-modify-writes form one release sequence)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t done = atomicAdd(a.counter, 1u);
    s_last = done == gridDim.x - 1 ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  // The last workgroup: every other partial has been counted; the acquire makes
  // them visible.  Its first wave adds them -- lane l takes partials l, l + 64,
  // ... in order, then the lanes meet along the shuffle butterfly -- with no
  // barrier.
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  if (tid >= kWave) return;
  const int nparts = (int)gridDim.x;
  re = dd{0.0, 0.0};
  im = dd{0.0, 0.0};
  for (int k = tid; k < nparts; k += kWave) {
    const double* p = a.partials + 4 * (size_t)k;
    re = dd_add(re, dd{p[0], p[1]});
    im = dd_add(im, dd{p[2], p[3]});
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (tid == 0) {
    int32_t es = 0;
    for (int i = 0; i < N; ++i) es += s_exp[i];
    DevResult* r = a.res;
    r->v[0] = re.hi;
    r->v[1] = re.lo;
    r->v[2] = im.hi;
    r->v[3] = im.lo;
    r->iw[0] = 0;
    r->iw[1] = 0;
    r->drift = -1.0;
    r->status = ok ? kStOk : kStNonFinite;
    r->exp_sum = es;
    r->bound = 0.0;
    r->variant = 1;  // reported as walk_variant: the one-launch path ran
    r->ones0 = 0;
    const unsigned long long start = atomicExch((unsigned long long*)a.t0, ~0ull);
    r->ticks = (uint64_t)wall_clock64() - (uint64_t)start;
    atomicExch(a.counter, 0u);  // ready for the next call on these buffers
    // the record is complete (and visible to the host) before the flag
    __threadfence_system();
    *(volatile uint32_t*)&r->done = 1u;
  }
}

template <int N, bool CPLX>
hipError_t dispatch(int mode, const FusedArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), blk(kBlock);
  switch (mode) {
    case 0: hipLaunchKernelGGL((fused_kernel<N, CPLX, 0>), g, blk, 0, s, a); break;
    case 1: hipLaunchKernelGGL((fused_kernel<N, CPLX, 1>), g, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((fused_kernel<N, CPLX, 2>), g, blk, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t dispatch_n(bool cplx, int mode, const FusedArgs& a, int grid, hipStream_t s) {
  return cplx ? dispatch<N, true>(mode, a, grid, s) : dispatch<N, false>(mode, a, grid, s);
}

}  // namespace

hipError_t launch_fused(bool cplx, int n, int mode, const FusedArgs& a, int grid, hipStream_t s) {
  switch (n) {
#define PERM_FUSED_CASE(N) \
  case N:                  \
    return dispatch_n<N>(cplx, mode, a, grid, s);
    PERM_FUSED_CASE(2) PERM_FUSED_CASE(3) PERM_FUSED_CASE(4) PERM_FUSED_CASE(5)
    PERM_FUSED_CASE(6) PERM_FUSED_CASE(7) PERM_FUSED_CASE(8) PERM_FUSED_CASE(9)
    PERM_FUSED_CASE(10) PERM_FUSED_CASE(11) PERM_FUSED_CASE(12) PERM_FUSED_CASE(13)
    PERM_FUSED_CASE(14) PERM_FUSED_CASE(15) PERM_FUSED_CASE(16) PERM_FUSED_CASE(17)
    PERM_FUSED_CASE(18) PERM_FUSED_CASE(19) PERM_FUSED_CASE(20) PERM_FUSED_CASE(21)
    PERM_FUSED_CASE(22) PERM_FUSED_CASE(23) PERM_FUSED_CASE(24)
#undef PERM_FUSED_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace perm
