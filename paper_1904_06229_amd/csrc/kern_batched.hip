// Batched permanents of many independent matrices (the random-matrix studies
// of Secs. III-VI evaluate many independent permanents).
//
//   stage    one workgroup per matrix: validate, row exponents, +A/-A copy
//   reset    queue head <- 0 (a kernel, so the sequence can be captured in a
//            HIP graph without memset nodes)
//   walk     persistent kernel: each wave takes the next item from the queue
//            (an atomic counter on the item array, which the host sorted by
//            size, largest first), walks its 64 lane chunks with the same
//            chunk walk as the single-matrix kernels, and writes the wave's
//            sum into the item's slot
//   finish   one thread per matrix adds its items' slots in item order
//            (fixed order, so results are reproducible) and scales by
//            2(-1)^n and the row-scaling factor
#include "perm_walk.hpp"

namespace perm {
namespace {

__global__ __launch_bounds__(kBlock) void batched_stage_kernel(
    const double* __restrict__ A, const int64_t* __restrict__ off, const int32_t* __restrict__ ns,
    int is_complex, int row_scaling, double* __restrict__ staged,
    const int64_t* __restrict__ st_off, int32_t* __restrict__ exp_sum,
    int32_t* __restrict__ mstatus) {
  __shared__ int32_t s_exp[kMaxBatchedN];
  __shared__ int32_t s_bad;
  const int m = blockIdx.x;
  const int n = ns[m];
  const int cw = is_complex ? 2 : 1;
  const double* a = A + off[m];
  double* st = staged + st_off[m];
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    double mx = 0.0;
    bool bad = false;
    for (int j = 0; j < n; ++j)
      for (int c = 0; c < cw; ++c) {
        const double v = a[cw * (i + j * n) + c];
        if (!isfinite(v)) bad = true;
        mx = fmax(mx, fabs(v));
      }
    int e = 0;
    if (!bad && row_scaling && mx > 0.0) {
      double ss = 0.0;
      for (int j = 0; j < n; ++j)
        for (int c = 0; c < cw; ++c) {
          const double v = a[cw * (i + j * n) + c] / mx;
          ss += v * v;
        }
      int k1, k2;
      frexp(mx, &k1);
      frexp(sqrt(ss), &k2);
      e = 2 - (k1 + k2);
      e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
    }
    s_exp[i] = e;
    if (bad) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  const int nn = n * n;
  for (int idx = tid; idx < nn; idx += kBlock) {
    const int i = idx % n;
    for (int c = 0; c < cw; ++c) {
      const double v = ldexp(a[cw * idx + c], s_exp[i]);
      st[cw * idx + c] = v;
      st[cw * (nn + idx) + c] = -v;
    }
  }
  if (tid == 0) {
    int32_t es = 0;
    for (int i = 0; i < n; ++i) es += s_exp[i];
    exp_sum[m] = es;
    mstatus[m] = s_bad ? kStNonFinite : kStOk;
  }
}

__global__ void batched_reset_kernel(unsigned int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) counter[0] = 0u;
}

typedef const __attribute__((address_space(4))) BatchItem* citem_ptr;
typedef const __attribute__((address_space(4))) int64_t* ci64_ptr;
typedef const __attribute__((address_space(4))) int32_t* ci32_ptr;

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One queue item.  Not inlined: each size gets its own register allocation
// (inlined into one switch, the sizes' code is merged and the kernel needs
// the registers of the largest size plus more).  Arguments of a call arrive
// in VGPRs, so the uniform ones are moved back to SGPRs first.
template <int N, int MODE, bool CPLX>
__device__ __attribute__((noinline)) void run_item(const double* st_arg, uint64_t task_arg,
                                                   int b_arg, uint64_t nchunks_arg,
                                                   double* slot_arg) {
  const double* st = (const double*)uniform64((uint64_t)st_arg);
  const uint64_t task = uniform64(task_arg);
  const int b = __builtin_amdgcn_readfirstlane(b_arg);
  const uint64_t nchunks = uniform64(nchunks_arg);
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t c = task_chunk(task, lane);
  const uint32_t gpar = (uint32_t)(task & 1);
  double dr = 0.0;
  dd re{0.0, 0.0}, im{0.0, 0.0};
  // n = 1 has a single term; every larger size is planned with b >= 1.
  if constexpr (CPLX) {
    const cdd p = (N == 1) ? single_term_complex<N, MODE>(st, c)
                           : walk_chunk_complex<N, MODE, false>(st, nullptr, c, b, gpar, dr);
    re = p.re;
    im = p.im;
  } else {
    re = (N == 1) ? single_term_real<N, MODE>(st, c)
                  : walk_chunk_real<N, MODE, false>(st, nullptr, c, b, gpar, dr);
  }
  if (c >= nchunks) {
    re = dd{0.0, 0.0};
    im = dd{0.0, 0.0};
  }
  re = wave_sum(re);
  if constexpr (CPLX) im = wave_sum(im);
  if (lane == 0) {
    slot_arg[0] = re.hi;
    slot_arg[1] = re.lo;
    slot_arg[2] = im.hi;
    slot_arg[3] = im.lo;
  }
}

#define PERM_BCASE(N)                                   \
  case N:                                               \
    if constexpr (N <= MAXN) run_item<N, MODE, CPLX>(st, it.task, it.b, it.nchunks, slot); \
    break;

template <int MAXN, int MODE, bool CPLX>
__global__ __launch_bounds__(kBlock) void batched_walk_kernel(BatchArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    unsigned int got = 0;
    if (lane == 0) got = atomicAdd(a.counter, 1u);
    const uint64_t idx = (uint64_t)__builtin_amdgcn_readfirstlane(__shfl(got, 0));
    if (idx >= a.nitems) break;  // every wave reaches this once the queue is drained
    const citem_ptr ip = (citem_ptr)a.items + idx;
    BatchItem it;
    it.mat = ip->mat;
    it.n = ip->n;
    it.b = ip->b;
    it.task = ip->task;
    it.nchunks = ip->nchunks;
    if (((ci32_ptr)a.mstatus)[it.mat] != kStOk) {
      if (lane == 0) {
        double* s = a.slots + 4 * idx;
        s[0] = s[1] = s[2] = s[3] = 0.0;
      }
      continue;
    }
    const double* st = a.staged + ((ci64_ptr)a.st_off)[it.mat];
    double* slot = a.slots + 4 * idx;
    switch (it.n) {
      PERM_BCASE(1) PERM_BCASE(2) PERM_BCASE(3) PERM_BCASE(4) PERM_BCASE(5) PERM_BCASE(6)
      PERM_BCASE(7) PERM_BCASE(8) PERM_BCASE(9) PERM_BCASE(10) PERM_BCASE(11) PERM_BCASE(12)
      PERM_BCASE(13) PERM_BCASE(14) PERM_BCASE(15) PERM_BCASE(16) PERM_BCASE(17)
      PERM_BCASE(18) PERM_BCASE(19) PERM_BCASE(20) PERM_BCASE(21) PERM_BCASE(22)
      PERM_BCASE(23) PERM_BCASE(24) PERM_BCASE(25) PERM_BCASE(26) PERM_BCASE(27)
      PERM_BCASE(28) PERM_BCASE(29) PERM_BCASE(30) PERM_BCASE(31) PERM_BCASE(32)
      default:
        break;
    }
  }
}

__global__ __launch_bounds__(kBlock) void batched_finish_kernel(
    const double* __restrict__ slots, const int64_t* __restrict__ item_first,
    const int32_t* __restrict__ item_count, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ exp_sum, const int32_t* __restrict__ mstatus, int count,
    double* __restrict__ out, int32_t* __restrict__ status_out) {
  const int m = blockIdx.x * kBlock + threadIdx.x;
  if (m >= count) return;
  dd re{0.0, 0.0}, im{0.0, 0.0};
  const int64_t f = item_first[m];
  const int32_t k = item_count[m];
  for (int32_t q = 0; q < k; ++q) {
    const double* s = slots + 4 * (f + q);
    re = dd_add(re, dd{s[0], s[1]});
    im = dd_add(im, dd{s[2], s[3]});
  }
  const int n = ns[m];
  const double sg = (n % 2 == 0) ? 2.0 : -2.0;  // per = 2 (-1)^n S
  const int e = -exp_sum[m];
  const int32_t st = mstatus[m];
  if (st == kStOk) {
    out[4 * m] = ldexp(sg * re.hi, e);
    out[4 * m + 1] = ldexp(sg * re.lo, e);
    out[4 * m + 2] = ldexp(sg * im.hi, e);
    out[4 * m + 3] = ldexp(sg * im.lo, e);
  } else {
    const double nan = __builtin_nan("");
    out[4 * m] = out[4 * m + 1] = out[4 * m + 2] = out[4 * m + 3] = nan;
  }
  if (status_out) status_out[m] = st;
}

template <int MODE, bool CPLX>
hipError_t launch_walk_maxn(int max_n, const BatchArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  if (max_n <= 16)
    hipLaunchKernelGGL((batched_walk_kernel<16, MODE, CPLX>), g, b, 0, s, a);
  else if (max_n <= 24)
    hipLaunchKernelGGL((batched_walk_kernel<24, MODE, CPLX>), g, b, 0, s, a);
  else
    hipLaunchKernelGGL((batched_walk_kernel<32, MODE, CPLX>), g, b, 0, s, a);
  return hipGetLastError();
}

}  // namespace

int batched_walk_blocks_per_cu(int is_complex, int mode, int max_n) {
  const void* f = nullptr;
#define PERM_PICK(MODE, C)                                                        \
  f = max_n <= 16 ? (const void*)batched_walk_kernel<16, MODE, C>                 \
                  : (max_n <= 24 ? (const void*)batched_walk_kernel<24, MODE, C>  \
                                 : (const void*)batched_walk_kernel<32, MODE, C>);
  if (mode == 0) {
    if (is_complex) { PERM_PICK(0, true) } else { PERM_PICK(0, false) }
  } else {
    if (is_complex) { PERM_PICK(1, true) } else { PERM_PICK(1, false) }
  }
#undef PERM_PICK
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

hipError_t launch_batched_stage(int is_complex, const double* A, const int64_t* d_off,
                                const int32_t* d_n, int count, int row_scaling, double* staged,
                                const int64_t* st_off, int32_t* rowexp_sum, int32_t* mstatus,
                                hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(batched_stage_kernel, dim3(count), dim3(kBlock), 0, s, A, d_off, d_n,
                     is_complex, row_scaling, staged, st_off, rowexp_sum, mstatus);
  return hipGetLastError();
}

hipError_t launch_batched_reset(unsigned int* counter, hipStream_t s) {
  hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_batched_walk(int is_complex, int mode, int max_n, const BatchArgs& a, int grid,
                               hipStream_t s) {
  if (mode == 0)
    return is_complex ? launch_walk_maxn<0, true>(max_n, a, grid, s)
                      : launch_walk_maxn<0, false>(max_n, a, grid, s);
  if (mode == 1)
    return is_complex ? launch_walk_maxn<1, true>(max_n, a, grid, s)
                      : launch_walk_maxn<1, false>(max_n, a, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batched_finish(const double* slots, const int64_t* item_first,
                                 const int32_t* item_count, const int32_t* d_n,
                                 const int32_t* rowexp_sum, const int32_t* mstatus, int count,
                                 double* d_out, int32_t* d_status, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (count + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(batched_finish_kernel, dim3(grid), dim3(kBlock), 0, s, slots, item_first,
                     item_count, d_n, rowexp_sum, mstatus, count, d_out, d_status);
  return hipGetLastError();
}

}  // namespace perm
