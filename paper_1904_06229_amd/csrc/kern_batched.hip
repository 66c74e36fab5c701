// Batched permanents of many independent matrices (the random-matrix studies
// of Secs. III-VI evaluate many independent permanents).
//
//   stage    one workgroup per matrix: validate, row exponents, +A/-A copy
//   walk     one persistent launch per matrix size (largest first): the
//            items of one size are contiguous in the item array and cost the
//            same, so wave w takes items w, w + W, w + 2W, ... (W waves in the
//            grid) with no queue; each item's 64 lane chunks are walked with
//            the same chunk walk as the single-matrix kernels, fully inlined
//            for that size, and the wave's sum goes into the item's slot
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

typedef const __attribute__((address_space(4))) BatchItem* citem_ptr;
typedef const __attribute__((address_space(4))) int64_t* ci64_ptr;
typedef const __attribute__((address_space(4))) int32_t* ci32_ptr;

// Complex sizes whose lanes walk two half-length chunks of the same parity in
// lockstep (walk_chunks_complex_twin): every scalar column read then serves
// two walks and each wave has two independent product chains, at two waves
// per SIMD.  Measured per size against one chunk per lane at four waves:
// faster at n = 17..20 (by 1.5-11%), slower below (short chunks) and from
// n = 21 on (the two walks' row sums spill).
template <int N>
constexpr bool twin_chunks() {
  return N >= 17 && N <= 20;
}

// Smallest waves per SIMD the compiler must keep for size N: up to n = 24
// the walk fits 4 waves (128 VGPRs) with at most a few spills outside the
// chunk loop, where it would otherwise take a few registers more and run
// with 3; the twin walk fits 2; larger sizes keep the compiler's choice.
template <int N, bool CPLX>
constexpr int batched_min_waves() {
  return (CPLX && twin_chunks<N>()) ? 2 : (N <= 24 ? 4 : 1);
}

// The items [item0, item0 + nitems), all of size N.
template <int N, int MODE, bool CPLX>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(batched_min_waves<N, CPLX>())))
void batched_size_kernel(BatchArgs a, uint64_t item0, uint64_t nitems) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = wave_id();
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  for (uint64_t q = wave; q < nitems; q += nwaves) {
    const uint64_t idx = item0 + q;
    const citem_ptr ip = (citem_ptr)a.items + idx;
    const int mat = ip->mat;
    const int b = ip->b;
    const uint64_t task = ip->task;
    const uint64_t nchunks = ip->nchunks;
    double* slot = a.slots + 4 * idx;
    if (((ci32_ptr)a.mstatus)[mat] != kStOk) {
      if (lane == 0) slot[0] = slot[1] = slot[2] = slot[3] = 0.0;
      continue;
    }
    const double* st = a.staged + ((ci64_ptr)a.st_off)[mat];
    const uint64_t c = task_chunk(task, lane);
    const uint32_t gpar = (uint32_t)(task & 1);
    double dr = 0.0;
    dd re{0.0, 0.0}, im{0.0, 0.0};
    // n = 1 has a single term; every larger size is planned with b >= 1.
    if constexpr (CPLX && twin_chunks<N>()) {
      if (b >= 2) {
        // the half-length chunks ca and ca + 2 (same parity); tasks 2k and
        // 2k + 1 (always both planned) cover the chunks 128k .. 128k + 127
        // that they cover with whole chunks
        const uint64_t ca = 4 * (uint64_t(kWave) * (task >> 1) + (uint64_t)lane) + (task & 1);
        cdd pa, pb;
        walk_chunks_complex_twin<N, MODE>(st, ca, ca + 2, b - 1, gpar, pa, pb);
        if (ca < 2 * nchunks) {
          re = pa.re;
          im = pa.im;
        }
        if (ca + 2 < 2 * nchunks) {
          re = dd_add(re, pb.re);
          im = dd_add(im, pb.im);
        }
      } else {
        const cdd p = walk_chunk_complex<N, MODE, false>(st, nullptr, c, b, gpar, dr);
        if (c < nchunks) {
          re = p.re;
          im = p.im;
        }
      }
    } else if constexpr (CPLX) {
      cdd p;
      if constexpr (N == 1)
        p = single_term_complex<N, MODE>(st, c);
      else
        p = walk_chunk_complex<N, MODE, false>(st, nullptr, c, b, gpar, dr);
      if (c < nchunks) {
        re = p.re;
        im = p.im;
      }
    } else {
      if constexpr (N == 1)
        re = single_term_real<N, MODE>(st, c);
      else
        re = walk_chunk_real<N, MODE, false>(st, nullptr, c, b, gpar, dr);
      if (c >= nchunks) re = dd{0.0, 0.0};
    }
    re = wave_sum(re);
    if constexpr (CPLX) im = wave_sum(im);
    if (lane == 0) {
      slot[0] = re.hi;
      slot[1] = re.lo;
      slot[2] = im.hi;
      slot[3] = im.lo;
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

template <int N, int MODE, bool CPLX>
const void* size_kernel() {
  return (const void*)batched_size_kernel<N, MODE, CPLX>;
}

template <int MODE, bool CPLX>
const void* size_kernel_by_n(int n) {
  switch (n) {
#define PERM_BK(N) \
  case N:          \
    return size_kernel<N, MODE, CPLX>();
    PERM_BK(1) PERM_BK(2) PERM_BK(3) PERM_BK(4) PERM_BK(5) PERM_BK(6) PERM_BK(7) PERM_BK(8)
    PERM_BK(9) PERM_BK(10) PERM_BK(11) PERM_BK(12) PERM_BK(13) PERM_BK(14) PERM_BK(15)
    PERM_BK(16) PERM_BK(17) PERM_BK(18) PERM_BK(19) PERM_BK(20) PERM_BK(21) PERM_BK(22)
    PERM_BK(23) PERM_BK(24) PERM_BK(25) PERM_BK(26) PERM_BK(27) PERM_BK(28) PERM_BK(29)
    PERM_BK(30) PERM_BK(31) PERM_BK(32)
#undef PERM_BK
    default:
      return nullptr;
  }
}

const void* size_kernel_ptr(int is_complex, int mode, int n) {
  if (mode == 0) return is_complex ? size_kernel_by_n<0, true>(n) : size_kernel_by_n<0, false>(n);
  if (mode == 1) return is_complex ? size_kernel_by_n<1, true>(n) : size_kernel_by_n<1, false>(n);
  return nullptr;
}

}  // namespace

int batched_walk_blocks_per_cu(int is_complex, int mode, int n) {
  const void* f = size_kernel_ptr(is_complex, mode, n);
  int nb = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, 0) != hipSuccess || nb < 1)
    nb = 1;
  return nb;
}

hipError_t launch_batched_size(int is_complex, int mode, int n, const BatchArgs& a,
                               uint64_t item0, uint64_t nitems, int grid, hipStream_t s) {
  const void* f = size_kernel_ptr(is_complex, mode, n);
  if (!f) return hipErrorInvalidValue;
  BatchArgs args = a;
  void* params[] = {&args, &item0, &nitems};
  return hipLaunchKernel(f, dim3(grid), dim3(kBlock), params, 0, s);
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
