// Staging and finishing kernels for the single-matrix path.
//
// Staging (one workgroup): checks the input, picks power-of-two row scales,
// and writes the walk's copy of the matrix (+A then -A, column-major, ld = n;
// for 0/1 input +2A then -2A as doubles).  Row scaling multiplies row i by
// 2^e_i; per(DA) = prod_i d_i per(A) for a diagonal D, so the factor is
// undone exactly at the end.  e_i is chosen so the row's 2-norm lies in
// [2, 4): the row sums w_i = 1/2 sum_j delta_j a_ij are then of order one,
// which keeps FP32 products of many of them inside FP32's range.
//
// Finishing (one workgroup): adds the per-workgroup partial sums of all walk
// launches in a fixed order (thread t takes partials t, t+256, ...; then the
// 256 thread sums are added along a fixed binary tree), so the result is bit-for-bit
// reproducible (the paper stores partial sums in an array before the final
// compensated sum instead of reducing them in arbitrary order, Sec. II.B).
#include "perm_device.hpp"
#include "perm_internal.hpp"

namespace perm {
namespace {

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Doubles of the matrix each thread copies into LDS (complex n = 64 at most).
constexpr int kStageLoads = (2 * kMaxN * kMaxN + kBlock - 1) / kBlock;

// The matrix is first copied into LDS (all threads; every load of a thread is
// issued before the first one is used), so the per-row statistics read LDS
// instead of walking a row of global memory one dependent load at a time.
__global__ __launch_bounds__(kBlock) void stage_float_kernel(const double* __restrict__ A, int n,
                                                             int ld, int is_complex,
                                                             int row_scaling, double* staged,
                                                             double* rowabs, int32_t* rowexp,
                                                             int32_t* status) {
  __shared__ double s_a[2 * kMaxN * kMaxN];  // column-major, ld = n (complex: pairs)
  __shared__ double s_abs[kMaxN * kMaxN];    // |a_ij| 2^e_i, column-major, ld = n
  __shared__ int32_t s_exp[kMaxN];
  __shared__ int32_t s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  const int cw = is_complex ? 2 : 1;  // doubles per entry
  const int nn = n * n;
  const int tot = cw * nn;
  {
    double v[kStageLoads];
#pragma unroll
    for (int u = 0; u < kStageLoads; ++u) {
      const int t = tid + u * kBlock;
      const int idx = t / cw, c = t - cw * (t / cw);
      const int i = idx % n, j = idx / n;
      v[u] = t < tot ? A[cw * ((size_t)i + (size_t)j * ld) + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kStageLoads; ++u) {
      const int t = tid + u * kBlock;
      if (t < tot) s_a[t] = v[u];
    }
  }
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    double mx = 0.0;
    bool bad = false;
    for (int j = 0; j < n; ++j) {
      for (int c = 0; c < cw; ++c) {
        const double v = s_a[cw * (i + j * n) + c];
        if (!finite(v)) bad = true;
        mx = fmax(mx, fabs(v));
      }
    }
    int e = 0;
    if (!bad && row_scaling && mx > 0.0) {
      double ss = 0.0;
      for (int j = 0; j < n; ++j)
        for (int c = 0; c < cw; ++c) {
          const double v = s_a[cw * (i + j * n) + c] / mx;
          ss += v * v;
        }
      // norm = mx sqrt(ss) in [2^(k-1), 2^k); the exponents of the two
      // factors are taken apart, so a row near the top of the double range
      // does not overflow the product
      int k1, k2;
      const double f = frexp(mx, &k1) * frexp(sqrt(ss), &k2);  // in [1/4, 1)
      int k = k1 + k2;
      if (f < 0.5) --k;
      e = 2 - k;
      e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
    }
    s_exp[i] = e;
    rowexp[i] = e;
    if (bad) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  for (int t = tid; t < tot; t += kBlock) {
    const int i = (t / cw) % n;
    const double v = ldexp(s_a[t], s_exp[i]);
    staged[t] = v;
    staged[tot + t] = -v;
  }
  // |a_ij| 2^e_i by all threads, then each row's sum in column order
  for (int idx = tid; idx < nn; idx += kBlock) {
    const int e = s_exp[idx % n];
    const int o = cw * idx;
    s_abs[idx] = is_complex ? hypot(ldexp(s_a[o], e), ldexp(s_a[o + 1], e))
                            : fabs(ldexp(s_a[o], e));
  }
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += s_abs[i + j * n];
    rowabs[i] = 0.5 * s;
  }
  if (tid == 0) status[0] = s_bad ? kStNonFinite : kStOk;
}

// 0/1 input: entries must be 0 or 1.  Writes +2A/-2A, d_i into rowabs, and
// checks (n-1) + sum_i log2(d_i!)/d_i < 127 (Bregman: per(A) <=
// prod_i (d_i!)^(1/d_i)), which keeps 2^(n-1) per(A) inside a signed 128-bit
// integer.
//
// With pair_rows = M > 0 (full permanents only: a permutation changes the
// terms, not the total) the copy is permuted: the column with the fewest
// ones becomes column 0 (the column flipped between the two terms of every
// pair), the rows with a one there come first, then the other rows by
// ascending degree up to M rows (group D).  Column 1 (flipped after every
// other pair) becomes the column with the fewest ones outside D; the rows
// after D are those with a one in it, then the others, each by ascending
// degree.  With E = (n - M) / 2, rows M .. M+E-1 form group E and the rest
// group S', whose rows have zeros in columns 0 and 1.  status[1] = 1 when
// column 0 has at most M ones and D's degrees multiply to less than 2^50
// (the pair-shared walk is exact); 2 when moreover column 1 has at most E ones
// outside D and the degrees of E and of S' each multiply to less than 2^50
// (the banded walk is exact); status[2] = the number of ones in column 0.
__global__ __launch_bounds__(kBlock) void stage_int01_kernel(const uint8_t* __restrict__ A, int n,
                                                             int ld, int range_check,
                                                             int pair_rows, double* staged,
                                                             double* rowabs, int32_t* rowexp,
                                                             int32_t* status, double* bound) {
  __shared__ uint8_t s_a[kMaxN * kMaxN];  // s_a[i * kMaxN + j] = a_ij
  __shared__ uint64_t s_cmask[kMaxN];      // bit i of s_cmask[j]: a_ij != 0
  __shared__ uint64_t s_less[kMaxN];       // bit q of s_less[i]: row q before row i by degree
  __shared__ int32_t s_row[kMaxN], s_col[kMaxN], s_deg[kMaxN], s_csum[kMaxN];
  __shared__ double s_term[kMaxN];
  __shared__ double s_lg[kMaxN + 1];      // log2(k)
  __shared__ int32_t s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  if (tid >= 2 && tid <= kMaxN) s_lg[tid] = log2((double)tid);
  __syncthreads();
  const int nn = n * n;
  {
    // thread t copies rows t mod 64 of the columns t/64, t/64 + 4, ...: every
    // load of a thread is issued before the first one is used
    constexpr int kCols = kMaxN / (kBlock / kMaxN);  // columns per thread
    const int i = tid % kMaxN, j0 = tid / kMaxN;
    uint8_t v[kCols];
#pragma unroll
    for (int u = 0; u < kCols; ++u) {
      const int j = j0 + u * (kBlock / kMaxN);
      v[u] = (i < n && j < n) ? A[(size_t)i + (size_t)j * ld] : 0;
    }
    int bad = 0;
#pragma unroll
    for (int u = 0; u < kCols; ++u) {
      const int j = j0 + u * (kBlock / kMaxN);
      if (i < n && j < n) {
        bad |= v[u] > 1;
        s_a[i * kMaxN + j] = v[u];
      }
      // the wave holds all rows of column j: its rows with a one, as a mask
      const uint64_t m = __ballot(i < n && j < n && v[u] != 0);
      if (i == 0 && j < n) s_cmask[j] = m;
    }
    if (bad) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  // row sums and Bregman terms (threads 0..n-1), column sums (threads 64..64+n-1)
  if (tid < n) {
    int d = 0;
    for (int j = 0; j < n; ++j) d += s_a[tid * kMaxN + j];
    s_deg[tid] = d;
    double lf = 0.0;
    for (int k = 2; k <= d; ++k) lf += s_lg[k];
    s_term[tid] = d > 0 ? lf / d : 0.0;
    s_row[tid] = tid;
    s_col[tid] = tid;
  } else if (tid >= kMaxN && tid < kMaxN + n) {
    const int j = tid - kMaxN;
    int c = 0;
    for (int i = 0; i < n; ++i) c += s_a[i * kMaxN + j];
    s_csum[j] = c;
  }
  __shared__ int32_t s_best, s_col1, s_ones1;
  __shared__ int32_t s_pos[kMaxN];  // place of row i in the staged order (group D)
  __shared__ uint64_t s_outd;       // the rows outside group D, as a mask
  __syncthreads();
  const bool permute = pair_rows > 0 && !s_bad;
  const int band = (n - pair_rows) / 2;  // rows of group E
  // the sparsest column (lowest index among equals): one wave's min-reduction
  if (permute && tid < kWave) {
    int key = tid < n ? (s_csum[tid] << 8) | tid : 0x7fffffff;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off));
    if (tid == 0) s_best = key & 0xff;
  }
  __syncthreads();
  if (permute && tid < n) {
    const int best = s_best;
    // rows: those with a one in the sparsest column first (in index order), then
    // the others by ascending degree (index order among equals); each row's
    // place is the number of rows that precede it
    const int i = tid;
    const uint64_t topm = s_cmask[best];
    const bool top = (topm >> i) & 1;
    uint64_t less = 0;  // rows before row i by (degree, index)
    for (int q = 0; q < n; ++q)
      if (s_deg[q] < s_deg[i] || (s_deg[q] == s_deg[i] && q < i)) less |= 1ull << q;
    const uint64_t below = i ? (~0ull >> (kMaxN - i)) : 0ull;  // rows 0..i-1
    const int rank = top ? __popcll(topm & below) : __popcll(topm) + __popcll(less & ~topm);
    s_row[rank] = i;
    s_pos[i] = rank;
    s_less[i] = less;
  }
  __syncthreads();
  if (permute && tid < kWave) {
    const uint64_t outd = __ballot(tid < n && s_pos[tid] >= pair_rows);
    // column 1: the fewest ones outside group D (lowest index among equals)
    const int c1 = tid < n ? __popcll(s_cmask[tid] & outd) : 0;
    int key = (tid < n && tid != s_best) ? (c1 << 8) | tid : 0x7fffffff;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off));
    if (tid == 0) {
      s_col1 = key & 0xff;
      s_ones1 = key >> 8;
      s_outd = outd;
    }
  }
  __syncthreads();
  if (permute && tid < n) {
    const int best = s_best, col1 = s_col1;
    // columns: the sparsest, then column 1, then the others in their order
    int src = best;
    if (tid == 1) {
      src = col1;
    } else if (tid >= 2) {
      // the (tid - 2)-th column, counting from 0, that is neither of those two
      int k = tid - 2;
      src = 0;
      while (src == best || src == col1 || k-- > 0) ++src;
    }
    s_col[tid] = src;
    // rows after group D: a one in column 1 first, then the others, each by
    // ascending degree (index order among equals)
    const int i = tid;
    const uint64_t outd = s_outd;
    if ((outd >> i) & 1) {
      const uint64_t em = s_cmask[col1] & outd;  // outside D with a one in column 1
      const uint64_t less = s_less[i];
      const int rank = pair_rows + (((em >> i) & 1) ? __popcll(less & em)
                                                     : __popcll(em) + __popcll(less & outd & ~em));
      s_row[rank] = i;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int pairs_ok = 0, ones0 = 0;
    if (permute) {
      // degree products are exact while below 2^53; only compared with 2^50
      auto degprod = [&](int lo, int hi) {
        double prod = 1.0;
        for (int i = lo; i < hi; ++i) prod *= (double)s_deg[s_row[i]];
        return prod;
      };
      constexpr double k2p50 = 1125899906842624.0;
      ones0 = s_csum[s_best];
      if (ones0 <= pair_rows && degprod(0, pair_rows) < k2p50) {
        pairs_ok = 1;
        if (band >= 1 && n - pair_rows - band >= 1 && s_ones1 <= band &&
            degprod(pair_rows, pair_rows + band) < k2p50 && degprod(pair_rows + band, n) < k2p50)
          pairs_ok = 2;
      }
    }
    double lb = 0.0;
    bool zero_row = false;
    for (int i = 0; i < n; ++i) {
      if (s_deg[i] == 0) zero_row = true;
      lb += s_term[i];
    }
    lb = zero_row ? 0.0 : (double)(n - 1) + lb;
    bound[0] = lb;
    int32_t st = kStOk;
    if (s_bad)
      st = kStInval;
    else if (range_check && lb >= 127.0)
      st = kStRange;
    status[0] = st;
    status[1] = pairs_ok;
    status[2] = ones0;
  }
  __syncthreads();
  for (int idx = tid; idx < nn; idx += kBlock) {
    const int i = idx % n, j = idx / n;  // staged position (row i, column j)
    const double v = 2.0 * s_a[s_row[i] * kMaxN + s_col[j]];
    staged[idx] = v;
    staged[nn + idx] = -v;
  }
  if (tid < n) {
    rowabs[tid] = (double)s_deg[s_row[tid]];
    rowexp[tid] = 0;
  }
}

template <class T, class Add>
__device__ __forceinline__ T tree_sum(T* s, Add add) {
  // fixed binary tree over kBlock values in shared memory; thread 0 gets the sum
  for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) s[threadIdx.x] = add(s[threadIdx.x], s[threadIdx.x + stride]);
    __syncthreads();
  }
  return s[0];
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void finish_kernel(const void* __restrict__ partials,
                                                        int nparts,
                                                        const double* __restrict__ drift_part,
                                                        int want_drift,
                                                        const int32_t* __restrict__ status,
                                                        const int32_t* __restrict__ rowexp, int n,
                                                        const double* __restrict__ bound,
                                                        DevResult* res) {
  const int tid = threadIdx.x;
  __shared__ dd s_re[kBlock], s_im[kBlock];
  __shared__ u128 s_i[kBlock];
  __shared__ double s_dr[kBlock];
  dd re{0.0, 0.0}, im{0.0, 0.0};
  u128 iv{0, 0};
  double dr = 0.0;
  for (int k = tid; k < nparts; k += kBlock) {
    if constexpr (KIND == kReal) {
      const double* p = (const double*)partials;
      re = dd_add(re, dd{p[2 * k], p[2 * k + 1]});
    } else if constexpr (KIND == kComplex) {
      const double* p = (const double*)partials;
      re = dd_add(re, dd{p[4 * k], p[4 * k + 1]});
      im = dd_add(im, dd{p[4 * k + 2], p[4 * k + 3]});
    } else {
      const uint64_t* p = (const uint64_t*)partials;
      iv = u128_add(iv, u128{p[2 * k], p[2 * k + 1]});
    }
    if (want_drift) dr = fmax(dr, drift_part[k]);
  }
  if constexpr (KIND == kInt01) {
    s_i[tid] = iv;
    __syncthreads();
    iv = tree_sum(s_i, u128_add);
  } else {
    s_re[tid] = re;
    if constexpr (KIND == kComplex) s_im[tid] = im;
    __syncthreads();
    re = tree_sum(s_re, dd_add);
    if constexpr (KIND == kComplex) im = tree_sum(s_im, dd_add);
  }
  if (want_drift) {
    s_dr[tid] = dr;
    __syncthreads();
    dr = tree_sum(s_dr, [](double x, double y) { return fmax(x, y); });
  }
  if (tid == 0) {
    int32_t es = 0;
    for (int i = 0; i < n; ++i) es += rowexp[i];
    res->v[0] = re.hi;
    res->v[1] = re.lo;
    res->v[2] = im.hi;
    res->v[3] = im.lo;
    res->iw[0] = iv.lo;
    res->iw[1] = iv.hi;
    res->drift = want_drift ? dr : -1.0;
    res->status = status[0];
    res->exp_sum = es;
    res->bound = bound ? bound[0] : 0.0;
    res->variant = KIND == kInt01 ? status[1] : 0;
    res->ones0 = KIND == kInt01 ? status[2] : 0;
  }
}

// The per-workgroup partials as caller records of 5 doubles (re hi, re lo,
// im hi, im lo, drift), scaled back to the unscaled matrix (2^-sum e_i,
// exact); 0/1 partials as their two 64-bit words.
__global__ __launch_bounds__(kBlock) void export_partials_kernel(
    int kind, const void* __restrict__ partials, const double* __restrict__ drift_part,
    int want_drift, int nparts, const int32_t* __restrict__ rowexp, int n, double* out) {
  __shared__ int32_t s_es;
  if (threadIdx.x == 0) {
    int32_t es = 0;
    for (int i = 0; i < n; ++i) es += rowexp[i];
    s_es = es;
  }
  __syncthreads();
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nparts) return;
  double* o = out + 5 * (size_t)k;
  const int e = -s_es;
  if (kind == kInt01) {
    const uint64_t* p = (const uint64_t*)partials;
    o[0] = __longlong_as_double((long long)p[2 * k]);
    o[1] = __longlong_as_double((long long)p[2 * k + 1]);
    o[2] = 0.0;
    o[3] = 0.0;
  } else if (kind == kComplex) {
    const double* p = (const double*)partials;
    o[0] = ldexp(p[4 * k], e);
    o[1] = ldexp(p[4 * k + 1], e);
    o[2] = ldexp(p[4 * k + 2], e);
    o[3] = ldexp(p[4 * k + 3], e);
  } else {
    const double* p = (const double*)partials;
    o[0] = ldexp(p[2 * k], e);
    o[1] = ldexp(p[2 * k + 1], e);
    o[2] = 0.0;
    o[3] = 0.0;
  }
  o[4] = want_drift ? drift_part[k] : -1.0;
}

}  // namespace

hipError_t launch_export_partials(int kind, const void* partials, const double* drift_part,
                                  int want_drift, int nparts, const int32_t* rowexp, int n,
                                  double* out, hipStream_t s) {
  if (nparts <= 0) return hipSuccess;
  hipLaunchKernelGGL(export_partials_kernel, dim3((nparts + kBlock - 1) / kBlock), dim3(kBlock),
                     0, s, kind, partials, drift_part, want_drift, nparts, rowexp, n, out);
  return hipGetLastError();
}

hipError_t launch_stage(int kind, const void* A, int n, int ld, int row_scaling, int range_check,
                        int pair_rows, double* staged, double* rowabs, int32_t* rowexp,
                        int32_t* status, double* bound, hipStream_t s) {
  if (kind == kInt01) {
    hipLaunchKernelGGL(stage_int01_kernel, dim3(1), dim3(kBlock), 0, s, (const uint8_t*)A, n, ld,
                       range_check, pair_rows, staged, rowabs, rowexp, status, bound);
  } else {
    hipLaunchKernelGGL(stage_float_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)A, n, ld,
                       kind == kComplex ? 1 : 0, row_scaling, staged, rowabs, rowexp, status);
  }
  return hipGetLastError();
}

hipError_t launch_finish(int kind, const void* partials, int nparts, const double* drift_part,
                         int want_drift, const int32_t* status, const int32_t* rowexp, int n,
                         const double* bound, DevResult* res, hipStream_t s) {
  switch (kind) {
    case kReal:
      hipLaunchKernelGGL(finish_kernel<kReal>, dim3(1), dim3(kBlock), 0, s, partials, nparts,
                         drift_part, want_drift, status, rowexp, n, bound, res);
      break;
    case kComplex:
      hipLaunchKernelGGL(finish_kernel<kComplex>, dim3(1), dim3(kBlock), 0, s, partials, nparts,
                         drift_part, want_drift, status, rowexp, n, bound, res);
      break;
    default:
      hipLaunchKernelGGL(finish_kernel<kInt01>, dim3(1), dim3(kBlock), 0, s, partials, nparts,
                         drift_part, want_drift, status, rowexp, n, bound, res);
      break;
  }
  return hipGetLastError();
}

}  // namespace perm
