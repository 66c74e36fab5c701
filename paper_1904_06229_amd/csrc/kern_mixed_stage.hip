// Staging for the mixed-radix Ryser walks (repeated columns, Eq. ryser2;
// sparse matrices, App. B) and the device greedypartition of App. B.
//
// Staging (one workgroup): checks the staged columns for NaN/infinity,
// picks power-of-two row scales (row i of the source scales row i of the
// matrix, so per(DA) = prod_i d_i per(A)), and writes
//   staged : [+cols | 0] [-cols | 0] (n x (ncols+1) each, column-major,
//            ld = n), then the two start columns (chunk parity 0, 1): the row
//            sums of the inner digits' values at the first step of a chunk
//   omega  : the signed weight of every value of every digit
//   dig    : radix, kind and omega offset per digit; digit and bit per column
//   qabs   : Q_k = r_0 ... r_{k-1} for k = 0..R
//   tin    : signed weight of the inner digits at step s of a chunk of parity
//            0 or 1
//   toff   : offset of the column added after step s (+c or -c; the zero
//            column after the chunk's last step).
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

__device__ __forceinline__ uint32_t gray32(uint32_t v) { return v ^ (v >> 1); }

__device__ __forceinline__ double load_entry(const void* A, int in_kind, int ld, int i, int j,
                                             int part) {
  const size_t o = (size_t)i + (size_t)j * ld;
  if (in_kind == 2) return part ? 0.0 : (double)((const uint8_t*)A)[o];
  if (in_kind == 1) return ((const double*)A)[2 * o + part];
  return part ? 0.0 : ((const double*)A)[o];
}

__global__ __launch_bounds__(kBlock) void stage_mix_kernel(const void* __restrict__ A, int in_kind,
                                                           int n, int ld, MixDigits dg, int b,
                                                           int L, int row_scaling, double* staged,
                                                           double* omega, double* tin,
                                                           int32_t* toff, int32_t* dig,
                                                           uint64_t* qabs, int32_t* rowexp,
                                                           int32_t* status) {
  __shared__ uint64_t s_pascal[kMaxN + 1][kMaxN + 1];
  __shared__ int32_t s_exp[kMaxN], s_wofs[kMaxN], s_r[kMaxN];
  __shared__ uint32_t s_Q[kMaxN + 1];
  __shared__ int32_t s_bad;
  const int tid = threadIdx.x;
  const int cw = in_kind == 1 ? 2 : 1;
  const int R = dg.R, nc = dg.ncols;
  if (tid == 0) {
    s_bad = 0;
    int w = 0;
    for (int k = 0; k < R; ++k) {
      s_wofs[k] = w;
      w += dg.radix[k];
    }
    s_Q[0] = 1;
    for (int k = 0; k < b; ++k) s_Q[k + 1] = s_Q[k] * (uint32_t)dg.radix[k];
  }
  if (tid < R) s_r[tid] = dg.radix[tid];
  if (tid <= kMaxN) s_pascal[0][tid] = tid == 0 ? 1 : 0;
  __syncthreads();
  for (int m = 1; m <= kMaxN; ++m) {
    if (tid <= kMaxN)
      s_pascal[m][tid] = (tid == 0 ? 0 : s_pascal[m - 1][tid - 1]) + s_pascal[m - 1][tid];
    __syncthreads();
  }
  if (tid < n) {
    const int i = tid;
    double mx = 0.0;
    bool bad = false;
    bool not01 = false;  // 0/1 input: the exact sums assume every entry is 0 or 1
    for (int c = 0; c < nc; ++c)
      for (int p = 0; p < cw; ++p) {
        const double v = load_entry(A, in_kind, ld, dg.row[i], dg.src[c], p);
        if (!isfinite(v)) bad = true;
        if (in_kind == 2 && v > 1.0) not01 = true;
        mx = fmax(mx, fabs(v));
      }
    int e = 0;
    if (!bad && row_scaling && mx > 0.0) {
      double ss = 0.0;  // squared 2-norm of row i of the matrix, over mx^2
      for (int c = 0; c < nc; ++c)
        for (int p = 0; p < cw; ++p) {
          const double v = load_entry(A, in_kind, ld, dg.row[i], dg.src[c], p) / mx;
          ss += (double)dg.cmult[c] * v * v;
        }
      // 2-norm = mx sqrt(ss) in [2^(q-1), 2^q); the exponents of the two
      // factors are taken apart, so a row near the top of the double range
      // does not overflow the product
      int q1, q2;
      const double f = frexp(mx, &q1) * frexp(sqrt(ss), &q2);  // in [1/4, 1)
      int q = q1 + q2;
      if (f < 0.5) --q;
      e = 2 - q;
      e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
    }
    s_exp[i] = e;
    rowexp[i] = e;
    if (bad) atomicOr(&s_bad, 1);
    if (not01) atomicOr(&s_bad, 2);
  }
  __syncthreads();
  const int cols = (nc + 1) * n;  // entries of [+cols | 0]
  for (int idx = tid; idx < cols; idx += kBlock) {
    const int i = idx % n, c = idx / n;
    for (int p = 0; p < cw; ++p) {
      const double v =
          c < nc ? ldexp(load_entry(A, in_kind, ld, dg.row[i], dg.src[c], p), s_exp[i]) : 0.0;
      staged[cw * idx + p] = v;
      staged[cw * (cols + idx) + p] = c < nc ? -v : 0.0;
    }
  }
  // omega: every value of every digit
  for (int k = 0; k < R; ++k)
    for (int v = tid; v < dg.radix[k]; v += kBlock) {
      double wv;
      if (dg.kind[k] == 0)
        wv = ((v & 1) ? -1.0 : 1.0) * (double)s_pascal[dg.mult[k]][v];
      else
        wv = (__popc(gray32((uint32_t)v + 1u)) & 1) ? -1.0 : 1.0;
      omega[s_wofs[k] + v] = wv;
    }
  if (tid < R) {
    dig[kDigRadix * kMaxN + tid] = dg.radix[tid];
    dig[kDigKind * kMaxN + tid] = dg.kind[tid];
    dig[kDigWofs * kMaxN + tid] = s_wofs[tid];
    for (int e = 0; e < dg.size[tid]; ++e) {
      dig[kDigColDigit * kMaxN + dg.first[tid] + e] = tid;
      dig[kDigColBit * kMaxN + dg.first[tid] + e] = e;
    }
  }
  if (tid == 0) {
    uint64_t q = 1;  // the product of all radices is at most 2^63
    for (int k = 0; k < R; ++k) {
      qabs[k] = q;
      q *= (uint64_t)dg.radix[k];
    }
    qabs[R] = q;
  }
  // inner-digit tables
  const uint32_t uL = (uint32_t)L;
  for (int t = tid; t < 2 * L; t += kBlock) {
    const uint32_t par = (uint32_t)(t / L), s = (uint32_t)(t % L);
    double wgt = 1.0;
    for (int k = 0; k < b; ++k) {
      const uint32_t f = inner_digit(s, k, par, uL, s_Q, s_r);
      if (dg.kind[k] == 0)
        wgt *= ((f & 1) ? -1.0 : 1.0) * (double)s_pascal[dg.mult[k]][f];
      else if (__popc(gray32(f + 1u)) & 1)
        wgt = -wgt;
    }
    tin[t] = wgt;
    int32_t off = nc * n * cw;  // zero column
    if (s + 1 < uL) {
      int j = b - 1;
      while (j > 0 && (s + 1) % s_Q[j] != 0) --j;
      const uint32_t f0 = inner_digit(s, j, par, uL, s_Q, s_r);
      const uint32_t f1 = inner_digit(s + 1, j, par, uL, s_Q, s_r);
      int col;
      bool add;
      if (dg.kind[j] == 0) {
        col = dg.first[j];
        add = f1 > f0;
      } else {
        const uint32_t s0 = gray32(f0 + 1u), s1 = gray32(f1 + 1u);
        const int e = __ffs(s0 ^ s1) - 1;
        col = dg.first[j] + e;
        add = ((s1 >> e) & 1u) != 0;
      }
      off = (add ? col : (nc + 1) + col) * n * cw;
    }
    toff[t] = off;
  }
  __syncthreads();  // staged +cols complete
  for (int t = tid; t < 2 * n; t += kBlock) {
    const uint32_t par = (uint32_t)(t / n);
    const int i = t % n;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < b; ++k) {
      const uint32_t f = inner_digit(0, k, par, uL, s_Q, s_r);
      if (dg.kind[k] == 0) {
        sr = fma((double)f, staged[cw * (i + dg.first[k] * n)], sr);
        if (cw == 2) si = fma((double)f, staged[cw * (i + dg.first[k] * n) + 1], si);
      } else {
        const uint32_t sub = gray32(f + 1u);
        for (int e = 0; e < dg.size[k]; ++e)
          if ((sub >> e) & 1u) {
            sr += staged[cw * (i + (dg.first[k] + e) * n)];
            if (cw == 2) si += staged[cw * (i + (dg.first[k] + e) * n) + 1];
          }
      }
    }
    const int o = cw * (2 * cols + t);
    staged[o] = sr;
    if (cw == 2) staged[o + 1] = si;
  }
  if (tid == 0) {
    status[0] = (s_bad & 2) ? kStInval : ((s_bad & 1) ? kStNonFinite : kStOk);
    status[1] = 0;
    status[2] = 0;
  }
}

// splitmix64 (Steele, Lea and Flood, 2014): a counter-based 64-bit hash.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr int kMaxTrials = kBlock;

__global__ __launch_bounds__(kBlock) void sparse_partition_kernel(const void* __restrict__ A,
                                                                  int in_kind, int n, int ld,
                                                                  int trials, uint64_t seed,
                                                                  SparsePart* out) {
  __shared__ uint64_t s_nb[kMaxN];
  __shared__ int32_t s_deg[kMaxN];
  __shared__ int8_t s_order[kMaxTrials][kMaxN];
  __shared__ int32_t s_nsel[kMaxTrials];
  __shared__ double s_score[kMaxTrials];
  const int tid = threadIdx.x;
  if (tid < n) {
    uint64_t m = 0;
    for (int j = 0; j < n; ++j) {
      const bool nz = load_entry(A, in_kind, ld, tid, j, 0) != 0.0 ||
                      (in_kind == 1 && load_entry(A, in_kind, ld, tid, j, 1) != 0.0);
      if (nz) m |= 1ull << j;
    }
    s_nb[tid] = m;
    s_deg[tid] = __popcll(m);
  }
  __syncthreads();
  if (tid < trials) {
    uint64_t alive = n == 64 ? ~0ull : ((1ull << n) - 1);
    int nsel = 0, step = 0, used = 0;
    double score = 0.0;
    while (alive) {
      int mind = kMaxN + 1, cnt = 0;
      for (uint64_t a = alive; a; a &= a - 1) {
        const int i = __ffsll((long long)a) - 1;
        if (s_deg[i] < mind) {
          mind = s_deg[i];
          cnt = 1;
        } else if (s_deg[i] == mind) {
          ++cnt;
        }
      }
      int pick = 0;  // trial 0: the lowest index among rows of least degree
      if (tid > 0 && cnt > 1)
        pick = (int)(splitmix64(seed ^ splitmix64(((uint64_t)tid << 32) | (uint64_t)step)) %
                     (uint64_t)cnt);
      int k = -1;
      for (uint64_t a = alive; a; a &= a - 1) {
        const int i = __ffsll((long long)a) - 1;
        if (s_deg[i] == mind && pick-- == 0) {
          k = i;
          break;
        }
      }
      alive &= ~(1ull << k);
      for (uint64_t a = alive; a; a &= a - 1) {
        const int l = __ffsll((long long)a) - 1;
        if (s_nb[l] & s_nb[k]) alive &= ~(1ull << l);
      }
      s_order[tid][nsel++] = (int8_t)k;
      if (s_deg[k] <= kSparseMaxBlock && s_deg[k] > 0) {
        used += s_deg[k];
        score += log2((double)((1u << s_deg[k]) - 1u));
      }
      ++step;
    }
    s_nsel[tid] = nsel;
    s_score[tid] = score + (double)(n - used);
  }
  __syncthreads();
  if (tid == 0) {
    int zero = 0;
    double ldp = 0.0, breg = 0.0;
    for (int i = 0; i < n; ++i) {
      if (s_deg[i] == 0) {
        zero = 1;
      } else {
        ldp += log2((double)s_deg[i]);
        double lf = 0.0;
        for (int q = 2; q <= s_deg[i]; ++q) lf += log2((double)q);
        breg += lf / s_deg[i];
      }
    }
    int best = 0;
    for (int t = 1; t < trials; ++t)
      if (s_score[t] < s_score[best]) best = t;
    uint64_t used = 0;
    int nb = 0, nc = 0;
    for (int q = 0; q < s_nsel[best]; ++q) {
      const int k = s_order[best][q];
      if (s_deg[k] > kSparseMaxBlock || s_deg[k] == 0) continue;
      out->bsize[nb++] = s_deg[k];
      for (uint64_t a = s_nb[k]; a; a &= a - 1) out->cols[nc++] = __ffsll((long long)a) - 1;
      used |= s_nb[k];
    }
    int nt = 0;
    for (int j = 0; j < n; ++j)
      if (!((used >> j) & 1)) {
        out->cols[nc++] = j;
        ++nt;
      }
    out->status = zero;
    out->nblocks = nb;
    out->ntail = nt;
    out->trial = best;
    out->log2_terms = s_score[best];
    out->log2_degprod = ldp;
    out->bregman = breg;
  }
  if (tid < n) out->deg[tid] = s_deg[tid];
}

}  // namespace

hipError_t launch_mix_stage(int in_kind, const void* A, int n, int ld, const MixDigits& dg,
                            int b, int L, int row_scaling, double* staged, double* omega,
                            double* tin, int32_t* toff, int32_t* dig, uint64_t* qabs,
                            int32_t* rowexp, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(stage_mix_kernel, dim3(1), dim3(kBlock), 0, s, A, in_kind, n, ld, dg, b, L,
                     row_scaling, staged, omega, tin, toff, dig, qabs, rowexp, status);
  return hipGetLastError();
}

hipError_t launch_sparse_partition(int in_kind, const void* A, int n, int ld, int trials,
                                   uint64_t seed, SparsePart* out, hipStream_t s) {
  if (trials < 1 || trials > kMaxTrials) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sparse_partition_kernel, dim3(1), dim3(kBlock), 0, s, A, in_kind, n, ld,
                     trials, seed, out);
  return hipGetLastError();
}

}  // namespace perm
