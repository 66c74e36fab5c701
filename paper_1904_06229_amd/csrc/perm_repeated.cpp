// C-ABI entry points for matrices with repeated columns (Sec. II.A,
// Eq. ryser2): perm_repeated and perm_repeated_partial.
//
// Launch sequence (caller's stream): stage (checks, row exponents, +C/-C,
// binomials, the inner-digit step tables) -> walk: head (single terms), body
// (chunks of L terms), tail (single terms) -> the fixed-order finish shared
// with the dense path -> copy of one record -> wait -> (-1)^n and the row
// scaling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "../../include/perm.h"
#include "perm_batched_host.hpp"
#include "perm_internal.hpp"

using namespace perm;

namespace {

constexpr int kMaxGrid = 65536;          // workgroups per walk launch
constexpr int kMaxRepParts = 3 * kMaxGrid;

struct RepWorkspace {
  int device = -1;
  int cu_count = 256;
  char* dmem = nullptr;
  DevResult* hres = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t* status = nullptr;
  int32_t* rowexp = nullptr;
  int32_t* radix = nullptr;
  DevResult* dres = nullptr;
  double* staged = nullptr;
  double* binom = nullptr;
  double* tin = nullptr;
  int32_t* toff = nullptr;
  void* partials = nullptr;
};

std::mutex g_mu;
std::map<int, RepWorkspace*> g_ws;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

perm_status hip_fail(const char* what, hipError_t e) {
  return set_error(PERM_EHIP, (std::string(what) + " failed: " + hipGetErrorString(e)).c_str());
}

#define REP_TRY(expr)                               \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(#expr, e_); \
  } while (0)

perm_status get_ws(RepWorkspace** out) {
  int dev = 0;
  REP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) {
    *out = it->second;
    return PERM_OK;
  }
  const size_t L = (size_t)1 << kRepMaxLog2Chunk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_status = take(64);
  const size_t o_rowexp = take(sizeof(int32_t) * kMaxN);
  const size_t o_radix = take(sizeof(int32_t) * kMaxN);
  const size_t o_res = take(sizeof(DevResult));
  const size_t o_staged = take(sizeof(double) * 2 * (2 * (kMaxN + 1) + 2) * kMaxN);
  const size_t o_binom = take(sizeof(double) * kMaxN * kRepBinomStride);
  const size_t o_tin = take(sizeof(double) * 2 * L);
  const size_t o_toff = take(sizeof(int32_t) * 2 * L);
  const size_t o_part = take(sizeof(double) * 4 * (size_t)kMaxRepParts);
  RepWorkspace* w = new RepWorkspace();
  w->device = dev;
  hipError_t e = hipMalloc((void**)&w->dmem, off);
  if (e != hipSuccess) {
    delete w;
    return set_error(PERM_ENOMEM, "hipMalloc of the repeated-column workspace failed");
  }
  e = hipHostMalloc((void**)&w->hres, sizeof(DevResult), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(w->dmem);
    delete w;
    return set_error(PERM_ENOMEM, "hipHostMalloc failed");
  }
  for (auto& ev : w->ev) REP_TRY(hipEventCreate(&ev));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    w->cu_count = prop.multiProcessorCount;
  w->status = (int32_t*)(w->dmem + o_status);
  w->rowexp = (int32_t*)(w->dmem + o_rowexp);
  w->radix = (int32_t*)(w->dmem + o_radix);
  w->dres = (DevResult*)(w->dmem + o_res);
  w->staged = (double*)(w->dmem + o_staged);
  w->binom = (double*)(w->dmem + o_binom);
  w->tin = (double*)(w->dmem + o_tin);
  w->toff = (int32_t*)(w->dmem + o_toff);
  w->partials = (void*)(w->dmem + o_part);
  g_ws[dev] = w;
  *out = w;
  return PERM_OK;
}

int floor_log2(uint64_t x) { return x ? 63 - __builtin_clzll(x) : -1; }

hipError_t launch_rep_walk(bool cplx, int n, bool single, const RepArgs& a, int grid,
                           hipStream_t s) {
  if (cplx)
    return n <= 32 ? launch_rep_walk_complex_lo(n, single, a, grid, s)
                   : launch_rep_walk_complex_hi(n, single, a, grid, s);
  return n <= 32 ? launch_rep_walk_real_lo(n, single, a, grid, s)
                 : launch_rep_walk_real_hi(n, single, a, grid, s);
}

perm_status rep_call(int dtype, const double* dC, int n, int R, int ld, const int32_t* mult,
                     uint64_t start, uint64_t count, bool full, const perm_opts* opts,
                     perm_result* out, hipStream_t stream) {
  if (!out) return set_error(PERM_EINVAL, "out is NULL");
  if (dtype != PERM_DT_REAL && dtype != PERM_DT_COMPLEX)
    return set_error(PERM_EINVAL, "dtype must be PERM_DT_REAL or PERM_DT_COMPLEX");
  if (n < 1 || n > kMaxN) return set_error(PERM_EINVAL, "n must be in [1, 64]");
  if (R < 1 || R > n) return set_error(PERM_EINVAL, "R must be in [1, n]");
  if (ld < n) return set_error(PERM_EINVAL, "ld must be >= n");
  if (!dC || !mult) return set_error(PERM_EINVAL, "NULL argument");
  int total = 0;
  unsigned __int128 T = 1;
  RepMult rm{};
  for (int k = 0; k < R; ++k) {
    if (mult[k] < 1) return set_error(PERM_EINVAL, "every multiplicity must be >= 1");
    total += mult[k];
    if (total > n) break;
    rm.m[k] = mult[k];
    T *= (unsigned __int128)(mult[k] + 1);
  }
  if (total != n) return set_error(PERM_EINVAL, "the multiplicities must add up to n");
  if (T > ((unsigned __int128)1 << 63))
    return set_error(PERM_EINVAL, "prod (mult[k] + 1) exceeds 2^63");
  const uint64_t terms = (uint64_t)T;
  if (start > terms || count > terms - start)
    return set_error(PERM_EINVAL, "range outside [0, prod (mult[k] + 1))");
  perm_opts o{};
  if (opts) o = *opts;
  if (o.precision != PERM_FP64_DD)
    return set_error(PERM_ENOTIMPL, "repeated columns: only PERM_FP64_DD is provided");
  if (o.drift_check) return set_error(PERM_ENOTIMPL, "repeated columns: no drift check");
  if (o.log2_chunk < 0 || o.log2_chunk > kRepMaxLog2Chunk)
    return set_error(PERM_EINVAL, "log2_chunk out of range (max 14)");
  if (o.blocks < 0 || o.blocks > kMaxGrid) return set_error(PERM_EINVAL, "blocks out of range");
  if (o.reserved[0] || o.reserved[1]) return set_error(PERM_EINVAL, "reserved options must be 0");
  perm_result r{};
  r.max_drift = -1.0;
  if (count == 0) {
    *out = r;
    return PERM_OK;
  }
  const bool cplx = dtype == PERM_DT_COMPLEX;

  // Inner digits: as many leading digits as fit in the chunk cap (at least one).
  int cap_lg = o.log2_chunk;
  if (cap_lg == 0) {
    cap_lg = floor_log2(count) - 18;
    cap_lg = cap_lg < 4 ? 4 : (cap_lg > 12 ? 12 : cap_lg);
  }
  const uint64_t cap = 1ull << cap_lg;
  int b = 0;
  uint64_t L = 1;
  while (b < R && L * (uint64_t)(mult[b] + 1) <= cap) L *= (uint64_t)(mult[b++] + 1);
  if (b == 0) {
    b = 1;
    L = (uint64_t)(mult[0] + 1);
  }
  const uint64_t end = start + count;
  uint64_t a0 = (start + L - 1) / L * L;
  if (a0 > end) a0 = end;
  const uint64_t a1 = a0 + (end - a0) / L * L;

  RepWorkspace* ws = nullptr;
  perm_status st = get_ws(&ws);
  if (st != PERM_OK) return st;
  const int grid_cap = o.blocks > 0 ? o.blocks : 8 * ws->cu_count;
  REP_TRY(hipEventRecord(ws->ev[0], stream));
  REP_TRY(launch_rep_stage(cplx ? 1 : 0, dC, n, R, ld, rm, b, (int)L, o.no_row_scaling ? 0 : 1,
                           ws->staged, ws->binom, ws->tin, ws->toff, ws->radix, ws->rowexp,
                           ws->status, stream));
  int nparts = 0, body_grid = 0;
  const size_t part_bytes = cplx ? 32 : 16;
  auto walk = [&](uint64_t first, uint64_t nchunks, bool single, int* grid_out) -> perm_status {
    if (nchunks == 0) return PERM_OK;
    RepArgs a;
    a.staged = ws->staged;
    a.binom = ws->binom;
    a.tin = ws->tin;
    a.toff = ws->toff;
    a.radix = ws->radix;
    a.status = ws->status;
    a.first = first;
    a.nchunks = nchunks;
    a.ntasks = 2 * ((nchunks + 2 * kWave - 1) / (2 * kWave));
    a.R = R;
    a.b = b;
    a.L = (int32_t)L;
    a.pad = 0;
    a.partials = (char*)ws->partials + part_bytes * nparts;
    uint64_t blocks = (a.ntasks + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > (uint64_t)grid_cap) blocks = (uint64_t)grid_cap;
    if (blocks < 1) blocks = 1;
    const int grid = (int)blocks;
    if (grid_out) *grid_out = grid;
    nparts += grid;
    const hipError_t e = launch_rep_walk(cplx, n, single, a, grid, stream);
    if (e != hipSuccess) return hip_fail("repeated-column walk launch", e);
    return PERM_OK;
  };
  REP_TRY(hipEventRecord(ws->ev[1], stream));
  if ((st = walk(start, a0 - start, true, nullptr)) != PERM_OK) return st;
  if ((st = walk(a0 / L, (a1 - a0) / L, false, &body_grid)) != PERM_OK) return st;
  if ((st = walk(a1, end - a1, true, nullptr)) != PERM_OK) return st;
  REP_TRY(hipEventRecord(ws->ev[2], stream));
  REP_TRY(launch_finish(cplx ? kComplex : kReal, ws->partials, nparts, nullptr, 0, ws->status,
                        ws->rowexp, n, nullptr, ws->dres, stream));
  REP_TRY(hipMemcpyAsync(ws->hres, ws->dres, sizeof(DevResult), hipMemcpyDeviceToHost, stream));
  REP_TRY(hipEventRecord(ws->ev[3], stream));
  REP_TRY(hipStreamSynchronize(stream));
  const DevResult res = *ws->hres;
  if (res.status == kStNonFinite)
    return set_error(PERM_ENONFINITE, "matrix has a NaN or infinite entry");
  if (res.status != kStOk) return set_error(PERM_EHIP, "unexpected device status");
  // per = (-1)^n S (whole sum only), then undo the row scaling 2^(sum e_i).
  const double f = (full && (n % 2)) ? -1.0 : 1.0;
  const int e = -res.exp_sum;
  r.re_hi = std::ldexp(f * res.v[0], e);
  r.re_lo = std::ldexp(f * res.v[1], e);
  r.im_hi = std::ldexp(f * res.v[2], e);
  r.im_lo = std::ldexp(f * res.v[3], e);
  r.terms = count;
  r.chunks = (a1 - a0) / L + (a0 - start) + (end - a1);
  r.log2_chunk = b;
  r.blocks = body_grid;
  (void)hipEventElapsedTime(&r.kernel_ms, ws->ev[1], ws->ev[2]);
  (void)hipEventElapsedTime(&r.total_ms, ws->ev[0], ws->ev[3]);
  *out = r;
  return PERM_OK;
}

}  // namespace

namespace perm {
void repeated_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_ws) {
    RepWorkspace* w = kv.second;
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    for (auto& ev : w->ev)
      if (ev) (void)hipEventDestroy(ev);
    if (w->hres) (void)hipHostFree(w->hres);
    if (w->dmem) (void)hipFree(w->dmem);
    delete w;
  }
  g_ws.clear();
  (void)hipSetDevice(cur);
}
}  // namespace perm

extern "C" {

perm_status perm_repeated(int dtype, const double* dC, int n, int R, int ld, const int32_t* mult,
                          const perm_opts* opts, perm_result* out, void* stream) {
  // whole range: start 0, count = prod (mult[k] + 1) (checked inside)
  uint64_t T = 1;
  if (mult && R >= 1 && R <= kMaxN) {
    unsigned __int128 t = 1;
    for (int k = 0; k < R; ++k) {
      t *= (unsigned __int128)(mult[k] > 0 ? mult[k] + 1 : 1);
      if (t > ((unsigned __int128)1 << 63)) break;
    }
    T = t > ((unsigned __int128)1 << 63) ? 0 : (uint64_t)t;
  }
  if (T == 0) return set_error(PERM_EINVAL, "prod (mult[k] + 1) exceeds 2^63");
  return rep_call(dtype, dC, n, R, ld, mult, 0, T, true, opts, out, (hipStream_t)stream);
}

perm_status perm_repeated_partial(int dtype, const double* dC, int n, int R, int ld,
                                  const int32_t* mult, uint64_t start, uint64_t count,
                                  const perm_opts* opts, perm_result* out, void* stream) {
  return rep_call(dtype, dC, n, R, ld, mult, start, count, false, opts, out,
                  (hipStream_t)stream);
}

}  // extern "C"
