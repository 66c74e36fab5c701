// C-ABI entry points of the mixed-radix Ryser walks: perm_repeated and
// perm_repeated_partial (repeated columns, Eq. ryser2), perm_sparse,
// perm_sparse_partial and perm_sparse_partition (sparse matrices, App. B).
//
// Launch sequence (caller's stream): [sparse: greedypartition on the device,
// then one small record back to the host] -> stage (checks, row exponents,
// +cols/-cols, digit weights, the inner-digit step tables) -> walk: head
// (single terms), body (chunks of L terms), tail (single terms) -> the
// fixed-order finish shared with the dense path -> copy of one record ->
// wait -> (-1)^n and the row scaling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "../../include/perm.h"
#include "perm_batched_host.hpp"
#include "perm_internal.hpp"

using namespace perm;

namespace {

constexpr int kMaxGrid = 65536;  // workgroups per walk launch
constexpr int kMaxMixParts = 3 * kMaxGrid;
constexpr int kMaxSparseTrials = 256;

struct MixWorkspace {
  int device = -1;
  int cu_count = 256;
  char* dmem = nullptr;
  DevResult* hres = nullptr;
  SparsePart* hpart = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t* status = nullptr;
  int32_t* rowexp = nullptr;
  int32_t* dig = nullptr;
  uint64_t* qabs = nullptr;
  DevResult* dres = nullptr;
  SparsePart* dpart = nullptr;
  double* staged = nullptr;
  double* omega = nullptr;
  double* tin = nullptr;
  int32_t* toff = nullptr;
  void* partials = nullptr;
  std::mutex call_mu;  // held for a whole call: calls on one device take turns
};

std::mutex g_mu;
std::map<int, MixWorkspace*> g_ws;

// Holds a device's workspace for the length of one call.  On the way out
// (also after an error) the stream is drained before the next call may
// enter, so a call on another stream or thread never finds kernels of this
// one still using the buffers.
struct CallGuard {
  std::unique_lock<std::mutex> lk;
  hipStream_t s;
  CallGuard(MixWorkspace* w, hipStream_t st) : lk(w->call_mu), s(st) {}
  ~CallGuard() { (void)hipStreamSynchronize(s); }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

perm_status hip_fail(const char* what, hipError_t e) {
  return set_error(PERM_EHIP, (std::string(what) + " failed: " + hipGetErrorString(e)).c_str());
}

#define MIX_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(#expr, e_); \
  } while (0)

perm_status get_ws(MixWorkspace** out) {
  int dev = 0;
  MIX_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find(dev);
  if (it != g_ws.end()) {
    *out = it->second;
    return PERM_OK;
  }
  const size_t L = (size_t)1 << kMixMaxLog2Chunk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_status = take(64);
  const size_t o_rowexp = take(sizeof(int32_t) * kMaxN);
  const size_t o_dig = take(sizeof(int32_t) * kDigFields * kMaxN);
  const size_t o_qabs = take(sizeof(uint64_t) * (kMaxN + 1));
  const size_t o_res = take(sizeof(DevResult));
  const size_t o_part = take(sizeof(SparsePart));
  const size_t o_staged = take(sizeof(double) * 2 * (2 * (kMaxN + 1) + 2) * kMaxN);
  const size_t o_omega = take(sizeof(double) * kMixMaxOmega);
  const size_t o_tin = take(sizeof(double) * 2 * L);
  const size_t o_toff = take(sizeof(int32_t) * 2 * L);
  const size_t o_parts = take(sizeof(double) * 4 * (size_t)kMaxMixParts);
  MixWorkspace* w = new MixWorkspace();
  w->device = dev;
  if (hipMalloc((void**)&w->dmem, off) != hipSuccess) {
    delete w;
    return set_error(PERM_ENOMEM, "hipMalloc of the mixed-radix workspace failed");
  }
  if (hipHostMalloc((void**)&w->hres, sizeof(DevResult), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&w->hpart, sizeof(SparsePart), hipHostMallocDefault) != hipSuccess) {
    if (w->hres) (void)hipHostFree(w->hres);
    (void)hipFree(w->dmem);
    delete w;
    return set_error(PERM_ENOMEM, "hipHostMalloc failed");
  }
  for (auto& ev : w->ev) MIX_TRY(hipEventCreate(&ev));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    w->cu_count = prop.multiProcessorCount;
  w->status = (int32_t*)(w->dmem + o_status);
  w->rowexp = (int32_t*)(w->dmem + o_rowexp);
  w->dig = (int32_t*)(w->dmem + o_dig);
  w->qabs = (uint64_t*)(w->dmem + o_qabs);
  w->dres = (DevResult*)(w->dmem + o_res);
  w->dpart = (SparsePart*)(w->dmem + o_part);
  w->staged = (double*)(w->dmem + o_staged);
  w->omega = (double*)(w->dmem + o_omega);
  w->tin = (double*)(w->dmem + o_tin);
  w->toff = (int32_t*)(w->dmem + o_toff);
  w->partials = (void*)(w->dmem + o_parts);
  g_ws[dev] = w;
  *out = w;
  return PERM_OK;
}

int floor_log2(uint64_t x) { return x ? 63 - __builtin_clzll(x) : -1; }

hipError_t launch_walk(bool cplx, int n, bool single, bool exact, int groups, const MixArgs& a,
                       int grid, hipStream_t s) {
  if (cplx)
    return n <= 32 ? launch_mix_walk_complex_lo(n, single, exact, groups, a, grid, s)
                   : launch_mix_walk_complex_hi(n, single, exact, groups, a, grid, s);
  return n <= 32 ? launch_mix_walk_real_lo(n, single, exact, groups, a, grid, s)
                 : launch_mix_walk_real_hi(n, single, exact, groups, a, grid, s);
}

// Exact 0/1 products: deal the rows into kg equal groups (ceil(n / kg) rows,
// the last shorter) so that every group's product of row degrees is below
// 2^50.  A row sum of a 0/1 matrix over any column set is at most the row's
// degree, so every partial product of a group is then an exact double.  Rows
// are taken by decreasing degree, each into the open group with the smallest
// log-degree sum; row[] lists group 0's rows, then group 1's, ...  Returns
// false when some group's product reaches 2^50.
bool group_rows(const int32_t* deg, int n, int kg, int32_t* row) {
  const int gs = (n + kg - 1) / kg;
  if (kg < 1 || kg > kMixMaxRowGroups || (kg - 1) * gs >= n) return false;
  int order[kMaxN];
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order, order + n, [&](int x, int y) { return deg[x] > deg[y]; });
  double lsum[kMixMaxRowGroups] = {};
  int cnt[kMixMaxRowGroups] = {};
  int member[kMixMaxRowGroups][kMaxN];
  for (int q = 0; q < n; ++q) {
    const int i = order[q];
    int best = -1;
    for (int g = 0; g < kg; ++g) {
      const int cap = g + 1 < kg ? gs : n - (kg - 1) * gs;
      if (cnt[g] < cap && (best < 0 || lsum[g] < lsum[best])) best = g;
    }
    member[best][cnt[best]++] = i;
    lsum[best] += std::log2((double)(deg[i] > 0 ? deg[i] : 1));
  }
  int k = 0;
  for (int g = 0; g < kg; ++g) {
    uint64_t prod = 1;
    std::sort(member[g], member[g] + cnt[g]);
    for (int t = 0; t < cnt[g]; ++t) {
      const uint64_t d = (uint64_t)(deg[member[g][t]] > 0 ? deg[member[g][t]] : 1);
      prod *= d;  // stays below 2^50 * 64 before the check fails
      if (prod >= (1ull << 50)) return false;
      row[k++] = member[g][t];
    }
  }
  return true;
}

// The options the mixed-radix walks take: precision PERM_FP64_DD, log2_chunk
// <= 14, blocks, row scaling.
perm_status check_opts(const perm_opts& o) {
  if (o.precision != PERM_FP64_DD)
    return set_error(PERM_ENOTIMPL, "mixed-radix walks: only PERM_FP64_DD is provided");
  if (o.drift_check) return set_error(PERM_ENOTIMPL, "mixed-radix walks: no drift check");
  if (o.use_graph) return set_error(PERM_ENOTIMPL, "mixed-radix walks: no graph replay");
  if (o.log2_chunk < 0 || o.log2_chunk > kMixMaxLog2Chunk)
    return set_error(PERM_EINVAL, "log2_chunk out of range (max 14)");
  if (o.blocks < 0 || o.blocks > kMaxGrid) return set_error(PERM_EINVAL, "blocks out of range");
  if (o.reserved) return set_error(PERM_EINVAL, "reserved options must be 0");
  if (o.partials_out) return set_error(PERM_ENOTIMPL, "partials_out is not provided here");
  return PERM_OK;
}

struct Walked {
  DevResult res;
  int b;
  uint64_t chunks;
  int blocks;
  float kernel_ms, total_ms;
};

// Stage and walk Gray indices [start, start + count) of the digit order.
// exact: 128-bit integer sums (0/1 data, weights +-1).
perm_status run_mixed(MixWorkspace* ws, int in_kind, const void* dA, int n, int ld,
                      const MixDigits& dg, uint64_t start, uint64_t count, const perm_opts& o,
                      int row_scaling, bool exact, int groups, hipStream_t stream,
                      Walked* wk) {
  const bool cplx = in_kind == 1;
  // Inner digits: as many leading digits as fit in the chunk cap (at least one).
  int cap_lg = o.log2_chunk;
  if (cap_lg == 0) {
    cap_lg = floor_log2(count) - 18;
    cap_lg = cap_lg < 4 ? 4 : (cap_lg > 12 ? 12 : cap_lg);
  }
  if (exact && cap_lg > kMixExactMaxLog2Chunk) cap_lg = kMixExactMaxLog2Chunk;
  const uint64_t cap = 1ull << cap_lg;
  int b = 0;
  uint64_t L = 1;
  while (b < dg.R && L * (uint64_t)dg.radix[b] <= cap) L *= (uint64_t)dg.radix[b++];
  if (b == 0) {
    b = 1;
    L = (uint64_t)dg.radix[0];
  }
  const uint64_t end = start + count;
  uint64_t a0 = (start + L - 1) / L * L;
  if (a0 > end) a0 = end;
  const uint64_t a1 = a0 + (end - a0) / L * L;
  const int grid_cap = o.blocks > 0 ? o.blocks : 8 * ws->cu_count;
  MIX_TRY(hipEventRecord(ws->ev[0], stream));
  MIX_TRY(launch_mix_stage(in_kind, dA, n, ld, dg, b, (int)L, row_scaling, ws->staged, ws->omega,
                           ws->tin, ws->toff, ws->dig, ws->qabs, ws->rowexp, ws->status,
                           stream));
  int nparts = 0, body_grid = 0;
  const size_t part_bytes = (cplx && !exact) ? 32 : 16;
  auto walk = [&](uint64_t first, uint64_t nchunks, bool single, int* grid_out) -> perm_status {
    if (nchunks == 0) return PERM_OK;
    MixArgs a;
    a.staged = ws->staged;
    a.omega = ws->omega;
    a.tin = ws->tin;
    a.toff = ws->toff;
    a.dig = ws->dig;
    a.qabs = ws->qabs;
    a.status = ws->status;
    a.first = first;
    a.nchunks = nchunks;
    a.ntasks = 2 * ((nchunks + 2 * kWave - 1) / (2 * kWave));
    a.R = dg.R;
    a.b = b;
    a.L = (int32_t)L;
    a.ncols = dg.ncols;
    a.outer_col = b < dg.R ? dg.first[b] : dg.ncols;
    a.pad = 0;
    a.partials = (char*)ws->partials + part_bytes * nparts;
    uint64_t blocks = (a.ntasks + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > (uint64_t)grid_cap) blocks = (uint64_t)grid_cap;
    if (blocks < 1) blocks = 1;
    const int grid = (int)blocks;
    if (grid_out) *grid_out = grid;
    nparts += grid;
    const hipError_t e = launch_walk(cplx, n, single, exact, groups, a, grid, stream);
    if (e != hipSuccess) return hip_fail("mixed-radix walk launch", e);
    return PERM_OK;
  };
  perm_status st;
  MIX_TRY(hipEventRecord(ws->ev[1], stream));
  if ((st = walk(start, a0 - start, true, nullptr)) != PERM_OK) return st;
  if ((st = walk(a0 / L, (a1 - a0) / L, false, &body_grid)) != PERM_OK) return st;
  if ((st = walk(a1, end - a1, true, nullptr)) != PERM_OK) return st;
  MIX_TRY(hipEventRecord(ws->ev[2], stream));
  MIX_TRY(launch_finish(exact ? kInt01 : (cplx ? kComplex : kReal), ws->partials, nparts,
                        nullptr, 0, ws->status, ws->rowexp, n, nullptr, ws->dres, stream));
  MIX_TRY(hipMemcpyAsync(ws->hres, ws->dres, sizeof(DevResult), hipMemcpyDeviceToHost, stream));
  MIX_TRY(hipEventRecord(ws->ev[3], stream));
  MIX_TRY(hipStreamSynchronize(stream));
  wk->res = *ws->hres;
  wk->b = b;
  wk->chunks = (a1 - a0) / L + (a0 - start) + (end - a1);
  wk->blocks = body_grid;
  wk->kernel_ms = wk->total_ms = 0.0f;
  (void)hipEventElapsedTime(&wk->kernel_ms, ws->ev[1], ws->ev[2]);
  (void)hipEventElapsedTime(&wk->total_ms, ws->ev[0], ws->ev[3]);
  if (wk->res.status == kStNonFinite)
    return set_error(PERM_ENONFINITE, "matrix has a NaN or infinite entry");
  if (wk->res.status == kStInval)
    return set_error(PERM_EINVAL, "0/1 matrix has an entry other than 0 or 1");
  if (wk->res.status != kStOk) return set_error(PERM_EHIP, "unexpected device status");
  return PERM_OK;
}

// Product of the radices, or 0 above 2^63.
uint64_t digit_terms(const MixDigits& dg) {
  unsigned __int128 t = 1;
  for (int k = 0; k < dg.R; ++k) {
    t *= (unsigned __int128)dg.radix[k];
    if (t > ((unsigned __int128)1 << 63)) return 0;
  }
  return (uint64_t)t;
}

void fill_float(const Walked& wk, double sign, uint64_t count, perm_result* r) {
  const int e = -wk.res.exp_sum;
  r->re_hi = std::ldexp(sign * wk.res.v[0], e);
  r->re_lo = std::ldexp(sign * wk.res.v[1], e);
  r->im_hi = std::ldexp(sign * wk.res.v[2], e);
  r->im_lo = std::ldexp(sign * wk.res.v[3], e);
  r->max_drift = -1.0;
  r->terms = count;
  r->chunks = wk.chunks;
  r->log2_chunk = wk.b;
  r->blocks = wk.blocks;
  r->kernel_ms = wk.kernel_ms;
  r->total_ms = wk.total_ms;
}

// ------------------------------------------------------- repeated columns ----

perm_status rep_call(int dtype, const double* dC, int n, int R, int ld, const int32_t* mult,
                     bool whole, uint64_t start, uint64_t count, const perm_opts* opts,
                     perm_result* out, hipStream_t stream) {
  if (!out) return set_error(PERM_EINVAL, "out is NULL");
  if (dtype != PERM_DT_REAL && dtype != PERM_DT_COMPLEX)
    return set_error(PERM_EINVAL, "dtype must be PERM_DT_REAL or PERM_DT_COMPLEX");
  if (n < 1 || n > kMaxN) return set_error(PERM_EINVAL, "n must be in [1, 64]");
  if (R < 1 || R > n) return set_error(PERM_EINVAL, "R must be in [1, n]");
  if (ld < n) return set_error(PERM_EINVAL, "ld must be >= n");
  if (!dC || !mult) return set_error(PERM_EINVAL, "NULL argument");
  MixDigits dg;
  std::memset(&dg, 0, sizeof dg);
  for (int i = 0; i < n; ++i) dg.row[i] = i;
  dg.R = R;
  dg.ncols = R;
  int total = 0;
  for (int k = 0; k < R; ++k) {
    if (mult[k] < 1) return set_error(PERM_EINVAL, "every multiplicity must be >= 1");
    total += mult[k];
    if (total > n) break;
    dg.kind[k] = 0;
    dg.radix[k] = mult[k] + 1;
    dg.first[k] = k;
    dg.size[k] = 1;
    dg.mult[k] = mult[k];
    dg.src[k] = k;
    dg.cmult[k] = mult[k];
  }
  if (total != n) return set_error(PERM_EINVAL, "the multiplicities must add up to n");
  const uint64_t T = digit_terms(dg);
  if (T == 0) return set_error(PERM_EINVAL, "prod (mult[k] + 1) exceeds 2^63");
  if (whole) {
    start = 0;
    count = T;
  }
  if (start > T || count > T - start)
    return set_error(PERM_EINVAL, "range outside [0, prod (mult[k] + 1))");
  perm_opts o{};
  if (opts) o = *opts;
  perm_status st = check_opts(o);
  if (st != PERM_OK) return st;
  perm_result r{};
  r.max_drift = -1.0;
  if (count == 0) {
    *out = r;
    return PERM_OK;
  }
  MixWorkspace* ws = nullptr;
  if ((st = get_ws(&ws)) != PERM_OK) return st;
  CallGuard guard(ws, stream);
  Walked wk;
  st = run_mixed(ws, dtype == PERM_DT_COMPLEX ? 1 : 0, dC, n, ld, dg, start, count, o,
                 o.no_row_scaling ? 0 : 1, false, 0, stream, &wk);
  if (st != PERM_OK) return st;
  fill_float(wk, (whole && (n % 2)) ? -1.0 : 1.0, count, &r);  // per = (-1)^n S
  *out = r;
  return PERM_OK;
}

// ---------------------------------------------------------------- sparse ----

perm_status sparse_args(int dtype, const void* dA, int n, int ld, int trials, perm_result* out) {
  if (!out) return set_error(PERM_EINVAL, "out is NULL");
  if (dtype < PERM_DT_REAL || dtype > PERM_DT_INT01) return set_error(PERM_EINVAL, "bad dtype");
  if (n < 1 || n > kMaxN) return set_error(PERM_EINVAL, "n must be in [1, 64]");
  if (ld < n) return set_error(PERM_EINVAL, "ld must be >= n");
  if (!dA) return set_error(PERM_EINVAL, "dA is NULL");
  if (trials < 1 || trials > kMaxSparseTrials)
    return set_error(PERM_EINVAL, "trials must be in [1, 256]");
  return PERM_OK;
}

int in_kind_of(int dtype) { return dtype == PERM_DT_COMPLEX ? 1 : (dtype == PERM_DT_INT01 ? 2 : 0); }

// greedypartition on the device, brought back to the host.
perm_status partition(MixWorkspace* ws, int dtype, const void* dA, int n, int ld, int trials,
                      uint64_t seed, hipStream_t stream, SparsePart* part) {
  MIX_TRY(launch_sparse_partition(in_kind_of(dtype), dA, n, ld, trials, seed, ws->dpart, stream));
  MIX_TRY(hipMemcpyAsync(ws->hpart, ws->dpart, sizeof(SparsePart), hipMemcpyDeviceToHost, stream));
  MIX_TRY(hipStreamSynchronize(stream));
  *part = *ws->hpart;
  return PERM_OK;
}

// Digits of the sparse enumeration: blocks (kind 1), then the columns of T.
void sparse_digits(const SparsePart& p, int n, MixDigits* dg) {
  std::memset(dg, 0, sizeof *dg);
  for (int i = 0; i < n; ++i) dg->row[i] = i;
  int c = 0, d = 0;
  for (int l = 0; l < p.nblocks; ++l, ++d) {
    dg->kind[d] = 1;
    dg->radix[d] = (1 << p.bsize[l]) - 1;
    dg->first[d] = c;
    dg->size[d] = p.bsize[l];
    c += p.bsize[l];
  }
  for (int t = 0; t < p.ntail; ++t, ++d) {
    dg->kind[d] = 0;
    dg->radix[d] = 2;
    dg->first[d] = c++;
    dg->size[d] = 1;
    dg->mult[d] = 1;
  }
  dg->R = d;
  dg->ncols = n;
  for (int j = 0; j < n; ++j) {
    dg->src[j] = p.cols[j];
    dg->cmult[j] = 1;
  }
}

perm_status sparse_call(int dtype, const void* dA, int n, int ld, int trials, uint64_t seed,
                        bool whole, uint64_t start, uint64_t count, const perm_opts* opts,
                        perm_result* out, hipStream_t stream) {
  perm_status st = sparse_args(dtype, dA, n, ld, trials, out);
  if (st != PERM_OK) return st;
  perm_opts o{};
  if (opts) o = *opts;
  if ((st = check_opts(o)) != PERM_OK) return st;
  MixWorkspace* ws = nullptr;
  if ((st = get_ws(&ws)) != PERM_OK) return st;
  CallGuard guard(ws, stream);
  SparsePart p;
  if ((st = partition(ws, dtype, dA, n, ld, trials, seed, stream, &p)) != PERM_OK) return st;
  perm_result r{};
  r.max_drift = -1.0;
  if (p.status) {  // a zero row: per(A) = 0 and nothing to enumerate
    if (!whole && (start != 0 || count != 0))
      return set_error(PERM_EINVAL, "range outside the (empty) enumeration");
    *out = r;
    return PERM_OK;
  }
  MixDigits dg;
  sparse_digits(p, n, &dg);
  const uint64_t T = digit_terms(dg);
  if (T == 0) return set_error(PERM_EINVAL, "the enumeration has more than 2^63 column sets");
  if (whole) {
    start = 0;
    count = T;
  }
  if (start > T || count > T - start) return set_error(PERM_EINVAL, "range outside [0, terms)");
  const bool exact = dtype == PERM_DT_INT01;
  if (exact && whole && p.bregman >= 127.0)
    return set_error(PERM_ERANGE, "exact 0/1 result may exceed 128 bits (Bregman bound >= 127)");
  if (count == 0) {
    *out = r;
    return PERM_OK;
  }
  Walked wk;
  int groups = 0;  // exact: the fewest row groups whose degree products fit
  if (exact) {
    const int k = int01_group_rows(n);
    const int kdef = (n + k - 1) / k;
    for (int kg = 1; kg < kdef && kg <= kMixMaxRowGroups && !groups; ++kg)
      if (group_rows(p.deg, n, kg, dg.row)) groups = kg;
    if (!groups)
      for (int i = 0; i < n; ++i) dg.row[i] = i;
  }
  st = run_mixed(ws, in_kind_of(dtype), dA, n, ld, dg, start, count, o,
                 (exact || o.no_row_scaling) ? 0 : 1, exact, groups, stream, &wk);
  if (st != PERM_OK) return st;
  fill_float(wk, (whole && (n % 2)) ? -1.0 : 1.0, count, &r);
  if (exact) {
    r.walk_variant = groups;
    // S = sum over the sets of (-1)^|J| prod_i r_i modulo 2^128; per = (-1)^n S
    unsigned __int128 u = ((unsigned __int128)wk.res.iw[1] << 64) | wk.res.iw[0];
    if (whole && (n % 2)) u = (unsigned __int128)0 - u;
    const __int128 v = (__int128)u;
    r.int_lo = (uint64_t)u;
    r.int_hi = (int64_t)(u >> 64);
    const double h = (double)v;
    r.re_hi = h;
    r.re_lo = std::fabs(h) >= 1.7014118346046923e38 ? 0.0 : (double)(v - (__int128)h);
    r.im_hi = r.im_lo = 0.0;
  }
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
    MixWorkspace* w = kv.second;
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    for (auto& ev : w->ev)
      if (ev) (void)hipEventDestroy(ev);
    if (w->hres) (void)hipHostFree(w->hres);
    if (w->hpart) (void)hipHostFree(w->hpart);
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
  return rep_call(dtype, dC, n, R, ld, mult, true, 0, 0, opts, out, (hipStream_t)stream);
}

perm_status perm_repeated_partial(int dtype, const double* dC, int n, int R, int ld,
                                  const int32_t* mult, uint64_t start, uint64_t count,
                                  const perm_opts* opts, perm_result* out, void* stream) {
  return rep_call(dtype, dC, n, R, ld, mult, false, start, count, opts, out, (hipStream_t)stream);
}

perm_status perm_sparse(int dtype, const void* dA, int n, int ld, int trials, uint64_t seed,
                        const perm_opts* opts, perm_result* out, void* stream) {
  return sparse_call(dtype, dA, n, ld, trials, seed, true, 0, 0, opts, out, (hipStream_t)stream);
}

perm_status perm_sparse_partial(int dtype, const void* dA, int n, int ld, int trials,
                                uint64_t seed, uint64_t start, uint64_t count,
                                const perm_opts* opts, perm_result* out, void* stream) {
  return sparse_call(dtype, dA, n, ld, trials, seed, false, start, count, opts, out,
                     (hipStream_t)stream);
}

perm_status perm_sparse_partition(int dtype, const void* dA, int n, int ld, int trials,
                                  uint64_t seed, int32_t* block_of_col, int32_t* nblocks,
                                  uint64_t* terms, void* stream) {
  perm_result dummy;
  perm_status st = sparse_args(dtype, dA, n, ld, trials, &dummy);
  if (st != PERM_OK) return st;
  if (!block_of_col || !nblocks || !terms) return set_error(PERM_EINVAL, "NULL argument");
  MixWorkspace* ws = nullptr;
  if ((st = get_ws(&ws)) != PERM_OK) return st;
  CallGuard guard(ws, (hipStream_t)stream);
  SparsePart p;
  if ((st = partition(ws, dtype, dA, n, ld, trials, seed, (hipStream_t)stream, &p)) != PERM_OK)
    return st;
  if (p.status) return set_error(PERM_EINVAL, "the matrix has a zero row (per = 0)");
  for (int j = 0; j < n; ++j) block_of_col[j] = -1;
  int c = 0;
  for (int l = 0; l < p.nblocks; ++l)
    for (int e = 0; e < p.bsize[l]; ++e) block_of_col[p.cols[c++]] = l;
  *nblocks = p.nblocks;
  MixDigits dg;
  sparse_digits(p, n, &dg);
  *terms = digit_terms(dg);
  return PERM_OK;
}

}  // extern "C"
