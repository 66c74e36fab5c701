// Host side of the batched path: queue construction, per-device plan cache,
// HIP graph capture and replay, and the chunk-length autotuner.
//
// The items: matrices are sorted by size, largest first, and each matrix of
// size n contributes 2*ceil(C/128) wave items, C = 2^(n-1-b) lane chunks of
// 2^b terms.  b comes from the autotuned table for n, or from
// opts->log2_chunk, or from a default that gives items of about 2^16 terms.
// The items of one size are contiguous and cost the same: each size runs as
// one persistent launch of that size's kernel (its own register allocation),
// the waves taking the items round-robin.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "perm_batched_host.hpp"
#include "perm_internal.hpp"

using namespace perm;

namespace {

std::mutex g_bmu;

struct TuneTable {
  int b[2][kMaxBatchedN + 1];  // [is_complex][n], -1 = not tuned
  bool loaded_env = false;
  TuneTable() {
    for (auto& row : b)
      for (int& x : row) x = -1;
  }
};
TuneTable g_tune;

struct Plan {
  int device = -1;
  // key
  const double* dA = nullptr;
  int count = 0, is_complex = 0, mode = 0, lc = 0, row_scaling = 1;
  double* d_out = nullptr;
  int32_t* d_status = nullptr;
  std::vector<int32_t> n;
  std::vector<int64_t> off;
  int tune_stamp = 0;
  // device buffers (one allocation)
  char* mem = nullptr;
  int64_t* d_off = nullptr;
  int32_t* d_n = nullptr;
  int64_t* st_off = nullptr;
  double* staged = nullptr;
  int32_t* exp_sum = nullptr;
  int32_t* mstatus = nullptr;
  BatchItem* items = nullptr;
  int64_t* item_first = nullptr;
  int32_t* item_count = nullptr;
  double* slots = nullptr;
  uint64_t nitems = 0;
  struct Group {
    int n;
    uint64_t item0, nitems;
    int grid;
  };
  std::vector<Group> groups;  // by size, largest first
  hipGraphExec_t gexec = nullptr;
  hipStream_t gstream = nullptr;
  // Stream order of the plan's buffers: `done` is recorded after each call's
  // work; a call on another stream first waits for it, and the buffers are
  // freed only once it has completed.
  hipEvent_t done = nullptr;
  hipStream_t last = nullptr;
  bool used = false;
};

std::vector<Plan*> g_plans;  // one per device
int g_tune_stamp = 0;

void free_plan(Plan* p) {
  if (!p) return;
  if (p->done) {
    if (p->used) (void)hipEventSynchronize(p->done);
    (void)hipEventDestroy(p->done);
  }
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->mem) (void)hipFree(p->mem);
  delete p;
}

// Default chunk length: one wave pair per matrix while that keeps chunks at
// or below 2^10 terms (n <= 18), then 2^10-term chunks and more items.
int default_log2_chunk(int n) {
  int b = n - 1 - 7;
  if (b > 10) b = 10;
  if (b < 1) b = 1;
  return b;
}

int pick_b(int is_complex, int n, int lc) {
  int b;
  if (lc > 0)
    b = lc;
  else if (g_tune.b[is_complex][n] >= 0)
    b = g_tune.b[is_complex][n];
  else
    b = default_log2_chunk(n);
  if (b > n - 1) b = n - 1;
  if (b < 1) b = n > 1 ? 1 : 0;  // the batched walk takes b >= 1 except for n = 1
  return b;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool same_key(const Plan* p, const double* dA, const int32_t* h_n, const int64_t* h_off, int count,
              int is_complex, int mode, int lc, int rs, double* d_out, int32_t* d_status, int dev) {
  if (!p || p->device != dev || p->dA != dA || p->count != count || p->is_complex != is_complex ||
      p->mode != mode || p->lc != lc || p->row_scaling != rs || p->d_out != d_out ||
      p->d_status != d_status || p->tune_stamp != g_tune_stamp)
    return false;
  return std::equal(p->n.begin(), p->n.end(), h_n) && std::equal(p->off.begin(), p->off.end(), h_off);
}

perm_status build_plan(Plan* p, int dev) {
  const int count = p->count;
  const int cw = p->is_complex ? 2 : 1;
  std::vector<int64_t> st_off(count);
  int64_t st_total = 0;
  for (int m = 0; m < count; ++m) {
    st_off[m] = st_total;
    st_total += (int64_t)cw * 2 * p->n[m] * p->n[m];
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->n[a] > p->n[b]; });
  std::vector<BatchItem> items;
  std::vector<int64_t> item_first(count);
  std::vector<int32_t> item_count(count);
  p->groups.clear();
  for (int m : order) {
    const int n = p->n[m];
    if (p->groups.empty() || p->groups.back().n != n)
      p->groups.push_back(Plan::Group{n, (uint64_t)items.size(), 0, 0});
    const int b = pick_b(p->is_complex, n, p->lc);
    const uint64_t C = 1ull << (n - 1 - b);
    const uint64_t tasks = 2 * ((C + 2 * kWave - 1) / (2 * kWave));
    item_first[m] = (int64_t)items.size();
    item_count[m] = (int32_t)tasks;
    for (uint64_t t = 0; t < tasks; ++t) {
      BatchItem it;
      it.mat = m;
      it.n = n;
      it.b = b;
      it.pad = 0;
      it.task = t;
      it.nchunks = C;
      items.push_back(it);
    }
    p->groups.back().nitems += tasks;
  }
  p->nitems = items.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 8), 256);
    return o;
  };
  const size_t o_off = take(sizeof(int64_t) * count);
  const size_t o_n = take(sizeof(int32_t) * count);
  const size_t o_st = take(sizeof(int64_t) * count);
  const size_t o_staged = take(sizeof(double) * (size_t)st_total);
  const size_t o_exp = take(sizeof(int32_t) * count);
  const size_t o_ms = take(sizeof(int32_t) * count);
  const size_t o_items = take(sizeof(BatchItem) * items.size());
  const size_t o_if = take(sizeof(int64_t) * count);
  const size_t o_ic = take(sizeof(int32_t) * count);
  const size_t o_slots = take(sizeof(double) * 4 * items.size());
  hipError_t e = hipMalloc((void**)&p->mem, off);
  if (e != hipSuccess) {
    p->mem = nullptr;
    return set_error(PERM_ENOMEM, "hipMalloc of the batched plan failed");
  }
  p->d_off = (int64_t*)(p->mem + o_off);
  p->d_n = (int32_t*)(p->mem + o_n);
  p->st_off = (int64_t*)(p->mem + o_st);
  p->staged = (double*)(p->mem + o_staged);
  p->exp_sum = (int32_t*)(p->mem + o_exp);
  p->mstatus = (int32_t*)(p->mem + o_ms);
  p->items = (BatchItem*)(p->mem + o_items);
  p->item_first = (int64_t*)(p->mem + o_if);
  p->item_count = (int32_t*)(p->mem + o_ic);
  p->slots = (double*)(p->mem + o_slots);
  struct Up {
    void* dst;
    const void* src;
    size_t bytes;
  } ups[] = {{p->d_off, p->off.data(), sizeof(int64_t) * count},
             {p->d_n, p->n.data(), sizeof(int32_t) * count},
             {p->st_off, st_off.data(), sizeof(int64_t) * count},
             {p->items, items.data(), sizeof(BatchItem) * items.size()},
             {p->item_first, item_first.data(), sizeof(int64_t) * count},
             {p->item_count, item_count.data(), sizeof(int32_t) * count}};
  for (auto& u : ups)
    if (u.bytes && hipMemcpy(u.dst, u.src, u.bytes, hipMemcpyHostToDevice) != hipSuccess)
      return set_error(PERM_EHIP, "upload of the batched plan failed");
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  for (Plan::Group& g : p->groups) {
    const int nb = batched_walk_blocks_per_cu(p->is_complex, p->mode, g.n);
    uint64_t grid = (uint64_t)cus * nb;
    const uint64_t need = (g.nitems + kWavesPerBlock - 1) / kWavesPerBlock;
    if (grid > need) grid = need;
    g.grid = (int)std::max<uint64_t>(grid, 1);
  }
  return PERM_OK;
}

perm_status enqueue(Plan* p, hipStream_t s) {
  BatchArgs a;
  a.staged = p->staged;
  a.st_off = p->st_off;
  a.mstatus = p->mstatus;
  a.items = p->items;
  a.slots = p->slots;
  hipError_t e = launch_batched_stage(p->is_complex, p->dA, p->d_off, p->d_n, p->count,
                                      p->row_scaling, p->staged, p->st_off, p->exp_sum,
                                      p->mstatus, s);
  for (const Plan::Group& g : p->groups)
    if (e == hipSuccess)
      e = launch_batched_size(p->is_complex, p->mode, g.n, a, g.item0, g.nitems, g.grid, s);
  if (e == hipSuccess)
    e = launch_batched_finish(p->slots, p->item_first, p->item_count, p->d_n, p->exp_sum,
                              p->mstatus, p->count, p->d_out, p->d_status, s);
  if (e != hipSuccess)
    return set_error(PERM_EHIP, (std::string("batched launch failed: ") + hipGetErrorString(e)).c_str());
  return PERM_OK;
}

// The plan's launches on s: directly, or as a HIP graph captured once per
// stream and replayed.
perm_status launch_plan(Plan* p, hipStream_t s, bool use_graph) {
  if (!use_graph) return enqueue(p, s);
  if (!p->gexec || p->gstream != s) {
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      p->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(PERM_EHIP, "hipStreamBeginCapture failed (graphs need a non-default stream)");
    perm_status st = enqueue(p, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != PERM_OK) return st;
    if (e != hipSuccess) return set_error(PERM_EHIP, "hipStreamEndCapture failed");
    e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->gexec = nullptr;
      return set_error(PERM_EHIP, "hipGraphInstantiate failed");
    }
    p->gstream = s;
  }
  if (hipGraphLaunch(p->gexec, s) != hipSuccess) return set_error(PERM_EHIP, "hipGraphLaunch failed");
  return PERM_OK;
}


// ------------------------------------------------------------ tune cache ----

void write_cache(const char* path) {
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{\"arch\": \"gfx950\"");
  const char* names[2] = {"real", "complex"};
  for (int c = 0; c < 2; ++c) {
    std::fprintf(f, ", \"%s\": {", names[c]);
    bool first = true;
    for (int n = 1; n <= kMaxBatchedN; ++n)
      if (g_tune.b[c][n] >= 0) {
        std::fprintf(f, "%s\"%d\": %d", first ? "" : ", ", n, g_tune.b[c][n]);
        first = false;
      }
    std::fprintf(f, "}");
  }
  // the same choice as lanes per matrix: 2^(n-1-b) lane chunks of 2^b terms
  for (int c = 0; c < 2; ++c) {
    std::fprintf(f, ", \"lanes_%s\": {", names[c]);
    bool first = true;
    for (int n = 1; n <= kMaxBatchedN; ++n)
      if (g_tune.b[c][n] >= 0) {
        std::fprintf(f, "%s\"%d\": %llu", first ? "" : ", ", n,
                     (unsigned long long)(1ull << (n - 1 - g_tune.b[c][n])));
        first = false;
      }
    std::fprintf(f, "}");
  }
  std::fprintf(f, "}\n");
  std::fclose(f);
}

// Reads the file written above: sections "real"/"complex" of "n": b pairs.
void read_cache(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
  std::fclose(f);
  const char* names[2] = {"\"real\"", "\"complex\""};
  for (int c = 0; c < 2; ++c) {
    size_t pos = txt.find(names[c]);
    if (pos == std::string::npos) continue;
    size_t open = txt.find('{', pos), close = txt.find('}', pos);
    if (open == std::string::npos || close == std::string::npos) continue;
    std::string sec = txt.substr(open + 1, close - open - 1);
    size_t q = 0;
    while ((q = sec.find('"', q)) != std::string::npos) {
      int n = 0, b = 0;
      if (std::sscanf(sec.c_str() + q, "\"%d\": %d", &n, &b) == 2 && n >= 1 &&
          n <= kMaxBatchedN && b >= 0 && b < n)
        g_tune.b[c][n] = b;
      size_t end = sec.find('"', q + 1);
      if (end == std::string::npos) break;
      q = end + 1;
    }
  }
  ++g_tune_stamp;
}

}  // namespace

namespace perm {
void batched_release() {
  std::lock_guard<std::mutex> lk(g_bmu);
  for (Plan* p : g_plans) free_plan(p);
  g_plans.clear();
}
}  // namespace perm

extern "C" {

perm_status perm_batched(const double* dA, const int32_t* h_n, const int64_t* h_offset, int count,
                         int is_complex, const perm_opts* opts, double* d_out, int32_t* d_status,
                         void* stream) {
  if (count < 0) return set_error(PERM_EINVAL, "count must be >= 0");
  if (count == 0) return PERM_OK;
  if (!dA || !h_n || !h_offset || !d_out) return set_error(PERM_EINVAL, "NULL argument");
  perm_opts o{};
  if (opts) o = *opts;
  if (o.precision != PERM_FP64_DD && o.precision != PERM_FP64)
    return set_error(PERM_ENOTIMPL, "perm_batched supports PERM_FP64_DD and PERM_FP64");
  if (o.log2_chunk < 0 || o.log2_chunk > 24) return set_error(PERM_EINVAL, "log2_chunk out of range");
  if (o.drift_check) return set_error(PERM_ENOTIMPL, "perm_batched has no drift check");
  if (o.reserved) return set_error(PERM_EINVAL, "reserved options must be 0");
  if (o.partials_out) return set_error(PERM_ENOTIMPL, "partials_out is not provided here");
  for (int m = 0; m < count; ++m) {
    if (h_n[m] < 1 || h_n[m] > kMaxBatchedN) return set_error(PERM_EINVAL, "batched n must be in [1, 32]");
    if (h_offset[m] < 0) return set_error(PERM_EINVAL, "negative offset");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(PERM_EHIP, "hipGetDevice failed");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_bmu);
  if (!g_tune.loaded_env) {
    g_tune.loaded_env = true;
    if (const char* path = std::getenv("PERM_AUTOTUNE_CACHE")) read_cache(path);
  }
  const int rs = o.no_row_scaling ? 0 : 1;
  Plan* p = nullptr;
  for (Plan* q : g_plans)
    if (q->device == dev) p = q;
  if (!same_key(p, dA, h_n, h_offset, count, is_complex ? 1 : 0, o.precision, o.log2_chunk, rs,
                d_out, d_status, dev)) {
    if (p) {
      g_plans.erase(std::find(g_plans.begin(), g_plans.end(), p));
      free_plan(p);
    }
    p = new Plan();
    p->device = dev;
    p->dA = dA;
    p->count = count;
    p->is_complex = is_complex ? 1 : 0;
    p->mode = o.precision;
    p->lc = o.log2_chunk;
    p->row_scaling = rs;
    p->d_out = d_out;
    p->d_status = d_status;
    p->n.assign(h_n, h_n + count);
    p->off.assign(h_offset, h_offset + count);
    p->tune_stamp = g_tune_stamp;
    perm_status st = build_plan(p, dev);
    if (st == PERM_OK && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess) {
      p->done = nullptr;
      st = set_error(PERM_EHIP, "hipEventCreate failed");
    }
    if (st != PERM_OK) {
      free_plan(p);
      return st;
    }
    g_plans.push_back(p);
  }
  if (p->used && p->last != s && hipStreamWaitEvent(s, p->done, 0) != hipSuccess)
    return set_error(PERM_EHIP, "hipStreamWaitEvent failed");
  perm_status st = launch_plan(p, s, o.use_graph != 0);
  if (st != PERM_OK) return st;
  if (hipEventRecord(p->done, s) != hipSuccess) {
    // the order of later calls can no longer be kept: drain and forget the plan
    (void)hipStreamSynchronize(s);
    g_plans.erase(std::find(g_plans.begin(), g_plans.end(), p));
    p->used = false;
    free_plan(p);
    return set_error(PERM_EHIP, "hipEventRecord failed");
  }
  p->last = s;
  p->used = true;
  return PERM_OK;
}

perm_status perm_autotune(int is_complex, int n_lo, int n_hi, const char* cache_path,
                          void* stream) {
  if (n_lo < 1 || n_hi > kMaxBatchedN || n_lo > n_hi)
    return set_error(PERM_EINVAL, "autotune range must satisfy 1 <= n_lo <= n_hi <= 32");
  hipStream_t s = (hipStream_t)stream;
  const int c = is_complex ? 1 : 0;
  const int cw = c ? 2 : 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_error(PERM_EHIP, "hipEventCreate failed");
  perm_status result = PERM_OK;
  for (int n = n_lo; n <= n_hi && result == PERM_OK; ++n) {
    // Synthetic batch: enough matrices for about 2^30 terms (at least 64, at
    // most 16384), so that every chunk length is timed on a grid that fills the
    // device several times over, as a large batch does (a small batch favours
    // short chunks, which a large one pays for in chunk starts).
    const int64_t per = 1ll << (n - 1);
    int count = (int)std::min<int64_t>(16384, std::max<int64_t>(64, (1ll << 30) / per));
    const size_t elems = (size_t)count * n * n * cw;
    std::vector<double> h(elems);
    uint64_t x = 0x9E3779B97F4A7C15ull ^ (uint64_t)n;
    for (double& v : h) {  // xorshift64*, uniform in [-1, 1)
      x ^= x >> 12;
      x ^= x << 25;
      x ^= x >> 27;
      v = (double)((x * 2685821657736338717ull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
    std::vector<int32_t> ns(count, n);
    std::vector<int64_t> offs(count);
    for (int m = 0; m < count; ++m) offs[m] = (int64_t)m * n * n * cw;
    double *dA = nullptr, *dOut = nullptr;
    if (hipMalloc((void**)&dA, elems * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&dOut, (size_t)count * 4 * sizeof(double)) != hipSuccess) {
      if (dA) (void)hipFree(dA);
      result = set_error(PERM_ENOMEM, "autotune allocation failed");
      break;
    }
    (void)hipMemcpy(dA, h.data(), elems * sizeof(double), hipMemcpyHostToDevice);
    int best_b = -1;
    float best_ms = 1e30f;
    const int b_lo = std::max(1, n - 1 - 16), b_hi = std::min(n - 1, 14);
    for (int b = b_lo; b <= b_hi; ++b) {
      perm_opts o{};
      o.log2_chunk = b;
      float tmin = 1e30f;
      for (int rep = 0; rep < 4 && result == PERM_OK; ++rep) {
        (void)hipEventRecord(e0, s);
        result = perm_batched(dA, ns.data(), offs.data(), count, is_complex, &o, dOut, nullptr, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tmin = std::min(tmin, ms);  // first run builds the plan
      }
      if (result != PERM_OK) break;
      if (tmin < best_ms) {
        best_ms = tmin;
        best_b = b;
      }
    }
    (void)hipFree(dA);
    (void)hipFree(dOut);
    {
      std::lock_guard<std::mutex> lk(g_bmu);
      if (best_b >= 0) g_tune.b[c][n] = best_b;
      ++g_tune_stamp;
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_bmu);
    // plans built on the synthetic batches are of no further use
    for (Plan* p : g_plans) free_plan(p);
    g_plans.clear();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result == PERM_OK && cache_path) write_cache(cache_path);
  return result;
}

}  // extern "C"
