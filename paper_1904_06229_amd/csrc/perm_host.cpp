// C-ABI runtime of the permanent library: argument checks, the chunk plan,
// per-device workspace, launch sequence and result assembly.
//
// Launch sequence of a single-matrix call (all on the caller's stream):
//   stage (validate, row exponents, +A/-A)  ->  walk: head (single terms),
//   body (aligned chunks), tail (single terms)  ->  finish (fixed-order sum of
//   the per-workgroup partials, written straight into a pinned host record)
//   ->  wait for the stream  ->  scale by 2(-1)^n and 2^-(row exponents).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "../../include/perm.h"
#include "perm_batched_host.hpp"
#include "perm_internal.hpp"

using namespace perm;

namespace {

thread_local std::string g_last_error;

perm_status fail(perm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(PERM_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxParts = 3 * 65536;
constexpr int kFloatChunkCap = 24;
constexpr int kInt01ChunkCap = 10;

struct Workspace {
  int device = -1;
  char* dmem = nullptr;
  char* fmem = nullptr;           // one-launch path: workgroup slots, counter, start time
  DevResult* hres = nullptr;      // pinned host record
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  CallBuffers buf;                // device sub-buffers of dmem, the record, two events
};

constexpr size_t kFusedSlotBytes = sizeof(double) * (size_t)kFusedMaxBlocks * kFusedSlotDoubles;

// Workspaces are leased, one per call: a call takes an idle workspace of the
// current device (or allocates one) and gives it back when it returns, after
// its stream has finished with it.  Calls from several host threads or on
// several streams therefore never share device buffers.
std::mutex g_mu;
std::map<int, std::vector<Workspace*>> g_idle;  // idle workspaces per device
std::vector<Workspace*> g_all;                  // every workspace, for perm_release

void destroy_workspace(Workspace* w) {
  for (auto& ev : w->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (w->hres) (void)hipHostFree(w->hres);
  if (w->dmem) (void)hipFree(w->dmem);
  if (w->fmem) (void)hipFree(w->fmem);
  delete w;
}

perm_status create_workspace(int dev, Workspace** out) {
  Workspace* w = new Workspace();
  w->device = dev;
  hipError_t e = hipMalloc((void**)&w->dmem, call_buffer_bytes(kMaxParts));
  if (e != hipSuccess) {
    w->dmem = nullptr;
    destroy_workspace(w);
    return fail(PERM_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
  }
  e = hipHostMalloc((void**)&w->hres, sizeof(DevResult), hipHostMallocDefault);
  if (e != hipSuccess) {
    w->hres = nullptr;
    destroy_workspace(w);
    return fail(PERM_ENOMEM, std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
  }
  e = hipMalloc((void**)&w->fmem, kFusedSlotBytes + 256);
  if (e != hipSuccess) {
    w->fmem = nullptr;
    destroy_workspace(w);
    return fail(PERM_ENOMEM, std::string("hipMalloc of workspace failed: ") + hipGetErrorString(e));
  }
  CallBuffers& b = w->buf;
  carve_call_buffers(w->dmem, kMaxParts, &b);
  b.fused_slots = (double*)w->fmem;
  b.counter = (uint32_t*)(w->fmem + kFusedSlotBytes);
  b.t0 = (uint64_t*)(w->fmem + kFusedSlotBytes + 8);
  // counter 0, start time all ones (set once; every launch leaves them so)
  e = hipMemset(b.counter, 0, 8);
  if (e == hipSuccess) e = hipMemset(b.t0, 0xff, 8);
  if (e != hipSuccess) {
    destroy_workspace(w);
    return fail(PERM_EHIP, std::string("hipMemset failed: ") + hipGetErrorString(e));
  }
  if (hipDeviceGetAttribute(&b.wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    b.wall_khz = 0;
  b.hres = w->hres;
  // The finishing kernel writes the result record straight into pinned host
  // memory (no separate copy); the stream synchronisation makes it visible.
  e = hipHostGetDevicePointer((void**)&b.hres_dev, w->hres, 0);
  if (e != hipSuccess) {
    destroy_workspace(w);
    return fail(PERM_EHIP, std::string("hipHostGetDevicePointer failed: ") + hipGetErrorString(e));
  }
  for (auto& ev : w->ev) {
    e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      ev = nullptr;
      destroy_workspace(w);
      return fail(PERM_EHIP, std::string("hipEventCreate failed: ") + hipGetErrorString(e));
    }
  }
  b.ev_start = w->ev[1];
  b.ev_stop = w->ev[2];
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) b.cu_count = prop.multiProcessorCount;
  if (b.cu_count <= 0) b.cu_count = 256;
  *out = w;
  return PERM_OK;
}

perm_status acquire_workspace(Workspace** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<Workspace*>& idle = g_idle[dev];
    if (!idle.empty()) {
      *out = idle.back();
      idle.pop_back();
      return PERM_OK;
    }
  }
  Workspace* w = nullptr;
  perm_status st = create_workspace(dev, &w);
  if (st != PERM_OK) return st;
  std::lock_guard<std::mutex> lk(g_mu);
  g_all.push_back(w);
  *out = w;
  return PERM_OK;
}

// A leased workspace; it goes back to the idle list when the call returns.
struct Lease {
  Workspace* w = nullptr;
  ~Lease() {
    if (!w) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_idle[w->device].push_back(w);
  }
};

// If a call leaves early after enqueueing work (an error after a launch),
// the stream is drained first so that no kernel still uses its buffers.
struct Drain {
  hipStream_t s = nullptr;
  bool pending = false;
  ~Drain() {
    if (pending) (void)hipStreamSynchronize(s);
  }
};

uint64_t total_terms(int n) { return n >= 64 ? (1ull << 63) : (1ull << (n - 1)); }

int floor_log2(uint64_t x) { return x ? 63 - __builtin_clzll(x) : -1; }

// Automatic chunk length: enough chunks to give every SIMD several waves
// (2^18 lane chunks), chunks no longer than the cap, and at least 2^3 terms
// (when the range has them) so that small sizes walk instead of forming
// every term from scratch.  (20 x 20 complex: 18.2 us per walk at 2^3,
// 21.0 at 2^4, 26.0 at 2^5; the grid size made no difference.)
int auto_log2_chunk(uint64_t count, int cap) {
  const int lg = floor_log2(count);
  int b = lg - 18;
  const int lo = lg < 3 ? (lg > 0 ? lg : 0) : 3;
  if (b < lo) b = lo;
  if (b > cap) b = cap;
  return b;
}

int grid_for(uint64_t tasks, int cap_blocks) {
  uint64_t blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > (uint64_t)cap_blocks) blocks = (uint64_t)cap_blocks;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

perm_status check_opts(const perm_opts* o, int is_int01) {
  if (!o) return PERM_OK;
  if (o->precision < 0 || o->precision > 2) return fail(PERM_EINVAL, "precision must be 0, 1 or 2");
  const int cap = is_int01 ? kInt01ChunkCap : kFloatChunkCap;
  if (o->log2_chunk < 0 || o->log2_chunk > cap)
    return fail(PERM_EINVAL, "log2_chunk out of range (max " + std::to_string(cap) + ")");
  if (o->blocks < 0 || o->blocks > kMaxParts / 3) return fail(PERM_EINVAL, "blocks out of range");
  if (o->drift_check < 0 || o->drift_check > 1) return fail(PERM_EINVAL, "drift_check must be 0 or 1");
  if (o->reserved) return fail(PERM_EINVAL, "reserved options must be 0");
  if (o->partials_out && o->partials_cap < 0) return fail(PERM_EINVAL, "partials_cap must be >= 0");
  return PERM_OK;
}

int to_int(perm_status s) { return (int)s; }

struct Raw {
  DevResult r;
  perm_plan_info plan;
  float kernel_ms, total_ms;
  int blocks;
  int parts;  // partial sums added by the finish
};

perm_status launch_walk(int kind, int n, int mode, bool drift, int variant, const WalkArgs& a,
                        int grid, hipStream_t s) {
  hipError_t e;
  const bool lo = n <= 32;
  if (kind == kReal)
    e = lo ? launch_walk_real_lo(n, mode, drift, a, grid, s)
           : launch_walk_real_hi(n, mode, drift, a, grid, s);
  else if (kind == kComplex)
    e = lo ? launch_walk_complex_lo(n, mode, drift, a, grid, s)
           : launch_walk_complex_hi(n, mode, drift, a, grid, s);
  else
    e = lo ? launch_walk_int01_lo(n, drift, variant, a, grid, s)
           : launch_walk_int01_hi(n, drift, variant, a, grid, s);
  if (e != hipSuccess) return fail(PERM_EHIP, std::string("walk launch failed: ") + hipGetErrorString(e));
  return PERM_OK;
}

// Automatic chunk length of the one-launch path.  Every workgroup stages its
// own copy, so fewer, longer-walking workgroups pay off there: measured on
// one MI355X (host time per call, complex; real alike), the best lengths were
// 2^2 at n = 16 (23.8 us), 2^4 at n = 20 (31.0 us, against 32.3 at 2^3),
// 2^5 at n = 22 (41.6 us) and 2^7 at n = 24 (75.6 us).
int fused_log2_chunk(int n) {
  const int lg = n - 1;
  const int b = lg <= 19 ? lg - 15 : lg - 16;
  return std::min(lg, std::max(2, b));
}

// The whole sum of a small real or complex matrix in one launch (stage, walk
// and the fixed-order finish in kern_fused.hip), when the buffers have the
// workgroup slots and the options ask for nothing that launch lacks.
bool fused_eligible(const CallBuffers& bf, int kind, int n, const perm_opts& o,
                    const perm_plan_info& plan) {
  return bf.fused_slots && kind != kInt01 && n >= 2 && n <= kFusedMaxN && !o.drift_check &&
         o.blocks == 0 && !o.partials_out && plan.log2_chunk >= 1 && plan.head_count == 0 &&
         plan.tail_count == 0;
}

perm_status run_fused_on(const CallBuffers& bf, int kind, const void* dA, int n, int ld,
                         const perm_opts& o, const perm_plan_info& plan, hipStream_t s, Raw* raw) {
  const auto t_call = std::chrono::steady_clock::now();
  FusedArgs a;
  a.A = (const double*)dA;
  a.ld = ld;
  a.row_scaling = o.no_row_scaling ? 0 : 1;
  a.slots = bf.fused_slots;
  const uint64_t cw = kind == kComplex ? 2 : 1;
  a.slot_stride = (2 * cw * n * n + 31) / 32 * 32;  // 256-byte aligned slots
  a.ntasks = plan.body_tasks;
  a.nchunks = plan.body_chunks;
  a.b = plan.log2_chunk;
  a.pad = 0;
  a.partials = (double*)bf.partials;
  a.counter = bf.counter;
  a.t0 = bf.t0;
  a.res = bf.hres ? bf.hres_dev : bf.dres;
  const int grid = grid_for(plan.body_tasks, std::min(8 * bf.cu_count, kFusedMaxBlocks));
  Drain drain;
  drain.s = s;
  drain.pending = true;
  volatile uint32_t* done = bf.hres ? &bf.hres->done : nullptr;
  if (done) {
    *done = 0u;
    std::atomic_thread_fence(std::memory_order_seq_cst);
  }
  hipError_t e = launch_fused(kind == kComplex, n, o.precision, a, grid, s);
  if (e != hipSuccess) return fail(PERM_EHIP, std::string("fused launch failed: ") + hipGetErrorString(e));
  if (done) {
    // The kernel writes the record into pinned host memory and sets `done`
    // last: watching the flag returns as soon as the result is there, without
    // the stream synchronisation's wake-up.  The stream is queried now and
    // then, so an error (or a launch that never ran) ends the wait too.
    for (uint32_t spin = 1; *done == 0u; ++spin) {
      if ((spin & 1023u) == 0u && hipStreamQuery(s) != hipErrorNotReady) break;
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    if (*done == 0u) HIP_TRY(hipStreamSynchronize(s));
    if (*done == 0u) return fail(PERM_EHIP, "one-launch kernel ended without its result");
    raw->r = *bf.hres;
  } else {
    HIP_TRY(hipMemcpyAsync(&raw->r, bf.dres, sizeof(DevResult), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  drain.pending = false;
  raw->plan = plan;
  raw->blocks = grid;
  raw->parts = grid;
  raw->kernel_ms = bf.wall_khz > 0 ? (float)((double)raw->r.ticks / bf.wall_khz) : 0.0f;
  raw->total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_call).count();
  return PERM_OK;
}

// Stage, walk [start, start+count), finish, and bring the record back, on the
// device buffers `bf`.
// full: the range is the whole sum, so the 0/1 path may permute rows and
// columns and use the pair-shared walk.
perm_status run_range_on(const CallBuffers& bf, int kind, const void* dA, int n, int ld,
                         uint64_t start, uint64_t count, const perm_opts* opts, int range_check,
                         bool full, hipStream_t s, Raw* raw) {
  perm_opts o{};
  if (opts) o = *opts;
  const int is_int = kind == kInt01;
  perm_plan_info plan;
  perm_status st = perm_plan(n, start, count, o.log2_chunk, is_int, &plan);
  if (st != PERM_OK) return st;
  if (full && fused_eligible(bf, kind, n, o, plan)) {
    perm_plan_info fplan = plan;
    if (o.log2_chunk == 0 &&
        perm_plan(n, start, count, fused_log2_chunk(n), is_int, &fplan) != PERM_OK)
      fplan = plan;
    if (fused_eligible(bf, kind, n, o, fplan))
      return run_fused_on(bf, kind, dA, n, ld, o, fplan, s, raw);
    return run_fused_on(bf, kind, dA, n, ld, o, plan, s, raw);
  }
  // 8 workgroups (32 waves) per CU: more than can be resident, so the
  // dispatcher hands out the remaining workgroups as others finish, which
  // evens out the tail.  Three launches (head, body, tail) fit the partials.
  const int cap = std::min(o.blocks > 0 ? o.blocks : 8 * bf.cu_count, bf.max_parts / 3);
  const bool drift = o.drift_check != 0;
  const int mode = is_int ? 0 : o.precision;
  const bool timed = bf.ev_start && bf.ev_stop;

  const int pair_rows = (is_int && full && !drift && plan.log2_chunk >= 1 &&
                         plan.head_count == 0 && plan.tail_count == 0 &&
                         n / 3 >= kInt01PairMinRows)
                            ? n / 3
                            : 0;
  // The partial-sum slots the three walk launches will fill (checked against
  // the caller's records before anything is enqueued).
  auto tasks_of = [](uint64_t nchunks) { return 2 * ((nchunks + 2 * kWave - 1) / (2 * kWave)); };
  const int total_parts = (plan.head_count ? grid_for(tasks_of(plan.head_count), cap) : 0) +
                          (plan.body_chunks ? grid_for(tasks_of(plan.body_chunks), cap) : 0) +
                          (plan.tail_count ? grid_for(tasks_of(plan.tail_count), cap) : 0);
  if (o.partials_out && total_parts > o.partials_cap)
    return fail(PERM_EINVAL, "partials_out holds " + std::to_string(o.partials_cap) +
                                 " records, the call needs " + std::to_string(total_parts));
  // Only the walk is timed with events (each record is a marker packet in the
  // stream, a few microseconds of gap); the whole call is timed on the host.
  const auto t_call = std::chrono::steady_clock::now();
  Drain drain;
  drain.s = s;
  drain.pending = true;
  HIP_TRY(launch_stage(kind, dA, n, ld, o.no_row_scaling ? 0 : 1, range_check, pair_rows,
                       bf.staged, bf.rowabs, bf.rowexp, bf.status, bf.bound, s));

  int nparts = 0;
  int body_grid = 0;
  char* part_base = (char*)bf.partials;
  const size_t part_bytes = (kind == kComplex) ? 32 : 16;
  auto walk = [&](uint64_t first, uint64_t nchunks, int b, int variant,
                  int* grid_out) -> perm_status {
    if (nchunks == 0) return PERM_OK;
    WalkArgs a;
    a.staged = bf.staged;
    a.rowabs = bf.rowabs;
    a.status = bf.status;
    a.first = first;
    a.nchunks = nchunks;
    a.ntasks = 2 * ((nchunks + 2 * kWave - 1) / (2 * kWave));
    a.b = b;
    a.drift = drift ? 1 : 0;
    a.partials = part_base + part_bytes * nparts;
    a.drift_part = bf.drift + nparts;
    const int grid = grid_for(a.ntasks, cap);
    if (grid_out) *grid_out = grid;
    nparts += grid;
    return launch_walk(kind, n, mode, drift, variant, a, grid, s);
  };

  if (timed) HIP_TRY(hipEventRecord(bf.ev_start, s));
  if ((st = walk(plan.head_start, plan.head_count, 0, 0, nullptr)) != PERM_OK) return st;
  // Pair-shared 0/1 walk: the walk kernel takes it when the staging kernel's
  // flag allows it, else walks plainly (one launch).
  if ((st = walk(plan.body_first_chunk, plan.body_chunks, plan.log2_chunk, pair_rows > 0 ? 1 : 0,
                 &body_grid)) != PERM_OK)
    return st;
  if ((st = walk(plan.tail_start, plan.tail_count, 0, 0, nullptr)) != PERM_OK) return st;
  if (timed) HIP_TRY(hipEventRecord(bf.ev_stop, s));
  HIP_TRY(launch_finish(kind, bf.partials, nparts, bf.drift, drift ? 1 : 0, bf.status, bf.rowexp,
                        n, bf.bound, bf.hres ? bf.hres_dev : bf.dres, s));
  if (o.partials_out)
    HIP_TRY(launch_export_partials(kind, bf.partials, bf.drift, drift ? 1 : 0, nparts, bf.rowexp,
                                   n, o.partials_out, s));
  if (bf.hres) {
    HIP_TRY(hipStreamSynchronize(s));
    raw->r = *bf.hres;
  } else {
    // no pinned record: copy the device record into host memory
    HIP_TRY(hipMemcpyAsync(&raw->r, bf.dres, sizeof(DevResult), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  drain.pending = false;
  raw->plan = plan;
  raw->blocks = body_grid;
  raw->parts = nparts;
  raw->kernel_ms = 0.0f;
  if (timed) (void)hipEventElapsedTime(&raw->kernel_ms, bf.ev_start, bf.ev_stop);
  raw->total_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_call).count();
  return PERM_OK;
}

// run_range_on with a leased workspace of the current device.
perm_status run_range(int kind, const void* dA, int n, int ld, uint64_t start, uint64_t count,
                      const perm_opts* opts, int range_check, bool full, hipStream_t s,
                      Raw* raw) {
  Lease lease;
  perm_status st = acquire_workspace(&lease.w);
  if (st != PERM_OK) return st;
  return run_range_on(lease.w->buf, kind, dA, n, ld, start, count, opts, range_check, full, s,
                      raw);
}

void fill_common(const Raw& raw, uint64_t count, perm_result* out) {
  out->max_drift = raw.r.drift;
  out->terms = count;
  out->chunks = raw.plan.body_chunks + raw.plan.head_count + raw.plan.tail_count;
  out->log2_chunk = raw.plan.log2_chunk;
  out->blocks = raw.blocks;
  out->kernel_ms = raw.kernel_ms;
  out->total_ms = raw.total_ms;
  // the banded walk needs chunks of at least 4 terms; with shorter ones the
  // pair-shared walk ran on the same staged layout
  out->walk_variant = (raw.r.variant == 2 && raw.plan.log2_chunk < 2) ? 1 : raw.r.variant;
  out->col0_nonzeros = raw.r.variant ? raw.r.ones0 : 0;
  out->parts = raw.parts;
}

perm_status status_from_device(int32_t st) {
  switch (st) {
    case kStOk: return PERM_OK;
    case kStNonFinite: return fail(PERM_ENONFINITE, "matrix has a NaN or infinite entry");
    case kStInval: return fail(PERM_EINVAL, "0/1 matrix has an entry other than 0 or 1");
    case kStRange:
      return fail(PERM_ERANGE, "exact 0/1 result may exceed 128 bits (Bregman bound >= 127)");
    default: return fail(PERM_EHIP, "unexpected device status");
  }
}

void pair_from_i128(__int128 v, double* hi, double* lo) {
  const double h = (double)v;
  *hi = h;
  if (std::fabs(h) >= 1.7014118346046923e38) {  // 2^127: no exact difference in 128 bits
    *lo = 0.0;
    return;
  }
  *lo = (double)(v - (__int128)h);
}

// Accurate double-double addition on the host (two TwoSums and two
// renormalisations, as the device reductions).  This file is compiled with
// -ffp-contract=off, so nothing is fused.
struct HostDD {
  double hi, lo;
};

HostDD host_dd_add(HostDD a, HostDD b) {
  double s = a.hi + b.hi;
  double bs = s - a.hi;
  double e = (a.hi - (s - bs)) + (b.hi - bs);
  double t = a.lo + b.lo;
  double bt = t - a.lo;
  double f = (a.lo - (t - bt)) + (b.lo - bt);
  e += t;
  double s2 = s + e;
  e = e - (s2 - s);
  e += f;
  double s3 = s2 + e;
  e = e - (s3 - s2);
  return HostDD{s3, e};
}

perm_status float_call(int kind, const double* dA, int n, int ld, const perm_opts* opts,
                       perm_result* out, void* stream) {
  if (!out) return fail(PERM_EINVAL, "out is NULL");
  if (n < 0 || n > kMaxN) return fail(PERM_EINVAL, "n must be in [0, 64]");
  if (ld < std::max(n, 1)) return fail(PERM_EINVAL, "ld must be >= n");
  perm_status st = check_opts(opts, 0);
  if (st != PERM_OK) return st;
  if (n == 0) {
    perm_result r{};
    r.re_hi = 1.0;
    r.max_drift = -1.0;
    *out = r;
    return PERM_OK;
  }
  if (!dA) return fail(PERM_EINVAL, "dA is NULL");
  const uint64_t T = total_terms(n);
  Raw raw;
  st = run_range(kind, dA, n, ld, 0, T, opts, 0, true, (hipStream_t)stream, &raw);
  if (st != PERM_OK) return st;
  st = status_from_device(raw.r.status);
  if (st != PERM_OK) return st;
  // per = 2 (-1)^n S, then undo the row scaling 2^(sum e_i).
  const double f = (n % 2 == 0) ? 2.0 : -2.0;
  const int e = -raw.r.exp_sum;
  perm_result r{};
  r.re_hi = std::ldexp(f * raw.r.v[0], e);
  r.re_lo = std::ldexp(f * raw.r.v[1], e);
  r.im_hi = std::ldexp(f * raw.r.v[2], e);
  r.im_lo = std::ldexp(f * raw.r.v[3], e);
  fill_common(raw, T, &r);
  *out = r;
  return PERM_OK;
}

perm_status partial_impl(const CallBuffers* bf, int dtype, const void* dA, int n, int ld,
                         uint64_t start, uint64_t count, const perm_opts* opts, perm_result* out,
                         void* stream) {
  if (!out) return fail(PERM_EINVAL, "out is NULL");
  if (dtype < 0 || dtype > 2) return fail(PERM_EINVAL, "dtype must be 0, 1 or 2");
  if (n < 1 || n > kMaxN) return fail(PERM_EINVAL, "n must be in [1, 64]");
  if (ld < n) return fail(PERM_EINVAL, "ld must be >= n");
  if (!dA) return fail(PERM_EINVAL, "dA is NULL");
  const int kind = dtype == PERM_DT_REAL ? kReal : (dtype == PERM_DT_COMPLEX ? kComplex : kInt01);
  perm_status st = check_opts(opts, kind == kInt01);
  if (st != PERM_OK) return st;
  if (bf && opts && opts->blocks > bf->max_parts / 3)
    return fail(PERM_EINVAL, "blocks exceeds the " + std::to_string(bf->max_parts / 3) +
                                 " workgroups the fixed device array holds partials for");
  const uint64_t T = total_terms(n);
  if (start > T || count > T - start) return fail(PERM_EINVAL, "range outside [0, 2^(n-1))");
  perm_result r{};
  r.max_drift = -1.0;
  if (count == 0) {
    *out = r;
    return PERM_OK;
  }
  Raw raw;
  st = bf ? run_range_on(*bf, kind, dA, n, ld, start, count, opts, 0, false, (hipStream_t)stream,
                         &raw)
          : run_range(kind, dA, n, ld, start, count, opts, 0, false, (hipStream_t)stream, &raw);
  if (st != PERM_OK) return st;
  st = status_from_device(raw.r.status);
  if (st != PERM_OK) return st;
  if (kind == kInt01) {
    r.int_lo = raw.r.iw[0];
    r.int_hi = (int64_t)raw.r.iw[1];
    const __int128 v = (__int128)(((unsigned __int128)raw.r.iw[1] << 64) | raw.r.iw[0]);
    pair_from_i128(v, &r.re_hi, &r.re_lo);
  } else {
    const int e = -raw.r.exp_sum;
    r.re_hi = std::ldexp(raw.r.v[0], e);
    r.re_lo = std::ldexp(raw.r.v[1], e);
    r.im_hi = std::ldexp(raw.r.v[2], e);
    r.im_lo = std::ldexp(raw.r.v[3], e);
  }
  fill_common(raw, count, &r);
  *out = r;
  return PERM_OK;
}

}  // namespace

extern "C" {

perm_status perm_plan(int n, uint64_t start, uint64_t count, int log2_chunk, int is_int01,
                      perm_plan_info* out) {
  if (!out) return fail(PERM_EINVAL, "out is NULL");
  if (n < 1 || n > kMaxN) return fail(PERM_EINVAL, "n must be in [1, 64]");
  const uint64_t T = total_terms(n);
  if (start > T || count > T - start) return fail(PERM_EINVAL, "range outside [0, 2^(n-1))");
  const int cap = is_int01 ? kInt01ChunkCap : kFloatChunkCap;
  if (log2_chunk < 0 || log2_chunk > cap) return fail(PERM_EINVAL, "log2_chunk out of range");
  int b = log2_chunk > 0 ? log2_chunk : auto_log2_chunk(count, is_int01 ? kInt01ChunkCap : 12);
  const uint64_t L = 1ull << b;
  const uint64_t end = start + count;
  uint64_t a0 = (start + L - 1) / L * L;
  if (a0 > end || a0 < start) a0 = end;
  const uint64_t a1 = a0 + (end - a0) / L * L;
  perm_plan_info p{};
  p.log2_chunk = b;
  p.head_start = start;
  p.head_count = a0 - start;
  p.body_first_chunk = a0 / L;
  p.body_chunks = (a1 - a0) / L;
  p.tail_start = a1;
  p.tail_count = end - a1;
  p.body_tasks = 2 * ((p.body_chunks + 2 * kWave - 1) / (2 * kWave));
  *out = p;
  return PERM_OK;
}

double perm_int01_bound(const int32_t* d, int n) {
  if (n <= 0) return 0.0;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    if (d[i] <= 0) return 0.0;
    double lf = 0.0;
    for (int k = 2; k <= d[i]; ++k) lf += std::log2((double)k);
    s += lf / d[i];
  }
  return (double)(n - 1) + s;
}

perm_status perm_real(const double* dA, int n, int ld, const perm_opts* opts, perm_result* out,
                      void* stream) {
  return float_call(kReal, dA, n, ld, opts, out, stream);
}

perm_status perm_complex(const double* dA, int n, int ld, const perm_opts* opts,
                         perm_result* out, void* stream) {
  return float_call(kComplex, dA, n, ld, opts, out, stream);
}

perm_status perm_int01(const uint8_t* dA, int n, int ld, const perm_opts* opts, perm_result* out,
                       void* stream) {
  if (!out) return fail(PERM_EINVAL, "out is NULL");
  if (n < 0 || n > kMaxN) return fail(PERM_EINVAL, "n must be in [0, 64]");
  if (ld < std::max(n, 1)) return fail(PERM_EINVAL, "ld must be >= n");
  perm_status st = check_opts(opts, 1);
  if (st != PERM_OK) return st;
  if (n == 0) {
    perm_result r{};
    r.re_hi = 1.0;
    r.int_lo = 1;
    r.max_drift = -1.0;
    *out = r;
    return PERM_OK;
  }
  if (!dA) return fail(PERM_EINVAL, "dA is NULL");
  const uint64_t T = total_terms(n);
  Raw raw;
  st = run_range(kInt01, dA, n, ld, 0, T, opts, 1, true, (hipStream_t)stream, &raw);
  if (st != PERM_OK) return st;
  st = status_from_device(raw.r.status);
  if (st != PERM_OK) return st;
  // S = (-1)^n 2^(n-1) per(A) modulo 2^128, with |S| < 2^127 by the guard.
  const unsigned __int128 u = ((unsigned __int128)raw.r.iw[1] << 64) | raw.r.iw[0];
  const __int128 S = (__int128)u;
  const unsigned __int128 low_mask = (((unsigned __int128)1) << (n - 1)) - 1;
  if ((u & low_mask) != 0)
    return fail(PERM_EHIP, "internal check failed: 0/1 sum not divisible by 2^(n-1)");
  __int128 per = S >> (n - 1);  // exact division (low bits are zero)
  if (n % 2) per = -per;
  perm_result r{};
  r.int_lo = (uint64_t)(unsigned __int128)per;
  r.int_hi = (int64_t)(per >> 64);
  pair_from_i128(per, &r.re_hi, &r.re_lo);
  fill_common(raw, T, &r);
  *out = r;
  return PERM_OK;
}

perm_status perm_partial(int dtype, const void* dA, int n, int ld, uint64_t start, uint64_t count,
                         const perm_opts* opts, perm_result* out, void* stream) {
  return partial_impl(nullptr, dtype, dA, n, ld, start, count, opts, out, stream);
}

perm_status perm_combine(int dtype, int n, const perm_result* parts, int count,
                         perm_result* out) {
  if (!out || !parts) return fail(PERM_EINVAL, "NULL argument");
  if (dtype < 0 || dtype > 2) return fail(PERM_EINVAL, "dtype must be 0, 1 or 2");
  if (n < 1 || n > kMaxN) return fail(PERM_EINVAL, "n must be in [1, 64]");
  if (count < 1) return fail(PERM_EINVAL, "count must be >= 1");
  const uint64_t T = total_terms(n);
  uint64_t terms = 0, chunks = 0;
  int64_t nparts = 0;
  double drift = -1.0;
  float kms = 0.0f, tms = 0.0f;
  for (int k = 0; k < count; ++k) {
    if (parts[k].terms > T - terms) return fail(PERM_EINVAL, "the parts hold more than 2^(n-1) terms");
    terms += parts[k].terms;
    chunks += parts[k].chunks;
    nparts += parts[k].parts;
    drift = std::max(drift, parts[k].max_drift);
    kms += parts[k].kernel_ms;
    tms += parts[k].total_ms;
  }
  if (terms != T) return fail(PERM_EINVAL, "the parts do not cover all 2^(n-1) terms");
  perm_result r{};
  r.terms = T;
  r.chunks = chunks;
  r.max_drift = drift;
  r.kernel_ms = kms;
  r.total_ms = tms;
  r.log2_chunk = parts[0].log2_chunk;
  r.blocks = parts[0].blocks;
  r.parts = (int32_t)std::min<int64_t>(nparts, INT32_MAX);
  if (dtype == PERM_DT_INT01) {
    // The parts hold sum (-1)^(g+1) prod_i r_i = (-1)^n 2^(n-1) per(A), mod 2^128.
    unsigned __int128 u = 0;
    for (int k = 0; k < count; ++k)
      u += ((unsigned __int128)(uint64_t)parts[k].int_hi << 64) | parts[k].int_lo;
    const unsigned __int128 low_mask = (((unsigned __int128)1) << (n - 1)) - 1;
    if ((u & low_mask) != 0)
      return fail(PERM_EINVAL, "the parts do not add up to a multiple of 2^(n-1)");
    __int128 per = ((__int128)u) >> (n - 1);
    if (n % 2) per = -per;
    r.int_lo = (uint64_t)(unsigned __int128)per;
    r.int_hi = (int64_t)(per >> 64);
    pair_from_i128(per, &r.re_hi, &r.re_lo);
  } else {
    HostDD re{0.0, 0.0}, im{0.0, 0.0};
    for (int k = 0; k < count; ++k) {
      re = host_dd_add(re, HostDD{parts[k].re_hi, parts[k].re_lo});
      im = host_dd_add(im, HostDD{parts[k].im_hi, parts[k].im_lo});
    }
    const double f = (n % 2 == 0) ? 2.0 : -2.0;  // per = 2 (-1)^n S
    r.re_hi = f * re.hi;
    r.re_lo = f * re.lo;
    r.im_hi = f * im.hi;
    r.im_lo = f * im.lo;
  }
  *out = r;
  return PERM_OK;
}

const char* perm_strerror(perm_status s) {
  switch (s) {
    case PERM_OK: return "success";
    case PERM_EINVAL: return "invalid argument";
    case PERM_ERANGE: return "exact result out of the 128-bit range";
    case PERM_ENONFINITE: return "non-finite matrix entry";
    case PERM_ENOMEM: return "out of memory";
    case PERM_EHIP: return "HIP runtime error";
    case PERM_ENOTIMPL: return "not implemented";
  }
  return "unknown status";
}

const char* perm_last_error(void) { return g_last_error.c_str(); }

const char* perm_version(void) { return "perm-mi355x 0.1 (gfx950)"; }

void perm_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (Workspace* w : g_all) {
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    destroy_workspace(w);
  }
  g_all.clear();
  g_idle.clear();
  perm::batched_release();
  perm::repeated_release();
  perm::band_release();
  (void)hipSetDevice(cur);
}

}  // extern "C"

namespace perm {
perm_status set_error(perm_status s, const char* msg) { return fail(s, msg); }

perm_status partial_on_buffers(const CallBuffers& bf, int dtype, const void* dA, int n, int ld,
                               uint64_t start, uint64_t count, const perm_opts* opts,
                               perm_result* out, void* stream) {
  return partial_impl(&bf, dtype, dA, n, ld, start, count, opts, out, stream);
}
}  // namespace perm
