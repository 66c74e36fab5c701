// C-ABI entry point perm_band: permanents of band matrices by the transfer
// matrix of App. C, one wavefront per matrix.  The sizes and offsets are
// copied to a library-owned device array through pinned memory; the call
// waits for its stream before returning, so the caller's host arrays and the
// staging memory are free again on return.
#include <hip/hip_runtime.h>

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

constexpr int kBandMaxN = 65536;

struct BandWorkspace {
  int device = -1;
  int cu_count = 256;
  size_t cap = 0;           // matrices the buffers hold
  char* dmem = nullptr;     // n (int32) then offsets (int64)
  char* hmem = nullptr;     // pinned staging, same layout
  int blocks_per_cu[2][kBandMaxK + 1] = {};  // occupancy by (complex, k); 0 = not queried
  std::mutex call_mu;       // held for a whole call: calls on one device take turns
};

std::mutex g_mu;
std::map<int, BandWorkspace*> g_ws;

perm_status hip_fail(const char* what, hipError_t e) {
  return set_error(PERM_EHIP, (std::string(what) + " failed: " + hipGetErrorString(e)).c_str());
}

size_t layout_bytes(size_t cap, size_t* o_off) {
  *o_off = (cap * sizeof(int32_t) + 255) / 256 * 256;
  return *o_off + cap * sizeof(int64_t);
}

perm_status get_ws(BandWorkspace** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail("hipGetDevice", e);
  std::lock_guard<std::mutex> lk(g_mu);
  BandWorkspace*& w = g_ws[dev];
  if (!w) {
    w = new BandWorkspace();
    w->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      w->cu_count = prop.multiProcessorCount;
  }
  *out = w;
  return PERM_OK;
}

// Grows the size/offset buffers to hold `count` matrices.  Called with the
// workspace's call lock held, after the previous call's stream has drained.
perm_status ensure_cap(BandWorkspace* w, size_t count) {
  if (w->cap >= count) return PERM_OK;
  size_t cap = 1024;
  while (cap < count) cap *= 2;
  size_t o_off;
  const size_t bytes = layout_bytes(cap, &o_off);
  char* d = nullptr;
  char* h = nullptr;
  if (hipMalloc((void**)&d, bytes) != hipSuccess)
    return set_error(PERM_ENOMEM, "hipMalloc of the band workspace failed");
  if (hipHostMalloc((void**)&h, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(d);
    return set_error(PERM_ENOMEM, "hipHostMalloc of the band staging failed");
  }
  if (w->dmem) (void)hipFree(w->dmem);
  if (w->hmem) (void)hipHostFree(w->hmem);
  w->dmem = d;
  w->hmem = h;
  w->cap = cap;
  return PERM_OK;
}

// Holds a device's workspace for the length of one call; on the way out
// (also after an error) the stream is drained before the next call enters.
struct CallGuard {
  std::unique_lock<std::mutex> lk;
  hipStream_t s;
  CallGuard(BandWorkspace* w, hipStream_t st) : lk(w->call_mu), s(st) {}
  ~CallGuard() { (void)hipStreamSynchronize(s); }
};

}  // namespace

namespace perm {
void band_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_ws) {
    BandWorkspace* w = kv.second;
    if (!w) continue;
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    if (w->dmem) (void)hipFree(w->dmem);
    if (w->hmem) (void)hipHostFree(w->hmem);
    delete w;
  }
  g_ws.clear();
  (void)hipSetDevice(cur);
}
}  // namespace perm

extern "C" perm_status perm_band(int dtype, const double* dA, const int32_t* h_n,
                                 const int64_t* h_offset, int count, int k,
                                 const perm_opts* opts, double* d_out, int32_t* d_status,
                                 void* stream) {
  if (dtype != PERM_DT_REAL && dtype != PERM_DT_COMPLEX)
    return set_error(PERM_EINVAL, "dtype must be PERM_DT_REAL or PERM_DT_COMPLEX");
  if (count < 0) return set_error(PERM_EINVAL, "count must be >= 0");
  if (k < 0 || k > kBandMaxK) return set_error(PERM_EINVAL, "k must be in [0, 5]");
  if (count == 0) return PERM_OK;
  if (!dA || !h_n || !h_offset || !d_out) return set_error(PERM_EINVAL, "NULL argument");
  perm_opts o{};
  if (opts) o = *opts;
  if (o.precision != PERM_FP64_DD || o.log2_chunk || o.drift_check || o.use_graph)
    return set_error(PERM_ENOTIMPL, "perm_band takes only the blocks option");
  if (o.blocks < 0 || o.blocks > 65536) return set_error(PERM_EINVAL, "blocks out of range");
  if (o.reserved) return set_error(PERM_EINVAL, "reserved options must be 0");
  if (o.partials_out) return set_error(PERM_ENOTIMPL, "partials_out is not provided here");
  for (int m = 0; m < count; ++m) {
    if (h_n[m] < 1 || h_n[m] > kBandMaxN) return set_error(PERM_EINVAL, "n must be in [1, 65536]");
    if (h_offset[m] < 0) return set_error(PERM_EINVAL, "offsets must be >= 0");
  }
  BandWorkspace* ws = nullptr;
  perm_status st = get_ws(&ws);
  if (st != PERM_OK) return st;
  CallGuard guard(ws, (hipStream_t)stream);
  if ((st = ensure_cap(ws, (size_t)count)) != PERM_OK) return st;
  size_t o_off;
  const size_t bytes = layout_bytes(ws->cap, &o_off);
  std::memcpy(ws->hmem, h_n, sizeof(int32_t) * count);
  std::memcpy(ws->hmem + o_off, h_offset, sizeof(int64_t) * count);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(ws->dmem, ws->hmem, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail("hipMemcpyAsync of the band plan", e);
  BandArgs a;
  a.A = dA;
  a.n = (const int32_t*)ws->dmem;
  a.off = (const int64_t*)(ws->dmem + o_off);
  a.count = count;
  a.pad = 0;
  a.out = d_out;
  a.status = d_status;
  int& per_cu = ws->blocks_per_cu[dtype == PERM_DT_COMPLEX ? 1 : 0][k];
  if (per_cu == 0) per_cu = band_blocks_per_cu(dtype == PERM_DT_COMPLEX, k);
  int grid = o.blocks > 0 ? o.blocks : per_cu * ws->cu_count;
  const int need = (int)((count + kWavesPerBlock - 1) / kWavesPerBlock);  // a wave per matrix
  if (grid > need) grid = need;
  e = launch_band(dtype == PERM_DT_COMPLEX, k, a, grid, s);
  if (e != hipSuccess) return hip_fail("band launch", e);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail("hipStreamSynchronize", e);
  return PERM_OK;
}
