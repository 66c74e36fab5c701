// perm_partial_noalloc: perm_partial on a fixed device array instead of
// library-allocated workspace, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The array `scratch` holds the buffers of one call (staging status, row
// exponents, the staged +A/-A copy, per-workgroup partial sums, the result
// record) for at most kNoAllocMaxBlocks workgroups per walk launch.  Every
// device the library runs on holds its own copy until the process ends.  In
// host code the name `scratch` is only a stand-in for the device variable, so
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is handed to the kernels and
// copies.  All calls on one device share the array: calls that overlap on
// one device race and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/perm.h"
#include "perm_batched_host.hpp"
#include "perm_internal.hpp"

namespace {

constexpr int kNoAllocMaxBlocks = PERM_NOALLOC_MAX_BLOCKS;  // workgroups per walk launch
constexpr int kNoAllocMaxParts = 3 * kNoAllocMaxBlocks;        // head, body and tail launches
constexpr size_t kScratchBytes = perm::call_buffer_bytes(kNoAllocMaxParts);
constexpr int kMaxDevices = 64;

static_assert(kScratchBytes <= 512 * 1024, "the fixed device array is meant to stay small");

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device
int g_cus[kMaxDevices] = {};

// Device address and CU count of the current device, looked up on the first
// call on that device.
perm_status scratch_of_current(char** ptr, int* cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return perm::set_error(PERM_EHIP, (std::string("hipGetDevice failed: ") +
                                       hipGetErrorString(e)).c_str());
  if (dev < 0 || dev >= kMaxDevices)
    return perm::set_error(PERM_EINVAL, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return perm::set_error(PERM_EHIP, (std::string("hipGetSymbolAddress(scratch) failed: ") +
                                         hipGetErrorString(e)).c_str());
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0)
      cu = 256;
    g_cus[dev] = cu;
    g_ptr[dev] = (char*)p;
  }
  *ptr = g_ptr[dev];
  *cus = g_cus[dev];
  return PERM_OK;
}

}  // namespace

extern "C" perm_status perm_partial_noalloc(int dtype, const void* dA, int n, int ld,
                                            uint64_t start, uint64_t count,
                                            const perm_opts* opts, perm_result* out,
                                            void* stream) {
  if (opts && opts->blocks > kNoAllocMaxBlocks)
    return perm::set_error(PERM_EINVAL, ("blocks exceeds the no-allocation limit of " +
                                         std::to_string(kNoAllocMaxBlocks)).c_str());
  char* base = nullptr;
  int cus = 0;
  perm_status st = scratch_of_current(&base, &cus);
  if (st != PERM_OK) return st;
  perm::CallBuffers bf;
  perm::carve_call_buffers(base, kNoAllocMaxParts, &bf);
  bf.cu_count = cus;  // no pinned record and no events: nothing is allocated
  return perm::partial_on_buffers(bf, dtype, dA, n, ld, start, count, opts, out, stream);
}
