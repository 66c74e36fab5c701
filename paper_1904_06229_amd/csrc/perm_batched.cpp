// Batched permanents: placeholder until the persistent kernel lands.
#include "perm_batched_host.hpp"

namespace perm {
void batched_release() {}
}  // namespace perm

extern "C" {
perm_status perm_batched(const double*, const int32_t*, const int64_t*, int, int,
                         const perm_opts*, double*, int32_t*, void*) {
  return perm::set_error(PERM_ENOTIMPL, "perm_batched not built yet");
}
perm_status perm_autotune(int, int, int, const char*, void*) {
  return perm::set_error(PERM_ENOTIMPL, "perm_autotune not built yet");
}
}
