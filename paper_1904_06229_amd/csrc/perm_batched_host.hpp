// Host-side helpers shared by the runtime files: release of the batched
// (perm_batched, perm_autotune) repeated-column (perm_repeated) and band (perm_band)
// workspaces,
// and the thread-local error text.
#pragma once

#include "../../include/perm.h"

namespace perm {
void batched_release();
void repeated_release();
void band_release();
perm_status set_error(perm_status s, const char* msg);
}  // namespace perm
