// Host side of the batched path (perm_batched, perm_autotune).
#pragma once

#include "../../include/perm.h"

namespace perm {
void batched_release();
perm_status set_error(perm_status s, const char* msg);
}  // namespace perm
