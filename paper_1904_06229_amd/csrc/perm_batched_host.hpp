// Host-side helpers shared by the runtime files: release of the batched
// (perm_batched, perm_autotune) repeated-column (perm_repeated) and band (perm_band)
// workspaces, the thread-local error text, and perm_partial on caller-chosen
// device buffers.
#pragma once

#include "../../include/perm.h"
#include "perm_internal.hpp"

namespace perm {
void batched_release();
void repeated_release();
void band_release();
perm_status set_error(perm_status s, const char* msg);
// perm_partial with its stage / walk / finish buffers in `bf` (no workspace
// is leased; bf.max_parts / 3 caps the workgroups of each walk launch).
perm_status partial_on_buffers(const CallBuffers& bf, int dtype, const void* dA, int n, int ld,
                               uint64_t start, uint64_t count, const perm_opts* opts,
                               perm_result* out, void* stream);
}  // namespace perm
