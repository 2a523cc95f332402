// Helpers shared by the translation units of the library (not exported).
#pragma once

#include "../../include/pbcgs.h"

#define PBCGS_HIDDEN __attribute__((visibility("hidden")))

// The HIP stream a context works on.
PBCGS_HIDDEN void* pbcgs_internal_stream(pbcgs_ctx_t ctx);
// Record an error message on ctx (or globally) and return code.
PBCGS_HIDDEN int pbcgs_internal_fail(pbcgs_ctx_t ctx, int code, const char* msg);
