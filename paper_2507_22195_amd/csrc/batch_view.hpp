// Internal to the library: what the batch calls (mehdg_batch.hip) need of a
// context beyond the public API.
#pragma once
#include <cstdint>

#include "../../include/mehdg.h"

extern "C" {
// The context works on the first n (<= the n_macro it was created with) of its
// macros, reading mesh sizes d_h [n][3], wall flags d_bc [n][6] (or NULL) and
// writing status codes d_status [n] in the caller's device arrays, until the
// next view or mehdg_batch_ctx_unview.  Host call, no device work.
mehdg_err mehdg_batch_ctx_view(mehdg_ctx* ctx, int64_t n, const double* d_h, const uint8_t* d_bc,
                               int32_t* d_status);
mehdg_err mehdg_batch_ctx_unview(mehdg_ctx* ctx);
// Device bytes per macro a context of degree p holds after an FP64 step.
int64_t mehdg_batch_ctx_bytes(int p);
}
