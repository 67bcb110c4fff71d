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

// One group's arrays for the two passes of an assembly (device pointers).
typedef struct {
    const double *v, *vhat, *v_old;
    double *R_q, *R_v, *R_vhat, *entropy;
} mehdg_batch_slices;

// The residual pass (residual, entropy production, pointwise Jacobian
// coefficients) of ng <= 4 contexts of distinct degrees in one persistent
// launch over a queue of their macros in descending degree; counter is one
// device word of the caller's (reset by the launch).  Then, per context,
// mehdg_batch_ctx_rows completes the assembly (bordered rows, NaN outputs of
// flagged macros) as mehdg_assemble(want_blocks = 1) would.
mehdg_err mehdg_batch_ctx_residual(mehdg_ctx* const* ctxs, const mehdg_batch_slices* sl, int ng,
                                   unsigned long long* counter, mehdg_stream stream);
mehdg_err mehdg_batch_ctx_rows(mehdg_ctx* ctx, const mehdg_batch_slices* sl, mehdg_stream stream);
}
