// Internal interface between the two translation units of the library: the
// dense condensation kernels (blocked pivoted LU of S, the X rows, the Schur
// product) applied to bordered matrices [[S, -Y, r_V], [X, A', r_hat]] with
// the sizes of a tetrahedral macro-element of degree p (NV = 5n, NH = 20 nf).
// Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/mehdg.h"

struct TetCondWork {
    double* B;          // [n_macro][rows][ld] bordered matrices, factored in place
    int32_t* ipiv;      // [n_macro][NV]
    double* tri;        // [n_macro][tri] triangular inverses of the blocked LU
    int32_t* perm;      // [n_macro][perm] composed interchanges of the current block
    int32_t* status;    // [n_macro] status codes (zero pivot: ESINGULAR)
    int64_t n_macro;
};

// Per-macro sizes at degree p: out = {rows, ld, tri doubles, perm ints}.
bool tet_cond_sizes(int p, int64_t out[4]);

// Factors every macro's bordered matrix and writes Ahat = A' + X S^-1 Y,
// bhat = r_hat - X S^-1 r_V (eq. R5a-b); flagged macros get NaN in Ahat, bhat.
mehdg_err tet_condense(int p, const TetCondWork& w, double* Ahat, double* bhat, hipStream_t st);

// The stored factors applied to a new right-hand side (eq. R4, R5b): bhat =
// r_hat - X S^-1 r_V (r_hat NULL: zero), and the right-hand-side column of
// the factored bordered matrices replaced so that the next recovery gives
// dV = S^-1 (r_V + Y dVhat).
mehdg_err tet_condense_rhs(int p, const TetCondWork& w, const double* r_v, const double* r_hat, double* bhat,
                           hipStream_t st);

// Overwrites with NaN the outputs a[per_a], b[per_b] (either may be NULL) of
// every macro whose status code is set: the error contract of the compute
// calls (a flagged macro's outputs are NaN).
mehdg_err poison_flagged(const int32_t* status, int64_t n_macro, double* a, int64_t per_a, double* b,
                         int64_t per_b, hipStream_t st);
