// Persistent residual pass of a batch of macro-elements of mixed degree:
// one launch whose workgroups take macros from a device queue (descending
// degree) and run the residual body of each macro's degree (residual_macro
// of k_residual.hpp, the code of the per-degree kernel).
#pragma once
#include "k_residual.hpp"

namespace mehdg {

// One degree group of a batch for the persistent residual pass.
struct ResidualGroup {
    int p;
    DevParams pr;
    const double *v, *vhat, *v_old, *hs;
    const Tab1D* tab;
    double *R_q, *R_v, *R_vh, *ent, *scratch, *coefV, *coefF;
    const uint8_t* bc;
    int32_t* status;
};

// The groups in the order of the work queue (descending degree: the longest
// items first); queue positions [first[i], first[i+1]) are group i's macros.
struct ResidualBatch {
    ResidualGroup g[4];
    int64_t first[5];
    int ng;
};

__global__ void k_reset_counter(unsigned long long* counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0ull;
}

// The residual and pointwise Jacobian coefficients of every macro of a batch
// of mixed degree in one persistent launch: each workgroup takes the next
// queue position from the device counter until the queue is empty (every
// workgroup then returns), and runs the body of its macro's degree.
__global__ void __launch_bounds__(256) k_residual_batch(ResidualBatch b, unsigned long long* counter) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ long long item;
    const int64_t total = b.first[b.ng];
    while (true) {
        if (threadIdx.x == 0) item = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t it = item;
        __syncthreads();                 // all have read it before thread 0 takes the next
        if (it >= total) return;
        int gi = 0;
        while (gi + 1 < b.ng && it >= b.first[gi + 1]) ++gi;
        const ResidualGroup& g = b.g[gi];
        const int64_t m = it - b.first[gi];
        switch (g.p) {
#define MEHDG_BATCH_RESIDUAL(PP)                                                                                  \
    case PP:                                                                                                      \
        residual_macro<PP, true>(m, smem_raw, g.v, g.vhat, nullptr, g.v_old, g.hs, g.pr, g.tab, g.R_q, g.R_v,      \
                                 g.R_vh, g.ent, g.scratch, g.coefV, g.coefF, g.bc, g.status);                      \
        break;
            MEHDG_BATCH_RESIDUAL(1)
            MEHDG_BATCH_RESIDUAL(2)
            MEHDG_BATCH_RESIDUAL(3)
            MEHDG_BATCH_RESIDUAL(4)
#undef MEHDG_BATCH_RESIDUAL
            default: break;
        }
        __syncthreads();                 // the LDS is reused by the next macro
    }
}

}  // namespace mehdg
