// Host runtime and C ABI of the macro-element HDG local-work library.
//
// One translation unit: the kernel families are included as headers so that
// every kernel template is instantiated here for p = 1..3.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mehdg.h"
#include "common.hpp"
#include "k_residual.hpp"
#include "tables.hpp"

using namespace mehdg;

struct mehdg_ctx {
    int p = 0;
    int64_t n_macro = 0;
    mehdg_params prm{};
    DevParams dp{};
    Tab1D tab{};
    double* d_h = nullptr;          // [n_macro][3]
    Tab1D* d_tab = nullptr;
    int32_t* d_status = nullptr;    // [n_macro]
    double* d_scratch = nullptr;    // residual scratch
    int64_t bytes = 0;
    int stage = 0;                  // 0 nothing, 1 blocks assembled, 2 condensed
};

namespace {

constexpr int kMaxP = 3;

int64_t res_scratch_doubles(int p) {
    const int nq1 = 2 * (p + 1);
    return (int64_t)RES_FIELDS * nq1 * nq1 * nq1;
}

template <int P>
size_t res_lds() { return sizeof(ResLds<P>); }

mehdg_err hip_ok(hipError_t e) { return e == hipSuccess ? MEHDG_OK : MEHDG_EHIP; }

template <typename T>
mehdg_err dev_alloc(mehdg_ctx* c, T** ptr, int64_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return MEHDG_ENOMEM;
    }
    c->bytes += (int64_t)count * sizeof(T);
    *ptr = static_cast<T*>(p);
    return MEHDG_OK;
}

template <int P>
mehdg_err launch_residual(mehdg_ctx* c, const double* v, const double* vhat, const double* q,
                          const double* v_old, double* R_q, double* R_v, double* R_vhat, double* ent,
                          hipStream_t st) {
    const size_t lds = res_lds<P>();
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_residual<P>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return MEHDG_EHIP;
        attr = true;
    }
    hipLaunchKernelGGL(k_residual<P>, dim3((unsigned)c->n_macro), dim3(256), lds, st, v, vhat, q, v_old,
                       c->d_h, c->dp, c->d_tab, R_q, R_v, R_vhat, ent, c->d_scratch, c->d_status);
    return hip_ok(hipGetLastError());
}

}  // namespace

extern "C" {

mehdg_err mehdg_sizes(int32_t p, int64_t out[5]) {
    if (!out || p < 1 || p > 4) return MEHDG_EINVAL;
    const int64_t n1d = 2 * p + 1;
    out[0] = n1d * n1d * n1d;
    out[1] = n1d * n1d;
    out[2] = 5 * out[0];
    out[3] = 15 * out[0];
    out[4] = 30 * out[1];
    return MEHDG_OK;
}

mehdg_err mehdg_destroy(mehdg_ctx* c) {
    if (!c) return MEHDG_EINVAL;
    (void)hipFree(c->d_h);
    (void)hipFree(c->d_tab);
    (void)hipFree(c->d_status);
    (void)hipFree(c->d_scratch);
    delete c;
    return MEHDG_OK;
}

mehdg_err mehdg_create(const mehdg_mesh* mesh, const mehdg_params* prm, mehdg_ctx** out) {
    if (!out) return MEHDG_EINVAL;
    *out = nullptr;
    if (!mesh || !prm || !mesh->h || mesh->n_macro <= 0 || mesh->p < 1 || mesh->p > kMaxP)
        return MEHDG_EINVAL;
    if (!(prm->gamma > 1.0) || prm->flux < 0 || prm->flux > 2 || !(prm->logmean_eps >= 0.0))
        return MEHDG_EINVAL;
    if (mesh->n_macro > (int64_t)0x7fffffff) return MEHDG_EINVAL;
    for (int64_t i = 0; i < 3 * mesh->n_macro; ++i)
        if (!(mesh->h[i] > 0.0)) return MEHDG_EINVAL;
    mehdg_ctx* c = new (std::nothrow) mehdg_ctx();
    if (!c) return MEHDG_ENOMEM;
    c->p = mesh->p;
    c->n_macro = mesh->n_macro;
    c->prm = *prm;
    DevParams& d = c->dp;
    d.gamma = prm->gamma;
    d.mu = prm->viscous ? prm->mu : 0.0;
    d.kappa = prm->viscous ? prm->kappa : 0.0;
    d.lam = prm->lam;
    for (int k = 0; k < 5; ++k) d.sv[k] = prm->viscous ? prm->sigma_vis[k] : 0.0;
    d.alpha_t = prm->alpha_t;
    d.alpha_ps = prm->alpha_ps;
    d.eps = prm->logmean_eps;
    d.flux = prm->flux;
    d.viscous = prm->viscous ? 1 : 0;
    if (!build_tables(c->p, c->tab)) {
        delete c;
        return MEHDG_EINVAL;
    }
    mehdg_err e;
    if ((e = dev_alloc(c, &c->d_h, 3 * c->n_macro)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_tab, 1)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_status, c->n_macro)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_scratch, c->n_macro * res_scratch_doubles(c->p))) != MEHDG_OK) {
        mehdg_destroy(c);
        return e;
    }
    if (hipMemcpy(c->d_h, mesh->h, 3 * c->n_macro * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_tab, &c->tab, sizeof(Tab1D), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->d_status, 0, c->n_macro * sizeof(int32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        mehdg_destroy(c);
        return MEHDG_EHIP;
    }
    *out = c;
    return MEHDG_OK;
}

mehdg_err mehdg_assemble(mehdg_ctx* c, const double* v, const double* vhat, const double* q,
                         const double* v_old, double* R_q, double* R_v, double* R_vhat, double* entropy,
                         int32_t want_blocks, mehdg_stream stream) {
    if (!c || !v || !vhat || !v_old || !R_q || !R_v || !R_vhat || !entropy) return MEHDG_EINVAL;
    if (want_blocks) return MEHDG_EINVAL;   // block assembly not yet available
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_residual<1>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, st); break;
        case 2: e = launch_residual<2>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, st); break;
        case 3: e = launch_residual<3>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, st); break;
        default: break;
    }
    return e;
}

mehdg_err mehdg_condense(mehdg_ctx* c, double* Ahat, double* bhat, mehdg_stream stream) {
    (void)Ahat;
    (void)stream;
    if (!c || !bhat) return MEHDG_EINVAL;
    if (c->stage < 1) return MEHDG_ESTATE;
    return MEHDG_EINVAL;
}

mehdg_err mehdg_recover(mehdg_ctx* c, const double* R_q, const double* dvhat, double* dv, double* dq,
                        mehdg_stream stream) {
    (void)stream;
    if (!c || !R_q || !dvhat || !dv || !dq) return MEHDG_EINVAL;
    if (c->stage < 2) return MEHDG_ESTATE;
    return MEHDG_EINVAL;
}

mehdg_err mehdg_status(mehdg_ctx* c, int32_t* status, mehdg_stream stream) {
    if (!c || !status) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(status, c->d_status, c->n_macro * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    if (hipMemsetAsync(c->d_status, 0, c->n_macro * sizeof(int32_t), st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    for (int64_t i = 0; i < c->n_macro; ++i)
        if (status[i] != 0) return static_cast<mehdg_err>(status[i]);
    return MEHDG_OK;
}

int64_t mehdg_workspace_bytes(const mehdg_ctx* c) { return c ? c->bytes : 0; }

}  // extern "C"
