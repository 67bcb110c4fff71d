// Host runtime and C ABI of tetrahedral macro-elements (mehdg_tet_*): the
// residual, its JVP, and the local work of a Newton step (assembly of the
// bordered matrices from columns of the reduced Jacobian, the dense
// condensation shared with the hexahedral path through tet_cond.hpp, and the
// recovery).  A separate translation unit of the same library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mehdg.h"
#include "k_recover.hpp"
#include "k_tet.hpp"
#include "tet_cond.hpp"
#include "tet_tables.hpp"

using namespace mehdg;

struct mehdg_tet_ctx {
    int p = 0;
    int64_t n_macro = 0;
    DevParams dp{};
    TetTab tab;
    TetDevTab dt{};
    double* d_tab = nullptr;       // all double tables
    int* d_itab = nullptr;         // all int tables
    double* d_geo = nullptr;       // [n_macro][TET_GEO]
    uint8_t* d_bc = nullptr;       // [n_macro][4] or nullptr
    int32_t* d_status = nullptr;   // [n_macro]
    // local work of a Newton step (allocated by the first mehdg_tet_assemble)
    double* d_B = nullptr;         // [n_macro][rows][ld] bordered matrices
    int32_t* d_ipiv = nullptr;     // [n_macro][N_V]
    double* d_tri = nullptr;       // [n_macro][tri]
    int32_t* d_perm = nullptr;     // [n_macro][perm]
    double* d_coef = nullptr;      // pointwise Jacobian coefficients [n_macro][G][TET_CV] then [n_macro][FP][TET_CF]
    double* d_ctab = nullptr;      // weak-gradient tables of the columns
    int* d_citab = nullptr;        // local-index maps of the columns
    TetColTab ct{};
    int64_t rows = 0, ld = 0, per_tri = 0, per_perm = 0;
    int stage = 0;                 // 0 nothing, 1 assembled, 2 condensed
};

namespace {

template <int P, bool LIN>
size_t tet_lds() { return sizeof(TetLds<P, LIN>); }

template <bool LIN>
size_t tet_lds_bytes(int p) { return p == 1 ? tet_lds<1, LIN>() : p == 2 ? tet_lds<2, LIN>() : tet_lds<3, LIN>(); }

template <int P>
bool tet_allow_lds() {
    auto set = [](const void* k, size_t b) {
        return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b) == hipSuccess;
    };
    return set(reinterpret_cast<const void*>(&k_tet<P, 0>), tet_lds<P, false>()) &&
           set(reinterpret_cast<const void*>(&k_tet<P, 1>), tet_lds<P, true>()) &&
           set(reinterpret_cast<const void*>(&k_tet<P, 2>), sizeof(TetColLds<P>)) &&
           set(reinterpret_cast<const void*>(&k_tet_coef<P>), tet_lds<P, false>()) &&
           set(reinterpret_cast<const void*>(&k_tet_recover<P>), sizeof(TetRecLds<P>));
}

// g = J_r^T w from the assembled bordered matrices (before the condensation
// overwrites them): g[j] = sum_i B[i][j] w[i] over the rows i < NV + NH; one
// workgroup per macro, lanes along the columns (coalesced row reads).
__global__ void __launch_bounds__(256) k_tet_vjp_b(const double* __restrict__ B, const double* __restrict__ w_v,
                                                   const double* __restrict__ w_h, int NV, int NH, int ld,
                                                   int64_t per_macro, double* __restrict__ g_v,
                                                   double* __restrict__ g_h) {
    const int64_t m = blockIdx.x;
    const int rows = NV + NH;
    const double* Bm = B + m * per_macro;
    for (int j0 = 0; j0 < rows; j0 += 4 * blockDim.x) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < rows; ++i) {
            const double wi = i < NV ? w_v[m * NV + i] : w_h[m * NH + i - NV];
            const double* row = Bm + (int64_t)i * ld;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * blockDim.x + threadIdx.x;
                if (j < rows) acc[u] += row[j] * wi;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = j0 + u * blockDim.x + threadIdx.x;
            if (j < NV) g_v[m * NV + j] = acc[u];
            else if (j < rows) g_h[m * NH + j - NV] = acc[u];
        }
    }
}

// doubles of the pointwise coefficients per macro (volume part, total)
int64_t tet_coef_volume(int p) { return (int64_t)8 * (p + 1) * (p + 1) * (p + 1) * TET_CV; }
int64_t tet_coef_doubles(int p) { return tet_coef_volume(p) + (int64_t)16 * (p + 1) * (p + 1) * TET_CF; }

// -B[:, NV + NH] = R: the right-hand-side column of the bordered matrices.
__global__ void __launch_bounds__(256) k_tet_rhs(const double* __restrict__ R_v, const double* __restrict__ R_vh,
                                                 int NV, int NH, int ld, int64_t per_macro, double* __restrict__ B) {
    const int64_t m = blockIdx.x;
    for (int i = threadIdx.x; i < NV + NH; i += blockDim.x) {
        const double r = i < NV ? R_v[m * NV + i] : R_vh[m * NH + i - NV];
        B[m * per_macro + (int64_t)i * ld + NV + NH] = -r;
    }
}

// J^-1, |det J|, outward normals and twice the areas of one macro; false if degenerate.
bool tet_geometry(const double* X, double* out) {
    double J[3][3];
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) J[d][e] = X[(e + 1) * 3 + d] - X[d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!std::isfinite(det) || std::fabs(det) < 1e-300) return false;
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[i * 3 + j] = inv[i][j];
    out[9] = std::fabs(det);
    const int FV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (int f = 0; f < 4; ++f) {
        const double* P0 = X + 3 * FV[f][0];
        const double* P1 = X + 3 * FV[f][1];
        const double* P2 = X + 3 * FV[f][2];
        const double* Pf = X + 3 * f;
        double e1[3], e2[3], c[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = P1[d] - P0[d];
            e2[d] = P2[d] - P0[d];
        }
        c[0] = e1[1] * e2[2] - e1[2] * e2[1];
        c[1] = e1[2] * e2[0] - e1[0] * e2[2];
        c[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double a = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(a > 0.0)) return false;
        const double out_dir = c[0] * (P0[0] - Pf[0]) + c[1] * (P0[1] - Pf[1]) + c[2] * (P0[2] - Pf[2]);
        const double sgn = out_dir > 0.0 ? 1.0 : -1.0;
        for (int d = 0; d < 3; ++d) out[10 + 3 * f + d] = sgn * c[d] / a;
        out[22 + f] = a;
    }
    for (int i = 26; i < TET_GEO; ++i) out[i] = 0.0;
    return true;
}

template <typename T>
bool upload(const std::vector<std::vector<T>*>& parts, T** dev, std::vector<const T*>& ptrs) {
    size_t total = 0;
    for (auto* v : parts) total += v->size();
    std::vector<T> host;
    host.reserve(total);
    for (auto* v : parts) host.insert(host.end(), v->begin(), v->end());
    void* d = nullptr;
    if (hipMalloc(&d, total * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (hipMemcpy(d, host.data(), total * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return false;
    }
    *dev = static_cast<T*>(d);
    size_t off = 0;
    for (auto* v : parts) {
        ptrs.push_back(*dev + off);
        off += v->size();
    }
    return true;
}

}  // namespace

extern "C" {

mehdg_err mehdg_tet_sizes(int32_t p, int64_t out[5]) {
    if (!out || p < 1 || p > 3) return MEHDG_EINVAL;
    const int64_t m = 2 * p;
    out[0] = (m + 1) * (m + 2) * (m + 3) / 6;
    out[1] = (m + 1) * (m + 2) / 2;
    out[2] = 5 * out[0];
    out[3] = 15 * out[0];
    out[4] = 20 * out[1];
    return MEHDG_OK;
}

mehdg_err mehdg_tet_destroy(mehdg_tet_ctx* c) {
    if (!c) return MEHDG_EINVAL;
    (void)hipFree(c->d_tab);
    (void)hipFree(c->d_itab);
    (void)hipFree(c->d_geo);
    (void)hipFree(c->d_bc);
    (void)hipFree(c->d_status);
    (void)hipFree(c->d_B);
    (void)hipFree(c->d_ipiv);
    (void)hipFree(c->d_tri);
    (void)hipFree(c->d_perm);
    (void)hipFree(c->d_coef);
    (void)hipFree(c->d_ctab);
    (void)hipFree(c->d_citab);
    delete c;
    return MEHDG_OK;
}

mehdg_err mehdg_tet_create(const mehdg_tet_mesh* mesh, const mehdg_params* prm, mehdg_tet_ctx** out) {
    if (!out) return MEHDG_EINVAL;
    *out = nullptr;
    if (!mesh || !prm || !mesh->X || mesh->n_macro <= 0 || mesh->n_macro > (int64_t)0x7fffffff ||
        mesh->p < 1 || mesh->p > 3)
        return MEHDG_EINVAL;
    if (!(prm->gamma > 1.0) || prm->flux < 0 || prm->flux > 2 || !(prm->logmean_eps >= 0.0)) return MEHDG_EINVAL;
    bool walls = false;
    if (mesh->face_bc) {
        for (int64_t i = 0; i < 4 * mesh->n_macro; ++i) {
            if (mesh->face_bc[i] > 1) return MEHDG_EINVAL;
            walls = walls || mesh->face_bc[i] == 1;
        }
        if (walls && !(prm->T_wall > 0.0)) return MEHDG_EINVAL;
    }
    std::vector<double> geo((size_t)mesh->n_macro * TET_GEO);
    for (int64_t m = 0; m < mesh->n_macro; ++m)
        if (!tet_geometry(mesh->X + 12 * m, geo.data() + m * TET_GEO)) return MEHDG_EINVAL;
    mehdg_tet_ctx* c = new (std::nothrow) mehdg_tet_ctx();
    if (!c) return MEHDG_ENOMEM;
    c->p = mesh->p;
    c->n_macro = mesh->n_macro;
    DevParams& d = c->dp;
    d.gamma = prm->gamma;
    d.mu = prm->viscous ? prm->mu : 0.0;
    d.kappa = prm->viscous ? prm->kappa : 0.0;
    d.lam = prm->lam;
    for (int k = 0; k < 5; ++k) d.sv[k] = prm->viscous ? prm->sigma_vis[k] : 0.0;
    d.alpha_t = prm->alpha_t;
    d.alpha_ps = prm->alpha_ps;
    d.eps = prm->logmean_eps;
    d.gT = walls ? prm->gamma / prm->T_wall : 0.0;
    d.flux = prm->flux;
    d.viscous = prm->viscous ? 1 : 0;
    if (!build_tet_tables(c->p, c->tab)) {
        delete c;
        return MEHDG_EINVAL;
    }
    TetTab& t = c->tab;
    std::vector<const double*> dp;
    std::vector<const int*> ip;
    if (!upload<double>({&t.phi, &t.dphi, &t.wv, &t.BiT, &t.psi, &t.wf, &t.Mt, &t.CT, &t.ChT, &t.DT, &t.DhT, &t.Mi},
                        &c->d_tab, dp) ||
        !upload<int>({&t.vnode, &t.fnode, &t.tnode, &t.vptr, &t.vinc, &t.fptr, &t.finc}, &c->d_itab, ip)) {
        mehdg_tet_destroy(c);
        return MEHDG_ENOMEM;
    }
    c->dt = TetDevTab{dp[0], dp[1], dp[2], dp[3], dp[4], dp[5], dp[6], dp[7], dp[8], dp[9], dp[10], dp[11],
                      ip[0], ip[1], ip[2], ip[3], ip[4], ip[5], ip[6]};
    std::vector<const double*> cdp;
    std::vector<const int*> cip;
    if (!upload<double>({&t.ED, &t.EDf, &t.EH, &t.EHf}, &c->d_ctab, cdp) ||
        !upload<int>({&t.vloc, &t.tloc, &t.fidx}, &c->d_citab, cip)) {
        mehdg_tet_destroy(c);
        return MEHDG_ENOMEM;
    }
    c->ct.ED = cdp[0];
    c->ct.EDf = cdp[1];
    c->ct.EH = cdp[2];
    c->ct.EHf = cdp[3];
    c->ct.vloc = cip[0];
    c->ct.tloc = cip[1];
    c->ct.fidx = cip[2];
    const size_t gbytes = geo.size() * sizeof(double);
    if (hipMalloc(&c->d_geo, gbytes) != hipSuccess ||
        hipMemcpy(c->d_geo, geo.data(), gbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&c->d_status, c->n_macro * sizeof(int32_t)) != hipSuccess ||
        hipMemset(c->d_status, 0, c->n_macro * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        mehdg_tet_destroy(c);
        return MEHDG_ENOMEM;
    }
    if (walls && (hipMalloc(&c->d_bc, 4 * c->n_macro) != hipSuccess ||
                  hipMemcpy(c->d_bc, mesh->face_bc, 4 * c->n_macro, hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipGetLastError();
        mehdg_tet_destroy(c);
        return MEHDG_ENOMEM;
    }
    const bool lds_ok = c->p == 1 ? tet_allow_lds<1>() : c->p == 2 ? tet_allow_lds<2>() : tet_allow_lds<3>();
    if (!lds_ok) {
        mehdg_tet_destroy(c);
        return MEHDG_EHIP;
    }
    *out = c;
    return MEHDG_OK;
}

mehdg_err mehdg_tet_residual(mehdg_tet_ctx* c, const double* v, const double* vhat, const double* q,
                             const double* v_old, double* R_q, double* R_v, double* R_vhat, double* entropy,
                             mehdg_stream stream) {
    if (!c || !v || !vhat || !v_old || !R_q || !R_v || !R_vhat || !entropy) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)c->n_macro), block(TET_THREADS);
    const size_t lds = tet_lds_bytes<false>(c->p);
#define MEHDG_TET_LAUNCH(PP)                                                                                   \
    hipLaunchKernelGGL((k_tet<PP, 0>), grid, block, lds, st, v, vhat, q, v_old, nullptr, nullptr, nullptr, c->d_geo, \
                       c->dt, c->dp, c->d_bc, R_q, R_v, R_vhat, entropy, c->d_status, nullptr, 0, (int64_t)0, TetColTab{})
    if (c->p == 1)
        MEHDG_TET_LAUNCH(1);
    else if (c->p == 2)
        MEHDG_TET_LAUNCH(2);
    else
        MEHDG_TET_LAUNCH(3);
#undef MEHDG_TET_LAUNCH
    return hipGetLastError() == hipSuccess ? MEHDG_OK : MEHDG_EHIP;
}

mehdg_err mehdg_tet_jvp(mehdg_tet_ctx* c, const double* v, const double* vhat, const double* q, const double* dv,
                        const double* dvhat, const double* dq, double* JR_q, double* JR_v, double* JR_vhat,
                        mehdg_stream stream) {
    if (!c || !v || !vhat || !dv || !dvhat || !JR_q || !JR_v || !JR_vhat) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)c->n_macro), block(TET_THREADS);
    const size_t lds = tet_lds_bytes<true>(c->p);
#define MEHDG_TET_LAUNCH(PP)                                                                                  \
    hipLaunchKernelGGL((k_tet<PP, 1>), grid, block, lds, st, v, vhat, q, nullptr, dv, dvhat, dq, c->d_geo, c->dt, \
                       c->dp, c->d_bc, JR_q, JR_v, JR_vhat, nullptr, c->d_status, nullptr, 0, (int64_t)0, TetColTab{})
    if (c->p == 1)
        MEHDG_TET_LAUNCH(1);
    else if (c->p == 2)
        MEHDG_TET_LAUNCH(2);
    else
        MEHDG_TET_LAUNCH(3);
#undef MEHDG_TET_LAUNCH
    return hipGetLastError() == hipSuccess ? MEHDG_OK : MEHDG_EHIP;
}

mehdg_err mehdg_tet_assemble(mehdg_tet_ctx* c, const double* v, const double* vhat, const double* v_old,
                             double* R_q, double* R_v, double* R_vhat, double* entropy, mehdg_stream stream) {
    if (!c || !v || !vhat || !v_old || !R_q || !R_v || !R_vhat || !entropy) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int64_t sz[5];
    (void)mehdg_tet_sizes(c->p, sz);
    const int NV = (int)sz[2], NH = (int)sz[4];
    if (!c->d_B) {
        int64_t cs[4];
        if (!tet_cond_sizes(c->p, cs)) return MEHDG_EINVAL;
        c->rows = cs[0];
        c->ld = cs[1];
        c->per_tri = cs[2];
        c->per_perm = cs[3];
        const int64_t M = c->n_macro;
        if (hipMalloc(&c->d_B, (size_t)(M * c->rows * c->ld) * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->d_ipiv, (size_t)(M * NV) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->d_tri, (size_t)(M * c->per_tri) * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->d_perm, (size_t)(M * c->per_perm) * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->d_coef, (size_t)(M * tet_coef_doubles(c->p)) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(c->d_B);
            (void)hipFree(c->d_ipiv);
            (void)hipFree(c->d_tri);
            (void)hipFree(c->d_perm);
            (void)hipFree(c->d_coef);
            c->d_coef = nullptr;
            c->d_B = nullptr;
            c->d_ipiv = nullptr;
            c->d_tri = nullptr;
            c->d_perm = nullptr;
            return MEHDG_ENOMEM;
        }
    }
    c->stage = 0;
    mehdg_err e = mehdg_tet_residual(c, v, vhat, nullptr, v_old, R_q, R_v, R_vhat, entropy, stream);
    if (e != MEHDG_OK) return e;
    const int64_t per = c->rows * c->ld;
    hipLaunchKernelGGL(k_tet_rhs, dim3((unsigned)c->n_macro), dim3(256), 0, st, R_v, R_vhat, NV, NH, (int)c->ld, per,
                       c->d_B);
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    // pointwise coefficients once per macro, then one column per workgroup
    TetColTab ct = c->ct;
    ct.coefV = c->d_coef;
    ct.coefF = c->d_coef + c->n_macro * tet_coef_volume(c->p);
    const dim3 block(TET_THREADS);
    const size_t lds0 = tet_lds_bytes<false>(c->p);
    const size_t ldsc = c->p == 1 ? sizeof(TetColLds<1>) : c->p == 2 ? sizeof(TetColLds<2>) : sizeof(TetColLds<3>);
    // column launches: blockIdx.x the column, blockIdx.y the macro (at most 65535 per launch)
    constexpr int64_t kMaxY = 65535;
#define MEHDG_TET_LAUNCH(PP)                                                                                    \
    hipLaunchKernelGGL(k_tet_coef<PP>, dim3((unsigned)c->n_macro), block, lds0, st, v, vhat, c->d_geo, c->dt,   \
                       c->dp, const_cast<double*>(ct.coefV), const_cast<double*>(ct.coefF), c->d_status);        \
    for (int64_t m0 = 0; m0 < c->n_macro; m0 += kMaxY) {                                                        \
        ct.m0 = m0;                                                                                             \
        const int64_t cnt = (c->n_macro - m0) < kMaxY ? (c->n_macro - m0) : kMaxY;                               \
        hipLaunchKernelGGL((k_tet<PP, 2>), dim3((unsigned)(NV + NH), (unsigned)cnt), block, ldsc, st, v, vhat,  \
                           nullptr, nullptr, nullptr, nullptr, nullptr, c->d_geo, c->dt, c->dp, c->d_bc, nullptr, \
                           nullptr, nullptr, nullptr, c->d_status, c->d_B, (int)c->ld, per, ct);                 \
    }
    if (c->p == 1) {
        MEHDG_TET_LAUNCH(1);
    } else if (c->p == 2) {
        MEHDG_TET_LAUNCH(2);
    } else {
        MEHDG_TET_LAUNCH(3);
    }
#undef MEHDG_TET_LAUNCH
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    c->stage = 1;
    return MEHDG_OK;
}

mehdg_err mehdg_tet_vjp(mehdg_tet_ctx* c, const double* w_v, const double* w_vhat, double* g_v, double* g_vhat,
                        mehdg_stream stream) {
    if (!c || !w_v || !w_vhat || !g_v || !g_vhat) return MEHDG_EINVAL;
    if (c->stage != 1) return MEHDG_ESTATE;
    int64_t sz[5];
    (void)mehdg_tet_sizes(c->p, sz);
    hipLaunchKernelGGL(k_tet_vjp_b, dim3((unsigned)c->n_macro), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       c->d_B, w_v, w_vhat, (int)sz[2], (int)sz[4], (int)c->ld, c->rows * c->ld, g_v, g_vhat);
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    return poison_flagged(c->d_status, c->n_macro, g_v, sz[2], g_vhat, sz[4], reinterpret_cast<hipStream_t>(stream));
}

mehdg_err mehdg_tet_condense(mehdg_tet_ctx* c, double* Ahat, double* bhat, mehdg_stream stream) {
    if (!c || !Ahat || !bhat) return MEHDG_EINVAL;
    if (c->stage != 1) return MEHDG_ESTATE;
    TetCondWork w{c->d_B, c->d_ipiv, c->d_tri, c->d_perm, c->d_status, c->n_macro};
    mehdg_err e = tet_condense(c->p, w, Ahat, bhat, reinterpret_cast<hipStream_t>(stream));
    if (e == MEHDG_OK) c->stage = 2;
    return e;
}

mehdg_err mehdg_tet_condense_rhs(mehdg_tet_ctx* c, const double* r_v, const double* r_hat, double* bhat,
                                 mehdg_stream stream) {
    if (!c || !r_v || !bhat) return MEHDG_EINVAL;
    if (c->stage != 2) return MEHDG_ESTATE;
    TetCondWork w{c->d_B, c->d_ipiv, c->d_tri, c->d_perm, c->d_status, c->n_macro};
    return tet_condense_rhs(c->p, w, r_v, r_hat, bhat, reinterpret_cast<hipStream_t>(stream));
}

mehdg_err mehdg_tet_recover(mehdg_tet_ctx* c, const double* R_q, const double* dvhat, double* dv, double* dq,
                            mehdg_stream stream) {
    if (!c || !R_q || !dvhat || !dv || !dq) return MEHDG_EINVAL;
    if (c->stage != 2) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
#define MEHDG_TET_LAUNCH(PP)                                                                                     \
    hipLaunchKernelGGL(k_tet_recover<PP>, dim3((unsigned)c->n_macro), dim3(1024), sizeof(TetRecLds<PP>), st,   \
                       c->d_B, R_q, dvhat, c->d_geo, c->dt, dv, dq)
    if (c->p == 1)
        MEHDG_TET_LAUNCH(1);
    else if (c->p == 2)
        MEHDG_TET_LAUNCH(2);
    else
        MEHDG_TET_LAUNCH(3);
#undef MEHDG_TET_LAUNCH
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    int64_t sz[5];
    (void)mehdg_tet_sizes(c->p, sz);
    return poison_flagged(c->d_status, c->n_macro, dv, sz[2], dq, sz[3], st);
}

mehdg_err mehdg_tet_status(mehdg_tet_ctx* c, int32_t* status, mehdg_stream stream) {
    if (!c || !status) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(status, c->d_status, c->n_macro * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    for (int64_t i = 0; i < c->n_macro; ++i)
        if (status[i] != 0) return static_cast<mehdg_err>(status[i]);
    return MEHDG_OK;
}

}  // extern "C"
