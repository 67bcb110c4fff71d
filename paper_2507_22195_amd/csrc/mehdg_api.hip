// Host runtime and C ABI of the macro-element HDG local-work library.
//
// One translation unit: the kernel families are included as headers so that
// every kernel template is instantiated here for p = 1..3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mehdg.h"
#include "common.hpp"
#include "k_batch.hpp"
#include "k_linear.hpp"
#include "k_mixed.hpp"
#include "k_recover.hpp"
#include "k_trace.hpp"
#include "tables.hpp"
#include "tet_cond.hpp"
#include "tile_table.hpp"
#include "batch_view.hpp"

using namespace mehdg;

struct mehdg_ctx {
    int p = 0;
    int64_t n_macro = 0;
    int tile[MEHDG_NTILE_SITES] = {};   // product tile variant per call site
    int lu_depth = 0;                   // outer blocks per group of delayed updates (0: the degree's default)
    int lu_width = 0;                   // columns per group of the last condensation (0: the default's)
    int inner_prec = MEHDG_FP64;        // factors read by FGMRES's inner iterations
    float* d_mf32 = nullptr;            // their single-precision copies
    int64_t cond_count = 0, mf32_count = -1;   // FP64 condensations; the one the copies hold
    int64_t cap = 0;                    // macros the per-macro workspaces hold
    double* base_h = nullptr;           // the context's own mesh, status and wall arrays
    int32_t* base_status = nullptr;     // (d_h, d_status, d_bc point here unless a
    uint8_t* base_bc = nullptr;         // batch has set a view of its own arrays)
    double base_gT = 0.0;
    mehdg_params prm{};
    DevParams dp{};
    Tab1D tab{};
    double* d_h = nullptr;          // [n_macro][3]
    Tab1D* d_tab = nullptr;
    int32_t* d_status = nullptr;    // [n_macro]
    double* d_scratch = nullptr;    // residual scratch
    double* d_coefV = nullptr;      // pointwise Jacobian coefficients (volume)
    double* d_coefF = nullptr;      // pointwise Jacobian coefficients (faces)
    double* d_minvrq = nullptr;     // M^-1 R_Q per macro
    double* d_B = nullptr;          // bordered matrices
    int32_t* d_ipiv = nullptr;      // pivot rows of the LU of S
    double* d_tri = nullptr;        // inverses of the diagonal blocks of the current outer block
    int32_t* d_perm = nullptr;      // composed row interchange of the current panel or outer block
    int64_t bytes = 0;
    // kernel timing with HIP events (mehdg_profile_*)
    bool prof = false;
    struct Mark { int slot; hipEvent_t a, b; };
    std::vector<Mark> marks;
    double prof_ms[MEHDG_NPROF] = {};
    int64_t prof_calls[MEHDG_NPROF] = {};
    int stage = 0;                  // 0 nothing, 1 blocks assembled, 2 condensed
    bool have_coef = false;         // pointwise coefficients of some state stored (mehdg_jvp / mehdg_vjp)
    uint8_t* d_bc = nullptr;        // [n_macro][6] wall flags, or nullptr (no wall faces)
    // global trace system (mehdg_trace_*)
    int64_t n_faces = 0;
    int64_t* d_fid = nullptr;       // [n_macro][6] global face of each local face
    int64_t* d_side = nullptr;      // [n_faces][4] m1, f1, m2, f2
    double* d_yl = nullptr;         // [n_macro][N_VH] per-macro products
    double* d_mfw = nullptr;        // [n_macro][N_V] U12 x of the matrix-free product
    double* d_fZ = nullptr;         // FGMRES: preconditioned directions [restart][N]
    double* d_iV = nullptr;         // FGMRES: inner GMRES basis [inner + 1][N]
    int fg_restart = 0, fg_inner = 0;
    double* d_Dinv = nullptr;       // [n_faces][5nf][5nf] inverses of the diagonal face blocks
    double* d_V = nullptr;          // GMRES basis [restart + 1][N]
    double* d_w = nullptr;          // [N]
    double* d_z = nullptr;          // [N]
    double* d_part = nullptr;       // partial dot products [restart + 1][kDotBlocks]
    double* d_coef = nullptr;       // [restart + 1]
    int gm_restart = 0;
    std::vector<double> h_part, h_coef;
    // mixed-precision condensation: low-precision factors, solution, residual
    // and stopping sums of one wave of macros (mehdg_condense with FP32_IR / BF16_IR)
    int64_t lp_wave = 0;            // macros per wave the buffers hold
    float* d_slo = nullptr;         // [wave][N_V][lds] factors of S
    int32_t* d_lperm = nullptr;     // [wave][N_V] position -> row
    float* d_ltri = nullptr;        // [wave][panels][2][32][32] inverses of the diagonal blocks of L, U
    double* d_zb = nullptr;         // [wave][N_V][N_VH + 1] Z = S^-1 [-Y | r_V]
    double* d_rb = nullptr;         // [wave][N_V][N_VH + 1] right-hand sides / residuals
    float* d_yb = nullptr;          // [wave][N_V][ldy] solution of a solve with the FP32 factors
    double* d_nrm = nullptr;        // [wave][2] |correction|^2, |Z|^2
    int32_t* d_flags = nullptr;     // [wave] status codes raised by the refinement
    std::vector<double> h_nrm;
    std::vector<int32_t> h_flags;
    int32_t ir_iters = 0;           // refinement steps of the last mixed condensation (most in a wave)
};

namespace {

constexpr int kMaxP = 4;

// Brackets one launch with events when profiling is on.
struct Timed {
    mehdg_ctx* c;
    int slot;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(mehdg_ctx* c_, int slot_, hipStream_t st_) : c(c_), slot(slot_), st(st_) {
        if (c->prof && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
        else
            a = b = nullptr;
    }
    ~Timed() {
        if (a && b) {
            (void)hipEventRecord(b, st);
            c->marks.push_back({slot, a, b});
        }
    }
};

// per-macro doubles of the residual's global scratch (at least the fields,
// which the products of k_linear.hpp keep there for p >= 3)
int64_t res_scratch_doubles(int p) {
    const int nq1 = 2 * (p + 1);
    const int64_t fields = (int64_t)RES_FIELDS * nq1 * nq1 * nq1;
    switch (p) {
        case 4: return std::max<int64_t>(fields, ResScratch<4>::per_macro);
        default: return fields;
    }
}

template <int P>
size_t res_lds() { return ResScratch<P>::lds_bytes; }

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

template <typename K>
bool allow_lds(K* kern, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes) == hipSuccess;
}

template <int P>
mehdg_err ensure_coef_workspace(mehdg_ctx* c) {
    if (c->d_coefF) return MEHDG_OK;
    using D = Dims<P>;
    mehdg_err e;
    if (!c->d_coefV && (e = dev_alloc(c, &c->d_coefV, c->cap * (int64_t)D::G * COEF_V)) != MEHDG_OK) return e;
    return dev_alloc(c, &c->d_coefF, c->cap * (int64_t)6 * D::S * COEF_F);
}

template <int P>
mehdg_err ensure_block_workspace(mehdg_ctx* c) {
    mehdg_err e = ensure_coef_workspace<P>(c);
    if (e != MEHDG_OK) return e;
    if (c->d_B) return MEHDG_OK;
    using D = Dims<P>;
    if ((e = dev_alloc(c, &c->d_minvrq, c->cap * (int64_t)15 * D::n)) != MEHDG_OK) return e;
    if ((e = dev_alloc(c, &c->d_ipiv, c->cap * (int64_t)D::NV)) != MEHDG_OK) return e;
    if ((e = dev_alloc(c, &c->d_tri, c->cap * Panel<P>::TRI)) != MEHDG_OK) return e;
    if ((e = dev_alloc(c, &c->d_perm, c->cap * Panel<P>::PERM)) != MEHDG_OK) return e;
    if ((e = dev_alloc(c, &c->d_B, c->cap * Bdims<P>::per_macro)) != MEHDG_OK) return e;
    return MEHDG_OK;
}

// Device bytes per macro of a context after assemble(want_blocks = 1) and an
// FP64 condense: the workspaces above plus the residual scratch.
template <int P>
int64_t ctx_macro_bytes() {
    using D = Dims<P>;
    const int64_t doubles = (int64_t)D::G * COEF_V + (int64_t)6 * D::S * COEF_F + (int64_t)15 * D::n +
                            Panel<P>::TRI + Bdims<P>::per_macro + res_scratch_doubles(P) + 3;
    return doubles * 8 + (int64_t)D::NV * 4 + Panel<P>::PERM * 4 + 4 + 6;
}

template <int P>
mehdg_err launch_rows(mehdg_ctx* c, const double* R_q, const double* R_v, const double* R_vhat, hipStream_t st);

template <int P>
mehdg_err launch_assemble(mehdg_ctx* c, const double* v, const double* vhat, const double* q,
                          const double* v_old, double* R_q, double* R_v, double* R_vhat, double* ent,
                          int mode, hipStream_t st) {
    const size_t lds = res_lds<P>();
    const unsigned M = (unsigned)c->n_macro;
    if (mode == 0) {
        if (!allow_lds(&k_residual<P, false>, lds)) return MEHDG_EHIP;
        Timed t(c, MEHDG_PROF_RESIDUAL, st);
        hipLaunchKernelGGL((k_residual<P, false>), dim3(M), dim3(256), lds, st, v, vhat, q, v_old, c->d_h, c->dp,
                           c->d_tab, R_q, R_v, R_vhat, ent, c->d_scratch, (double*)nullptr, (double*)nullptr,
                           (const uint8_t*)c->d_bc, c->d_status);
        return hip_ok(hipGetLastError());
    }
    mehdg_err e = (mode == 1) ? ensure_block_workspace<P>(c) : ensure_coef_workspace<P>(c);
    if (e != MEHDG_OK) return e;
    if (!allow_lds(&k_residual<P, true>, lds)) return MEHDG_EHIP;
    {
        Timed t(c, MEHDG_PROF_RESIDUAL, st);
        hipLaunchKernelGGL((k_residual<P, true>), dim3(M), dim3(256), lds, st, v, vhat, q, v_old, c->d_h, c->dp,
                           c->d_tab, R_q, R_v, R_vhat, ent, c->d_scratch, c->d_coefV, c->d_coefF,
                           (const uint8_t*)c->d_bc, c->d_status);
    }
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    if (mode == 2) return MEHDG_OK;
    return launch_rows<P>(c, R_q, R_v, R_vhat, st);
}

// The rows of the bordered matrix from the residual pass's outputs and
// coefficients: M^-1 R_Q, the interior rows, the trace rows, the wall rows.
template <int P>
mehdg_err launch_rows(mehdg_ctx* c, const double* R_q, const double* R_v, const double* R_vhat, hipStream_t st) {
    using D = Dims<P>;
    const unsigned M = (unsigned)c->n_macro;
    {
        Timed t(c, MEHDG_PROF_MINV_RQ, st);
        hipLaunchKernelGGL(k_minv_rq<P>, dim3(M, MinvRqCfg<P>::GROUPS), dim3(256), 0, st, R_q, c->d_h, c->d_tab, c->d_minvrq);
    }
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    const size_t rl = sizeof(RowLds<P>), rlh = sizeof(RowLdsH<P>);
    if (!allow_lds(&k_rows_v<P>, rl) || !allow_lds(&k_rows_h<P>, rlh)) return MEHDG_EHIP;
    {
        Timed t(c, MEHDG_PROF_ROWS_V, st);
        hipLaunchKernelGGL(k_rows_v<P>, dim3(xcd_grid(D::n, c->n_macro)), dim3(RowCfg<P>::THREADS), rl, st, c->d_coefV,
                           c->d_coefF, R_v, c->d_minvrq, c->d_h, c->d_tab, c->dp.viscous, c->d_B, (int64_t)c->n_macro);
    }
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    {
        Timed t(c, MEHDG_PROF_ROWS_H, st);
        hipLaunchKernelGGL(k_rows_h<P>, dim3(xcd_grid(6 * D::nf, c->n_macro)), dim3(RowCfgH<P>::THREADS), rlh, st,
                           c->d_coefF, R_vhat, c->d_minvrq, c->d_h, c->d_tab, c->dp.viscous, c->d_B,
                           (int64_t)c->n_macro);
        if (c->d_bc)
            hipLaunchKernelGGL(k_wall_rows<P>, dim3((unsigned)(6 * c->n_macro)), dim3(256), 0, st,
                               (const uint8_t*)c->d_bc, R_vhat, c->d_h, c->d_tab, c->d_B);
    }
    return hip_ok(hipGetLastError());
}

// Outputs of the macro-elements whose status is not OK are set to NaN.
struct PoisonArgs {
    double* ptr[4];
    int64_t per[4];       // doubles per macro of each array
};

__global__ void __launch_bounds__(256) k_poison(const int32_t* __restrict__ status, PoisonArgs a) {
    const int64_t m = blockIdx.x;
    if (status[m] == 0) return;
    const double nan = __builtin_nan("");
    for (int k = 0; k < 4; ++k) {
        double* q = a.ptr[k];
        if (!q) continue;
        for (int64_t i = threadIdx.x; i < a.per[k]; i += blockDim.x) q[m * a.per[k] + i] = nan;
    }
}

mehdg_err launch_poison(mehdg_ctx* c, PoisonArgs a, hipStream_t st) {
    hipLaunchKernelGGL(k_poison, dim3((unsigned)c->n_macro), dim3(256), 0, st, c->d_status, a);
    return hip_ok(hipGetLastError());
}

// Compute units of the current device (cached per device).
int device_cus() {
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

template <int TAG, class T>
mehdg_err launch_gemm_t(GemmArgs g, int64_t n, hipStream_t st) {
    const int tr = (g.rows + T::TM - 1) / T::TM;
    g.tiles_c = (g.cols + T::TN - 1) / T::TN;
    if (tr <= 0 || g.tiles_c <= 0 || g.K <= 0 || n <= 0) return MEHDG_OK;
    g.tiles = tr * g.tiles_c;
    g.n_macro = n;
    hipLaunchKernelGGL((k_gemm<TAG, T>), dim3(xcd_grid(g.tiles, n)), dim3(T::NT), 0, st, g);
    return hip_ok(hipGetLastError());
}

// The batched product over the first n macros that the pointers start at, in
// the tile shape the context holds for the product's call site.
template <int TAG>
mehdg_err launch_gemm_n(mehdg_ctx* c, GemmArgs g, int64_t n, int slot, hipStream_t st) {
    const int site = TAG == 0 ? MEHDG_TILE_UPDATE : MEHDG_TILE_SCHUR;
    Timed t(c, slot, st);
    switch (c->tile[site]) {
#define MEHDG_LAUNCH_VARIANT(i, wm, wn, bi, bj, kc, occ) \
    case i: return launch_gemm_t<TAG, GTile<wm, wn, bi, bj, kc, occ>>(g, n, st);
        MEHDG_GEMM_VARIANTS(MEHDG_LAUNCH_VARIANT)
#undef MEHDG_LAUNCH_VARIANT
        default: return MEHDG_EINVAL;
    }
}

template <int TAG>
mehdg_err launch_gemm(mehdg_ctx* c, GemmArgs g, int slot, hipStream_t st) {
    return launch_gemm_n<TAG>(c, g, c->n_macro, slot, st);
}

// D(rows, cols) -= B[rows, kb0 : kb0+K] * B[kb0 : kb0+K, cols] inside one bordered matrix,
// origin (o_r, o_c), with the corner from (skip_r, skip_c) left alone
template <int P>
mehdg_err launch_update(mehdg_ctx* c, int kb0, int K, int o_r, int o_c, int rows, int cols, int skip_r,
                        int skip_c, hipStream_t st) {
    using BD = Bdims<P>;
    constexpr int ld = BD::ld;
    if (skip_r <= 0 && skip_c <= 0) return MEHDG_OK;   // all of it is the corner
    double* B = c->d_B;
    GemmArgs g{};
    g.A = B + (int64_t)o_r * ld + kb0;
    g.Bt = B + (int64_t)kb0 * ld + o_c;
    g.limA = BD::per_macro - ((int64_t)o_r * ld + kb0);
    g.limB = BD::per_macro - ((int64_t)kb0 * ld + o_c);
    g.C = B + (int64_t)o_r * ld + o_c;
    g.D = B + (int64_t)o_r * ld + o_c;
    g.D2 = nullptr;
    g.sA = g.sB = g.sC = g.sD = BD::per_macro;
    g.sD2 = 0;
    g.lda = g.ldb = g.ldc = g.ldd = ld;
    g.ldd2 = 0;
    g.rows = rows;
    g.cols = cols;
    g.K = K;
    g.dsplit = cols;
    g.skip_r = skip_r;
    g.skip_c = skip_c;
    return launch_gemm<0>(c, g, MEHDG_PROF_UPDATE, st);
}

// Outer blocks per group of delayed trailing updates of the LU of S, by
// degree from the tuned table (other element families: 1).
constexpr int lu_depth_default(int p) { return p >= 1 && p <= 4 ? kLuDepth[p] : 1; }

// Columns per group of delayed trailing updates: depth outer blocks (the
// context's, else the degree's default).
template <int P>
int lu_group_width(const mehdg_ctx* c) {
    int depth = c->lu_depth > 0 ? c->lu_depth : lu_depth_default(P);
    const int nblk = (Dims<P>::NV + Panel<P>::OB - 1) / Panel<P>::OB;
    if (depth > nblk) depth = nblk;
    return depth * Panel<P>::OB;
}

template <int P>
mehdg_err launch_perm_rows(mehdg_ctx* c, int kb0, int w, int c_lo, int c_hi, hipStream_t st) {
    const int ct = (c_hi - c_lo + GT - 1) / GT;
    if (ct <= 0) return MEHDG_OK;
    Timed t(c, MEHDG_PROF_ROWBLOCK, st);
    hipLaunchKernelGGL(k_perm_rows<P>, dim3(xcd_grid(ct, c->n_macro)), dim3(GTHREADS), 0, st, c->d_B, c->d_perm,
                       kb0, w, c_lo, c_hi, ct, (int64_t)c->n_macro);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_tri(mehdg_ctx* c, TriArgs a, hipStream_t st) {
    using D = Dims<P>;
    a.ct = a.c_hi > a.c_lo ? (a.c_hi - a.c_lo + GT - 1) / GT : 0;
    if (a.ct == 0) return MEHDG_OK;
    Timed t(c, MEHDG_PROF_ROWBLOCK, st);
    if (a.kpre > 0)
        hipLaunchKernelGGL((k_tri<P, true>), dim3(xcd_grid(a.ct, c->n_macro)), dim3(GTHREADS), 0, st, c->d_B,
                           c->d_tri, c->d_perm, a, (int64_t)c->n_macro);
    else
        hipLaunchKernelGGL((k_tri<P, false>), dim3(xcd_grid(a.ct, c->n_macro)), dim3(GTHREADS), 0, st,
                           c->d_B, c->d_tri, c->d_perm, a, (int64_t)c->n_macro);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_condense(mehdg_ctx* c, double* Ahat, double* bhat, hipStream_t st) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NV = D::NV, NH = D::NH, ld = BD::ld, NB = PN::NB;
    const unsigned M = (unsigned)c->n_macro;
    double* B = c->d_B;
    mehdg_err e;
    auto panel = [&](int kb, int kb0) {
        Timed t(c, MEHDG_PROF_PANEL, st);
        // more rows than threads: the 64-wide register segments would spill, so
        // the panel goes in left-looking 8-column sub-panels
        if constexpr (PN::RPT > 1)
            hipLaunchKernelGGL((k_panel_sub<P, 8>), dim3(M), dim3(PN::THREADS), 0, st, B, kb, kb0, c->d_ipiv, c->d_perm,
                               c->d_tri, c->d_status);
        else
            hipLaunchKernelGGL(k_panel<P>, dim3(M), dim3(PN::THREADS), 0, st, B, kb, kb0, c->d_ipiv, c->d_perm,
                               c->d_tri, c->d_status);
        return hip_ok(hipGetLastError());
    };
    // outer blocks in groups of delayed trailing updates, gw columns each
    const int gw = lu_group_width<P>(c);
    c->lu_width = gw;
    constexpr int ncol = NV + NH + 1;
    for (int kb0 = 0; kb0 < NV; kb0 += PN::OB) {
        const int w = (NV - kb0) < PN::OB ? (NV - kb0) : PN::OB;
        const int kg = kb0 - kb0 % gw;               // first column of the group
        const int kpre = kb0 - kg;                   // columns of its earlier blocks
        const bool group_end = kb0 + w - kg >= gw || kb0 + w >= NV;
        // the earlier blocks' pending update of this block's columns
        if (kpre > 0 && (e = launch_update<P>(c, kg, kpre, kb0, kb0, NV - kb0, w, NV - kb0, w, st)) != MEHDG_OK)
            return e;
        if ((e = panel(kb0, kb0)) != MEHDG_OK) return e;
        TriArgs a{};
        a.kb0 = kb0;
        if (w > NB) {
            // first panel: its U rows over the second panel's columns
            a.w = NB;
            a.loff = PN::LINV1;
            a.ldl = NB;
            a.c_lo = kb0 + NB;
            a.c_hi = kb0 + w;
            if ((e = launch_tri<P>(c, a, st)) != MEHDG_OK) return e;
            // the second panel's columns, S rows below the first panel
            const int o = kb0 + NB;
            if ((e = launch_update<P>(c, kb0, NB, o, o, NV - o, w - NB, NV - o, w - NB, st)) != MEHDG_OK)
                return e;
            if ((e = panel(kb0 + NB, kb0)) != MEHDG_OK) return e;
            a.loff = PN::LINVW;
            a.ldl = PN::OB;
        } else {
            a.loff = PN::LINV1;
            a.ldl = NB;
        }
        // the earlier blocks' multipliers follow this block's interchange
        if (kpre > 0 && (e = launch_perm_rows<P>(c, kb0, w, kg, kb0, st)) != MEHDG_OK) return e;
        // the whole block: U rows right of it (after the group's pending update of them)
        a.w = w;
        a.c_lo = kb0 + w;
        a.c_hi = ld;
        a.kpre = kpre;
        if ((e = launch_tri<P>(c, a, st)) != MEHDG_OK) return e;
        // after the group: trailing update of the S rows (S and border columns)
        if (group_end) {
            const int o = kb0 + w;
            if ((e = launch_update<P>(c, kg, o - kg, o, o, NV - o, ncol - o, NV - o, ncol - o, st)) != MEHDG_OK)
                return e;
        }
    }
    // L21 of the X rows, panel by panel
    {
        const int tiles = (NH + GM - 1) / GM;
        for (int q = 0; q < PN::NPAN; ++q) {
            Timed t(c, MEHDG_PROF_TRSM, st);
            hipLaunchKernelGGL(k_trsm_x<P>, dim3(xcd_grid(tiles, c->n_macro)), dim3(GTHREADS), 0, st, c->d_B,
                               c->d_tri, q, (int64_t)c->n_macro);
            if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
        }
    }
    // Ahat = A' - L21 U12, bhat = r_hat - L21 y
    GemmArgs g{};
    g.A = B + (int64_t)NV * ld;
    g.limA = BD::per_macro - (int64_t)NV * ld;
    g.sA = g.sB = g.sC = BD::per_macro;
    g.lda = g.ldb = g.ldc = ld;
    g.rows = NH;
    g.K = NV;
    g.skip_r = NH;
    g.skip_c = NH + 1;
    if (Ahat) {
        g.Bt = B + NV;
        g.limB = BD::per_macro - NV;
        g.C = B + (int64_t)NV * ld + NV;
        g.D = Ahat;
        g.sD = (int64_t)NH * NH;
        g.ldd = NH;
        g.D2 = bhat;
        g.sD2 = NH;
        g.ldd2 = 1;
        g.cols = NH + 1;
        g.dsplit = NH;
    } else {
        g.Bt = B + NV + NH;
        g.limB = BD::per_macro - (NV + NH);
        g.C = B + (int64_t)NV * ld + NV + NH;
        g.D = bhat;
        g.sD = NH;
        g.ldd = 1;
        g.D2 = bhat;
        g.sD2 = NH;
        g.ldd2 = 1;
        g.cols = 1;
        g.dsplit = 0;
    }
    return launch_gemm<1>(c, g, MEHDG_PROF_SCHUR, st);
}

// Device memory the mixed-precision condensation may hold for one wave.
constexpr int64_t kLpBudget = (int64_t)32 << 30;

template <int P>
int64_t lp_bytes_per_macro() {
    using LD = LpDims<P>;
    return LD::per_s * 4 + LD::per_t * 4 + 2 * LD::per_z * 8 + LpTrsmDims<P>::per_y * 4 + (int64_t)LD::NV * 4 +
           2 * 8 + 4;
}

template <int P>
mehdg_err ensure_lp_workspace(mehdg_ctx* c, int64_t wave) {
    using LD = LpDims<P>;
    if (c->lp_wave >= wave) return MEHDG_OK;
    (void)hipFree(c->d_slo);
    (void)hipFree(c->d_lperm);
    (void)hipFree(c->d_ltri);
    (void)hipFree(c->d_zb);
    (void)hipFree(c->d_rb);
    (void)hipFree(c->d_yb);
    (void)hipFree(c->d_nrm);
    (void)hipFree(c->d_flags);
    c->d_yb = nullptr;
    c->d_slo = nullptr;
    c->d_lperm = nullptr;
    c->d_ltri = nullptr;
    c->d_zb = c->d_rb = c->d_nrm = nullptr;
    c->d_flags = nullptr;
    c->lp_wave = 0;
    mehdg_err e;
    if ((e = dev_alloc(c, &c->d_slo, wave * LD::per_s)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_lperm, wave * LD::NV)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_ltri, wave * LD::per_t)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_zb, wave * LD::per_z)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_rb, wave * LD::per_z)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_yb, wave * LpTrsmDims<P>::per_y)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_nrm, 2 * wave)) != MEHDG_OK || (e = dev_alloc(c, &c->d_flags, wave)) != MEHDG_OK)
        return e;
    c->h_nrm.assign((size_t)(2 * wave), 0.0);
    c->h_flags.assign((size_t)wave, 0);
    c->lp_wave = wave;
    return MEHDG_OK;
}

// Mixed-precision condensation (precision modes FP32_IR, BF16_IR), macros in
// waves that fit kLpBudget: FP32 LU of S (BF16 MFMA trailing updates for
// BF16_IR), Z = S^-1 [-Y | r_V] refined with FP64 residuals until the
// forward-error estimate |d_k| rho_k / (1 - rho_k) / |Z| <= ir_tol
// (rho_k = |d_k| / |d_{k-1}|, the observed contraction; d_0 = Z_0), at most
// ir_maxit refinement steps (else MEHDG_EIRNOCONV for the macro), then
// [Ahat | bhat] = [A' | r_hat] - X Z in FP64 and Z stashed for the recovery.
template <int P>
mehdg_err launch_condense_mixed(mehdg_ctx* c, bool bf16, double* Ahat, double* bhat, hipStream_t st) {
    using LD = LpDims<P>;
    using BD = Bdims<P>;
    constexpr int NV = LD::NV, NH = LD::NH, NR = LD::NR, ld = BD::ld;
    const int64_t per = lp_bytes_per_macro<P>();
    const int64_t nwave = (c->n_macro * per + kLpBudget - 1) / kLpBudget;
    const int64_t Wmax = (c->n_macro + nwave - 1) / nwave;
    mehdg_err e = ensure_lp_workspace<P>(c, Wmax);
    if (e != MEHDG_OK) return e;
    const double tol = c->prm.ir_tol;
    const int maxit = c->prm.ir_maxit;
    c->ir_iters = 0;
    for (int64_t m0 = 0; m0 < c->n_macro; m0 += Wmax) {
        const int64_t W = (c->n_macro - m0) < Wmax ? (c->n_macro - m0) : Wmax;
        {
            Timed t(c, MEHDG_PROF_LP_MOVE, st);
            hipLaunchKernelGGL(k_lp_init<P>, dim3((unsigned)NV, (unsigned)W), dim3(256), 0, st, c->d_B, m0, W,
                               c->d_slo, c->d_lperm, c->d_zb, c->d_rb);
        }
        if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
        for (int kb = 0; kb < NV; kb += LP_NB) {
            {
                Timed t(c, MEHDG_PROF_LP_PANEL, st);
                hipLaunchKernelGGL(k_lp_panel<P>, dim3((unsigned)W), dim3(LD::PT), 0, st, c->d_slo, c->d_lperm,
                                   c->d_ltri, kb, m0, c->d_status);
            }
            if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
            const int rows = NV - kb - LP_NB;
            if (rows <= 0) continue;
            const int tc = (rows + 63) / 64, tiles = ((rows + 127) / 128) * tc;
            {
                Timed t(c, MEHDG_PROF_LP_UPDATE, st);
                if (bf16)
                    hipLaunchKernelGGL((k_lp_update<P, true>), dim3(xcd_grid(tiles, W)), dim3(LP_UT), 0, st,
                                       c->d_slo, c->d_lperm, kb, tc, tiles, W);
                else
                    hipLaunchKernelGGL((k_lp_update<P, false>), dim3(xcd_grid(tiles, W)), dim3(LP_UT), 0, st,
                                       c->d_slo, c->d_lperm, kb, tc, tiles, W);
            }
            if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
        }
        // x = S^-1 R with the low-precision factors (R in d_rb), Z += x
        auto solve = [&]() -> mehdg_err {
            hipLaunchKernelGGL(k_lp_fill, dim3((unsigned)((2 * W + 255) / 256)), dim3(256), 0, st, c->d_nrm, 2 * W, 0.0);
            const dim3 grid(xcd_grid(LpTrsmDims<P>::TILES, W));
            Timed t(c, MEHDG_PROF_LP_SOLVE, st);
            for (int q = 0; q < LD::NPAN; ++q)
                hipLaunchKernelGGL((k_lp_trsm<P, true>), grid, dim3(LPT_T), 0, st, c->d_slo, c->d_lperm, c->d_ltri,
                                   c->d_rb, c->d_yb, q, W);
            for (int q = LD::NPAN - 1; q >= 0; --q)
                hipLaunchKernelGGL((k_lp_trsm<P, false>), grid, dim3(LPT_T), 0, st, c->d_slo, c->d_lperm, c->d_ltri,
                                   c->d_rb, c->d_yb, q, W);
            hipLaunchKernelGGL(k_lp_zadd<P>, dim3((unsigned)((NV + 31) / 32), (unsigned)W), dim3(256), 0, st, c->d_yb,
                               c->d_zb, c->d_nrm, W);
            return hip_ok(hipGetLastError());
        };
        if ((e = solve()) != MEHDG_OK) return e;
        // refinement: R = [-Y | r_V] - S Z in FP64, Z += solve(R)
        GemmArgs g{};
        g.A = c->d_B + m0 * BD::per_macro;
        g.lda = ld;
        g.sA = BD::per_macro;
        g.limA = BD::per_macro;
        g.Bt = c->d_zb;
        g.ldb = NR;
        g.sB = LD::per_z;
        g.limB = LD::per_z;
        g.C = c->d_B + m0 * BD::per_macro + NV;
        g.ldc = ld;
        g.sC = BD::per_macro;
        g.D = c->d_rb;
        g.ldd = NR;
        g.sD = LD::per_z;
        g.rows = NV;
        g.cols = NR;
        g.K = NV;
        g.dsplit = NR;
        g.skip_r = NV;
        g.skip_c = NR;
        std::vector<double> prev((size_t)W, 1.0);
        std::vector<char> done((size_t)W, 0);
        int it = 0;
        bool all = false;
        while (!all && it < maxit) {
            if ((e = launch_gemm_n<2>(c, g, W, MEHDG_PROF_IR_RESID, st)) != MEHDG_OK) return e;
            if ((e = solve()) != MEHDG_OK) return e;
            ++it;
            if (hipMemcpyAsync(c->h_nrm.data(), c->d_nrm, sizeof(double) * 2 * W, hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return MEHDG_EHIP;
            all = true;
            for (int64_t i = 0; i < W; ++i) {
                const double dx = std::sqrt(c->h_nrm[2 * i]), zz = std::sqrt(c->h_nrm[2 * i + 1]);
                if (!std::isfinite(dx) || !std::isfinite(zz)) {
                    done[i] = 2;
                    continue;
                }
                const double rel = zz > 0.0 ? dx / zz : 0.0;
                const double rho = prev[i] > 0.0 ? rel / prev[i] : 0.0;
                prev[i] = rel;
                if (!done[i] && (rel == 0.0 || (rho < 1.0 && rel * rho / (1.0 - rho) <= tol))) done[i] = 1;
                if (!done[i]) all = false;
            }
        }
        if (it > c->ir_iters) c->ir_iters = it;
        bool any = false;
        for (int64_t i = 0; i < W; ++i) {
            c->h_flags[i] = done[i] == 1 ? 0 : (done[i] == 2 ? ST_NONFINITE : ST_IRNOCONV);
            any = any || c->h_flags[i] != 0;
        }
        if (any) {
            if (hipMemcpyAsync(c->d_flags, c->h_flags.data(), sizeof(int32_t) * W, hipMemcpyHostToDevice, st) !=
                hipSuccess)
                return MEHDG_EHIP;
            hipLaunchKernelGGL(k_lp_flag, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, st, c->d_flags, m0, W,
                               c->d_status);
            if (hipStreamSynchronize(st) != hipSuccess) return MEHDG_EHIP;   // h_flags is reused by the next wave
        }
        // [Ahat | bhat] = [A' | r_hat] - X Z
        GemmArgs s{};
        s.A = c->d_B + m0 * BD::per_macro + (int64_t)NV * ld;
        s.lda = ld;
        s.sA = BD::per_macro;
        s.limA = BD::per_macro - (int64_t)NV * ld;
        s.Bt = c->d_zb;
        s.ldb = NR;
        s.sB = LD::per_z;
        s.limB = LD::per_z;
        s.C = c->d_B + m0 * BD::per_macro + (int64_t)NV * ld + NV;
        s.ldc = ld;
        s.sC = BD::per_macro;
        s.rows = NH;
        s.K = NV;
        s.skip_r = NH;
        s.skip_c = NR;
        if (Ahat) {
            s.D = Ahat + m0 * (int64_t)NH * NH;
            s.ldd = NH;
            s.sD = (int64_t)NH * NH;
            s.D2 = bhat + m0 * NH;
            s.ldd2 = 1;
            s.sD2 = NH;
            s.cols = NR;
            s.dsplit = NH;
        } else {
            s.Bt = c->d_zb + NH;
            s.limB = LD::per_z - NH;
            s.C = c->d_B + m0 * BD::per_macro + (int64_t)NV * ld + NV + NH;
            s.D = bhat + m0 * NH;
            s.ldd = 1;
            s.sD = NH;
            s.D2 = bhat + m0 * NH;
            s.ldd2 = 1;
            s.sD2 = NH;
            s.cols = 1;
            s.dsplit = 0;
        }
        if ((e = launch_gemm_n<1>(c, s, W, MEHDG_PROF_SCHUR, st)) != MEHDG_OK) return e;
        {
            Timed t(c, MEHDG_PROF_LP_MOVE, st);
            hipLaunchKernelGGL(k_lp_stash<P>, dim3((unsigned)((NR + 31) / 32), (unsigned)((NV + 31) / 32), (unsigned)W),
                               dim3(256), 0, st, c->d_zb, m0, W, c->d_B);
        }
        if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    }
    return MEHDG_OK;
}

template <int P>
mehdg_err launch_recover_z(mehdg_ctx* c, const double* R_q, const double* dvhat, double* dv, double* dq,
                           hipStream_t st) {
    const size_t lds = sizeof(RecLds<P>);
    if (!allow_lds(&k_recover_z<P>, lds)) return MEHDG_EHIP;
    Timed t(c, MEHDG_PROF_RECOVER, st);
    hipLaunchKernelGGL(k_recover_z<P>, dim3((unsigned)c->n_macro), dim3(1024), lds, st, c->d_B, R_q, dvhat, c->d_h,
                       c->d_tab, dv, dq);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_recover(mehdg_ctx* c, const double* R_q, const double* dvhat, double* dv, double* dq,
                         hipStream_t st) {
    const size_t lds = sizeof(RecLds<P>);
    if (!allow_lds(&k_recover<P>, lds)) return MEHDG_EHIP;
    Timed t(c, MEHDG_PROF_RECOVER, st);
    // up to p = 3 the LDS holds two macros per CU: two 512-thread workgroups
    // overlap one macro's serial block solves with the other's loads
    const unsigned threads = P <= 3 ? 512 : 1024;
    hipLaunchKernelGGL(k_recover<P>, dim3((unsigned)c->n_macro), dim3(threads), lds, st, c->d_B, R_q, dvhat, c->d_h,
                       c->d_tab, dv, dq);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_jvp(mehdg_ctx* c, const double* dv, const double* dvh, const double* dq, double* J_q, double* J_v,
                     double* J_vh, hipStream_t st) {
    const size_t lds = res_lds<P>();
    if (!allow_lds(&k_jvp<P>, lds)) return MEHDG_EHIP;
    Timed t(c, MEHDG_PROF_JVP, st);
    hipLaunchKernelGGL(k_jvp<P>, dim3((unsigned)c->n_macro), dim3(256), lds, st, dv, dvh, dq, c->d_h, c->d_tab,
                       c->d_coefV, c->d_coefF, c->dp.viscous, (const uint8_t*)c->d_bc, J_q, J_v, J_vh,
                       c->d_scratch);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_vjp(mehdg_ctx* c, const double* wq, const double* wv, const double* wvh, double* g_q, double* g_v,
                     double* g_vh, hipStream_t st) {
    const size_t lds = res_lds<P>();
    if (!allow_lds(&k_vjp<P>, lds)) return MEHDG_EHIP;
    Timed t(c, MEHDG_PROF_VJP, st);
    hipLaunchKernelGGL(k_vjp<P>, dim3((unsigned)c->n_macro), dim3(256), lds, st, wq, wv, wvh, c->d_h, c->d_tab,
                       c->d_coefV, c->d_coefF, c->dp.viscous, (const uint8_t*)c->d_bc, g_q, g_v, g_vh,
                       c->d_scratch);
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err launch_fsolve(mehdg_ctx* c, const double* r_v, const double* r_h, double* bhat, hipStream_t st) {
    const size_t lds = sizeof(FsLds<P>);
    if (!allow_lds(&k_fsolve<P>, lds)) return MEHDG_EHIP;
    Timed t(c, MEHDG_PROF_FSOLVE, st);
    const int width = c->lu_width > 0 ? c->lu_width : lu_group_width<P>(c);
    hipLaunchKernelGGL(k_fsolve<P>, dim3((unsigned)c->n_macro), dim3(1024), lds, st, c->d_B, c->d_ipiv, r_v, r_h,
                       bhat, width);
    return hip_ok(hipGetLastError());
}

int64_t bordered_rows(int p) {
    switch (p) {
        case 1: return Bdims<1>::rows;
        case 2: return Bdims<2>::rows;
        case 3: return Bdims<3>::rows;
        case 4: return Bdims<4>::rows;
        default: return 0;
    }
}
int64_t bordered_ld(int p) {
    switch (p) {
        case 1: return Bdims<1>::ld;
        case 2: return Bdims<2>::ld;
        case 3: return Bdims<3>::ld;
        case 4: return Bdims<4>::ld;
        default: return 0;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Global trace system
namespace {

constexpr int kDotBlocks = 256;
constexpr int kMaxRestart = 60;

int64_t face_block(int p) { return 5 * (int64_t)(2 * p + 1) * (2 * p + 1); }

unsigned vec_grid(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

// K x; with Ahat NULL matrix-free from the factors of an FP64 condensation
// (Algorithm 1: Ahat_m x_m = A' x_m - L21 (U12 x_m), k_mf_w then k_mf_y)
template <int P>
mehdg_err trace_launch_apply(mehdg_ctx* c, const double* Ahat, const double* x, double* y, hipStream_t st,
                             bool inner = false) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    using MF = MfF32<P>;
    constexpr int RT = (D::NH + 63) / 64, RTV = (D::NV + 63) / 64, NV = D::NV, NH = D::NH, ld = BD::ld;
    if (Ahat) {
        hipLaunchKernelGGL(k_local_apply<P>, dim3(xcd_grid(RT, c->n_macro)), dim3(256), 0, st, Ahat, x, c->d_fid,
                           c->d_yl, (int64_t)c->n_macro);
    } else if (inner && c->inner_prec == MEHDG_FP32_IR) {
        const float* F = c->d_mf32;
        hipLaunchKernelGGL((k_mf_w<P, float>), dim3(xcd_grid(RTV, c->n_macro)), dim3(256), 0, st, F, MF::per_macro,
                           NH, x, c->d_fid, c->d_mfw, (int64_t)c->n_macro);
        hipLaunchKernelGGL((k_mf_y<P, float>), dim3(xcd_grid(RT, c->n_macro)), dim3(256), 0, st, F + MF::off_l21,
                           F + MF::off_ap, MF::per_macro, NV, NH, x, c->d_fid, c->d_mfw, c->d_yl,
                           (int64_t)c->n_macro);
    } else {
        const double* B = c->d_B;
        hipLaunchKernelGGL((k_mf_w<P, double>), dim3(xcd_grid(RTV, c->n_macro)), dim3(256), 0, st, B + NV,
                           BD::per_macro, ld, x, c->d_fid, c->d_mfw, (int64_t)c->n_macro);
        hipLaunchKernelGGL((k_mf_y<P, double>), dim3(xcd_grid(RT, c->n_macro)), dim3(256), 0, st,
                           B + (int64_t)NV * ld, B + (int64_t)NV * ld + NV, BD::per_macro, ld, ld, x, c->d_fid,
                           c->d_mfw, c->d_yl, (int64_t)c->n_macro);
    }
    hipLaunchKernelGGL(k_face_sum<P>, dim3((unsigned)c->n_faces), dim3(128), 0, st, c->d_yl, c->d_side, y,
                       c->n_faces);
    return hip_ok(hipGetLastError());
}

// Single-precision copies of the factors for the inner iterations, made once
// per FP64 condensation.
template <int P>
mehdg_err ensure_mf32(mehdg_ctx* c, hipStream_t st) {
    if (c->mf32_count == c->cond_count) return MEHDG_OK;
    if (!c->d_mf32) {
        mehdg_err e = dev_alloc(c, &c->d_mf32, c->n_macro * MfF32<P>::per_macro);
        if (e != MEHDG_OK) return e;
    }
    const unsigned gy = (unsigned)std::min<int64_t>(c->n_macro, 65535);
    hipLaunchKernelGGL(k_mf_to_f32<P>, dim3((unsigned)(Dims<P>::NV + Dims<P>::NH), gy), dim3(256), 0, st, c->d_B,
                       c->d_mf32, (int64_t)c->n_macro);
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    c->mf32_count = c->cond_count;
    return MEHDG_OK;
}

// inverses of K's diagonal face blocks; with Ahat NULL the blocks are formed
// from the factors first (k_mf_face_blocks)
template <int P>
mehdg_err trace_launch_precond_setup(mehdg_ctx* c, const double* Ahat, hipStream_t st) {
    const size_t lds = BlockInvCfg<P>::lds_bytes;
    if (Ahat) {
        if (!allow_lds(&k_face_block_inv<P, false>, lds)) return MEHDG_EHIP;
        hipLaunchKernelGGL((k_face_block_inv<P, false>), dim3((unsigned)c->n_faces), dim3(256), lds, st, Ahat,
                           c->d_side, c->d_Dinv, c->n_faces);
    } else {
        constexpr int BS = 5 * Dims<P>::nf;
        constexpr int tiles = ((BS + GM - 1) / GM) * ((BS + GT - 1) / GT);
        if (!allow_lds(&k_face_block_inv<P, true>, lds)) return MEHDG_EHIP;
        hipLaunchKernelGGL(k_mf_face_blocks<P>, dim3((unsigned)(c->n_faces * tiles)), dim3(GTHREADS), 0, st, c->d_B,
                           c->d_side, c->d_Dinv, c->n_faces);
        hipLaunchKernelGGL((k_face_block_inv<P, true>), dim3((unsigned)c->n_faces), dim3(256), lds, st, c->d_B,
                           c->d_side, c->d_Dinv, c->n_faces);
    }
    return hip_ok(hipGetLastError());
}

template <int P>
mehdg_err trace_launch_precond_apply(mehdg_ctx* c, const double* r, double* z, hipStream_t st) {
    hipLaunchKernelGGL(k_face_block_apply<P>, dim3((unsigned)c->n_faces), dim3(256), 0, st, c->d_Dinv, r, z,
                       c->n_faces);
    return hip_ok(hipGetLastError());
}

mehdg_err trace_ready(mehdg_ctx* c) {
    if (!c) return MEHDG_EINVAL;
    if (!c->d_side) return MEHDG_ESTATE;
    return MEHDG_OK;
}

mehdg_err ensure_trace_work(mehdg_ctx* c, bool precond) {
    mehdg_err e;
    const int64_t BS = face_block(c->p), NH = 6 * BS;
    if (!c->d_yl && (e = dev_alloc(c, &c->d_yl, c->n_macro * NH)) != MEHDG_OK) return e;
    if (precond && !c->d_Dinv && (e = dev_alloc(c, &c->d_Dinv, c->n_faces * BS * BS)) != MEHDG_OK) return e;
    return MEHDG_OK;
}

// The matrix-free operator reads the factors of an FP64 condensation.
mehdg_err ensure_matrix_free(mehdg_ctx* c) {
    if (c->stage != 2) return MEHDG_ESTATE;
    int64_t sz[5];
    (void)mehdg_sizes(c->p, sz);
    if (!c->d_mfw) return dev_alloc(c, &c->d_mfw, c->n_macro * sz[2]);
    return MEHDG_OK;
}

}  // namespace

// Partial sums of mehdg_dot_noalloc: a file-scope device array of kDotBlocks
// doubles, one copy per GPU for the life of the process.  Host code reaches
// it only through the address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[kDotBlocks];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocDevices] = {};

// The device address of this GPU's copy of the scratch array, looked up
// once per device with that device current.
mehdg_err scratch_on_device(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return MEHDG_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return MEHDG_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MEHDG_OK;
}

// sums of the partial dot products of nv vectors, in block order
mehdg_err host_dots(mehdg_ctx* c, const double* V, int64_t n, int nv, const double* w, double* out,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_dots, dim3(kDotBlocks), dim3(256), 0, st, V, n, nv, w, c->d_part);
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    if (hipMemcpyAsync(c->h_part.data(), c->d_part, sizeof(double) * nv * kDotBlocks, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    for (int i = 0; i < nv; ++i) {
        double s = 0.0;
        for (int b = 0; b < kDotBlocks; ++b) s += c->h_part[(size_t)i * kDotBlocks + b];
        out[i] = s;
    }
    return MEHDG_OK;
}

// w += sum_i coef[i] V[i]
mehdg_err host_combine(mehdg_ctx* c, const double* V, int64_t n, int nv, const double* coef, double* w,
                       hipStream_t st) {
    for (int i = 0; i < nv; ++i) c->h_coef[i] = coef[i];
    if (hipMemcpyAsync(c->d_coef, c->h_coef.data(), sizeof(double) * nv, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    hipLaunchKernelGGL(k_combine, dim3(vec_grid(n)), dim3(256), 0, st, V, n, nv, c->d_coef, w);
    return hip_ok(hipGetLastError());
}

mehdg_err host_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(vec_grid(n)), dim3(256), 0, st, n, a, x, b, y);
    return hip_ok(hipGetLastError());
}

// Right-preconditioned restarted GMRES with classical Gram-Schmidt applied
// twice; the (restart+1) x restart Hessenberg matrix and its Givens
// rotations live on the host.
template <int P>
mehdg_err trace_gmres(mehdg_ctx* c, const double* Ahat, const double* F, double* x, double rtol, int maxit,
                      int restart, int32_t* iters, double* relres, hipStream_t st) {
    const int64_t N = c->n_faces * face_block(P);
    mehdg_err e;
    if (restart > c->gm_restart) {
        (void)hipFree(c->d_V);
        (void)hipFree(c->d_part);
        (void)hipFree(c->d_coef);
        c->d_V = c->d_part = c->d_coef = nullptr;
        if ((e = dev_alloc(c, &c->d_V, (restart + 1) * N)) != MEHDG_OK ||
            (e = dev_alloc(c, &c->d_part, (int64_t)(restart + 1) * kDotBlocks)) != MEHDG_OK ||
            (e = dev_alloc(c, &c->d_coef, (int64_t)restart + 1)) != MEHDG_OK)
            return e;
        c->gm_restart = restart;
    }
    if (!c->d_w && (e = dev_alloc(c, &c->d_w, N)) != MEHDG_OK) return e;
    if (!c->d_z && (e = dev_alloc(c, &c->d_z, N)) != MEHDG_OK) return e;
    c->h_part.assign((size_t)(restart + 1) * kDotBlocks, 0.0);
    c->h_coef.assign((size_t)restart + 1, 0.0);
    if ((e = trace_launch_precond_setup<P>(c, Ahat, st)) != MEHDG_OK) return e;
    double* V = c->d_V;
    double* w = c->d_w;
    double* z = c->d_z;
    double bn2;
    if ((e = host_dots(c, F, N, 1, F, &bn2, st)) != MEHDG_OK) return e;
    const double bnorm = std::sqrt(bn2);
    int it = 0;
    double res = 0.0;
    if (!(bnorm > 0.0)) {
        if ((e = host_axpby(N, 0.0, F, 0.0, x, st)) != MEHDG_OK) return e;
        *iters = 0;
        *relres = 0.0;
        return MEHDG_OK;
    }
    std::vector<double> H((size_t)(restart + 1) * restart, 0.0), cs(restart), sn(restart), g(restart + 1),
        y(restart), h(restart + 1), h2(restart + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * restart + j]; };
    while (true) {
        // r = F - K x
        if ((e = trace_launch_apply<P>(c, Ahat, x, w, st)) != MEHDG_OK) return e;
        if ((e = host_axpby(N, 1.0, F, -1.0, w, st)) != MEHDG_OK) return e;
        double b2;
        if ((e = host_dots(c, w, N, 1, w, &b2, st)) != MEHDG_OK) return e;
        const double beta = std::sqrt(b2);
        res = beta;
        if (beta <= rtol * bnorm || it >= maxit || !std::isfinite(beta)) break;
        if ((e = host_axpby(N, 1.0 / beta, w, 0.0, V, st)) != MEHDG_OK) return e;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        while (j < restart && it < maxit) {
            double* vj = V + (int64_t)j * N;
            if ((e = trace_launch_precond_apply<P>(c, vj, z, st)) != MEHDG_OK) return e;
            if ((e = trace_launch_apply<P>(c, Ahat, z, w, st)) != MEHDG_OK) return e;
            for (int pass = 0; pass < 2; ++pass) {
                double* hh = pass ? h2.data() : h.data();
                if ((e = host_dots(c, V, N, j + 1, w, hh, st)) != MEHDG_OK) return e;
                for (int i = 0; i <= j; ++i) hh[i] = -hh[i];
                if ((e = host_combine(c, V, N, j + 1, hh, w, st)) != MEHDG_OK) return e;
            }
            for (int i = 0; i <= j; ++i) Hij(i, j) = -(h[i] + h2[i]);
            double hn2;
            if ((e = host_dots(c, w, N, 1, w, &hn2, st)) != MEHDG_OK) return e;
            const double hn = std::sqrt(hn2);
            Hij(j + 1, j) = hn;
            if (hn > 0.0 && (e = host_axpby(N, 1.0 / hn, w, 0.0, V + (int64_t)(j + 1) * N, st)) != MEHDG_OK)
                return e;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
                Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
                Hij(i, j) = t;
            }
            const double rr = std::hypot(Hij(j, j), Hij(j + 1, j));
            cs[j] = rr > 0.0 ? Hij(j, j) / rr : 1.0;
            sn[j] = rr > 0.0 ? Hij(j + 1, j) / rr : 0.0;
            Hij(j, j) = rr;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            res = std::fabs(g[j + 1]);
            ++it;
            ++j;
            if (res <= rtol * bnorm || hn == 0.0) break;
        }
        // x += M^-1 (V y),  H y = g
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= Hij(i, k) * y[k];
            y[i] = s / Hij(i, i);
        }
        if ((e = host_axpby(N, 0.0, F, 0.0, w, st)) != MEHDG_OK) return e;
        if ((e = host_combine(c, V, N, j, y.data(), w, st)) != MEHDG_OK) return e;
        if ((e = trace_launch_precond_apply<P>(c, w, z, st)) != MEHDG_OK) return e;
        if ((e = host_axpby(N, 1.0, z, 1.0, x, st)) != MEHDG_OK) return e;
    }
    *iters = it;
    *relres = res / bnorm;
    return MEHDG_OK;
}

// z ~ K^-1 r by `inner` iterations of GMRES from z = 0, right-preconditioned
// with the face-block Jacobi inverses (no restart, no stopping test: a fixed
// polynomial-plus-Jacobi preconditioner, different for every r, which is
// why the outer solver is flexible).  inner = 0: z = Jacobi(r).
template <int P>
mehdg_err inner_gmres(mehdg_ctx* c, const double* Ahat, const double* r, double* z, int inner, hipStream_t st) {
    const int64_t N = c->n_faces * face_block(P);
    mehdg_err e;
    if (inner <= 0) return trace_launch_precond_apply<P>(c, r, z, st);
    double* V = c->d_iV;
    double* w = c->d_w;
    double b2;
    if ((e = host_dots(c, r, N, 1, r, &b2, st)) != MEHDG_OK) return e;
    const double beta = std::sqrt(b2);
    if (!(beta > 0.0) || !std::isfinite(beta)) return host_axpby(N, 0.0, r, 0.0, z, st);
    if ((e = host_axpby(N, 1.0 / beta, r, 0.0, V, st)) != MEHDG_OK) return e;
    std::vector<double> H((size_t)(inner + 1) * inner, 0.0), cs(inner), sn(inner), g(inner + 1, 0.0), y(inner),
        h(inner + 1), h2(inner + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * inner + j]; };
    g[0] = beta;
    int j = 0;
    for (; j < inner; ++j) {
        double* vj = V + (int64_t)j * N;
        if ((e = trace_launch_precond_apply<P>(c, vj, z, st)) != MEHDG_OK) return e;
        if ((e = trace_launch_apply<P>(c, Ahat, z, w, st, true)) != MEHDG_OK) return e;
        for (int pass = 0; pass < 2; ++pass) {
            double* hh = pass ? h2.data() : h.data();
            if ((e = host_dots(c, V, N, j + 1, w, hh, st)) != MEHDG_OK) return e;
            for (int i = 0; i <= j; ++i) hh[i] = -hh[i];
            if ((e = host_combine(c, V, N, j + 1, hh, w, st)) != MEHDG_OK) return e;
        }
        for (int i = 0; i <= j; ++i) Hij(i, j) = -(h[i] + h2[i]);
        double hn2;
        if ((e = host_dots(c, w, N, 1, w, &hn2, st)) != MEHDG_OK) return e;
        const double hn = std::sqrt(hn2);
        Hij(j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
            Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
            Hij(i, j) = t;
        }
        const double rr = std::hypot(Hij(j, j), Hij(j + 1, j));
        cs[j] = rr > 0.0 ? Hij(j, j) / rr : 1.0;
        sn[j] = rr > 0.0 ? Hij(j + 1, j) / rr : 0.0;
        Hij(j, j) = rr;
        Hij(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        if (!(hn > 0.0) || j + 1 == inner) {
            ++j;
            break;
        }
        if ((e = host_axpby(N, 1.0 / hn, w, 0.0, V + (int64_t)(j + 1) * N, st)) != MEHDG_OK) return e;
    }
    for (int i = j - 1; i >= 0; --i) {
        double sacc = g[i];
        for (int k = i + 1; k < j; ++k) sacc -= Hij(i, k) * y[k];
        y[i] = Hij(i, i) != 0.0 ? sacc / Hij(i, i) : 0.0;
    }
    // z = Jacobi (V y)
    if ((e = host_axpby(N, 0.0, r, 0.0, w, st)) != MEHDG_OK) return e;
    if ((e = host_combine(c, V, N, j, y.data(), w, st)) != MEHDG_OK) return e;
    return trace_launch_precond_apply<P>(c, w, z, st);
}

// Flexible GMRES (Saad 1993) on K dVhat = F, Sec. 6.4: the preconditioner of
// every outer direction is `inner` iterations of the inner GMRES above, so
// the preconditioned directions Z_j are kept; classical Gram-Schmidt twice;
// x += Z y at every restart.  Ahat NULL: K applied matrix-free from the
// stored factors and the Jacobi blocks formed from them.
template <int P>
mehdg_err trace_fgmres(mehdg_ctx* c, const double* Ahat, const double* F, double* x, double rtol, int maxit,
                       int restart, int inner, int32_t* iters, int32_t* inner_total, double* relres,
                       hipStream_t st) {
    const int64_t N = c->n_faces * face_block(P);
    mehdg_err e;
    const int nbasis = restart > inner ? restart : inner;
    if (nbasis > c->gm_restart) {
        (void)hipFree(c->d_V);
        (void)hipFree(c->d_part);
        (void)hipFree(c->d_coef);
        c->d_V = c->d_part = c->d_coef = nullptr;
        if ((e = dev_alloc(c, &c->d_V, (nbasis + 1) * N)) != MEHDG_OK ||
            (e = dev_alloc(c, &c->d_part, (int64_t)(nbasis + 1) * kDotBlocks)) != MEHDG_OK ||
            (e = dev_alloc(c, &c->d_coef, (int64_t)nbasis + 1)) != MEHDG_OK)
            return e;
        c->gm_restart = nbasis;
    }
    if (restart > c->fg_restart) {
        (void)hipFree(c->d_fZ);
        c->d_fZ = nullptr;
        if ((e = dev_alloc(c, &c->d_fZ, (int64_t)restart * N)) != MEHDG_OK) return e;
        c->fg_restart = restart;
    }
    if (inner > c->fg_inner) {
        (void)hipFree(c->d_iV);
        c->d_iV = nullptr;
        if ((e = dev_alloc(c, &c->d_iV, (int64_t)(inner + 1) * N)) != MEHDG_OK) return e;
        c->fg_inner = inner;
    }
    if (!c->d_w && (e = dev_alloc(c, &c->d_w, N)) != MEHDG_OK) return e;
    if (!c->d_z && (e = dev_alloc(c, &c->d_z, N)) != MEHDG_OK) return e;
    c->h_part.assign((size_t)(nbasis + 1) * kDotBlocks, 0.0);
    c->h_coef.assign((size_t)nbasis + 1, 0.0);
    if ((e = trace_launch_precond_setup<P>(c, Ahat, st)) != MEHDG_OK) return e;
    if (!Ahat && c->inner_prec == MEHDG_FP32_IR && inner > 0 && (e = ensure_mf32<P>(c, st)) != MEHDG_OK) return e;
    double* V = c->d_V;
    double* Z = c->d_fZ;
    double* w = c->d_w;
    double bn2;
    if ((e = host_dots(c, F, N, 1, F, &bn2, st)) != MEHDG_OK) return e;
    const double bnorm = std::sqrt(bn2);
    int it = 0, itot = 0;
    double res = 0.0;
    *inner_total = 0;
    if (!(bnorm > 0.0)) {
        if ((e = host_axpby(N, 0.0, F, 0.0, x, st)) != MEHDG_OK) return e;
        *iters = 0;
        *relres = 0.0;
        return MEHDG_OK;
    }
    std::vector<double> H((size_t)(restart + 1) * restart, 0.0), cs(restart), sn(restart), g(restart + 1),
        y(restart), h(restart + 1), h2(restart + 1);
    auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * restart + j]; };
    while (true) {
        if ((e = trace_launch_apply<P>(c, Ahat, x, w, st)) != MEHDG_OK) return e;
        if ((e = host_axpby(N, 1.0, F, -1.0, w, st)) != MEHDG_OK) return e;
        double b2;
        if ((e = host_dots(c, w, N, 1, w, &b2, st)) != MEHDG_OK) return e;
        const double beta = std::sqrt(b2);
        res = beta;
        if (beta <= rtol * bnorm || it >= maxit || !std::isfinite(beta)) break;
        if ((e = host_axpby(N, 1.0 / beta, w, 0.0, V, st)) != MEHDG_OK) return e;
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        while (j < restart && it < maxit) {
            double* zj = Z + (int64_t)j * N;
            if ((e = inner_gmres<P>(c, Ahat, V + (int64_t)j * N, zj, inner, st)) != MEHDG_OK) return e;
            itot += inner;
            if ((e = trace_launch_apply<P>(c, Ahat, zj, w, st)) != MEHDG_OK) return e;
            for (int pass = 0; pass < 2; ++pass) {
                double* hh = pass ? h2.data() : h.data();
                if ((e = host_dots(c, V, N, j + 1, w, hh, st)) != MEHDG_OK) return e;
                for (int i = 0; i <= j; ++i) hh[i] = -hh[i];
                if ((e = host_combine(c, V, N, j + 1, hh, w, st)) != MEHDG_OK) return e;
            }
            for (int i = 0; i <= j; ++i) Hij(i, j) = -(h[i] + h2[i]);
            double hn2;
            if ((e = host_dots(c, w, N, 1, w, &hn2, st)) != MEHDG_OK) return e;
            const double hn = std::sqrt(hn2);
            Hij(j + 1, j) = hn;
            if (hn > 0.0 && (e = host_axpby(N, 1.0 / hn, w, 0.0, V + (int64_t)(j + 1) * N, st)) != MEHDG_OK)
                return e;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
                Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
                Hij(i, j) = t;
            }
            const double rr = std::hypot(Hij(j, j), Hij(j + 1, j));
            cs[j] = rr > 0.0 ? Hij(j, j) / rr : 1.0;
            sn[j] = rr > 0.0 ? Hij(j + 1, j) / rr : 0.0;
            Hij(j, j) = rr;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            res = std::fabs(g[j + 1]);
            ++it;
            ++j;
            if (res <= rtol * bnorm || hn == 0.0) break;
        }
        // x += Z y,  H y = g
        for (int i = j - 1; i >= 0; --i) {
            double sacc = g[i];
            for (int k = i + 1; k < j; ++k) sacc -= Hij(i, k) * y[k];
            y[i] = sacc / Hij(i, i);
        }
        if ((e = host_combine(c, Z, N, j, y.data(), x, st)) != MEHDG_OK) return e;
    }
    *iters = it;
    *inner_total = itot;
    *relres = res / bnorm;
    return MEHDG_OK;
}

}  // namespace

// --------------------------------------------------------------------------
// condensation of tetrahedral bordered matrices (tet_cond.hpp)
// --------------------------------------------------------------------------
template <int P>
void tet_cond_sizes_of(int64_t out[4]) {
    out[0] = Bdims<P>::rows;
    out[1] = Bdims<P>::ld;
    out[2] = Panel<P>::TRI;
    out[3] = Panel<P>::PERM;
}

bool tet_cond_sizes(int p, int64_t out[4]) {
    switch (p) {
        case 1: tet_cond_sizes_of<TET_TAG + 1>(out); return true;
        case 2: tet_cond_sizes_of<TET_TAG + 2>(out); return true;
        case 3: tet_cond_sizes_of<TET_TAG + 3>(out); return true;
        default: return false;
    }
}

mehdg_err tet_condense(int p, const TetCondWork& w, double* Ahat, double* bhat, hipStream_t st) {
    // a context that only lends the workspace pointers to the launchers;
    // nothing is allocated or freed through it
    mehdg_ctx c;
    c.p = TET_TAG + p;
    c.n_macro = w.n_macro;
    c.d_B = w.B;
    c.d_ipiv = w.ipiv;
    c.d_tri = w.tri;
    c.d_perm = w.perm;
    c.d_status = w.status;
    mehdg_err e = MEHDG_EINVAL;
    int64_t NH = 0;
    switch (p) {
        case 1: e = launch_condense<TET_TAG + 1>(&c, Ahat, bhat, st); NH = Dims<TET_TAG + 1>::NH; break;
        case 2: e = launch_condense<TET_TAG + 2>(&c, Ahat, bhat, st); NH = Dims<TET_TAG + 2>::NH; break;
        case 3: e = launch_condense<TET_TAG + 3>(&c, Ahat, bhat, st); NH = Dims<TET_TAG + 3>::NH; break;
        default: break;
    }
    if (e == MEHDG_OK) e = launch_poison(&c, PoisonArgs{{Ahat, bhat, nullptr, nullptr}, {NH * NH, NH, 0, 0}}, st);
    return e;
}

mehdg_err tet_condense_rhs(int p, const TetCondWork& w, const double* r_v, const double* r_hat, double* bhat,
                           hipStream_t st) {
    mehdg_ctx c;   // lends the workspace pointers to the launcher, as in tet_condense
    c.p = TET_TAG + p;
    c.n_macro = w.n_macro;
    c.d_B = w.B;
    c.d_ipiv = w.ipiv;
    c.d_status = w.status;
    mehdg_err e = MEHDG_EINVAL;
    int64_t NH = 0;
    switch (p) {
        case 1: e = launch_fsolve<TET_TAG + 1>(&c, r_v, r_hat, bhat, st); NH = Dims<TET_TAG + 1>::NH; break;
        case 2: e = launch_fsolve<TET_TAG + 2>(&c, r_v, r_hat, bhat, st); NH = Dims<TET_TAG + 2>::NH; break;
        case 3: e = launch_fsolve<TET_TAG + 3>(&c, r_v, r_hat, bhat, st); NH = Dims<TET_TAG + 3>::NH; break;
        default: break;
    }
    if (e == MEHDG_OK) e = launch_poison(&c, PoisonArgs{{bhat, nullptr, nullptr, nullptr}, {NH, 0, 0, 0}}, st);
    return e;
}

mehdg_err poison_flagged(const int32_t* status, int64_t n_macro, double* a, int64_t per_a, double* b,
                         int64_t per_b, hipStream_t st) {
    hipLaunchKernelGGL(k_poison, dim3((unsigned)n_macro), dim3(256), 0, st, status,
                       PoisonArgs{{a, b, nullptr, nullptr}, {per_a, per_b, 0, 0}});
    return hip_ok(hipGetLastError());
}

extern "C" {

mehdg_err mehdg_sizes(int32_t p, int64_t out[5]) {
    if (!out || p < 1 || p > kMaxP) return MEHDG_EINVAL;
    const int64_t n1d = 2 * p + 1;
    out[0] = n1d * n1d * n1d;
    out[1] = n1d * n1d;
    out[2] = 5 * out[0];
    out[3] = 15 * out[0];
    out[4] = 30 * out[1];
    return MEHDG_OK;
}

static void drop_marks(mehdg_ctx* c) {
    for (auto& mk : c->marks) {
        (void)hipEventDestroy(mk.a);
        (void)hipEventDestroy(mk.b);
    }
    c->marks.clear();
}

mehdg_err mehdg_destroy(mehdg_ctx* c) {
    if (!c) return MEHDG_EINVAL;
    drop_marks(c);
    (void)hipFree(c->base_h);
    (void)hipFree(c->d_tab);
    (void)hipFree(c->base_status);
    (void)hipFree(c->base_bc);
    (void)hipFree(c->d_scratch);
    (void)hipFree(c->d_coefV);
    (void)hipFree(c->d_coefF);
    (void)hipFree(c->d_minvrq);
    (void)hipFree(c->d_ipiv);
    (void)hipFree(c->d_tri);
    (void)hipFree(c->d_perm);
    (void)hipFree(c->d_B);
    (void)hipFree(c->d_fid);
    (void)hipFree(c->d_side);
    (void)hipFree(c->d_yl);
    (void)hipFree(c->d_mfw);
    (void)hipFree(c->d_fZ);
    (void)hipFree(c->d_iV);
    (void)hipFree(c->d_mf32);
    (void)hipFree(c->d_Dinv);
    (void)hipFree(c->d_V);
    (void)hipFree(c->d_w);
    (void)hipFree(c->d_z);
    (void)hipFree(c->d_part);
    (void)hipFree(c->d_coef);
    (void)hipFree(c->d_slo);
    (void)hipFree(c->d_lperm);
    (void)hipFree(c->d_ltri);
    (void)hipFree(c->d_zb);
    (void)hipFree(c->d_rb);
    (void)hipFree(c->d_yb);
    (void)hipFree(c->d_nrm);
    (void)hipFree(c->d_flags);
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
    bool walls = false;
    if (mesh->face_bc) {
        for (int64_t i = 0; i < 6 * mesh->n_macro; ++i) {
            if (mesh->face_bc[i] > 1) return MEHDG_EINVAL;
            walls = walls || mesh->face_bc[i] == 1;
        }
        if (walls && !(prm->T_wall > 0.0)) return MEHDG_EINVAL;
    }
    mehdg_ctx* c = new (std::nothrow) mehdg_ctx();
    if (!c) return MEHDG_ENOMEM;
    c->p = mesh->p;
    c->n_macro = mesh->n_macro;
    c->prm = *prm;
    for (int site = 0; site < MEHDG_NTILE_SITES; ++site) c->tile[site] = kTileTable[c->p][site];
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
    if (!build_tables(c->p, c->tab)) {
        delete c;
        return MEHDG_EINVAL;
    }
    mehdg_err e;
    if ((e = dev_alloc(c, &c->base_h, 3 * c->n_macro)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_tab, 1)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->base_status, c->n_macro)) != MEHDG_OK ||
        (e = dev_alloc(c, &c->d_scratch, c->n_macro * res_scratch_doubles(c->p))) != MEHDG_OK) {
        mehdg_destroy(c);
        return e;
    }
    c->d_h = c->base_h;
    c->d_status = c->base_status;
    if (walls && ((e = dev_alloc(c, &c->base_bc, 6 * c->n_macro)) != MEHDG_OK ||
                  hipMemcpy(c->base_bc, mesh->face_bc, 6 * c->n_macro, hipMemcpyHostToDevice) != hipSuccess)) {
        mehdg_destroy(c);
        return e != MEHDG_OK ? e : MEHDG_EHIP;
    }
    c->d_bc = c->base_bc;
    c->cap = c->n_macro;
    c->base_gT = c->dp.gT;
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
    if (want_blocks < 0 || want_blocks > 2) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int mode = want_blocks;
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_assemble<1>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, mode, st); break;
        case 2: e = launch_assemble<2>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, mode, st); break;
        case 3: e = launch_assemble<3>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, mode, st); break;
        case 4:
            if (mode != 2) e = launch_assemble<4>(c, v, vhat, q, v_old, R_q, R_v, R_vhat, entropy, mode, st);
            break;
        default: break;
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{R_q, R_v, R_vhat, entropy}, {sz[3], sz[2], sz[4], 1}}, st);
    }
    if (e == MEHDG_OK && mode == 1) c->stage = 1;
    if (e == MEHDG_OK && mode != 0) c->have_coef = true;
    return e;
}

mehdg_err mehdg_jvp(mehdg_ctx* c, const double* dv, const double* dvhat, const double* dq, double* JR_q,
                    double* JR_v, double* JR_vhat, mehdg_stream stream) {
    if (!c || !dv || !dvhat || !JR_q || !JR_v || !JR_vhat) return MEHDG_EINVAL;
    if (!c->have_coef) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_jvp<1>(c, dv, dvhat, dq, JR_q, JR_v, JR_vhat, st); break;
        case 2: e = launch_jvp<2>(c, dv, dvhat, dq, JR_q, JR_v, JR_vhat, st); break;
        case 3: e = launch_jvp<3>(c, dv, dvhat, dq, JR_q, JR_v, JR_vhat, st); break;
        default: break;
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{JR_q, JR_v, JR_vhat, nullptr}, {sz[3], sz[2], sz[4], 0}}, st);
    }
    return e;
}

mehdg_err mehdg_vjp(mehdg_ctx* c, const double* w_q, const double* w_v, const double* w_vhat, double* g_q,
                    double* g_v, double* g_vhat, mehdg_stream stream) {
    if (!c || !w_v || !w_vhat || !g_v || !g_vhat || (w_q == nullptr) != (g_q == nullptr)) return MEHDG_EINVAL;
    if (!c->have_coef) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_vjp<1>(c, w_q, w_v, w_vhat, g_q, g_v, g_vhat, st); break;
        case 2: e = launch_vjp<2>(c, w_q, w_v, w_vhat, g_q, g_v, g_vhat, st); break;
        case 3: e = launch_vjp<3>(c, w_q, w_v, w_vhat, g_q, g_v, g_vhat, st); break;
        default: break;
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{g_q, g_v, g_vhat, nullptr}, {sz[3], sz[2], sz[4], 0}}, st);
    }
    return e;
}

mehdg_err mehdg_condense(mehdg_ctx* c, int32_t prec, double* Ahat, double* bhat, mehdg_stream stream) {
    if (!c || !bhat || prec < MEHDG_FP64 || prec > MEHDG_BF16_IR) return MEHDG_EINVAL;
    if (prec != MEHDG_FP64 && (!(c->prm.ir_tol > 0.0) || c->prm.ir_maxit < 1 || c->p > 3)) return MEHDG_EINVAL;
    if (c->stage != 1) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    const bool bf = prec == MEHDG_BF16_IR;
    if (prec == MEHDG_FP64) {
        switch (c->p) {
            case 1: e = launch_condense<1>(c, Ahat, bhat, st); break;
            case 2: e = launch_condense<2>(c, Ahat, bhat, st); break;
            case 3: e = launch_condense<3>(c, Ahat, bhat, st); break;
            case 4: e = launch_condense<4>(c, Ahat, bhat, st); break;
            default: break;
        }
    } else {
        switch (c->p) {
            case 1: e = launch_condense_mixed<1>(c, bf, Ahat, bhat, st); break;
            case 2: e = launch_condense_mixed<2>(c, bf, Ahat, bhat, st); break;
            case 3: e = launch_condense_mixed<3>(c, bf, Ahat, bhat, st); break;
            default: break;
        }
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{Ahat, bhat, nullptr, nullptr}, {sz[4] * sz[4], sz[4], 0, 0}}, st);
    }
    if (e == MEHDG_OK) {
        c->stage = prec == MEHDG_FP64 ? 2 : 3;
        if (prec == MEHDG_FP64) ++c->cond_count;
    } else {
        c->stage = 0;   // the bordered matrices are partly factored: assemble again
    }
    return e;
}

int32_t mehdg_ir_iterations(const mehdg_ctx* c) { return c ? c->ir_iters : 0; }

mehdg_err mehdg_condense_rhs(mehdg_ctx* c, const double* r_v, const double* r_hat, double* bhat,
                             mehdg_stream stream) {
    if (!c || !r_v || !bhat) return MEHDG_EINVAL;
    if (c->stage != 2) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_fsolve<1>(c, r_v, r_hat, bhat, st); break;
        case 2: e = launch_fsolve<2>(c, r_v, r_hat, bhat, st); break;
        case 3: e = launch_fsolve<3>(c, r_v, r_hat, bhat, st); break;
        default: break;
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{bhat, nullptr, nullptr, nullptr}, {sz[4], 0, 0, 0}}, st);
    }
    return e;
}

mehdg_err mehdg_recover(mehdg_ctx* c, const double* R_q, const double* dvhat, double* dv, double* dq,
                        mehdg_stream stream) {
    if (!c || !R_q || !dvhat || !dv || !dq) return MEHDG_EINVAL;
    if (c->stage != 2 && c->stage != 3) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    if (c->stage == 3) {
        switch (c->p) {
            case 1: e = launch_recover_z<1>(c, R_q, dvhat, dv, dq, st); break;
            case 2: e = launch_recover_z<2>(c, R_q, dvhat, dv, dq, st); break;
            case 3: e = launch_recover_z<3>(c, R_q, dvhat, dv, dq, st); break;
            default: break;
        }
    } else {
        switch (c->p) {
            case 1: e = launch_recover<1>(c, R_q, dvhat, dv, dq, st); break;
            case 2: e = launch_recover<2>(c, R_q, dvhat, dv, dq, st); break;
            case 3: e = launch_recover<3>(c, R_q, dvhat, dv, dq, st); break;
            case 4: e = launch_recover<4>(c, R_q, dvhat, dv, dq, st); break;
            default: break;
        }
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{dv, dq, nullptr, nullptr}, {sz[2], sz[3], 0, 0}}, st);
    }
    return e;
}

mehdg_err mehdg_copy_bordered(mehdg_ctx* c, int64_t m, double* out, int64_t* rows, int64_t* ld) {
    if (!c || m < 0 || m >= c->n_macro || !rows || !ld) return MEHDG_EINVAL;
    *rows = bordered_rows(c->p);
    *ld = bordered_ld(c->p);
    if (!out) return MEHDG_OK;
    if (!c->d_B || c->stage < 1) return MEHDG_ESTATE;
    const int64_t count = (*rows) * (*ld);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(out, c->d_B + m * count, count * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return MEHDG_EHIP;
    return MEHDG_OK;
}

mehdg_err mehdg_load_bordered(mehdg_ctx* c, int64_t m, const double* in) {
    if (!c || m < 0 || m >= c->n_macro || !in) return MEHDG_EINVAL;
    if (!c->d_B || c->stage < 1) return MEHDG_ESTATE;
    const int64_t count = bordered_rows(c->p) * bordered_ld(c->p);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(c->d_B + m * count, in, count * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return MEHDG_EHIP;
    c->stage = 1;
    return MEHDG_OK;
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

// Views for the batch calls (batch_view.hpp): the context works on the first n
// of its cap macros with mesh sizes, wall flags and status codes read from
// the caller's device arrays.
mehdg_err mehdg_batch_ctx_view(mehdg_ctx* c, int64_t n, const double* d_h, const uint8_t* d_bc, int32_t* d_status) {
    if (!c || n < 1 || n > c->cap || !d_h || !d_status) return MEHDG_EINVAL;
    if (d_bc && !(c->prm.T_wall > 0.0)) return MEHDG_EINVAL;
    c->n_macro = n;
    c->d_h = const_cast<double*>(d_h);
    c->d_bc = const_cast<uint8_t*>(d_bc);
    c->d_status = d_status;
    c->dp.gT = d_bc ? c->prm.gamma / c->prm.T_wall : 0.0;
    return MEHDG_OK;
}

mehdg_err mehdg_batch_ctx_unview(mehdg_ctx* c) {
    if (!c) return MEHDG_EINVAL;
    c->n_macro = c->cap;
    c->d_h = c->base_h;
    c->d_bc = c->base_bc;
    c->d_status = c->base_status;
    c->dp.gT = c->base_gT;
    return MEHDG_OK;
}

int64_t mehdg_batch_ctx_bytes(int p) {
    switch (p) {
        case 1: return ctx_macro_bytes<1>();
        case 2: return ctx_macro_bytes<2>();
        case 3: return ctx_macro_bytes<3>();
        case 4: return ctx_macro_bytes<4>();
        default: return 0;
    }
}

mehdg_err mehdg_batch_ctx_residual(mehdg_ctx* const* ctxs, const mehdg_batch_slices* sl, int ng,
                                   unsigned long long* counter, mehdg_stream stream) {
    if (!ctxs || !sl || ng < 1 || ng > 4 || !counter) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int order[4];
    for (int i = 0; i < ng; ++i) {
        if (!ctxs[i] || !sl[i].v || !sl[i].vhat || !sl[i].v_old || !sl[i].R_q || !sl[i].R_v || !sl[i].R_vhat ||
            !sl[i].entropy)
            return MEHDG_EINVAL;
        order[i] = i;
    }
    std::sort(order, order + ng, [&](int a, int b2) { return ctxs[a]->p > ctxs[b2]->p; });
    ResidualBatch b{};
    b.ng = ng;
    int64_t pos = 0;
    size_t lds = 0;
    for (int k = 0; k < ng; ++k) {
        mehdg_ctx* c = ctxs[order[k]];
        const mehdg_batch_slices& s = sl[order[k]];
        mehdg_err e = MEHDG_EINVAL;
        size_t l = 0;
        switch (c->p) {
            case 1: e = ensure_block_workspace<1>(c); l = res_lds<1>(); break;
            case 2: e = ensure_block_workspace<2>(c); l = res_lds<2>(); break;
            case 3: e = ensure_block_workspace<3>(c); l = res_lds<3>(); break;
            case 4: e = ensure_block_workspace<4>(c); l = res_lds<4>(); break;
            default: break;
        }
        if (e != MEHDG_OK) return e;
        lds = std::max(lds, l);
        ResidualGroup& g = b.g[k];
        g.p = c->p;
        g.pr = c->dp;
        g.v = s.v;
        g.vhat = s.vhat;
        g.v_old = s.v_old;
        g.hs = c->d_h;
        g.tab = c->d_tab;
        g.R_q = s.R_q;
        g.R_v = s.R_v;
        g.R_vh = s.R_vhat;
        g.ent = s.entropy;
        g.scratch = c->d_scratch;
        g.coefV = c->d_coefV;
        g.coefF = c->d_coefF;
        g.bc = c->d_bc;
        g.status = c->d_status;
        b.first[k] = pos;
        pos += c->n_macro;
    }
    b.first[ng] = pos;
    if (pos == 0) return MEHDG_OK;
    if (!allow_lds(&k_residual_batch, lds)) return MEHDG_EHIP;
    // as many workgroups as the CUs hold at once with this LDS (at most 8 of 256 threads)
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, 163840 / (lds + 1024)));
    const int64_t grid = std::min<int64_t>(pos, (int64_t)device_cus() * per_cu);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
    hipLaunchKernelGGL(k_residual_batch, dim3((unsigned)grid), dim3(256), lds, st, b, counter);
    return hip_ok(hipGetLastError());
}

mehdg_err mehdg_batch_ctx_rows(mehdg_ctx* c, const mehdg_batch_slices* s, mehdg_stream stream) {
    if (!c || !s || !s->R_q || !s->R_v || !s->R_vhat || !s->entropy) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    mehdg_err e = MEHDG_EINVAL;
    switch (c->p) {
        case 1: e = launch_rows<1>(c, s->R_q, s->R_v, s->R_vhat, st); break;
        case 2: e = launch_rows<2>(c, s->R_q, s->R_v, s->R_vhat, st); break;
        case 3: e = launch_rows<3>(c, s->R_q, s->R_v, s->R_vhat, st); break;
        case 4: e = launch_rows<4>(c, s->R_q, s->R_v, s->R_vhat, st); break;
        default: break;
    }
    if (e == MEHDG_OK) {
        int64_t sz[5];
        (void)mehdg_sizes(c->p, sz);
        e = launch_poison(c, PoisonArgs{{s->R_q, s->R_v, s->R_vhat, s->entropy}, {sz[3], sz[2], sz[4], 1}}, st);
    }
    if (e == MEHDG_OK) {
        c->stage = 1;
        c->have_coef = true;
    }
    return e;
}

mehdg_err mehdg_tile_variants(int32_t* count, int32_t* shapes) {
    if (!count) return MEHDG_EINVAL;
    *count = kGemmVariants;
    if (shapes) {
#define MEHDG_SHAPE_VARIANT(i, wm, wn, bi, bj, kc, occ) \
    {                                                   \
        const int32_t v[6] = {wm, wn, bi, bj, kc, occ}; \
        for (int k = 0; k < 6; ++k) shapes[6 * i + k] = v[k]; \
    }
        MEHDG_GEMM_VARIANTS(MEHDG_SHAPE_VARIANT)
#undef MEHDG_SHAPE_VARIANT
    }
    return MEHDG_OK;
}

mehdg_err mehdg_set_tile(mehdg_ctx* c, int32_t site, int32_t variant) {
    if (!c || site < 0 || site >= MEHDG_NTILE_SITES || variant < -1 || variant >= kGemmVariants)
        return MEHDG_EINVAL;
    c->tile[site] = variant < 0 ? kTileTable[c->p][site] : variant;
    return MEHDG_OK;
}

mehdg_err mehdg_get_tile(const mehdg_ctx* c, int32_t site, int32_t* variant) {
    if (!c || !variant || site < 0 || site >= MEHDG_NTILE_SITES) return MEHDG_EINVAL;
    *variant = c->tile[site];
    return MEHDG_OK;
}

mehdg_err mehdg_set_lu_depth(mehdg_ctx* c, int32_t depth) {
    if (!c || depth < 0 || depth > 1024) return MEHDG_EINVAL;
    c->lu_depth = depth;
    return MEHDG_OK;
}

mehdg_err mehdg_get_lu_depth(const mehdg_ctx* c, int32_t* depth) {
    if (!c || !depth) return MEHDG_EINVAL;
    int w = 0;
    switch (c->p) {
        case 1: w = lu_group_width<1>(c); break;
        case 2: w = lu_group_width<2>(c); break;
        case 3: w = lu_group_width<3>(c); break;
        case 4: w = lu_group_width<4>(c); break;
        default: return MEHDG_EINVAL;
    }
    *depth = w / Panel<1>::OB;
    return MEHDG_OK;
}


mehdg_err mehdg_trace_setup(mehdg_ctx* c, const int64_t* face_ids, int64_t n_faces) {
    if (!c || !face_ids || n_faces <= 0) return MEHDG_EINVAL;
    const int64_t M = c->n_macro;
    // wall flags of the macros' faces (host copy of the mesh's face_bc)
    std::vector<uint8_t> bc;
    if (c->d_bc) {
        bc.resize((size_t)(6 * M));
        if (hipMemcpy(bc.data(), c->d_bc, 6 * M, hipMemcpyDeviceToHost) != hipSuccess) return MEHDG_EHIP;
    }
    std::vector<int64_t> side((size_t)n_faces * 4, -1);
    std::vector<int> cnt((size_t)n_faces, 0), walls((size_t)n_faces, 0);
    for (int64_t m = 0; m < M; ++m)
        for (int f = 0; f < 6; ++f) {
            const int64_t g = face_ids[m * 6 + f];
            if (g < 0 || g >= n_faces || cnt[g] >= 2) return MEHDG_EINVAL;
            side[g * 4 + 2 * cnt[g]] = m;
            side[g * 4 + 2 * cnt[g] + 1] = f;
            ++cnt[g];
            if (!bc.empty() && bc[m * 6 + f]) ++walls[g];
        }
    // an interior face has two sides and no wall; a wall face is a face of
    // one macro only (side 2 = -1)
    for (int64_t g = 0; g < n_faces; ++g)
        if (!((cnt[g] == 2 && walls[g] == 0) || (cnt[g] == 1 && walls[g] == 1))) return MEHDG_EINVAL;
    (void)hipFree(c->d_fid);
    (void)hipFree(c->d_side);
    (void)hipFree(c->d_Dinv);
    (void)hipFree(c->d_w);
    (void)hipFree(c->d_z);
    (void)hipFree(c->d_V);
    c->d_fid = c->d_side = nullptr;
    c->d_Dinv = c->d_w = c->d_z = c->d_V = nullptr;
    c->gm_restart = 0;
    c->n_faces = n_faces;
    mehdg_err e;
    if ((e = dev_alloc(c, &c->d_fid, M * 6)) != MEHDG_OK || (e = dev_alloc(c, &c->d_side, n_faces * 4)) != MEHDG_OK)
        return e;
    if (hipMemcpy(c->d_fid, face_ids, sizeof(int64_t) * M * 6, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_side, side.data(), sizeof(int64_t) * n_faces * 4, hipMemcpyHostToDevice) != hipSuccess)
        return MEHDG_EHIP;
    return ensure_trace_work(c, false);
}

mehdg_err mehdg_trace_rhs(mehdg_ctx* c, const double* bhat, double* F, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!bhat || !F) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: hipLaunchKernelGGL(k_face_sum<1>, dim3((unsigned)c->n_faces), dim3(128), 0, st, bhat, c->d_side, F, c->n_faces); break;
        case 2: hipLaunchKernelGGL(k_face_sum<2>, dim3((unsigned)c->n_faces), dim3(128), 0, st, bhat, c->d_side, F, c->n_faces); break;
        case 3: hipLaunchKernelGGL(k_face_sum<3>, dim3((unsigned)c->n_faces), dim3(128), 0, st, bhat, c->d_side, F, c->n_faces); break;
        default: return MEHDG_EINVAL;
    }
    return hip_ok(hipGetLastError());
}

mehdg_err mehdg_trace_gather(mehdg_ctx* c, const double* xg, double* xl, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!xg || !xl) return MEHDG_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)c->n_macro);
    switch (c->p) {
        case 1: hipLaunchKernelGGL(k_face_gather<1>, grid, dim3(256), 0, st, xg, c->d_fid, xl, (int64_t)c->n_macro); break;
        case 2: hipLaunchKernelGGL(k_face_gather<2>, grid, dim3(256), 0, st, xg, c->d_fid, xl, (int64_t)c->n_macro); break;
        case 3: hipLaunchKernelGGL(k_face_gather<3>, grid, dim3(256), 0, st, xg, c->d_fid, xl, (int64_t)c->n_macro); break;
        default: return MEHDG_EINVAL;
    }
    return hip_ok(hipGetLastError());
}

mehdg_err mehdg_trace_apply(mehdg_ctx* c, const double* Ahat, const double* x, double* y, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!x || !y) return MEHDG_EINVAL;
    if (!Ahat && (e = ensure_matrix_free(c)) != MEHDG_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: return trace_launch_apply<1>(c, Ahat, x, y, st);
        case 2: return trace_launch_apply<2>(c, Ahat, x, y, st);
        case 3: return trace_launch_apply<3>(c, Ahat, x, y, st);
        default: return MEHDG_EINVAL;
    }
}

mehdg_err mehdg_trace_precond_setup(mehdg_ctx* c, const double* Ahat, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!Ahat && (e = ensure_matrix_free(c)) != MEHDG_OK) return e;
    if ((e = ensure_trace_work(c, true)) != MEHDG_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: return trace_launch_precond_setup<1>(c, Ahat, st);
        case 2: return trace_launch_precond_setup<2>(c, Ahat, st);
        case 3: return trace_launch_precond_setup<3>(c, Ahat, st);
        default: return MEHDG_EINVAL;
    }
}

mehdg_err mehdg_trace_precond_apply(mehdg_ctx* c, const double* r, double* z, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!r || !z) return MEHDG_EINVAL;
    if (!c->d_Dinv) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: return trace_launch_precond_apply<1>(c, r, z, st);
        case 2: return trace_launch_precond_apply<2>(c, r, z, st);
        case 3: return trace_launch_precond_apply<3>(c, r, z, st);
        default: return MEHDG_EINVAL;
    }
}

mehdg_err mehdg_trace_solve(mehdg_ctx* c, const double* Ahat, const double* F, double* x, double rtol,
                            int32_t maxit, int32_t restart, int32_t* iters, double* relres, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!F || !x || !iters || !relres || !(rtol > 0.0) || maxit < 0 || restart < 1 || restart > kMaxRestart)
        return MEHDG_EINVAL;
    if (!Ahat && (e = ensure_matrix_free(c)) != MEHDG_OK) return e;
    if ((e = ensure_trace_work(c, true)) != MEHDG_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: return trace_gmres<1>(c, Ahat, F, x, rtol, maxit, restart, iters, relres, st);
        case 2: return trace_gmres<2>(c, Ahat, F, x, rtol, maxit, restart, iters, relres, st);
        case 3: return trace_gmres<3>(c, Ahat, F, x, rtol, maxit, restart, iters, relres, st);
        default: return MEHDG_EINVAL;
    }
}

mehdg_err mehdg_trace_set_inner_precision(mehdg_ctx* c, int32_t prec) {
    if (!c || (prec != MEHDG_FP64 && prec != MEHDG_FP32_IR)) return MEHDG_EINVAL;
    c->inner_prec = prec;
    return MEHDG_OK;
}

mehdg_err mehdg_trace_solve_fgmres(mehdg_ctx* c, const double* Ahat, const double* F, double* x, double rtol,
                                   int32_t maxit, int32_t restart, int32_t inner, int32_t* iters,
                                   int32_t* inner_iters, double* relres, mehdg_stream stream) {
    mehdg_err e = trace_ready(c);
    if (e != MEHDG_OK) return e;
    if (!F || !x || !iters || !inner_iters || !relres || !(rtol > 0.0) || maxit < 0 || restart < 1 ||
        restart > kMaxRestart || inner < 0 || inner > kMaxRestart)
        return MEHDG_EINVAL;
    if (!Ahat && (e = ensure_matrix_free(c)) != MEHDG_OK) return e;
    if ((e = ensure_trace_work(c, true)) != MEHDG_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (c->p) {
        case 1: return trace_fgmres<1>(c, Ahat, F, x, rtol, maxit, restart, inner, iters, inner_iters, relres, st);
        case 2: return trace_fgmres<2>(c, Ahat, F, x, rtol, maxit, restart, inner, iters, inner_iters, relres, st);
        case 3: return trace_fgmres<3>(c, Ahat, F, x, rtol, maxit, restart, inner, iters, inner_iters, relres, st);
        default: return MEHDG_EINVAL;
    }
}


mehdg_err mehdg_profile_enable(mehdg_ctx* c, int32_t enable) {
    if (!c) return MEHDG_EINVAL;
    c->prof = enable != 0;
    return MEHDG_OK;
}

mehdg_err mehdg_profile_read(mehdg_ctx* c, double* ms, int64_t* calls, int32_t n) {
    if (!c || !ms || !calls || n < 0) return MEHDG_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return MEHDG_EHIP;
    for (auto& mk : c->marks) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, mk.a, mk.b) == hipSuccess) {
            c->prof_ms[mk.slot] += t;
            c->prof_calls[mk.slot] += 1;
        }
    }
    drop_marks(c);
    for (int i = 0; i < n && i < MEHDG_NPROF; ++i) {
        ms[i] = c->prof_ms[i];
        calls[i] = c->prof_calls[i];
        c->prof_ms[i] = 0.0;
        c->prof_calls[i] = 0;
    }
    return MEHDG_OK;
}


mehdg_err mehdg_add_source(mehdg_ctx* c, const double* s, double* R_v, mehdg_stream stream) {
    if (!c || !s || !R_v) return MEHDG_EINVAL;
    if (c->stage != 1) return MEHDG_ESTATE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)c->n_macro);
    switch (c->p) {
        case 1: hipLaunchKernelGGL(k_add_source<1>, grid, dim3(256), 0, st, s, R_v, c->d_B, (int64_t)c->n_macro); break;
        case 2: hipLaunchKernelGGL(k_add_source<2>, grid, dim3(256), 0, st, s, R_v, c->d_B, (int64_t)c->n_macro); break;
        case 3: hipLaunchKernelGGL(k_add_source<3>, grid, dim3(256), 0, st, s, R_v, c->d_B, (int64_t)c->n_macro); break;
        default: return MEHDG_EINVAL;
    }
    return hip_ok(hipGetLastError());
}

mehdg_err mehdg_set_pseudo_time(mehdg_ctx* c, double alpha_ps) {
    if (!c || !(alpha_ps >= 0.0) || !std::isfinite(alpha_ps)) return MEHDG_EINVAL;
    c->prm.alpha_ps = alpha_ps;
    c->dp.alpha_ps = alpha_ps;
    return MEHDG_OK;
}

mehdg_err mehdg_axpby(int64_t n, double a, const double* x, double b, double* y, mehdg_stream stream) {
    if (n < 0 || (n > 0 && (!x || !y))) return MEHDG_EINVAL;
    if (n == 0) return MEHDG_OK;
    return host_axpby(n, a, x, b, y, reinterpret_cast<hipStream_t>(stream));
}

mehdg_err mehdg_dot_noalloc(int64_t n, const double* x, const double* y, double* out, mehdg_stream stream) {
    if (n < 0 || !out || (n > 0 && (!x || !y))) return MEHDG_EINVAL;
    if (n == 0) {
        *out = 0.0;
        return MEHDG_OK;
    }
    double* part = nullptr;
    mehdg_err e = scratch_on_device(&part);
    if (e != MEHDG_OK) return e;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // every block writes its own partial, so nothing needs clearing first
    hipLaunchKernelGGL(k_dots, dim3(kDotBlocks), dim3(256), 0, st, x, n, 1, y, part);
    if (hipGetLastError() != hipSuccess) return MEHDG_EHIP;
    double h[kDotBlocks];
    if (hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return MEHDG_EHIP;
    double sum = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) sum += h[b];
    *out = sum;
    return MEHDG_OK;
}

mehdg_err mehdg_dot(mehdg_ctx* c, int64_t n, const double* x, const double* y, double* out, mehdg_stream stream) {
    if (!c || n < 0 || !out || (n > 0 && (!x || !y))) return MEHDG_EINVAL;
    if (n == 0) {
        *out = 0.0;
        return MEHDG_OK;
    }
    mehdg_err e;
    if (!c->d_part && (e = dev_alloc(c, &c->d_part, (int64_t)kDotBlocks)) != MEHDG_OK) return e;
    if (c->h_part.size() < (size_t)kDotBlocks) c->h_part.assign(kDotBlocks, 0.0);
    return host_dots(c, x, n, 1, y, out, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
