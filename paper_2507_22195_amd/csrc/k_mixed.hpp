// Mixed-precision static condensation (Sec. 6.2 eq. R4-R5): the interior
// block S factored in FP32 on MFMA, the solves with those factors refined to
// FP64 accuracy by FP64 residuals, the Schur product in FP64.
//
// Per wave of macros (the low-precision workspace holds a wave, not the batch):
//   k_lp_init     S_lo = fl32(S) (row-major, a row per identity), Z = 0,
//                 R = [-Y | r_V] (the right-hand sides, FP64), perm = identity;
//   k_lp_panel    one workgroup per macro: 32-column panel of the partial-pivot
//                 LU of S_lo, rows never move (perm maps position -> row), then
//                 U12 = L11^-1 A12 of the panel's pivot rows on the trailing
//                 columns;
//   k_lp_update   trailing update A22 -= L21 U12 (K = 32) on FP32 MFMA, or on
//                 BF16 MFMA with FP32 accumulation (operands rounded to BF16);
//   k_lp_trsm     x = U^-1 L^-1 P R by 32-row blocks, one launch per block and
//                 direction, each a batched FP32-MFMA product with the solved
//                 part followed by the stored inverse of the diagonal block;
//   k_lp_zadd     Z += x, per-macro sums of |x|^2 and |Z|^2;
//   residual      R = [-Y | r_V] - S Z in FP64 (k_gemm on FP64 MFMA), then
//                 the solve again, until the forward-error estimate of Z is
//                 below ir_tol (decided on the host from the sums);
//   Schur         [Ahat | bhat] = [A' | r_hat] - X Z in FP64 (k_gemm);
//   k_lp_stash    Z_Y^T to the rows of X, z_r to the r_V column of the
//                 bordered matrix, which the recovery then reads:
//                 dV = S^-1 (r_V + Y dVhat) = z_r - Z_Y dVhat (Z = S^-1 [-Y | r_V]).
//
// The factor layout: row id of S_lo at position pos = position of id holds
// L(pos, c) for c < pos (unit diagonal implied) and U(pos, c) for c >= pos;
// column c is the unknown c of S (partial pivoting permutes rows only), so
// L y = P r runs over positions and U x = y gives x in natural order.
#pragma once
#include <climits>

#include "k_condense.hpp"

namespace mehdg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int LP_NB = 32;       // panel width, and row block of the solves
constexpr int LP_UT = 512;      // update threads (8 waves, 128 x 64 tile)

template <int P>
struct LpDims {
    static constexpr int NV = Dims<P>::NV, NH = Dims<P>::NH, NR = NH + 1;
    static constexpr int lds = (NV + 3) / 4 * 4;               // row length of S_lo (floats)
    static constexpr int64_t per_s = (int64_t)NV * lds;        // floats per macro
    static constexpr int64_t per_z = (int64_t)NV * NR;         // doubles per macro (Z, R)
    static constexpr int NPAN = (NV + LP_NB - 1) / LP_NB;
    static constexpr int PT0 = ((NV + 63) / 64) * 64;
    static constexpr int PT = PT0 > 1024 ? 1024 : (PT0 < 128 ? 128 : PT0);   // panel threads
    static constexpr int RPT = (NV + PT - 1) / PT;             // rows per panel thread
    // inverses of the diagonal blocks of L and U, per panel: [NPAN][2][32][32]
    static constexpr int64_t per_t = (int64_t)NPAN * 2 * LP_NB * LP_NB;
};

// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(256) k_lp_init(const double* __restrict__ B, int64_t m0, int64_t W,
                                                 float* __restrict__ S, int32_t* __restrict__ perm,
                                                 double* __restrict__ Z, double* __restrict__ R) {
    using LD = LpDims<P>;
    using BD = Bdims<P>;
    constexpr int NV = LD::NV, NR = LD::NR;
    const int64_t m = blockIdx.y;
    const int r = blockIdx.x;
    if (m >= W || r >= NV) return;
    const double* Br = B + (m0 + m) * BD::per_macro + (int64_t)r * BD::ld;
    float* Sr = S + m * LD::per_s + (int64_t)r * LD::lds;
    double* Rr = R + m * LD::per_z + (int64_t)r * NR;
    double* Zr = Z + m * LD::per_z + (int64_t)r * NR;
    for (int c = threadIdx.x; c < LD::lds; c += blockDim.x) Sr[c] = c < NV ? (float)Br[c] : 0.0f;
    for (int c = threadIdx.x; c < NR; c += blockDim.x) {
        Rr[c] = Br[NV + c];
        Zr[c] = 0.0;
    }
    if (threadIdx.x == 0) perm[m * NV + r] = r;
}

// ---------------------------------------------------------------------------
// Panel kb .. kb+nb (nb <= 32) of the LU of one macro's S_lo.  Each thread owns
// RPT rows (by identity) among the positions kb .. NV-1; a row's 32 panel
// values stay in registers.  Column j: arg-max of |z_j| over the rows that
// are not pivots yet (wave shuffles, then the waves through LDS; ties to the
// lower identity), the pivot row broadcast through LDS, rank-1 update of the
// remaining columns; the multiplier replaces z_j.  Two barriers per column,
// the LDS buffers alternating by column parity.  Then the interchanges are
// replayed in LAPACK order on the position map, the panel is written back to
// the rows' own storage, the inverses of the diagonal blocks L11 and U11 are
// formed (one column per lane) and stored for the solves, and the pivot
// rows' trailing columns become U12 = L11^-1 A12 (one column per thread).
template <int P>
__global__ void __launch_bounds__(LpDims<P>::PT) k_lp_panel(float* __restrict__ S, int32_t* __restrict__ perm,
                                                            float* __restrict__ tinv, int kb, int64_t m0,
                                                            int32_t* __restrict__ status) {
    using LD = LpDims<P>;
    constexpr int NV = LD::NV, PT = LD::PT, RPT = LD::RPT, NB = LP_NB, NW = PT / 64, lds = LD::lds;
    __shared__ int mp[NV];              // position -> row (positions >= kb)
    __shared__ int ps[NV];              // row -> position
    __shared__ float prow[2][NB];
    __shared__ float redv[2][NW];
    __shared__ int redi[2][NW];
    __shared__ int pidj[NB];
    __shared__ float L11[NB][NB + 1];   // the pivot rows' panel values (L below, U on and above the diagonal)
    __shared__ float Li[NB][NB + 1];    // L11^-1 (unit lower)
    __shared__ float Ui[NB][NB + 1];    // U11^-1
    const int64_t m = blockIdx.x;
    float* Sm = S + m * LD::per_s;
    int32_t* pm = perm + m * NV;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    for (int i = kb + tid; i < NV; i += PT) {
        const int id = pm[i];
        mp[i] = id;
        ps[id] = i;
    }
    __syncthreads();
    float z[RPT][NB];
    int id[RPT];
    bool live[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int pos = kb + tid + r * PT;
        id[r] = pos < NV ? mp[pos] : -1;
        live[r] = pos < NV;
#pragma unroll
        for (int c = 0; c < NB; ++c) z[r][c] = (live[r] && c < nb) ? Sm[(int64_t)id[r] * lds + kb + c] : 0.0f;
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j >= nb) break;
        const int bf = j & 1;
        float best = -1.0f;
        int bi = INT_MAX;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            float a = fabsf(z[r][j]);
            if (!(a >= 0.0f)) a = 0.0f;           // NaN
            if (live[r] && (a > best || (a == best && id[r] < bi))) {
                best = a;
                bi = id[r];
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) {
            redv[bf][wave] = best;
            redi[bf][wave] = bi;
        }
        __syncthreads();
        float pbest = redv[bf][0];
        int p = redi[bf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
            if (redv[bf][w] > pbest || (redv[bf][w] == pbest && redi[bf][w] < p)) {
                pbest = redv[bf][w];
                p = redi[bf][w];
            }
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (live[r] && id[r] == p) {
#pragma unroll
                for (int c = 0; c < NB; ++c) prow[bf][c] = z[r][c];
                live[r] = false;
            }
        if (tid == 0) pidj[j] = p;
        __syncthreads();
        const float piv = prow[bf][j];
        const bool ok = piv != 0.0f && isfinite(piv);
        if (!ok) bad = true;
        const float inv = ok ? 1.0f / piv : 0.0f;
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (live[r]) {
                const float l = z[r][j] * inv;
                z[r][j] = l;
#pragma unroll
                for (int c = j + 1; c < NB; ++c) z[r][c] -= l * prow[bf][c];
            }
    }
    __syncthreads();
    if (tid == 0) {
        for (int j = 0; j < nb; ++j) {
            const int pid = pidj[j], pp = ps[pid], other = mp[kb + j];
            mp[kb + j] = pid;
            ps[pid] = kb + j;
            mp[pp] = other;
            ps[other] = pp;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        if (id[r] < 0) continue;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < nb) Sm[(int64_t)id[r] * lds + kb + c] = z[r][c];
        const int j = ps[id[r]] - kb;
        if (j >= 0 && j < nb) {
#pragma unroll
            for (int c = 0; c < NB; ++c) L11[j][c] = c < nb ? z[r][c] : 0.0f;
        }
    }
    // a short last panel: identity rows and columns beyond nb
    for (int e = tid; e < NB * NB; e += PT) {
        const int i = e / NB, c = e % NB;
        if (i >= nb || c >= nb) L11[i][c] = i == c ? 1.0f : 0.0f;
    }
    for (int i = kb + tid; i < NV; i += PT) pm[i] = mp[i];
    __syncthreads();
    // inverses of the diagonal blocks, one column per lane: wave 0 the unit
    // lower L11^-1 (forward), wave 1 U11^-1 (backward)
    if (wave == 0 && lane < NB) {
        const int c = lane;
        for (int i = 0; i < NB; ++i) {
            float sacc = i == c ? 1.0f : 0.0f;
            for (int k = 0; k < i; ++k) sacc -= L11[i][k] * Li[k][c];
            Li[i][c] = sacc;
        }
    } else if (wave == 1 && lane < NB) {
        const int c = lane;
        for (int i = NB - 1; i >= 0; --i) {
            float sacc = i == c ? 1.0f : 0.0f;
            for (int k = i + 1; k < NB; ++k) sacc -= L11[i][k] * Ui[k][c];
            Ui[i][c] = sacc / L11[i][i];
        }
    }
    __syncthreads();
    float* tm = tinv + m * LD::per_t + (int64_t)(kb / NB) * 2 * NB * NB;
    for (int e = tid; e < NB * NB; e += PT) {
        tm[e] = Li[e / NB][e % NB];
        tm[NB * NB + e] = Ui[e / NB][e % NB];
    }
    // U12 = L11^-1 A12 on the pivot rows' trailing columns, one column per thread
    for (int c = kb + nb + tid; c < NV; c += PT) {
        float a[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) a[i] = i < nb ? Sm[(int64_t)pidj[i] * lds + c] : 0.0f;
        for (int j = 0; j < nb; ++j) {
            float x = 0.0f;
#pragma unroll
            for (int i = 0; i < NB; ++i) x += Li[j][i] * a[i];
            Sm[(int64_t)pidj[j] * lds + c] = x;
        }
    }
    if (bad && tid == 0) record_status(status, m0 + m, ST_SINGULAR);
}

// ---------------------------------------------------------------------------
// Trailing update after the full panel at kb: for the positions and columns
// kb+32 .. NV-1, A[row(pos)][c] -= sum_j L[row(pos)][kb+j] U12[j][c] with
// U12[j][c] = S_lo[row(kb+j)][c].  128 x 64 tile per workgroup, eight waves in
// 4 x 2, each 2 x 2 blocks of 16 x 16; MFMA lane layouts (measured on gfx950):
// f32 16x16x4: A lane l <- A[l%16][l/16], B lane l <- B[l/16][l%16];
// bf16 16x16x32: A lane l <- A[l%16][8(l/16)+e], B lane l <- B[8(l/16)+e][l%16];
// result register r of lane l = D[4(l/16)+r][l%16] for both.
template <int P, bool BF>
__global__ void __launch_bounds__(LP_UT) k_lp_update(float* __restrict__ S, const int32_t* __restrict__ perm,
                                                     int kb, int tiles_c, int tiles, int64_t W) {
    using LD = LpDims<P>;
    constexpr int NV = LD::NV, NB = LP_NB, lds = LD::lds, TM = 128, TN = 64;
    __shared__ float As[TM][NB + 1];
    __shared__ float Bs[NB][TN + 1];
    __shared__ int rid[TM];
    __shared__ int pid[NB];
    int64_t m;
    int tile;
    xcd_tile(tiles, m, tile);
    if (m >= W) return;
    const int n0 = kb + NB, rows = NV - n0;
    const int r0 = (tile / tiles_c) * TM, c0 = (tile % tiles_c) * TN;
    float* Sm = S + m * LD::per_s;
    const int32_t* pm = perm + m * NV;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wr = wave >> 1, wc = wave & 1;
    for (int i = tid; i < TM; i += LP_UT) rid[i] = (r0 + i < rows) ? pm[n0 + r0 + i] : -1;
    if (tid < NB) pid[tid] = pm[kb + tid];
    __syncthreads();
    for (int e = tid; e < TM * NB; e += LP_UT) {
        const int i = e / NB, j = e % NB;
        As[i][j] = rid[i] >= 0 ? Sm[(int64_t)rid[i] * lds + kb + j] : 0.0f;
    }
    for (int e = tid; e < NB * TN; e += LP_UT) {
        const int j = e / TN, c = e % TN;
        Bs[j][c] = (c0 + c < rows) ? Sm[(int64_t)pid[j] * lds + n0 + c0 + c] : 0.0f;
    }
    // the C tile's current values, fetched before the products
    float cr[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * 32 + bi * 16 + 4 * (lane >> 4) + r;
                const int col = c0 + wc * 32 + bj * 16 + (lane & 15);
                const int rr = rid[row];
                cr[bi][bj][r] = (rr >= 0 && col < rows) ? Sm[(int64_t)rr * lds + n0 + col] : 0.0f;
            }
    __syncthreads();
    v4f acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (BF) {
        v8bf a[2], b[2];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * (lane >> 4) + e;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t][e] = (__bf16)As[wr * 32 + t * 16 + (lane & 15)][k];
                b[t][e] = (__bf16)Bs[k][wc * 32 + t * 16 + (lane & 15)];
            }
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    } else {
#pragma unroll
        for (int ks = 0; ks < NB; ks += 4) {
            const int k = ks + (lane >> 4);
            const float a0 = As[wr * 32 + (lane & 15)][k], a1 = As[wr * 32 + 16 + (lane & 15)][k];
            const float b0 = Bs[k][wc * 32 + (lane & 15)], b1 = Bs[k][wc * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * 32 + bi * 16 + 4 * (lane >> 4) + r;
                const int col = c0 + wc * 32 + bj * 16 + (lane & 15);
                const int rr = rid[row];
                if (rr >= 0 && col < rows) Sm[(int64_t)rr * lds + n0 + col] = cr[bi][bj][r] - acc[bi][bj][r];
            }
}

// ---------------------------------------------------------------------------
// Solves with the low-precision factors, one launch per 32-row block q
// (positions q0 = 32q ..), a 32 x 128 tile of right-hand-side columns per
// workgroup (4 waves, 32 x 32 each):
//   forward  (FWD):  Y[q] = L_qq^-1 (R[row(q0 + i)] - L[q, <q0] Y[<q0])
//   backward (!FWD): Y[q] = U_qq^-1 (Y[q] - U[q, >= q0+nb] Y[>= q0+nb])
// Y (FP32, [N_V][ldy], rows in position order) ends holding x = S^-1 R in
// natural order: U's column c is unknown c.  The block product runs on FP32
// MFMA over K chunks of 32, the factor rows (gathered through perm) and the Y
// rows staged through LDS with the next chunk's loads issued before the
// current chunk's products; then the stored inverse of the diagonal block
// (from k_lp_panel) is applied, a thread per 16 outputs.  Each launch reads
// only rows of Y that earlier launches wrote, and writes only its own block.
constexpr int LPT_TN = 128;     // columns per workgroup
constexpr int LPT_T = 256;      // threads
constexpr int LPT_KC = 32;      // K chunk

template <int P>
struct LpTrsmDims {
    static constexpr int ldy = (LpDims<P>::NR + 3) / 4 * 4;
    static constexpr int64_t per_y = (int64_t)LpDims<P>::NV * ldy;
    static constexpr int TILES = (LpDims<P>::NR + LPT_TN - 1) / LPT_TN;
};

template <int P, bool FWD>
__global__ void __launch_bounds__(LPT_T) k_lp_trsm(const float* __restrict__ S, const int32_t* __restrict__ perm,
                                                   const float* __restrict__ tinv, const double* __restrict__ R,
                                                   float* __restrict__ Y, int q, int64_t W) {
    using LD = LpDims<P>;
    using TD = LpTrsmDims<P>;
    constexpr int NV = LD::NV, NR = LD::NR, NB = LP_NB, lds = LD::lds, ldy = TD::ldy, TN = LPT_TN, KC = LPT_KC;
    constexpr int LA = NB * KC / LPT_T, LB = KC * TN / LPT_T;   // staged elements per thread
    __shared__ float As[2][NB][KC + 1];
    __shared__ float Bs[2][KC][TN + 1];
    __shared__ float Ti[NB][NB + 1];
    __shared__ int rid[NB];
    int64_t m;
    int tile;
    xcd_tile(TD::TILES, m, tile);
    if (m >= W) return;
    const int q0 = q * NB, nbq = (NV - q0) < NB ? (NV - q0) : NB, t0 = tile * TN;
    const float* Sm = S + m * LD::per_s;
    float* Ym = Y + m * TD::per_y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < NB) rid[tid] = tid < nbq ? perm[m * NV + q0 + tid] : -1;
    const float* Tq = tinv + m * LD::per_t + (int64_t)q * 2 * NB * NB + (FWD ? 0 : NB * NB);
    for (int e = tid; e < NB * NB; e += LPT_T) Ti[e / NB][e % NB] = Tq[e];
    __syncthreads();
    const int klo = FWD ? 0 : q0 + nbq, khi = FWD ? q0 : NV;
    v4f acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    float ra[LA], rb[LB];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + LPT_T * i, r = e / KC, k = k0 + e % KC;
            ra[i] = (rid[r] >= 0 && k < khi) ? Sm[(int64_t)rid[r] * lds + k] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = tid + LPT_T * i, k = k0 + e / TN, c = t0 + e % TN;
            rb[i] = (k < khi && c < NR) ? Ym[(int64_t)k * ldy + c] : 0.0f;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = tid + LPT_T * i;
            As[buf][e / KC][e % KC] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = tid + LPT_T * i;
            Bs[buf][e / TN][e % TN] = rb[i];
        }
    };
    const int nch = khi > klo ? (khi - klo + KC - 1) / KC : 0;
    if (nch > 0) {
        load(klo);
        stash(0);
    }
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(klo + (ch + 1) * KC);
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int k = ks + (lane >> 4);
            const float a0 = As[buf][lane & 15][k], a1 = As[buf][16 + (lane & 15)][k];
            const float b0 = Bs[buf][k][wave * 32 + (lane & 15)], b1 = Bs[buf][k][wave * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (ch + 1 < nch) stash(buf ^ 1);
        __syncthreads();
    }
    // t = (right-hand side of the block) - product, into Bs[0] as a 32 x 128 tile
    float (*T)[TN + 1] = Bs[0];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = bi * 16 + 4 * (lane >> 4) + r, cl = wave * 32 + bj * 16 + (lane & 15), c = t0 + cl;
                float t = 0.0f;
                if (i < nbq && c < NR) {
                    if constexpr (FWD) t = (float)(R[m * LD::per_z + (int64_t)rid[i] * NR + c] - (double)acc[bi][bj][r]);
                    else t = Ym[(int64_t)(q0 + i) * ldy + c] - acc[bi][bj][r];
                }
                T[i][cl] = t;
            }
    __syncthreads();
    // Y[q] = (inverse of the diagonal block) t: thread -> column cl, rows i0 .. i0+16
    {
        const int cl = tid % TN, i0 = (tid / TN) * 16, c = t0 + cl;
        float x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] = 0.0f;
#pragma unroll 2
        for (int j = 0; j < NB; ++j) {
            const float tj = T[j][cl];
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i] += Ti[i0 + i][j] * tj;
        }
        if (c < NR) {
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i0 + i < nbq) Ym[(int64_t)(q0 + i0 + i) * ldy + c] = x[i];
        }
    }
}

// Z += Y (x of the solve, natural order) and the per-macro sums |x|^2, |Z|^2
// for the stopping test; grid (row chunks of 32, W).
template <int P>
__global__ void __launch_bounds__(256) k_lp_zadd(const float* __restrict__ Y, double* __restrict__ Z,
                                                 double* __restrict__ nrm, int64_t W) {
    using LD = LpDims<P>;
    using TD = LpTrsmDims<P>;
    constexpr int NV = LD::NV, NR = LD::NR, ldy = TD::ldy;
    __shared__ double red[2][4];
    const int64_t m = blockIdx.y;
    if (m >= W) return;
    const int r0 = blockIdx.x * 32;
    const float* Ym = Y + m * TD::per_y;
    double* Zm = Z + m * LD::per_z;
    double sx = 0.0, sz = 0.0;
    for (int e = threadIdx.x; e < 32 * NR; e += 256) {
        const int r = r0 + e / NR, c = e % NR;
        if (r < NV) {
            const double xv = (double)Ym[(int64_t)r * ldy + c];
            double* zp = Zm + (int64_t)r * NR + c;
            const double zn = *zp + xv;
            *zp = zn;
            sx += xv * xv;
            sz += zn * zn;
        }
    }
    sx = wave_sum_f64(sx);
    sz = wave_sum_f64(sz);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = sx;
        red[1][wave] = sz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(nrm + 2 * m, (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
        atomicAdd(nrm + 2 * m + 1, (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
    }
}

__global__ void __launch_bounds__(256) k_lp_fill(double* __restrict__ x, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// Sets the refinement's code (flags[W], host-written) for the macros that
// have no code yet: a zero pivot or a non-physical state that made the
// refinement fail stays the reported cause.
__global__ void __launch_bounds__(256) k_lp_flag(const int32_t* __restrict__ flags, int64_t m0, int64_t W,
                                                 int32_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < W && flags[i] != 0 && status[m0 + i] == 0) status[m0 + i] = flags[i];
}

// ---------------------------------------------------------------------------
// Z_Y^T into the X rows of the bordered matrix (B[NV + i][c] = Z[c][i],
// i < NH) and z_r into its r_V column (B[c][NV + NH] = Z[c][NH]), through a
// 32 x 32 LDS tile per workgroup (grid: column tiles of Z, row tiles of Z, W).
template <int P>
__global__ void __launch_bounds__(256) k_lp_stash(const double* __restrict__ Z, int64_t m0, int64_t W,
                                                  double* __restrict__ B) {
    using LD = LpDims<P>;
    using BD = Bdims<P>;
    constexpr int NV = LD::NV, NH = LD::NH, NR = LD::NR, ld = BD::ld;
    __shared__ double t[32][33];
    const int64_t m = blockIdx.z;
    if (m >= W) return;
    const int i0 = blockIdx.x * 32, c0 = blockIdx.y * 32;   // Z columns i0.., Z rows c0..
    const double* Zm = Z + m * LD::per_z;
    double* Bm = B + (m0 + m) * BD::per_macro;
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const int cr = e / 32, ic = e % 32;
        const int c = c0 + cr, i = i0 + ic;
        const double v = (c < NV && i < NR) ? Zm[(int64_t)c * NR + i] : 0.0;
        t[cr][ic] = v;
        if (c < NV && i == NH) Bm[(int64_t)c * ld + NV + NH] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
        const int ir = e / 32, cc = e % 32;
        const int i = i0 + ir, c = c0 + cc;
        if (i < NH && c < NV) Bm[(int64_t)(NV + i) * ld + c] = t[cc][ir];
    }
}

}  // namespace mehdg
