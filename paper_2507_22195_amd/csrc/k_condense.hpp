// Static condensation of every macro-element (Sec. 6.2 eq. R4, R5):
// partial-pivoted LU of S run over the bordered matrix
//
//   B = [[S, -Y, r_V], [X, A', r_hat]],
//
// with pivot rows chosen among the rows of S only.  After the N_V columns of
// S are eliminated the trailing block holds
//   A' - X S^-1 (-Y) = Ahat  (R5a),   r_hat - X S^-1 r_V = bhat  (R5b),
// and the top rows hold U (of S), U12 = L^-1 P (-Y) and y = L^-1 P r_V, which
// is all that back-substitution needs (the factor L of S is not kept).
//
// Schedule per 64-column panel [kb, kb+nb):
//   k_panel     one workgroup per macro: factor the S rows of the panel
//               (one row per thread, the panel segment in registers), then
//               the X rows of the panel by a triangular solve with U_kk;
//   k_rowblock  apply the panel's row interchanges to columns >= kb+nb and
//               solve L_kk U = P B for the top rows (one column per thread);
//   k_gemm      rank-nb trailing update on FP64 MFMA of the L-shaped region
//               (all rows x S columns, and S rows x border columns); the A'
//               block is left alone.
// Then one k_gemm with K = N_V forms Ahat = A' - L21 U12 and bhat = r_hat - L21 y
// directly in the caller's arrays.
#pragma once
#include "k_assemble.hpp"

namespace mehdg {

typedef double v4d __attribute__((ext_vector_type(4)));

// panel width of the blocked factorisation
template <int P>
struct Panel {
    static constexpr int NB = 64;
    static constexpr int NV = Dims<P>::NV;
    static constexpr int THREADS = ((NV + 63) / 64) * 64 > 1024 ? 1024 : ((NV + 63) / 64) * 64;
    static constexpr int RPT = (NV + THREADS - 1) / THREADS;   // S rows per thread
};

// ---------------------------------------------------------------------------
// Panel factorisation.  Rows of S in [kb, NV) are spread one (or RPT) per
// thread; column j of the panel: arg-max over those rows, interchange of the
// two rows' panel segments, scaling and rank-1 update in registers.
template <int P>
__global__ void __launch_bounds__(Panel<P>::THREADS) k_panel(double* __restrict__ B, int kb,
                                                             int32_t* __restrict__ ipiv,
                                                             int32_t* __restrict__ status) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, RPT = PN::RPT, ld = BD::ld, ROWS = BD::rows;
    constexpr int NW = PN::THREADS / 64;
    __shared__ double prow[NB];            // current pivot row segment
    __shared__ double xch[2][NB];          // row interchange buffer
    __shared__ double U[NB][NB + 1];       // U_kk for the X-row solve
    __shared__ double redv[NW];
    __shared__ int redi[NW];
    __shared__ int piv_sh;
    __shared__ int bad_sh;
    const int64_t m = blockIdx.x;
    double* Bm = B + m * BD::per_macro;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int tid = threadIdx.x;
    if (tid == 0) bad_sh = 0;

    double seg[RPT][NB];
    int rows[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        rows[r] = kb + tid + r * PN::THREADS;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            seg[r][c] = (rows[r] < NV && c < nb) ? Bm[(int64_t)rows[r] * ld + kb + c] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const int col = kb + j;
        // pivot search over rows [col, NV)
        double best = -1.0;
        int bi = col;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            double x = 0.0;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c == j) x = seg[r][c];
            const double ax = fabs(x);
            if (rows[r] >= col && rows[r] < NV && (ax > best || (ax == best && rows[r] < bi))) {
                best = ax;
                bi = rows[r];
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_down(best, off, 64);
            const int oi = __shfl_down(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if ((tid & 63) == 0) {
            redv[tid >> 6] = best;
            redi[tid >> 6] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = redv[0];
            int i = redi[0];
            for (int w = 1; w < NW; ++w)
                if (redv[w] > b || (redv[w] == b && redi[w] < i)) {
                    b = redv[w];
                    i = redi[w];
                }
            piv_sh = i;
            ipiv[m * NV + col] = i;
            if (!(b > 0.0) || !isfinite(b)) bad_sh = 1;
        }
        __syncthreads();
        const int p = piv_sh;
        // interchange rows col and p (panel segment only)
        if (p != col) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (rows[r] == col) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) xch[0][c] = seg[r][c];
                }
                if (rows[r] == p) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) xch[1][c] = seg[r][c];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (rows[r] == col) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) seg[r][c] = xch[1][c];
                }
                if (rows[r] == p) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) seg[r][c] = xch[0][c];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (rows[r] == col) {
#pragma unroll
                for (int c = 0; c < NB; ++c) prow[c] = seg[r][c];
            }
        __syncthreads();
        const double pv = prow[j];
        const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (rows[r] > col && rows[r] < NV) {
                double l = 0.0;
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c == j) l = seg[r][c] * inv;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (c == j) seg[r][c] = l;
                    else if (c > j) seg[r][c] -= l * prow[c];
                }
            }
        }
        __syncthreads();
    }
    // write back the S rows of the panel, keep U_kk for the X rows
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        if (rows[r] < NV) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nb) Bm[(int64_t)rows[r] * ld + kb + c] = seg[r][c];
        }
        const int i = rows[r] - kb;
        if (i >= 0 && i < nb) {
#pragma unroll
            for (int c = 0; c < NB; ++c) U[i][c] = seg[r][c];
        }
    }
    __syncthreads();
    // X rows: L21 = X_panel U_kk^-1 (forward substitution along the row)
    for (int r = NV + tid; r < ROWS; r += PN::THREADS) {
        double x[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) x[c] = (c < nb) ? Bm[(int64_t)r * ld + kb + c] : 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c < nb) {
                double s = x[c];
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i < c) s -= x[i] * U[i][c];
                x[c] = (U[c][c] != 0.0) ? s / U[c][c] : 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c < nb) Bm[(int64_t)r * ld + kb + c] = x[c];
    }
    if (tid == 0 && bad_sh) record_status(status, m, ST_SINGULAR);
}

// ---------------------------------------------------------------------------
// Row interchanges and L_kk solve for the top rows [kb, kb+nb) of every
// column c >= kb+nb (one column per thread).
template <int P>
__global__ void __launch_bounds__(256) k_rowblock(double* __restrict__ B, int kb,
                                                  const int32_t* __restrict__ ipiv) {
    using BD = Bdims<P>;
    constexpr int NB = Panel<P>::NB, NV = Dims<P>::NV, ld = BD::ld;
    __shared__ double Lk[NB][NB + 1];
    __shared__ int src_top[NB];          // original row whose value lands in row kb+i
    __shared__ int out_dst[NB], out_src[NB];
    __shared__ int n_out;
    __shared__ int map[NV];
    const int64_t m = blockIdx.y;
    double* Bm = B + m * BD::per_macro;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int tid = threadIdx.x;
    // the interchanges, composed into a gather
    for (int r = tid; r < NV; r += blockDim.x) map[r] = r;
    for (int i = tid; i < NB * NB; i += blockDim.x) {
        const int r = i / NB, c = i % NB;
        Lk[r][c] = (r < nb && c < nb) ? Bm[(int64_t)(kb + r) * ld + kb + c] : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < nb; ++i) {
            const int p = ipiv[m * NV + kb + i];
            const int t = map[kb + i];
            map[kb + i] = map[p];
            map[p] = t;
        }
        int no = 0;
        for (int i = 0; i < nb; ++i) {
            src_top[i] = map[kb + i];
            const int p = ipiv[m * NV + kb + i];
            if (p >= kb + nb && map[p] != p) {
                bool seen = false;
                for (int q = 0; q < no; ++q)
                    if (out_dst[q] == p) seen = true;
                if (!seen) {
                    out_dst[no] = p;
                    out_src[no] = map[p];
                    ++no;
                }
            }
        }
        n_out = no;
    }
    __syncthreads();
    const int c = kb + nb + blockIdx.x * blockDim.x + tid;
    if (c >= ld) return;
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) x[i] = (i < nb) ? Bm[(int64_t)src_top[i] * ld + c] : 0.0;
    const int no = n_out;
    double moved[NB];
    for (int q = 0; q < no; ++q) moved[q < NB ? q : 0] = Bm[(int64_t)out_src[q] * ld + c];
    for (int q = 0; q < no; ++q) Bm[(int64_t)out_dst[q] * ld + c] = moved[q < NB ? q : 0];
    // unit lower solve with L_kk
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        double s = x[i];
#pragma unroll
        for (int k = 0; k < NB; ++k)
            if (k < i) s -= Lk[i][k] * x[k];
        x[i] = s;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (i < nb) Bm[(int64_t)(kb + i) * ld + c] = x[i];
}

// ---------------------------------------------------------------------------
// Batched FP64 MFMA product  D = C - A * Bt  on a 64 x 64 tile per workgroup.
//   A  (rows r, K): A[m*sA + r*lda + k]
//   Bt (K, cols c): Bt[m*sB + k*ldb + c]
//   C  (rows, cols): C[m*sC + r*ldc + c];  D: same as C, except that columns
//   c >= dsplit go to D2[m*sD2 + r*ldd2 + (c - dsplit)] when D2 is given.
// Elements with r >= skip_r and c >= skip_c are neither read nor written.
struct GemmArgs {
    const double* A;
    const double* Bt;
    const double* C;
    double* D;
    double* D2;
    int64_t sA, sB, sC, sD, sD2;
    int lda, ldb, ldc, ldd, ldd2;
    int rows, cols, K;       // extent of the region (relative to its origin)
    int dsplit;              // first column that goes to D2 (cols if none)
    int skip_r, skip_c;      // masked corner (relative), rows/cols if none
    int tiles_c;             // column tiles
};

constexpr int GT = 64;       // tile edge
constexpr int GK = 16;       // K chunk staged in LDS

// TAG only separates the trailing-update launches (0) from the final Schur
// product (1) in profiles; the code is the same.
template <int TAG>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ double As[GT][GK + 1];
    __shared__ double Bs[GK][GT + 1];
    const int64_t m = blockIdx.y;
    const int tr = blockIdx.x / g.tiles_c, tc = blockIdx.x % g.tiles_c;
    const int r0 = tr * GT, c0 = tc * GT;
    if (r0 >= g.skip_r && c0 >= g.skip_c) return;   // tile entirely in the masked corner
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const double* A = g.A + m * g.sA;
    const double* Bt = g.Bt + m * g.sB;
    const double* C = g.C + m * g.sC;
    v4d acc[2][2];
    // initial accumulators: C
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr * 32 + bi * 16 + (lane >> 4) + 4 * q;
                const int c = c0 + wc * 32 + bj * 16 + (lane & 15);
                const bool in = r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c);
                acc[bi][bj][q] = in ? C[(int64_t)r * g.ldc + c] : 0.0;
            }
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        // stage -A (64 x 16) and Bt (16 x 64)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 256 * i;
            const int ar = e >> 4, ak = e & 15;
            const int r = r0 + ar, k = k0 + ak;
            As[ar][ak] = (r < g.rows && k < g.K) ? -A[(int64_t)r * g.lda + k] : 0.0;
            const int bk = e >> 6, bc = e & 63;
            const int kk = k0 + bk, c = c0 + bc;
            Bs[bk][bc] = (kk < g.K && c < g.cols) ? Bt[(int64_t)kk * g.ldb + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const int kq = ks + (lane >> 4);
            const double a0 = As[wr * 32 + (lane & 15)][kq];
            const double a1 = As[wr * 32 + 16 + (lane & 15)][kq];
            const double b0 = Bs[kq][wc * 32 + (lane & 15)];
            const double b1 = Bs[kq][wc * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    double* D = g.D + m * g.sD;
    double* D2 = g.D2 ? g.D2 + m * g.sD2 : nullptr;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr * 32 + bi * 16 + (lane >> 4) + 4 * q;
                const int c = c0 + wc * 32 + bj * 16 + (lane & 15);
                if (r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c)) {
                    if (D2 && c >= g.dsplit) D2[(int64_t)r * g.ldd2 + (c - g.dsplit)] = acc[bi][bj][q];
                    else D[(int64_t)r * g.ldd + c] = acc[bi][bj][q];
                }
            }
}

}  // namespace mehdg
