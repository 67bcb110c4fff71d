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
//               (one row per thread, the panel segment in registers) and
//               invert the diagonal blocks L_kk, U_kk;
//   k_tri       per 64-column tile right of the panel: apply the panel's row
//               interchanges to the tile and form U_top = L_kk^-1 (P B)_top on
//               MFMA; per 64-row tile of X: L21 = X_panel U_kk^-1 (in place);
//   k_gemm      rank-nb trailing update on FP64 MFMA of the L-shaped region
//               (all rows x S columns, and S rows x border columns); the A'
//               block is left alone.
// Then one k_gemm with K = N_V forms Ahat = A' - L21 U12 and bhat = r_hat - L21 y
// directly in the caller's arrays.
#pragma once
#include "k_assemble.hpp"

namespace mehdg {

typedef double v4d __attribute__((ext_vector_type(4)));

// Wave-wide maximum of a double with DPP row permutations (quad swaps, half
// and full row mirrors) and a read of the four row results; every lane gets
// the maximum.  NaN inputs are ignored by fmax.
__device__ __forceinline__ double dpp_perm_f64(double v, int ctrl) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (ctrl) {
        case 0:
            lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
            break;
        case 1:
            lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
            break;
        case 2:
            lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
            break;
        default:
            lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
            break;
    }
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane_f64(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_perm_f64(v, 0));
    v = fmax(v, dpp_perm_f64(v, 1));
    v = fmax(v, dpp_perm_f64(v, 2));
    v = fmax(v, dpp_perm_f64(v, 3));
    return fmax(fmax(read_lane_f64(v, 0), read_lane_f64(v, 16)), fmax(read_lane_f64(v, 32), read_lane_f64(v, 48)));
}

// panel width of the blocked factorisation
template <int P>
struct Panel {
    static constexpr int NB = 64;
    static constexpr int NV = Dims<P>::NV;
    static constexpr int THREADS = ((NV + 63) / 64) * 64 > 1024 ? 1024 : ((NV + 63) / 64) * 64;
    static constexpr int RPT = (NV + THREADS - 1) / THREADS;   // S rows per thread
    static constexpr int64_t TRI = 2 * NB * NB;                 // per macro: L_kk^-1, U_kk^-1
    static constexpr int64_t PERM = 3 * NB + 1;                 // per macro: composed interchange
};

// ---------------------------------------------------------------------------
// Panel factorisation.  Rows of S in [kb, NV) are spread one (or RPT) per
// thread with their panel segment in registers; the column loop is fully
// unrolled so every register index is a constant.  Column j: arg-max over the
// rows (DPP wave maximum, then every thread reduces the per-wave results),
// the pivot row and the row it displaces are exchanged through LDS, then
// scaling and rank-1 update in registers.  Look-ahead: column j+1 is updated
// first and its pivot search is issued before the rest of the update, and
// the LDS buffers alternate by column parity, so two barriers per column.
// Afterwards: the composed row interchange (for k_tri) and the inverses of
// the diagonal blocks L_kk (unit lower) and U_kk go to per-macro workspaces.
template <int P>
__global__ void __launch_bounds__(Panel<P>::THREADS) k_panel(double* __restrict__ B, int kb,
                                                             int32_t* __restrict__ ipiv,
                                                             int32_t* __restrict__ perm,
                                                             double* __restrict__ tri,
                                                             int32_t* __restrict__ status) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, RPT = PN::RPT, ld = BD::ld;
    constexpr int NW = PN::THREADS / 64;
    __shared__ double raw[3 * NB * (NB + 1)];   // T and the two inverses
    __shared__ double prow[2][NB];         // pivot row segment (by column parity)
    __shared__ double xch[2][NB];          // segment of the row the pivot displaces
    __shared__ double redv[2][NW];
    __shared__ int redi[2][NW];
    __shared__ int pivs[NB];
    __shared__ int mp[NV];
    __shared__ int mark[NV];
    const int64_t m = blockIdx.x;
    double* Bm = B + m * BD::per_macro;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    bool bad = false;

    double seg[RPT][NB];
    int rows[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) rows[r] = kb + tid + r * PN::THREADS;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c)
            seg[r][c] = (rows[r] < NV && c < nb) ? Bm[(int64_t)rows[r] * ld + kb + c] : 0.0;
    for (int r = tid; r < NV; r += PN::THREADS) {
        mp[r] = r;
        mark[r] = 0;
    }
    // candidate pivot of column j among rows >= kb+j: wave arg-max to LDS
    auto candidate = [&](int j, int bf, const double (&cv)[RPT]) {
        double best = -1.0;
        int bi = NV;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const double ax = fabs(cv[r]);
            if (rows[r] >= kb + j && rows[r] < NV && (ax > best || (ax == best && rows[r] < bi))) {
                best = ax;
                bi = rows[r];
            }
        }
        const double wm = wave_max_f64(best);
        const unsigned long long bal = __ballot(best == wm);
        const int ol = bal ? (__ffsll((long long)bal) - 1) : 0;
        const int wrow = __builtin_amdgcn_readlane(bi, ol);
        if (lane == 0) {
            redv[bf][wave] = wm;
            redi[bf][wave] = wrow;
        }
    };
    {
        double cv[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) cv[r] = seg[r][0];
        candidate(0, 0, cv);
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < NB; ++j) {
      if (j < nb) {                                // uniform: only the last panel is narrower
        const int col = kb + j, bf = j & 1;
        __syncthreads();
        double b = redv[bf][0];
        int p = redi[bf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
            if (redv[bf][w] > b || (redv[bf][w] == b && redi[bf][w] < p)) {
                b = redv[bf][w];
                p = redi[bf][w];
            }
        if (!(b > 0.0) || !isfinite(b) || p >= NV) {
            bad = true;
            p = col;
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (rows[r] == p) {
#pragma unroll
                for (int c = 0; c < NB; ++c) prow[bf][c] = seg[r][c];
            }
            if (rows[r] == col && p != col) {
#pragma unroll
                for (int c = 0; c < NB; ++c) xch[bf][c] = seg[r][c];
            }
        }
        if (tid == 0) pivs[j] = p;
        __syncthreads();
        const double pv = prow[bf][j];
        const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
        double l[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (rows[r] == col) {
#pragma unroll
                for (int c = 0; c < NB; ++c) seg[r][c] = prow[bf][c];
            } else if (p != col && rows[r] == p) {
#pragma unroll
                for (int c = 0; c < NB; ++c) seg[r][c] = xch[bf][c];
            }
            const bool below = rows[r] > col && rows[r] < NV;
            l[r] = below ? seg[r][j] * inv : 0.0;
            if (below) {
                seg[r][j] = l[r];
                if (j + 1 < NB) seg[r][(j + 1) % NB] -= l[r] * prow[bf][(j + 1) % NB];   // look-ahead column
            }
        }
        if (j + 1 < nb) {
            double cv[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) cv[r] = (j + 1 < NB) ? seg[r][(j + 1) % NB] : 0.0;
            candidate(j + 1, bf ^ 1, cv);
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (rows[r] > col && rows[r] < NV) {
#pragma unroll
                for (int c = j + 2; c < NB; ++c) seg[r][c] -= l[r] * prow[bf][c];
            }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        if (rows[r] < NV) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nb) Bm[(int64_t)rows[r] * ld + kb + c] = seg[r][c];
        }
    }
    __syncthreads();
    // diagonal block T and the two inverses X_L, X_U
    double (*T)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw);
    double (*XL)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw + NB * (NB + 1));
    double (*XU)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw + 2 * NB * (NB + 1));
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = rows[r] - kb;
        if (i >= 0 && i < NB) {
#pragma unroll
            for (int c = 0; c < NB; ++c) T[i][c] = (i < nb && c < nb) ? seg[r][c] : (i == c ? 1.0 : 0.0);
        }
    }
    for (int e = tid; e < NB * NB; e += PN::THREADS) {
        const int i = e / NB, c = e % NB;
        XL[i][c] = (i == c) ? 1.0 : 0.0;
        XU[i][c] = (i == c) ? 1.0 : 0.0;
    }
    if (tid < nb) ipiv[m * NV + kb + tid] = pivs[tid];
    __syncthreads();
    // composed interchange: after it row r holds the old row mp[r].  perm[m]:
    // [0, NB) source rows of the top block, [NB, 2NB) displaced rows below the
    // block, [2NB, 3NB) their source rows, [3NB] their number.
    if (tid == 0) {
        for (int i = 0; i < nb; ++i) {
            const int p = pivs[i];
            const int t = mp[kb + i];
            mp[kb + i] = mp[p];
            mp[p] = t;
        }
        int32_t* pm = perm + m * (3 * NB + 1);
        int nd = 0;
        for (int i = 0; i < nb; ++i) {
            pm[i] = mp[kb + i];
            const int p = pivs[i];
            if (p >= kb + nb && !mark[p]) {
                mark[p] = 1;
                pm[NB + nd] = p;
                pm[2 * NB + nd] = mp[p];
                ++nd;
            }
        }
        pm[3 * NB] = nd;
    }
    // L_kk^-1 (forward, unit diagonal) by one half of the workgroup and
    // U_kk^-1 (backward; rows scaled by 1/U_kk at the end) by the other, one
    // elimination step per barrier.
    constexpr int GN = PN::THREADS / 2;
    const bool gU = tid >= GN;
    const int gt = gU ? tid - GN : tid;
    for (int s = 0; s < NB; ++s) {
        if (!gU) {
            const int k = s;
            for (int e = gt; e < (NB - 1 - k) * NB; e += GN) {
                const int i = k + 1 + e / NB, c = e % NB;
                XL[i][c] -= T[i][k] * XL[k][c];
            }
        } else {
            const int k = NB - 1 - s;
            const double invd = 1.0 / T[k][k];
            for (int e = gt; e < k * NB; e += GN) {
                const int i = e / NB, c = e % NB;
                XU[i][c] -= T[i][k] * (XU[k][c] * invd);
            }
        }
        __syncthreads();
    }
    double* Ti = tri + m * PN::TRI;
    for (int e = tid; e < NB * NB; e += PN::THREADS) {
        const int i = e / NB, c = e % NB;
        Ti[e] = XL[i][c];
        Ti[NB * NB + e] = XU[i][c] / T[i][i];
    }
    if (bad && tid == 0) record_status(status, m, ST_SINGULAR);
}

// ---------------------------------------------------------------------------
// 64 x 64 FP64 MFMA tile: acc (+)= sgn * A[r0.., 0..K) * Bt[0..K, c0..)
// with four waves in 2 x 2, each owning 2 x 2 blocks of 16 x 16 (register r of
// lane l holds row (l >> 4) + 4 r, column l & 15 of its block).  K is staged
// through LDS in chunks of GK with the next chunk's global loads issued
// before the current chunk is multiplied.
constexpr int GT = 64;
constexpr int GK = 16;
constexpr int GL = GT * GK / 256;              // elements of each operand chunk per thread

struct TileSmem {
    double As[2][GT][GK + 1];
    double Bs[2][GK][GT + 1];
};

template <bool NEG>
__device__ __forceinline__ void tile_mma(const double* A, int lda, const double* Bt, int ldb, int K, int r0,
                                         int c0, int rows, int cols, v4d acc[2][2], TileSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const double sgn = NEG ? -1.0 : 1.0;
    double ra[GL], rb[GL];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < GL; ++i) {
            const int e = tid + 256 * i;
            const int ar = e / GK, ak = e % GK;        // A chunk GT x GK
            const int r = r0 + ar, k = k0 + ak;
            ra[i] = (r < rows && k < K) ? A[(int64_t)r * lda + k] : 0.0;
            const int bk = e / GT, bc = e % GT;        // B chunk GK x GT
            const int kk = k0 + bk, c = c0 + bc;
            rb[i] = (kk < K && c < cols) ? Bt[(int64_t)kk * ldb + c] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < GL; ++i) {
            const int e = tid + 256 * i;
            sm.As[buf][e / GK][e % GK] = sgn * ra[i];
            sm.Bs[buf][e / GT][e % GT] = rb[i];
        }
    };
    const int nchunk = (K + GK - 1) / GK;
    load(0);
    stash(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) load((ch + 1) * GK);
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const int kq = ks + (lane >> 4);
            const double a0 = sm.As[buf][wr * 32 + (lane & 15)][kq];
            const double a1 = sm.As[buf][wr * 32 + 16 + (lane & 15)][kq];
            const double b0 = sm.Bs[buf][kq][wc * 32 + (lane & 15)];
            const double b1 = sm.Bs[buf][kq][wc * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (ch + 1 < nchunk) stash(buf ^ 1);
        __syncthreads();
    }
}

// tile_mma with the K rows of Bt taken from rows srcrow[k] of Bfull.
__device__ __forceinline__ void tile_mma_gather(const double* A, int lda, const double* Bfull, int ldb,
                                                const int* srcrow, int K, int r0, int c0, int rows, int cols,
                                                v4d acc[2][2], TileSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int nchunk = (K + GK - 1) / GK;
    for (int ch = 0; ch < nchunk; ++ch) {
        const int k0 = ch * GK;
#pragma unroll
        for (int i = 0; i < GL; ++i) {
            const int e = tid + 256 * i;
            const int ar = e / GK, ak = e % GK;
            const int r = r0 + ar, k = k0 + ak;
            sm.As[0][ar][ak] = (r < rows && k < K) ? A[(int64_t)r * lda + k] : 0.0;
            const int bk = e / GT, bc = e % GT;
            const int kk = k0 + bk, c = c0 + bc;
            sm.Bs[0][bk][bc] = (kk < K && c < cols) ? Bfull[(int64_t)srcrow[kk] * ldb + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            const int kq = ks + (lane >> 4);
            const double a0 = sm.As[0][wr * 32 + (lane & 15)][kq];
            const double a1 = sm.As[0][wr * 32 + 16 + (lane & 15)][kq];
            const double b0 = sm.Bs[0][kq][wc * 32 + (lane & 15)];
            const double b1 = sm.Bs[0][kq][wc * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int tile_row(int r0, int bi, int q) {
    const int lane = threadIdx.x & 63, wr = (threadIdx.x >> 6) >> 1;
    return r0 + wr * 32 + bi * 16 + (lane >> 4) + 4 * q;
}
__device__ __forceinline__ int tile_col(int c0, int bj) {
    const int lane = threadIdx.x & 63, wc = (threadIdx.x >> 6) & 1;
    return c0 + wc * 32 + bj * 16 + (lane & 15);
}

// ---------------------------------------------------------------------------
// In-place triangular applications of one panel, on MFMA:
//   blocks [0, ct):      U_top[:, c-tile] <- L_kk^-1 U_top[:, c-tile]   (columns >= kb+nb)
//   blocks [ct, ct+rt):  L21[r-tile, :]   <- X_panel[r-tile, :] U_kk^-1 (rows NV..)
// Each workgroup reads the whole 64 x 64 (or 64 x nb) block it overwrites
// before writing it.
template <int P>
__global__ void __launch_bounds__(256) k_tri(double* B, int kb, const double* __restrict__ tri,
                                             const int32_t* __restrict__ perm) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, ld = BD::ld, ROWS = BD::rows;
    __shared__ TileSmem sm;
    __shared__ int pm[3 * NB + 1];
    const int64_t m = blockIdx.y;
    double* Bm = B + m * BD::per_macro;
    const double* Ti = tri + m * PN::TRI;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int c0 = kb + nb;
    const int ct = (ld - c0 + GT - 1) / GT;
    v4d acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
    if ((int)blockIdx.x < ct) {
        const int cc = c0 + blockIdx.x * GT;     // columns [cc, cc+64) of the S rows
        for (int i = threadIdx.x; i < 3 * NB + 1; i += blockDim.x) pm[i] = perm[m * (3 * NB + 1) + i];
        __syncthreads();
        const int nd = pm[3 * NB];
        // displaced rows below the block read their new values before anything is written
        double mvr[NB * GT / 256];
#pragma unroll
        for (int i = 0; i < NB * GT / 256; ++i) {
            const int e = threadIdx.x + 256 * i, q = e / GT, c = cc + e % GT;
            mvr[i] = (q < nd && c < ld) ? Bm[(int64_t)pm[2 * NB + q] * ld + c] : 0.0;
        }
        tile_mma_gather(Ti, NB, Bm, ld, pm, nb, 0, cc, nb, ld, acc, sm);
#pragma unroll
        for (int i = 0; i < NB * GT / 256; ++i) {
            const int e = threadIdx.x + 256 * i, q = e / GT, c = cc + e % GT;
            if (q < nd && c < ld) Bm[(int64_t)pm[NB + q] * ld + c] = mvr[i];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = tile_row(0, bi, q), c = tile_col(cc, bj);
                    if (r < nb && c < ld) Bm[(int64_t)(kb + r) * ld + c] = acc[bi][bj][q];
                }
    } else {
        const int rr = NV + (blockIdx.x - ct) * GT;   // rows [rr, rr+64) of the X block
        tile_mma<false>(Bm + kb, ld, Ti + NB * NB, NB, nb, rr, 0, ROWS, nb, acc, sm);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = tile_row(rr, bi, q), c = tile_col(0, bj);
                    if (r < ROWS && c < nb) Bm[(int64_t)r * ld + kb + c] = acc[bi][bj][q];
                }
    }
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

// TAG only separates the trailing-update launches (0) from the final Schur
// product (1) in profiles; the code is the same.
template <int TAG>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ TileSmem sm;
    const int64_t m = blockIdx.y;
    const int tr = blockIdx.x / g.tiles_c, tc = blockIdx.x % g.tiles_c;
    const int r0 = tr * GT, c0 = tc * GT;
    if (r0 >= g.skip_r && c0 >= g.skip_c) return;   // tile entirely in the masked corner
    const double* C = g.C + m * g.sC;
    // C is fetched first and only added after the K loop, so its latency
    // overlaps the staging and the MFMA work.
    double cr[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = tile_row(r0, bi, q), c = tile_col(c0, bj);
                const bool in = r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c);
                cr[bi][bj][q] = in ? C[(int64_t)r * g.ldc + c] : 0.0;
            }
    v4d acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
    tile_mma<true>(g.A + m * g.sA, g.lda, g.Bt + m * g.sB, g.ldb, g.K, r0, c0, g.rows, g.cols, acc, sm);
    double* D = g.D ? g.D + m * g.sD : nullptr;
    double* D2 = g.D2 ? g.D2 + m * g.sD2 : nullptr;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = tile_row(r0, bi, q), c = tile_col(c0, bj);
                if (r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c)) {
                    const double v = cr[bi][bj][q] + acc[bi][bj][q];
                    if (D2 && c >= g.dsplit) D2[(int64_t)r * g.ldd2 + (c - g.dsplit)] = v;
                    else if (D) D[(int64_t)r * g.ldd + c] = v;
                }
            }
}

}  // namespace mehdg
