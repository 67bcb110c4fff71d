// Global trace system of one Newton step (Sec. 6.2, Algorithm 1):
//   K dVhat = F,  K = sum_m P_m^T Ahat_m P_m,  F = sum_m P_m^T bhat_m,
// the linearisation of sum_m R_Vhat,m = 0 (conservation on every face) with
// the trace single-valued per global face.  P_m gathers the six faces of
// macro m; a global face has exactly two sides (m1, f1), (m2, f2), whose
// nodes are ordered alike (axis-aligned boxes of one orientation), so every
// face-local block of 5 nf unknowns maps one to one.
//
// Kernels: the face sums (F, and K x from per-macro products), the gather
// of a local trace, the matrix-free product Ahat_m x_m of every macro, the
// inverse of the diagonal face blocks of K (block Jacobi, Sec. 6.4) by
// in-place Gauss-Jordan with partial pivoting in LDS, its application, and
// the vector kernels of GMRES.
#pragma once
#include "k_condense.hpp"

namespace mehdg {

// dst[g][e] = src[m1][f1][e] + src[m2][f2][e]  (face blocks of BS = 5 nf values)
// side[g] = {m1, f1, m2, f2}; m2 = -1 on a wall face (one side)
template <int P>
__global__ void __launch_bounds__(128) k_face_sum(const double* __restrict__ src, const int64_t* __restrict__ side,
                                                  double* __restrict__ dst, int64_t n_faces) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, NH = D::NH;
    const int64_t g = blockIdx.x;
    if (g >= n_faces) return;
    const int64_t m1 = side[4 * g], f1 = side[4 * g + 1], m2 = side[4 * g + 2], f2 = side[4 * g + 3];
    for (int e = threadIdx.x; e < BS; e += blockDim.x)
        dst[g * BS + e] = src[m1 * NH + f1 * BS + e] + (m2 >= 0 ? src[m2 * NH + f2 * BS + e] : 0.0);
}

// xl[m][f][e] = xg[fid[m][f]][e]
template <int P>
__global__ void __launch_bounds__(256) k_face_gather(const double* __restrict__ xg, const int64_t* __restrict__ fid,
                                                     double* __restrict__ xl, int64_t n_macro) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, NH = D::NH;
    const int64_t m = blockIdx.x;
    if (m >= n_macro) return;
    for (int i = threadIdx.x; i < NH; i += blockDim.x) xl[m * NH + i] = xg[fid[6 * m + i / BS] * BS + i % BS];
}

// yl[m] = Ahat_m (P_m x): 64 rows of one macro per workgroup, each wave
// RB = 8 rows at a time with lanes along the row and DPP wave sums.
template <int P>
__global__ void __launch_bounds__(256) k_local_apply(const double* __restrict__ Ahat, const double* __restrict__ xg,
                                                     const int64_t* __restrict__ fid, double* __restrict__ yl,
                                                     int64_t n_macro) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, NH = D::NH, RT = (NH + 63) / 64, RB = 8;
    __shared__ double x[NH];
    int64_t m;
    int tile;
    xcd_tile(RT, m, tile);
    if (m >= n_macro) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < NH; i += blockDim.x) x[i] = xg[fid[6 * m + i / BS] * BS + i % BS];
    __syncthreads();
    const double* A = Ahat + m * (int64_t)NH * NH;
    const int rlo = tile * 64, rhi = (rlo + 64) < NH ? (rlo + 64) : NH;
    for (int r0 = rlo + wave * RB; r0 < rhi; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < NH; c += 64) {
            const double xc = x[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < rhi) s[i] += A[(int64_t)(r0 + i) * NH + c] * xc;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < rhi) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            yl[m * NH + r0 + lane] = si;
        }
    }
}

// ---------------------------------------------------------------------------
// Matrix-free product with the reduced operator (Algorithm 1, the four stages
// of the local product), from the factors an FP64 condensation leaves in the
// bordered matrix: U12 = L^-1 P (-Y) in the S rows' trace columns and
// L21 = X U^-1 in place of X, with A' untouched.  Since
// S^-1 Y x = -U^-1 U12 x and X = L21 U,
//   Ahat_m x_m = A' x_m + X S^-1 Y x_m = A' x_m - L21 (U12 x_m),
// two products per macro and no triangular solve; Ahat is never formed.
// Phase 1: w_m = U12 x_m (N_V rows); phase 2: yl_m = A' x_m - L21 w_m (N_VH
// rows); 64 rows of one macro per workgroup, lanes along the rows (coalesced).
// The factors are read as T: double from the bordered matrix (stride sm per
// macro, leading dimension ld), or float from their single-precision copies
// (k_mf_to_f32) for the inner iterations of FGMRES; sums are FP64 in both.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_mf_w(const T* __restrict__ U12, int64_t sm, int ldu,
                                              const double* __restrict__ xg, const int64_t* __restrict__ fid,
                                              double* __restrict__ w, int64_t n_macro) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, NV = D::NV, NH = D::NH, RT = (NV + 63) / 64, RB = 8;
    __shared__ double x[NH];
    int64_t m;
    int tile;
    xcd_tile(RT, m, tile);
    if (m >= n_macro) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < NH; i += blockDim.x) x[i] = xg[fid[6 * m + i / BS] * BS + i % BS];
    __syncthreads();
    const T* U = U12 + m * sm;
    const int rlo = tile * 64, rhi = (rlo + 64) < NV ? (rlo + 64) : NV;
    for (int r0 = rlo + wave * RB; r0 < rhi; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < NH; c += 64) {
            const double xc = x[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < rhi) s[i] += (double)U[(int64_t)(r0 + i) * ldu + c] * xc;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < rhi) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            w[m * NV + r0 + lane] = si;
        }
    }
}

// L21 [NH][NV] (leading dimension ldl) and A' [NH][NH] (leading dimension
// lda), both at stride sm per macro.
template <int P, typename T>
__global__ void __launch_bounds__(256) k_mf_y(const T* __restrict__ L21, const T* __restrict__ Ap, int64_t sm,
                                              int ldl, int lda, const double* __restrict__ xg,
                                              const int64_t* __restrict__ fid, const double* __restrict__ w,
                                              double* __restrict__ yl, int64_t n_macro) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, NV = D::NV, NH = D::NH, RT = (NH + 63) / 64, RB = 8;
    __shared__ double x[NH];
    __shared__ double ws[NV];
    int64_t m;
    int tile;
    xcd_tile(RT, m, tile);
    if (m >= n_macro) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < NH; i += blockDim.x) x[i] = xg[fid[6 * m + i / BS] * BS + i % BS];
    for (int i = threadIdx.x; i < NV; i += blockDim.x) ws[i] = w[m * NV + i];
    __syncthreads();
    const T* Lm = L21 + m * sm;
    const T* Am = Ap + m * sm;
    const int rlo = tile * 64, rhi = (rlo + 64) < NH ? (rlo + 64) : NH;
    for (int r0 = rlo + wave * RB; r0 < rhi; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < NV; c += 64) {
            const double wc = ws[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < rhi) s[i] -= (double)Lm[(int64_t)(r0 + i) * ldl + c] * wc;
        }
        for (int c = lane; c < NH; c += 64) {
            const double xc = x[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < rhi) s[i] += (double)Am[(int64_t)(r0 + i) * lda + c] * xc;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < rhi) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            yl[m * NH + r0 + lane] = si;
        }
    }
}

// Single-precision copies of the factors the matrix-free product reads, per
// macro [U12: NV x NH | L21: NH x NV | A': NH x NH] (rounded to nearest),
// one row of the bordered matrix per workgroup row.
template <int P>
struct MfF32 {
    static constexpr int NV = Dims<P>::NV, NH = Dims<P>::NH;
    static constexpr int64_t per_macro = 2LL * NV * NH + (int64_t)NH * NH;
    static constexpr int64_t off_l21 = (int64_t)NV * NH, off_ap = 2LL * NV * NH;
};

template <int P>
__global__ void __launch_bounds__(256) k_mf_to_f32(const double* __restrict__ B, float* __restrict__ F32,
                                                   int64_t n_macro) {
    using BD = Bdims<P>;
    using MF = MfF32<P>;
    constexpr int NV = MF::NV, NH = MF::NH, ld = BD::ld;
    const int r = blockIdx.x;                     // bordered row, 0 .. NV + NH - 1
    for (int64_t m = blockIdx.y; m < n_macro; m += gridDim.y) {
        const double* row = B + m * BD::per_macro + (int64_t)r * ld;
        float* out = F32 + m * MF::per_macro;
        if (r < NV) {
            for (int c = threadIdx.x; c < NH; c += blockDim.x) out[(int64_t)r * NH + c] = (float)row[NV + c];
        } else {
            const int q = r - NV;
            for (int c = threadIdx.x; c < NV; c += blockDim.x)
                out[MF::off_l21 + (int64_t)q * NV + c] = (float)row[c];
            for (int c = threadIdx.x; c < NH; c += blockDim.x)
                out[MF::off_ap + (int64_t)q * NH + c] = (float)row[NV + c];
        }
    }
}

// Diagonal face blocks of K from the factors, without Ahat:
//   D_g = Ahat_m1[f1,f1] + Ahat_m2[f2,f2] (+ Ahat_m[f1,f2] + Ahat_m[f2,f1] when
//   both sides belong to one macro m),  Ahat_m[a,b] = A'[a,b] - L21[a,:] U12[:,b],
// each 128 x 64 tile of the BS x BS block on FP64 MFMA (K = N_V), written to
// the inverse workspace where k_face_block_inv<P, true> then inverts it.
template <int P>
__global__ void __launch_bounds__(GTHREADS, 4) k_mf_face_blocks(const double* __restrict__ B,
                                                                const int64_t* __restrict__ side,
                                                                double* __restrict__ Dblk, int64_t n_faces) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int BS = 5 * D::nf, NV = D::NV, ld = BD::ld;
    constexpr int TR = (BS + GM - 1) / GM, TC = (BS + GT - 1) / GT;
    __shared__ TileSmem sm;
    const int64_t g = blockIdx.x / (TR * TC);
    if (g >= n_faces) return;
    const int t = (int)(blockIdx.x % (TR * TC)), r0 = (t / TC) * GM, c0 = (t % TC) * GT;
    const int64_t m1 = side[4 * g], f1 = side[4 * g + 1], m2 = side[4 * g + 2], f2 = side[4 * g + 3];
    v4d acc[2][2];
    zero_acc(acc);
    // Ahat_m[a, b] tile: A' part added below, - L21[a rows] U12[b cols] accumulated here
    auto product = [&](int64_t m, int64_t fa, int64_t fb) {
        const double* Bm = B + m * BD::per_macro;
        tile_mma<true>(Bm + (int64_t)(NV + fa * BS) * ld, ld, Bm + NV + fb * BS, ld, NV, r0, c0, BS, BS, acc, sm);
        __syncthreads();
    };
    const bool same = m1 == m2, two = m2 >= 0;   // a wall face has one side
    product(m1, f1, f1);
    if (two) product(m2, f2, f2);
    if (same) {
        product(m1, f1, f2);
        product(m1, f2, f1);
    }
    double* out = Dblk + g * (int64_t)BS * BS;
    auto aprime = [&](int64_t m, int64_t fa, int64_t fb, int r, int c) {
        return B[m * BD::per_macro + (int64_t)(NV + fa * BS + r) * ld + NV + fb * BS + c];
    };
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = tile_row(r0, bi, q), c = tile_col(c0, bj);
                if (r < BS && c < BS) {
                    double d = acc[bi][bj][q] + aprime(m1, f1, f1, r, c) + (two ? aprime(m2, f2, f2, r, c) : 0.0);
                    if (same) d += aprime(m1, f1, f2, r, c) + aprime(m1, f2, f1, r, c);
                    out[(int64_t)r * BS + c] = d;
                }
            }
}

// Inverse of every diagonal face block of K:
//   D_g = Ahat_m1[f1, f1] + Ahat_m2[f2, f2]   (BS x BS),
// plus Ahat_m[f1, f2] + Ahat_m[f2, f1] when both sides belong to one macro m,
// in place in LDS by Gauss-Jordan elimination with row pivoting; the row
// interchanges become column interchanges of the inverse, undone at the end.
template <int P>
struct BlockInvLds {
    static constexpr int BS = 5 * Dims<P>::nf;
    double a[BS][BS + 1];
    double colk[BS];
    int piv[BS];
    double redv[4];
    int redi[4];
};

// Pivot column, pivots and reductions only: the block itself is eliminated in
// place in the global inverse workspace (blocks too large for LDS, p = 3:
// 245 x 245).  Every step then sweeps the block through L2; correct, not fast.
template <int P>
struct BlockInvSmall {
    static constexpr int BS = 5 * Dims<P>::nf;
    double colk[BS];
    int piv[BS];
    double redv[4];
    int redi[4];
};

template <int P>
struct BlockInvCfg {
    static constexpr bool in_lds = sizeof(BlockInvLds<P>) <= 150 * 1024;
    static constexpr size_t lds_bytes = in_lds ? sizeof(BlockInvLds<P>) : sizeof(BlockInvSmall<P>);
};

// Inverse of the diagonal face block of K by Gauss-Jordan with row pivoting.
// FROM_BLOCK: the block was already formed in Dinv (k_mf_face_blocks) and Ahat is unused.
template <int P, bool FROM_BLOCK>
__global__ void __launch_bounds__(256) k_face_block_inv(const double* __restrict__ Ahat,
                                                        const int64_t* __restrict__ side, double* __restrict__ Dinv,
                                                        int64_t n_faces) {
    using D = Dims<P>;
    using CFG = BlockInvCfg<P>;
    constexpr int BS = 5 * D::nf, NH = D::NH;
    constexpr int lda = CFG::in_lds ? BS + 1 : BS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    BlockInvLds<P>& LL = *reinterpret_cast<BlockInvLds<P>*>(smem_raw);
    BlockInvSmall<P>& LS = *reinterpret_cast<BlockInvSmall<P>*>(smem_raw);
    double* colk = CFG::in_lds ? LL.colk : LS.colk;
    int* piv = CFG::in_lds ? LL.piv : LS.piv;
    double* redv = CFG::in_lds ? LL.redv : LS.redv;
    int* redi = CFG::in_lds ? LL.redi : LS.redi;
    const int64_t g = blockIdx.x;
    if (g >= n_faces) return;
    double* out = Dinv + g * (int64_t)BS * BS;
    double* a = CFG::in_lds ? &LL.a[0][0] : out;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m1 = side[4 * g], f1 = side[4 * g + 1], m2 = side[4 * g + 2], f2 = side[4 * g + 3];
    const bool two = m2 >= 0;   // a wall face has one side
    const double* A1 = Ahat + m1 * (int64_t)NH * NH + (f1 * BS) * (int64_t)NH + f1 * BS;
    const double* A2 = two ? Ahat + m2 * (int64_t)NH * NH + (f2 * BS) * (int64_t)NH + f2 * BS : A1;
    // both sides on one macro (a periodic box one macro wide): K's block also
    // holds that macro's couplings between the two faces
    const bool same = m1 == m2;
    const double* A12 = Ahat + m1 * (int64_t)NH * NH + (f1 * BS) * (int64_t)NH + f2 * BS;
    const double* A21 = Ahat + m1 * (int64_t)NH * NH + (f2 * BS) * (int64_t)NH + f1 * BS;
    if constexpr (FROM_BLOCK) {
        if constexpr (CFG::in_lds)
            for (int e = tid; e < BS * BS; e += blockDim.x) a[(e / BS) * lda + e % BS] = out[e];
    } else {
        for (int e = tid; e < BS * BS; e += blockDim.x) {
            const int i = e / BS, j = e % BS;
            double d = A1[(int64_t)i * NH + j] + (two ? A2[(int64_t)i * NH + j] : 0.0);
            if (same) d += A12[(int64_t)i * NH + j] + A21[(int64_t)i * NH + j];
            a[i * lda + j] = d;
        }
    }
    __syncthreads();
    for (int k = 0; k < BS; ++k) {
        // pivot: largest |a[i][k]|, i >= k (ties to the lower row)
        double best = -1.0;
        int bi = BS;
        for (int i = k + tid; i < BS; i += blockDim.x) {
            const double v = fabs(a[i * lda + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        const double wm = wave_max_f64(best);
        const unsigned long long bal = __ballot(best == wm && bi < BS);
        const int ol = bal ? (__ffsll((long long)bal) - 1) : 0;
        const int wrow = __builtin_amdgcn_readlane(bi, ol);
        if (lane == 0) {
            redv[wave] = wm;
            redi[wave] = bal ? wrow : BS;
        }
        __syncthreads();
        int p = redi[0];
        double b = redv[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (redv[w] > b || (redv[w] == b && redi[w] < p)) {
                b = redv[w];
                p = redi[w];
            }
        if (p >= BS) p = k;
        if (tid == 0) piv[k] = p;
        if (p != k)
            for (int j = tid; j < BS; j += blockDim.x) {
                const double t = a[k * lda + j];
                a[k * lda + j] = a[p * lda + j];
                a[p * lda + j] = t;
            }
        __syncthreads();
        const double inv = 1.0 / a[k * lda + k];
        for (int i = tid; i < BS; i += blockDim.x) colk[i] = a[i * lda + k];
        __syncthreads();
        // row k scaled, a[k][k] <- 1 / pivot
        for (int j = tid; j < BS; j += blockDim.x) a[k * lda + j] = (j == k) ? inv : a[k * lda + j] * inv;
        __syncthreads();
        // every other row: a[i][j] -= a[i][k] a[k][j], with a[i][k] <- -a[i][k] / pivot
        for (int e = tid; e < BS * BS; e += blockDim.x) {
            const int i = e / BS, j = e % BS;
            if (i == k) continue;
            const double f = colk[i];
            if (j == k) a[i * lda + j] = -f * inv;
            else a[i * lda + j] -= f * a[k * lda + j];
        }
        __syncthreads();
    }
    // row interchanges of the elimination = column interchanges of the inverse, in reverse
    for (int k = BS - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k)
            for (int i = tid; i < BS; i += blockDim.x) {
                const double t = a[i * lda + k];
                a[i * lda + k] = a[i * lda + p];
                a[i * lda + p] = t;
            }
        __syncthreads();
    }
    if constexpr (CFG::in_lds)
        for (int e = tid; e < BS * BS; e += blockDim.x) out[e] = a[(e / BS) * lda + e % BS];
}

// z[g] = Dinv_g r[g]
template <int P>
__global__ void __launch_bounds__(256) k_face_block_apply(const double* __restrict__ Dinv, const double* __restrict__ r,
                                                          double* __restrict__ z, int64_t n_faces) {
    using D = Dims<P>;
    constexpr int BS = 5 * D::nf, RB = 8;
    __shared__ double x[BS];
    const int64_t g = blockIdx.x;
    if (g >= n_faces) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = threadIdx.x; i < BS; i += blockDim.x) x[i] = r[g * BS + i];
    __syncthreads();
    const double* A = Dinv + g * (int64_t)BS * BS;
    for (int r0 = wave * RB; r0 < BS; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < BS; c += 64) {
            const double xc = x[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < BS) s[i] += A[(int64_t)(r0 + i) * BS + c] * xc;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < BS) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            z[g * BS + r0 + lane] = si;
        }
    }
}

// ---------------------------------------------------------------------------
// Vector kernels of GMRES (n doubles per vector, nv <= 64 basis vectors).

// partial[i][b] = sum over block b's elements of V[i] * w
__global__ void __launch_bounds__(256) k_dots(const double* __restrict__ V, int64_t n, int nv,
                                              const double* __restrict__ w, double* __restrict__ partial) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int i = 0; i < nv; ++i) {
        const double* v = V + (int64_t)i * n;
        double s = 0.0;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) s += v[e] * w[e];
        s = wave_sum_f64(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[(int64_t)i * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// w += sum_i c[i] V[i]
__global__ void __launch_bounds__(256) k_combine(const double* __restrict__ V, int64_t n, int nv,
                                                 const double* __restrict__ c, double* __restrict__ w) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double s = w[e];
        for (int i = 0; i < nv; ++i) s += c[i] * V[(int64_t)i * n + e];
        w[e] = s;
    }
}

// y = a x + b y
__global__ void __launch_bounds__(256) k_axpby(int64_t n, double a, const double* __restrict__ x, double b,
                                               double* __restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        y[e] = (a == 0.0 ? 0.0 : a * x[e]) + (b == 0.0 ? 0.0 : b * y[e]);
}

// Constant source of a DIRK stage: R_v += s and r_V -= s in the bordered
// matrix (the rows of the interior equations), per macro.
template <int P>
__global__ void __launch_bounds__(256) k_add_source(const double* __restrict__ s, double* __restrict__ R_v,
                                                    double* __restrict__ B, int64_t n_macro) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int NV = D::NV, NH = D::NH, ld = BD::ld;
    const int64_t m = blockIdx.x;
    if (m >= n_macro) return;
    for (int a = threadIdx.x; a < NV; a += blockDim.x) {
        const double v = s[m * NV + a];
        R_v[m * NV + a] += v;
        B[m * BD::per_macro + (int64_t)a * ld + NV + NH] -= v;
    }
}

}  // namespace mehdg
