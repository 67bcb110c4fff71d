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
// Two-level blocking.  The columns of S go in outer blocks of OB = 128, each
// made of (up to) two register panels of NB = 64:
//   k_panel     one workgroup per macro: factor the S rows of one panel (one
//               row per thread, the panel segment in registers) and invert
//               its diagonal blocks L_kk, U_kk.  The second panel of a block
//               also re-orders the first panel's L columns by its own
//               interchanges, composes the interchanges of both panels and
//               forms the inverse of the block's unit-lower diagonal block;
//   k_tri       per 64-column tile right of the (panel or outer) block: apply
//               the composed row interchange and form U_top = L^-1 (P B)_top
//               on MFMA;
//   k_gemm      rank-nb update of the S rows on FP64 MFMA: inside the outer
//               block, the second panel's columns after the first panel;
//               after the block, the S rows right of it (S and border
//               columns) with K = 128.
// Delayed trailing updates: the outer blocks go in groups of G (the depth;
// G = 1 updates after every block, G >= the block count is left-looking).
// A block whose group has earlier blocks first takes their pending update
// on its own columns (k_gemm, K = the group's earlier columns), is factored
// as above, moves the earlier blocks' multipliers by its interchange
// (k_perm_rows, so that their rows stay in step with the rows they update),
// and k_tri subtracts their pending product from its U rows before the
// triangular solve.  After the last block of a group one k_gemm updates the
// S rows below with K = the group's width, so the trailing matrix is read and
// written once per group instead of once per block.
// The X rows take no part in the factorisation of S.  Afterwards, panel by
// panel, k_trsm_x forms L21 = X U^-1 left-looking,
//   L21[:, q] = (X[:, q] - L21[:, <q] U[<q, q]) U_qq^-1,
// long-K MFMA products written once, in place of X.  Then one k_gemm with
// K = N_V forms Ahat = A' - L21 U12 and bhat = r_hat - L21 y directly in the
// caller's arrays.
#pragma once
#include <type_traits>

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

// Wave-wide sum with the same permutations; every lane gets the sum.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_perm_f64(v, 0);
    v += dpp_perm_f64(v, 1);
    v += dpp_perm_f64(v, 2);
    v += dpp_perm_f64(v, 3);
    return (read_lane_f64(v, 0) + read_lane_f64(v, 16)) + (read_lane_f64(v, 32) + read_lane_f64(v, 48));
}

__device__ __forceinline__ double wave_max_f64(double v) {
    v = fmax(v, dpp_perm_f64(v, 0));
    v = fmax(v, dpp_perm_f64(v, 1));
    v = fmax(v, dpp_perm_f64(v, 2));
    v = fmax(v, dpp_perm_f64(v, 3));
    return fmax(fmax(read_lane_f64(v, 0), read_lane_f64(v, 16)), fmax(read_lane_f64(v, 32), read_lane_f64(v, 48)));
}

// panel and outer block widths of the blocked factorisation
template <int P>
struct Panel {
    static constexpr int NB = 64;
    static constexpr int OB = 2 * NB;
    static constexpr int NV = Dims<P>::NV;
    // one thread per S row, at least two waves (wave 0 inverts L_kk, wave 1
    // U_kk), at most 1024 threads
    static constexpr int THREADS_R = ((NV + 63) / 64) * 64 > 1024 ? 1024 : ((NV + 63) / 64) * 64;
    static constexpr int THREADS = THREADS_R < 128 ? 128 : THREADS_R;
    static constexpr int RPT = (NV + THREADS - 1) / THREADS;   // S rows per thread
    static constexpr int NPAN = (NV + NB - 1) / NB;             // panels of S
    // per macro: L^-1 of the first and of the second panel of the current
    // outer block (NB x NB each), L^-1 of the block's unit-lower diagonal block
    // (OB x OB), then U_kk^-1 of every panel (NPAN x NB x NB, kept for the
    // triangular solve of the X rows)
    static constexpr int LINV1 = 0, LINV2 = NB * NB, LINVW = 2 * NB * NB, UINV = 2 * NB * NB + OB * OB;
    static constexpr int64_t TRI = (int64_t)UINV + (int64_t)NPAN * NB * NB;
    // per macro: composed interchange of the current block: [0, OB) source
    // rows of the top rows, [OB, 2 OB) rows below the block that change,
    // [2 OB, 3 OB) their source rows, [3 OB] their number
    static constexpr int64_t PERM = 3 * OB + 1;
};

// 64 x 64 x 64 products of LDS matrices (leading dimension N + 1) on FP64
// MFMA: the sixteen 16 x 16 output tiles are dealt to the NW waves, TPW per
// wave; register r of lane l holds row (l >> 4) + 4 r, column l & 15 of a tile.
template <int N, int NW, int TPW>
__device__ __forceinline__ void lds_mm64(const double (*A)[N + 1], const double (*Bm)[N + 1], v4d (&acc)[TPW]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
        const int t = wave + NW * i;
        if (t < 16) {
            const int ti = t >> 2, tj = t & 3;
#pragma unroll
            for (int k0 = 0; k0 < N; k0 += 4) {
                const double a = A[ti * 16 + (lane & 15)][k0 + (lane >> 4)];
                const double b = Bm[k0 + (lane >> 4)][tj * 16 + (lane & 15)];
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
            }
        }
    }
}

template <int N, int NW, int TPW>
__device__ __forceinline__ void lds_mm64_store(const v4d (&acc)[TPW], double (*D)[N + 1], double scale) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int t = wave + NW * i;
        if (t < 16) {
            const int ti = t >> 2, tj = t & 3;
#pragma unroll
            for (int r = 0; r < 4; ++r) D[ti * 16 + (lane >> 4) + 4 * r][tj * 16 + (lane & 15)] = scale * acc[i][r];
        }
    }
}

template <int N, int NW, int TPW>
__device__ __forceinline__ void lds_mm64_store_global(const v4d (&acc)[TPW], double* D, int ldd, double scale) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int t = wave + NW * i;
        if (t < 16) {
            const int ti = t >> 2, tj = t & 3;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                D[(int64_t)(ti * 16 + (lane >> 4) + 4 * r) * ldd + tj * 16 + (lane & 15)] = scale * acc[i][r];
        }
    }
}

// D = sgn * A B for 32 x 32 LDS matrices (leading dimension LD) by one wave
// on FP64 MFMA: four 16 x 16 output tiles, K in steps of 4 (register r of lane
// l holds row (l >> 4) + 4 r, column l & 15 of a tile).
template <int LD>
__device__ __forceinline__ void wave_mm32(const double* A, const double* B, double* D, double sgn) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, kq = lane >> 4;
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
        const double a0 = A[r16 * LD + k0 + kq], a1 = A[(16 + r16) * LD + k0 + kq];
        const double b0 = B[(k0 + kq) * LD + r16], b1 = B[(k0 + kq) * LD + 16 + r16];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) D[(16 * i + kq + 4 * r) * LD + 16 * j + r16] = sgn * acc[i][j][r];
}

// LDS of a panel kernel that the common end of the panel (panel_finish) uses.
template <int P>
struct PanelShared {
    static constexpr int NB = Panel<P>::NB, NV = Panel<P>::NV;
    double raw[3 * NB * (NB + 1)];   // staging, then T and the two inverses
    int pidj[NB];                    // pivot row (identity) of each column
    int pivs[NB];                    // pivot position of each column (LAPACK order)
    int mvd[2 * NB], mvs[2 * NB];    // rows whose first-panel segment moves, and their sources
    int nmv;
    int pv1[NB];                     // the first panel's pivots (second panel only)
    int mp[NV];                      // position -> row identity
    int ps[NV];                      // row identity -> position
    int mark[NV];
};

// Common end of a panel once its rows sit at their final positions: the
// pivots, this panel's interchange as lists (perm for the first panel of an
// outer block; for the second, the rows whose first-panel multipliers move,
// which it then moves), the composed interchange of the block, and the
// inverses of the diagonal blocks (L_kk, U_kk; for the second panel the whole
// block's unit-lower inverse on MFMA).
template <int P>
__device__ __forceinline__ void panel_finish(PanelShared<P>& sh, double* __restrict__ Bm, int kb, int kb0, int nb,
                                             int64_t m, int32_t* __restrict__ ipiv, int32_t* __restrict__ perm,
                                             double* __restrict__ tri, bool bad, int32_t* __restrict__ status) {
    using PN = Panel<P>;
    constexpr int NB = PN::NB, OB = PN::OB, NV = PN::NV, ld = Bdims<P>::ld;
    constexpr int NT = PN::THREADS, NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool second = kb > kb0;
    double(&raw)[3 * NB * (NB + 1)] = sh.raw;
    int(&pivs)[NB] = sh.pivs;
    int(&mvd)[2 * NB] = sh.mvd;
    int(&mvs)[2 * NB] = sh.mvs;
    int& nmv = sh.nmv;
    int(&pv1)[NB] = sh.pv1;
    int(&mp)[NV] = sh.mp;
    int(&mark)[NV] = sh.mark;
    if (tid < nb) ipiv[m * NV + kb + tid] = pivs[tid];
    // this panel's interchange as lists: perm (first panel) or the rows whose
    // first-panel multipliers move (second panel)
    if (tid == 0) {
        int n = 0;
        int32_t* pm = perm + m * PN::PERM;
#pragma clang loop unroll(disable)
        for (int i = 0; i < nb; ++i) {
            const int r = kb + i;
            if (second && mp[r] != r) {
                mvd[n] = r;
                mvs[n] = mp[r];
                ++n;
            }
            if (!second) pm[i] = mp[r];
        }
        int nd = 0;
#pragma clang loop unroll(disable)
        for (int i = 0; i < nb; ++i) {
            const int q = pivs[i];
            if (q >= kb + nb && !mark[q]) {
                mark[q] = 1;
                if (second) {
                    mvd[n] = q;
                    mvs[n] = mp[q];
                    ++n;
                } else {
                    pm[OB + nd] = q;
                    pm[2 * OB + nd] = mp[q];
                    ++nd;
                }
            }
        }
        nmv = n;
        if (!second) pm[3 * OB] = nd;
    }
    __syncthreads();
    if (second) {
        // the first panel's multipliers follow this panel's interchange (read all, then write)
        const int cnt = nmv * NB;
        for (int e = tid; e < cnt; e += NT) raw[e] = Bm[(int64_t)mvs[e / NB] * ld + kb0 + e % NB];
        __syncthreads();
        for (int e = tid; e < cnt; e += NT) Bm[(int64_t)mvd[e / NB] * ld + kb0 + e % NB] = raw[e];
        // interchange of the whole outer block: the first panel's pivots, then this panel's
        for (int r = kb0 + tid; r < NV; r += NT) {
            mp[r] = r;
            mark[r] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            for (int i = 0; i < NB; ++i) {
                const int q = pv1[i];
                const int t = mp[kb0 + i];
                mp[kb0 + i] = mp[q];
                mp[q] = t;
            }
            for (int i = 0; i < nb; ++i) {
                const int q = pivs[i];
                const int t = mp[kb + i];
                mp[kb + i] = mp[q];
                mp[q] = t;
            }
            const int w = kb + nb - kb0;
            int32_t* pm = perm + m * PN::PERM;
            for (int i = 0; i < w; ++i) pm[i] = mp[kb0 + i];
            int nd = 0;
            for (int i = 0; i < NB + nb; ++i) {
                const int q = i < NB ? pv1[i] : pivs[i - NB];
                if (q >= kb0 + w && !mark[q]) {
                    mark[q] = 1;
                    pm[OB + nd] = q;
                    pm[2 * OB + nd] = mp[q];
                    ++nd;
                }
            }
            pm[3 * OB] = nd;
        }
        __syncthreads();
    }
    // diagonal block T (the pivot rows, now at kb..kb+nb) and the two inverses
    double (*T)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw);
    double (*XL)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw + NB * (NB + 1));
    double (*XU)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw + 2 * NB * (NB + 1));
    for (int e = tid; e < NB * NB; e += NT) {
        const int i = e / NB, c = e % NB;
        T[i][c] = (i < nb && c < nb) ? Bm[(int64_t)(kb + i) * ld + kb + c] : (i == c ? 1.0 : 0.0);
    }
    __syncthreads();
    // L_kk^-1 by wave 0 and U_kk^-1 by wave 1 in 32 x 32 blocks:
    //   L^-1 = [[A^-1, 0], [-D^-1 (C A^-1), D^-1]],  U^-1 = [[A^-1, -A^-1 (B D^-1)], [0, D^-1]].
    // Each lane inverts one column of a diagonal block in registers (lanes
    // 0..31 the first block, 32..63 the second; four partial sums per row),
    // then the wave forms the off-diagonal block with two 32 x 32 products on
    // MFMA, using the block of the result that stays zero as scratch.
    constexpr int H = NB / 2;
    static_assert(NB == 64, "the blocked inverse is written for 64-column panels");
    if (wave < 2) {
        const int hb = lane / H, cc = lane % H, o = hb * H;
        double x[H];
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < H; ++i) {
                double s0 = (i == cc) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int k = 0; k + 4 <= i; k += 4) {
                    s0 -= T[o + i][o + k] * x[k];
                    s1 -= T[o + i][o + k + 1] * x[k + 1];
                    s2 -= T[o + i][o + k + 2] * x[k + 2];
                    s3 -= T[o + i][o + k + 3] * x[k + 3];
                }
#pragma unroll
                for (int k = i & ~3; k < i; ++k) s0 -= T[o + i][o + k] * x[k];
                x[i] = (s0 + s1) + (s2 + s3);
            }
#pragma unroll
            for (int i = 0; i < H; ++i) XL[o + i][o + cc] = x[i];
        } else {
#pragma unroll
            for (int i = H - 1; i >= 0; --i) {
                double s0 = (i == cc) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int k = i + 1;
#pragma unroll
                for (; k + 4 <= H; k += 4) {
                    s0 -= T[o + i][o + k] * x[k];
                    s1 -= T[o + i][o + k + 1] * x[k + 1];
                    s2 -= T[o + i][o + k + 2] * x[k + 2];
                    s3 -= T[o + i][o + k + 3] * x[k + 3];
                }
#pragma unroll
                for (; k < H; ++k) s0 -= T[o + i][o + k] * x[k];
                x[i] = ((s0 + s1) + (s2 + s3)) / T[o + i][o + i];
            }
#pragma unroll
            for (int i = 0; i < H; ++i) XU[o + i][o + cc] = x[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (wave == 0) {
            wave_mm32<NB + 1>(&T[H][0], &XL[0][0], &XL[0][H], 1.0);     // C A^-1 into the zero block
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            wave_mm32<NB + 1>(&XL[H][H], &XL[0][H], &XL[H][0], -1.0);   // -D^-1 (C A^-1)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int i = 0; i < H; i += 2) XL[i + hb][H + cc] = 0.0;
        } else {
            wave_mm32<NB + 1>(&T[0][H], &XU[H][H], &XU[H][0], 1.0);     // B D^-1 into the zero block
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            wave_mm32<NB + 1>(&XU[0][0], &XU[H][0], &XU[0][H], -1.0);   // -A^-1 (B D^-1)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int i = 0; i < H; i += 2) XU[H + i + hb][cc] = 0.0;
        }
    }
    __syncthreads();
    double* Ti = tri + m * PN::TRI;
    double* Tl = Ti + (second ? PN::LINV2 : PN::LINV1);
    double* Tu = Ti + PN::UINV + (int64_t)(kb / NB) * NB * NB;
    for (int e = tid; e < NB * NB; e += NT) {
        const int i = e / NB, c = e % NB;
        Tl[e] = XL[i][c];
        Tu[e] = XU[i][c];
    }
    if (second) {
        // inverse of the block's unit-lower diagonal block [[L11, 0], [L21, L22]]:
        // [[L11^-1, 0], [-L22^-1 L21 L11^-1, L22^-1]]   (L22^-1 = XL), both products on MFMA
        __syncthreads();
        for (int e = tid; e < NB * NB; e += NT) {
            const int i = e / NB, c = e % NB;
            T[i][c] = (i < nb) ? Bm[(int64_t)(kb + i) * ld + kb0 + c] : 0.0;
            XU[i][c] = Ti[PN::LINV1 + e];
        }
        __syncthreads();
        constexpr int TPW = (16 + NW - 1) / NW;
        v4d acc[TPW];
        lds_mm64<NB, NW, TPW>(T, XU, acc);
        __syncthreads();
        lds_mm64_store<NB, NW, TPW>(acc, T, 1.0);
        __syncthreads();
        lds_mm64<NB, NW, TPW>(XL, T, acc);
        double* LW = Ti + PN::LINVW;
        lds_mm64_store_global<NB, NW, TPW>(acc, LW + NB * OB, OB, -1.0);
        for (int e = tid; e < OB * OB; e += NT) {
            const int i = e / OB, c = e % OB;
            if (i < NB) LW[e] = c < NB ? XU[i][c] : 0.0;
            else if (c >= NB) LW[e] = XL[i - NB][c - NB];
        }
    }
    if (bad && tid == 0) record_status(status, m, ST_SINGULAR);
}

// ---------------------------------------------------------------------------
// Panel factorisation.  Each thread owns one (or RPT) rows of S in [kb, NV)
// by identity: rows are never exchanged between threads, the pivot rows are
// only broadcast.  A row's 64 values live in registers as z[0..64) and move
// down by one register per column, so every column is the same code with
// constant register indices.  For a row that is not a pivot yet, after j
// columns z[0 .. 64-j) hold its current entries of columns j..63 and
// z[64-j .. 64) the multipliers of columns 0..j-1:
//   z[c] <- z[c+1] - l * prow[c+1]   (c < 63),   z[63] <- l,
// where the broadcast pivot row reads as zero over its multiplier part.  A
// pivot row takes l = 0 and z[63] <- z[0] instead, i.e. it just rotates, so
// after the last column every row's z[c] belongs to column (c + nb) mod 64.
// Column j: wave arg-max (DPP) and a reduction over the waves choose the
// pivot row, which is broadcast through LDS; the next column is updated
// first and its pivot search issued before the rest of the row (look-ahead),
// with the LDS buffers alternating by column parity: two barriers per column
// and no global memory traffic inside the column loop.  Afterwards the row
// interchanges are replayed (LAPACK order: position kb+j with the pivot's
// current position), rows go to their final positions through LDS
// (coalesced), the inverses of the diagonal blocks L_kk (unit lower) and
// U_kk are formed one column per lane, and the composed row interchange of
// the block goes to perm.  A panel with kb > kb0 is the second panel of the
// outer block that starts at kb0 (see the file comment).
template <int P>
__global__ void __launch_bounds__(Panel<P>::THREADS) k_panel(double* __restrict__ B, int kb, int kb0,
                                                             int32_t* __restrict__ ipiv,
                                                             int32_t* __restrict__ perm,
                                                             double* __restrict__ tri,
                                                             int32_t* __restrict__ status) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, RPT = PN::RPT, ld = BD::ld;
    constexpr int NT = PN::THREADS, NW = NT / 64;
    constexpr int CH = 3 * NB;                  // rows per staging chunk of raw
    __shared__ PanelShared<P> sh;
    __shared__ double prow[2][NB];              // pivot row (by column parity)
    __shared__ double redv[2][NW];
    __shared__ int redi[2][NW];
    double(&raw)[3 * NB * (NB + 1)] = sh.raw;
    int(&pidj)[NB] = sh.pidj;
    int(&pv1)[NB] = sh.pv1;
    int(&mp)[NV] = sh.mp;
    int(&ps)[NV] = sh.ps;
    int(&mark)[NV] = sh.mark;
    int(&pivs)[NB] = sh.pivs;
    const int64_t m = blockIdx.x;
    double* Bm = B + m * BD::per_macro;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool second = kb > kb0;
    const int nrows = NV - kb;
    double (*stage)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(raw);

    double z[RPT][NB];
    int id[RPT];
    bool done[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        id[r] = kb + tid + r * NT;
        done[r] = id[r] >= NV;
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c) z[r][c] = (!done[r] && c < nb) ? Bm[(int64_t)id[r] * ld + kb + c] : 0.0;
    for (int r = kb + tid; r < NV; r += NT) {
        mp[r] = r;
        ps[r] = r;
        mark[r] = 0;
    }
    // wave candidate over the rows that are not pivots yet, from their current
    // column values cv: arg-max to LDS (ties to the lower row)
    auto candidate = [&](int bf, const double (&cv)[RPT]) {
        double best = -1.0;
        int bi = NV;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            double ax = fabs(cv[r]);
            if (!(ax >= 0.0)) ax = 0.0;          // NaN
            if (!done[r] && (ax > best || (ax == best && id[r] < bi))) {
                best = ax;
                bi = id[r];
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
        for (int r = 0; r < RPT; ++r) cv[r] = z[r][0];
        candidate(0, cv);
    }
    bool bad = false;
    // one column; from column j0 on only z[0 .. 64-j0) can hold live entries
    // (the pivot row reads as zero beyond), so the segment starting at j0 is
    // compiled with AW = 64 - j0 live registers and moves the rest unchanged
    auto column = [&](int j, auto aw) {
        constexpr int AW = decltype(aw)::value;
        const int bf = j & 1;
        __syncthreads();
        double b = redv[bf][0];
        int p = redi[bf][0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
            if (redv[bf][w] > b || (redv[bf][w] == b && redi[bf][w] < p)) {
                b = redv[bf][w];
                p = redi[bf][w];
            }
        if (!(b > 0.0) || !isfinite(b)) bad = true;
        if (tid == 0) pidj[j] = p;
        // the pivot row publishes its values; its wave then zeroes the multiplier part
        bool own_wave = false;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const bool own = id[r] == p;
            if (own) {
#pragma unroll
                for (int c = 0; c < AW; ++c) prow[bf][c] = z[r][c];
                done[r] = true;
            }
            own_wave |= __ballot(own) != 0ull;
        }
        if (own_wave && lane >= NB - j && lane < AW) prow[bf][lane] = 0.0;   // same wave, after the row
        __syncthreads();
        const double pv = prow[bf][0];
        const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
        double l[RPT], nz0[RPT], z0[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            z0[r] = z[r][0];
            l[r] = done[r] ? 0.0 : z0[r] * inv;
            nz0[r] = z[r][1] - l[r] * prow[bf][1];       // look-ahead column
        }
        if (j + 1 < nb) candidate(bf ^ 1, nz0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
#pragma unroll
            for (int c = 1; c < AW - 1; ++c) z[r][c] = z[r][c + 1] - l[r] * prow[bf][c + 1];
#pragma unroll
            for (int c = (AW - 1 > 1 ? AW - 1 : 1); c < NB - 1; ++c) z[r][c] = z[r][c + 1];
            z[r][0] = nz0[r];
            z[r][NB - 1] = done[r] ? z0[r] : l[r];
        }
    };
    const int j1 = nb < 16 ? nb : 16, j2 = nb < 32 ? nb : 32, j3 = nb < 48 ? nb : 48;
#pragma clang loop unroll(disable)
    for (int j = 0; j < j1; ++j) column(j, std::integral_constant<int, 64>{});
#pragma clang loop unroll(disable)
    for (int j = j1; j < j2; ++j) column(j, std::integral_constant<int, 48>{});
#pragma clang loop unroll(disable)
    for (int j = j2; j < j3; ++j) column(j, std::integral_constant<int, 32>{});
#pragma clang loop unroll(disable)
    for (int j = j3; j < nb; ++j) column(j, std::integral_constant<int, 16>{});
    // replay of the interchanges: position kb+j with the pivot's current position
    if (second && tid < NB) pv1[tid] = ipiv[m * NV + kb0 + tid];
    __syncthreads();
    if (tid == 0) {
#pragma clang loop unroll(disable)
        for (int j = 0; j < nb; ++j) {
            const int pid = pidj[j], pp = ps[pid], other = mp[kb + j];
            mp[kb + j] = pid;
            ps[pid] = kb + j;
            mp[pp] = other;
            ps[other] = pp;
            pivs[j] = pp;
        }
    }
    __syncthreads();
    // every row to its final position, through LDS in chunks (coalesced); its
    // z[c] belongs to column (c + nb) mod 64
    for (int base = 0; base < RPT * NT; base += CH) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int sl = tid + r * NT - base;
            if (sl >= 0 && sl < CH) {
#pragma unroll
                for (int c = 0; c < NB; ++c) stage[sl][c] = z[r][c];
            }
        }
        __syncthreads();
        for (int e = tid; e < CH * NB; e += NT) {
            const int rr = base + e / NB, c = e % NB;
            if (rr < nrows && c < nb)
                Bm[(int64_t)ps[kb + rr] * ld + kb + c] = stage[e / NB][(c - nb) & (NB - 1)];
        }
        __syncthreads();
    }
    panel_finish<P>(sh, Bm, kb, kb0, nb, m, ipiv, perm, tri, bad, status);
}

// ---------------------------------------------------------------------------
// The same panel for S with more rows than the workgroup has threads (degree
// 3: 1715 rows, two per thread), whose 64-wide register segments would not
// fit: the panel goes in sub-panels of SW columns (8 at degree 3), left-looking.
// During the kernel a row keeps its panel values in its own storage row (its
// identity); before sub-panel s the pivot rows chosen so far get their U
// entries over its columns by a forward substitution among themselves
// (one column per lane, in LDS), every other row subtracts its stored
// multipliers times those entries, and then the sub-panel's columns are
// eliminated in registers as in k_panel (arg-max over the rows that are not
// pivots yet, the pivot row broadcast through LDS, rank-1 update).  The
// multipliers and U entries go back to the rows' storage.  Afterwards only
// the rows the interchanges move (at most 2 nb) are copied to their final
// positions, and panel_finish completes the panel as in k_panel.
template <int P, int SW>
__global__ void __launch_bounds__(Panel<P>::THREADS) k_panel_sub(double* __restrict__ B, int kb, int kb0,
                                                                 int32_t* __restrict__ ipiv,
                                                                 int32_t* __restrict__ perm,
                                                                 double* __restrict__ tri,
                                                                 int32_t* __restrict__ status) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, RPT = PN::RPT, ld = BD::ld;
    constexpr int NT = PN::THREADS, NW = NT / 64;
    static_assert(NB % SW == 0, "whole sub-panels");
    __shared__ PanelShared<P> sh;
    __shared__ double prow[2][SW];
    __shared__ double redv[2][NW];
    __shared__ int redi[2][NW];
    __shared__ int mvpos[2 * NB];
    __shared__ int nmov;
    int(&pidj)[NB] = sh.pidj;
    int(&pivs)[NB] = sh.pivs;
    int(&pv1)[NB] = sh.pv1;
    int(&mp)[NV] = sh.mp;
    int(&ps)[NV] = sh.ps;
    int(&mark)[NV] = sh.mark;
    double(&raw)[3 * NB * (NB + 1)] = sh.raw;
    // during the sub-panels (raw is free until the rows move): the multipliers
    // of the pivot rows among themselves, and their values over the current
    // sub-panel (at most NB - SW pivots before the last sub-panel)
    static_assert((NB - SW) * (NB + 1) + (NB - SW) * (SW + 1) <= 3 * NB * (NB + 1), "sub-panel tables fit in raw");
    double(*Lp)[NB + 1] = reinterpret_cast<double(*)[NB + 1]>(raw);
    double(*Us)[SW + 1] = reinterpret_cast<double(*)[SW + 1]>(raw + (NB - SW) * (NB + 1));
    const int64_t m = blockIdx.x;
    double* Bm = B + m * BD::per_macro;
    const int nb = (NV - kb) < NB ? (NV - kb) : NB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool second = kb > kb0;
    int id[RPT];
    bool done[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        id[r] = kb + tid + r * NT;
        done[r] = id[r] >= NV;
    }
    for (int r = kb + tid; r < NV; r += NT) {
        mp[r] = r;
        ps[r] = r;
        mark[r] = 0;
    }
    bool bad = false;
    double z[RPT][SW];
    for (int c0 = 0; c0 < nb; c0 += SW) {
        const int sw = (nb - c0) < SW ? (nb - c0) : SW;
        __syncthreads();
        if (c0 > 0) {
            // U entries of the pivots so far over this sub-panel
            for (int e = tid; e < c0 * c0; e += NT) {
                const int k = e / c0, i = e % c0;
                Lp[k][i] = i < k ? Bm[(int64_t)pidj[k] * ld + kb + i] : 0.0;
            }
            for (int e = tid; e < c0 * SW; e += NT) {
                const int k = e / SW, c = e % SW;
                Us[k][c] = c < sw ? Bm[(int64_t)pidj[k] * ld + kb + c0 + c] : 0.0;
            }
            __syncthreads();
            if (wave == 0 && lane < SW) {
                for (int k = 1; k < c0; ++k) {
                    double u = Us[k][lane];
                    for (int i = 0; i < k; ++i) u -= Lp[k][i] * Us[i][lane];
                    Us[k][lane] = u;
                }
            }
            __syncthreads();
            for (int e = tid; e < c0 * SW; e += NT) {
                const int k = e / SW, c = e % SW;
                if (c < sw) Bm[(int64_t)pidj[k] * ld + kb + c0 + c] = Us[k][c];
            }
        }
        // the rows that are not pivots yet: their sub-panel values, updated by
        // the earlier sub-panels
        bool act[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            act[r] = !done[r];
#pragma unroll
            for (int c = 0; c < SW; ++c) z[r][c] = (act[r] && c < sw) ? Bm[(int64_t)id[r] * ld + kb + c0 + c] : 0.0;
            if (act[r]) {
                for (int k = 0; k < c0; ++k) {
                    const double l = Bm[(int64_t)id[r] * ld + kb + k];
#pragma unroll
                    for (int c = 0; c < SW; ++c) z[r][c] -= l * Us[k][c];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < SW; ++j) {
            if (j < sw) {
                const int bf = j & 1;
                double best = -1.0;
                int bi = NV;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    double ax = fabs(z[r][j]);
                    if (!(ax >= 0.0)) ax = 0.0;          // NaN
                    if (!done[r] && (ax > best || (ax == best && id[r] < bi))) {
                        best = ax;
                        bi = id[r];
                    }
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
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
                double pbest = redv[bf][0];
                int p = redi[bf][0];
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    if (redv[bf][w] > pbest || (redv[bf][w] == pbest && redi[bf][w] < p)) {
                        pbest = redv[bf][w];
                        p = redi[bf][w];
                    }
                if (!(pbest > 0.0) || !isfinite(pbest)) bad = true;
#pragma unroll
                for (int r = 0; r < RPT; ++r)
                    if (!done[r] && id[r] == p) {
#pragma unroll
                        for (int c = 0; c < SW; ++c) prow[bf][c] = z[r][c];
                        done[r] = true;
                    }
                if (tid == 0) pidj[c0 + j] = p;
                __syncthreads();
                const double pv = prow[bf][j];
                const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
#pragma unroll
                for (int r = 0; r < RPT; ++r)
                    if (!done[r]) {
                        const double l = z[r][j] * inv;
                        z[r][j] = l;
#pragma unroll
                        for (int c = j + 1; c < SW; ++c) z[r][c] -= l * prow[bf][c];
                    }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (act[r]) {
#pragma unroll
                for (int c = 0; c < SW; ++c)
                    if (c < sw) Bm[(int64_t)id[r] * ld + kb + c0 + c] = z[r][c];
            }
    }
    // replay of the interchanges: position kb+j with the pivot's current position
    if (second && tid < NB) pv1[tid] = ipiv[m * NV + kb0 + tid];
    __syncthreads();
    if (tid == 0) {
        int n = 0;
#pragma clang loop unroll(disable)
        for (int j = 0; j < nb; ++j) {
            const int pid = pidj[j], pp = ps[pid], other = mp[kb + j];
            mp[kb + j] = pid;
            ps[pid] = kb + j;
            mp[pp] = other;
            ps[other] = pp;
            pivs[j] = pp;
        }
        // the positions whose row changes (each listed once)
#pragma clang loop unroll(disable)
        for (int j = 0; j < nb; ++j) {
            const int cand[2] = {kb + j, pivs[j]};
            for (int t = 0; t < 2; ++t) {
                const int q = cand[t];
                bool seen = mp[q] == q;
                for (int u = 0; u < n && !seen; ++u) seen = mvpos[u] == q;
                if (!seen) mvpos[n++] = q;
            }
        }
        nmov = n;
    }
    __syncthreads();
    // moved rows to their final positions (read all, then write)
    const int cnt = nmov * NB;
    for (int e = tid; e < cnt; e += NT) {
        const int c = e % NB;
        raw[e] = c < nb ? Bm[(int64_t)mp[mvpos[e / NB]] * ld + kb + c] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < cnt; e += NT) {
        const int c = e % NB;
        if (c < nb) Bm[(int64_t)mvpos[e / NB] * ld + kb + c] = raw[e];
    }
    __syncthreads();
    panel_finish<P>(sh, Bm, kb, kb0, nb, m, ipiv, perm, tri, bad, status);
}

// ---------------------------------------------------------------------------
// GM x GT = 128 x 64 FP64 MFMA tile: acc (+)= sgn * A[r0.., 0..K) * Bt[0..K, c0..)
// with eight waves in 4 x 2, each owning 2 x 2 blocks of 16 x 16 (register r
// of lane l holds row (l >> 4) + 4 r, column l & 15 of its block).  K is
// staged through LDS in chunks of GK with the next chunk's global loads
// issued before the current chunk is multiplied.
constexpr int GT = 64;
constexpr int GM = 128;
constexpr int GK = 16;
constexpr int GTHREADS = 512;
constexpr int GLA = GM * GK / GTHREADS;        // A elements of a chunk per thread
constexpr int GLB = GK * GT / GTHREADS;        // B elements of a chunk per thread

struct TileSmem {
    double As[2][GM][GK + 1];
    double Bs[2][GK][GT + 1];
};

template <bool NEG>
__device__ __forceinline__ void tile_mma(const double* A, int lda, const double* Bt, int ldb, int K, int r0,
                                         int c0, int rows, int cols, v4d acc[2][2], TileSmem& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const double sgn = NEG ? -1.0 : 1.0;
    double ra[GLA], rb[GLB];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < GLA; ++i) {
            const int e = tid + GTHREADS * i;
            const int ar = e / GK, ak = e % GK;
            const int r = r0 + ar, k = k0 + ak;
            ra[i] = (r < rows && k < K) ? A[(int64_t)r * lda + k] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < GLB; ++i) {
            const int e = tid + GTHREADS * i;
            const int bk = e / GT, bc = e % GT;
            const int kk = k0 + bk, c = c0 + bc;
            rb[i] = (kk < K && c < cols) ? Bt[(int64_t)kk * ldb + c] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < GLA; ++i) {
            const int e = tid + GTHREADS * i;
            sm.As[buf][e / GK][e % GK] = sgn * ra[i];
        }
#pragma unroll
        for (int i = 0; i < GLB; ++i) {
            const int e = tid + GTHREADS * i;
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

__device__ __forceinline__ int tile_row(int r0, int bi, int q) {
    const int lane = threadIdx.x & 63, wr = (threadIdx.x >> 6) >> 1;
    return r0 + wr * 32 + bi * 16 + (lane >> 4) + 4 * q;
}
__device__ __forceinline__ int tile_col(int c0, int bj) {
    const int lane = threadIdx.x & 63, wc = (threadIdx.x >> 6) & 1;
    return c0 + wc * 32 + bj * 16 + (lane & 15);
}

__device__ __forceinline__ void zero_acc(v4d acc[2][2]) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
}

// Tile shapes of the batched product (the sweep of the tile autotuner picks
// one per degree and call site): WM x WN waves, each owning BI x BJ blocks of
// 16 x 16, so a workgroup of 64 WM WN threads computes a TM x TN tile with
// TM = 16 WM BI, TN = 16 WN BJ; K is staged through LDS in chunks of KC, and
// OCC waves per SIMD are asked of the register allocator.
// Every shape adds the products of one output element in the same order (K
// ascending, four at a time per MFMA), so all shapes give the same bits.
template <int WM_, int WN_, int BI_, int BJ_, int KC_, int OCC_>
struct GTile {
    static constexpr int WM = WM_, WN = WN_, BI = BI_, BJ = BJ_, KC = KC_, OCC = OCC_;
    // from 6 waves per SIMD on (three 8-wave workgroups per CU) C is read
    // after the K loop instead of being held across it
    static constexpr bool C_LATE = OCC >= 6;
    static constexpr int TM = 16 * WM * BI, TN = 16 * WN * BJ, NT = 64 * WM * WN;
    static constexpr int LA = TM * KC / NT, LB = KC * TN / NT;   // staged elements per thread
    static_assert(LA * NT == TM * KC && LB * NT == KC * TN, "tile does not divide among the threads");
};

template <class T>
struct GTileSmem {
    double As[2][T::TM][T::KC + 1];
    double Bs[2][T::KC][T::TN + 1];
};

// The variants the library carries, in the order of their index.
#define MEHDG_GEMM_VARIANTS(X) \
    X(0, 4, 2, 2, 2, 16, 4)    \
    X(1, 4, 2, 2, 4, 16, 2)    \
    X(2, 2, 4, 4, 2, 16, 2)    \
    X(3, 4, 2, 2, 2, 32, 2)    \
    X(4, 2, 2, 2, 2, 16, 3)    \
    X(5, 4, 4, 2, 2, 16, 2)    \
    X(6, 2, 2, 2, 4, 16, 2)    \
    X(7, 4, 2, 2, 2, 16, 6)
constexpr int kGemmVariants = 8;

// acc += A[r0.., 0..K) * Bt[0..K, c0..) on a T tile.  The operands are read
// with buffer loads: each element a thread stages keeps one byte offset for
// the whole K loop, and each chunk moves the buffer's base (scalar work), so
// the loop spends no vector instructions on addresses or bounds.  Rows of A
// beyond the product's rows and columns of Bt beyond its columns are read
// as they stand (they only feed outputs that are never stored) and reads past
// a_bytes / b_bytes give 0; only the last chunk, when K is not a multiple of
// KC, zeroes the terms k >= K on both sides.
// GATHER: row k of Bt is row srcrow[k] of the matrix at Bt (b_bytes from its
// start); its offsets are formed per chunk from the list.
template <class T, bool GATHER = false>
__device__ __forceinline__ void tile_mma_t(const double* A, int lda, int64_t a_bytes, const double* Bt, int ldb,
                                           int64_t b_bytes, int K, int r0, int c0, v4d (&acc)[T::BI][T::BJ],
                                           GTileSmem<T>& sm, const int* srcrow = nullptr) {
    constexpr int KC = T::KC, TN = T::TN, NT = T::NT;
    constexpr int RA = NT / KC, RB = NT / TN;     // rows of A / of Bt between a thread's staged elements
    static_assert(RA * KC == NT && RB * TN == NT, "staging does not tile the chunk");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave / T::WN, wc = wave % T::WN;
    const int ak = tid % KC, bk = tid / TN;
    int va[T::LA], vb[T::LB];
#pragma unroll
    for (int i = 0; i < T::LA; ++i) va[i] = ((r0 + tid / KC + i * RA) * lda + ak) * 8;
#pragma unroll
    for (int i = 0; i < T::LB; ++i) vb[i] = ((bk + i * RB) * ldb + c0 + tid % TN) * 8;
    double ra[T::LA], rb[T::LB];
    // record counts as non-negative int32 (buffers here stay far below 2 GiB)
    auto clamp31 = [](int64_t b) { return (int)(b < 0 ? 0 : (b > 0x7fffffffll ? 0x7fffffffll : b)); };
    const int na = clamp31(a_bytes), nb = clamp31(b_bytes);
    const int sta = 8 * KC, stb = 8 * KC * ldb;   // bytes per chunk
    // descriptors are wave-uniform: readfirstlane keeps them in scalar registers
    auto rsrc = [](const double* p, int n) {
        const uint64_t a = (uint64_t)p;
        const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
        return __builtin_amdgcn_make_buffer_rsrc((void*)(lo | (hi << 32)), (short)0,
                                                 __builtin_amdgcn_readfirstlane(n), 0x00020000);
    };
    auto load = [&](int k0) {
        const int ch = k0 / KC;
        const auto sa = rsrc(A + k0, max(na - ch * sta, 0));
#pragma unroll
        for (int i = 0; i < T::LA; ++i)
            ra[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(sa, va[i], 0, 0));
        if constexpr (GATHER) {
            const auto sb = rsrc(Bt, nb);
#pragma unroll
            for (int i = 0; i < T::LB; ++i) {
                const int kk = k0 + bk + i * RB;
                const int off = kk < K ? (srcrow[kk] * ldb + c0 + tid % TN) * 8 : -1;
                rb[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(sb, off, 0, 0));
            }
        } else {
            const auto sb = rsrc(Bt + (int64_t)k0 * ldb, max(nb - ch * stb, 0));
#pragma unroll
            for (int i = 0; i < T::LB; ++i)
                rb[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(sb, vb[i], 0, 0));
        }
        if (k0 + KC > K) {                          // the last, partial chunk
#pragma unroll
            for (int i = 0; i < T::LA; ++i)
                if (k0 + ak >= K) ra[i] = 0.0;
#pragma unroll
            for (int i = 0; i < T::LB; ++i)
                if (k0 + bk + i * RB >= K) rb[i] = 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int i = 0; i < T::LA; ++i) {
            const int e = tid + NT * i;
            sm.As[buf][e / KC][e % KC] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < T::LB; ++i) {
            const int e = tid + NT * i;
            sm.Bs[buf][e / TN][e % TN] = rb[i];
        }
    };
    const int nchunk = (K + KC - 1) / KC;
    // one chunk: prefetch the next into registers, multiply this one from LDS
    // buffer BUF, stash the next into the other buffer; BUF is a constant of
    // the unrolled pair, so the LDS addresses are fixed offsets
    auto step = [&](int ch, auto bufc) {
        constexpr int BUF = decltype(bufc)::value;
        if (ch + 1 < nchunk) load((ch + 1) * KC);
#pragma unroll
        for (int ks = 0; ks < KC; ks += 4) {
            const int kq = ks + (lane >> 4);
            double a[T::BI], b[T::BJ];
#pragma unroll
            for (int bi = 0; bi < T::BI; ++bi) a[bi] = sm.As[BUF][(wr * T::BI + bi) * 16 + (lane & 15)][kq];
#pragma unroll
            for (int bj = 0; bj < T::BJ; ++bj) b[bj] = sm.Bs[BUF][kq][(wc * T::BJ + bj) * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < T::BI; ++bi)
#pragma unroll
                for (int bj = 0; bj < T::BJ; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
        }
        if (ch + 1 < nchunk) stash(BUF ^ 1);
        __syncthreads();
    };
    load(0);
    stash(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ch += 2) {
        step(ch, std::integral_constant<int, 0>{});
        if (ch + 1 < nchunk) step(ch + 1, std::integral_constant<int, 1>{});
    }
}

// The fixed 128 x 64 tile of the triangular kernels is variant 0's shape.
using GTri = GTile<4, 2, 2, 2, 16, 4>;

// ---------------------------------------------------------------------------
// In-place triangular application on MFMA after a panel or an outer block:
// per 64-column tile of [c_lo, c_hi), U_top[:, c-tile] <- L^-1 (P B)_top[:, c-tile];
// L^-1 is w x w, the top rows are [kb0, kb0+w) and P the composed interchange
// in perm.  With DELAYED (kpre > 0) the earlier blocks of the group have not
// updated these columns yet: the tile forms
//   T = (P B)_top - L[top, kb0-kpre : kb0] U[kb0-kpre : kb0, c-tile]
// (their multipliers already in the top rows' order), writes it to the top
// rows and solves U_top = L^-1 T.  Each workgroup reads everything it
// overwrites before writing it.
struct TriArgs {
    int kb0, w;          // top rows [kb0, kb0+w), also the K of the column tiles
    int loff, ldl;       // L^-1 of the top rows: offset in the per-macro workspace, leading dimension
    int c_lo, c_hi;      // columns that get U_top
    int ct;              // column tiles
    int kpre;            // columns of the group's earlier blocks whose update is pending (0: none)
};

template <int P, bool DELAYED>
__global__ void __launch_bounds__(GTHREADS) k_tri(double* B, const double* __restrict__ tri,
                                                  const int32_t* __restrict__ perm, TriArgs a, int64_t n_macro) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, OB = PN::OB, NV = PN::NV, ld = BD::ld, ROWS = BD::rows;
    constexpr int MV = OB * GT / GTHREADS;       // displaced-row elements per thread
    __shared__ TileSmem sm;
    __shared__ int pm[3 * OB + 1];
    static_assert(sizeof(TileSmem) == sizeof(GTileSmem<GTri>), "the two staging layouts coincide");
    GTileSmem<GTri>& gsm = *reinterpret_cast<GTileSmem<GTri>*>(&sm);
    int64_t m;
    int tile;
    xcd_tile(a.ct, m, tile);
    if (m >= n_macro) return;
    double* Bm = B + m * BD::per_macro;
    const double* Ti = tri + m * PN::TRI;
    v4d acc[2][2];
    zero_acc(acc);
    const int cc = a.c_lo + tile * GT;     // columns [cc, cc+64)
    for (int i = threadIdx.x; i < 3 * OB + 1; i += GTHREADS) pm[i] = perm[m * PN::PERM + i];
    __syncthreads();
    const int nd = pm[3 * OB];
    // rows below the block that change read their new values before anything is written
    double mvr[MV];
    if constexpr (DELAYED) {
        const int kg = a.kb0 - a.kpre;
        tile_mma_t<GTri>(Bm + kg, ld, ((int64_t)BD::per_macro - kg) * 8, Bm + (int64_t)kg * ld, ld,
                         ((int64_t)BD::per_macro - (int64_t)kg * ld) * 8, a.kpre, a.kb0, cc, acc, gsm);
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
            mvr[i] = (q < nd && c < a.c_hi) ? Bm[(int64_t)pm[2 * OB + q] * ld + c] : 0.0;
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = tile_row(0, bi, q), c = tile_col(cc, bj);
                    if (r < a.w && c < a.c_hi) acc[bi][bj][q] = Bm[(int64_t)pm[r] * ld + c] - acc[bi][bj][q];
                }
        __syncthreads();                 // every read of the rows this tile rewrites is done
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
            if (q < nd && c < a.c_hi) Bm[(int64_t)pm[OB + q] * ld + c] = mvr[i];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = tile_row(0, bi, q), c = tile_col(cc, bj);
                    if (r < a.w && c < a.c_hi) Bm[(int64_t)(a.kb0 + r) * ld + c] = acc[bi][bj][q];
                }
        __syncthreads();
        zero_acc(acc);
        tile_mma_t<GTri>(Ti + a.loff, a.ldl, ((int64_t)PN::TRI - a.loff) * 8, Bm + (int64_t)a.kb0 * ld, ld,
                         ((int64_t)BD::per_macro - (int64_t)a.kb0 * ld) * 8, a.w, 0, cc, acc, gsm);
    } else {
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
            mvr[i] = (q < nd && c < a.c_hi) ? Bm[(int64_t)pm[2 * OB + q] * ld + c] : 0.0;
        }
        tile_mma_t<GTri, true>(Ti + a.loff, a.ldl, ((int64_t)PN::TRI - a.loff) * 8, Bm, ld,
                               (int64_t)BD::per_macro * 8, a.w, 0, cc, acc, gsm, pm);
#pragma unroll
        for (int i = 0; i < MV; ++i) {
            const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
            if (q < nd && c < a.c_hi) Bm[(int64_t)pm[OB + q] * ld + c] = mvr[i];
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = tile_row(0, bi, q), c = tile_col(cc, bj);
                if (r < a.w && c < a.c_hi) Bm[(int64_t)(a.kb0 + r) * ld + c] = acc[bi][bj][q];
            }
}


// ---------------------------------------------------------------------------
// The composed row interchange of the current outer block (perm) applied to
// the columns [c_lo, c_hi) of the S rows [kb0, NV): position kb0+i takes row
// perm[i] (i < w) and each displaced row below the block takes its source.
// It moves the multipliers of the group's earlier blocks, whose update of
// these rows is still pending.  Per 64-column tile: every read, then every write.
template <int P>
__global__ void __launch_bounds__(GTHREADS) k_perm_rows(double* B, const int32_t* __restrict__ perm, int kb0, int w,
                                                        int c_lo, int c_hi, int ct, int64_t n_macro) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int OB = PN::OB, ld = BD::ld;
    constexpr int MV = 2 * OB * GT / GTHREADS;   // moved elements per thread
    __shared__ int pm[3 * OB + 1];
    int64_t m;
    int tile;
    xcd_tile(ct, m, tile);
    if (m >= n_macro) return;
    double* Bm = B + m * BD::per_macro;
    for (int i = threadIdx.x; i < 3 * OB + 1; i += GTHREADS) pm[i] = perm[m * PN::PERM + i];
    __syncthreads();
    const int nr = w + pm[3 * OB];
    const int cc = c_lo + tile * GT;
    double v[MV];
#pragma unroll
    for (int i = 0; i < MV; ++i) {
        const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
        v[i] = 0.0;
        if (q < nr && c < c_hi) v[i] = Bm[(int64_t)(q < w ? pm[q] : pm[2 * OB + q - w]) * ld + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MV; ++i) {
        const int e = threadIdx.x + GTHREADS * i, q = e / GT, c = cc + e % GT;
        if (q < nr && c < c_hi) Bm[(int64_t)(q < w ? kb0 + q : pm[OB + q - w]) * ld + c] = v[i];
    }
}

// ---------------------------------------------------------------------------
// L21 of the X rows for panel q (columns [kq, kq+nbq)), left-looking: per
// 128-row tile of X, acc = X[:, q] - L21[:, <q] U[<q, q] (K = kq, the earlier
// panels' L21 already in place of X), written in place, then
// L21[:, q] = acc U_qq^-1 (K = nbq) in place.  Each workgroup reads its own
// tile back only after writing it.
template <int P>
__global__ void __launch_bounds__(GTHREADS, 6) k_trsm_x(double* B, const double* __restrict__ tri, int q,
                                                     int64_t n_macro) {
    using BD = Bdims<P>;
    using PN = Panel<P>;
    constexpr int NB = PN::NB, NV = PN::NV, ld = BD::ld, ROWS = BD::rows;
    __shared__ GTileSmem<GTri> sm;
    int64_t m;
    int tile;
    xcd_tile((ROWS - NV + GM - 1) / GM, m, tile);
    if (m >= n_macro) return;
    double* Bm = B + m * BD::per_macro;
    const int kq = q * NB, nbq = (NV - kq) < NB ? (NV - kq) : NB;
    const int rr = NV + tile * GM;                 // rows [rr, rr+128) of X
    v4d acc[2][2];
    zero_acc(acc);
    if (kq > 0)
        tile_mma_t<GTri>(Bm, ld, (int64_t)BD::per_macro * 8, Bm + kq, ld, ((int64_t)BD::per_macro - kq) * 8, kq, rr,
                         0, acc, sm);
    // X[:, q] is read after the long product (not held across it: 6 waves per SIMD)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int r = tile_row(rr, bi, qq), c = tile_col(0, bj);
                if (r < ROWS && c < nbq)
                    Bm[(int64_t)r * ld + kq + c] = Bm[(int64_t)r * ld + kq + c] - acc[bi][bj][qq];
            }
    __syncthreads();
    zero_acc(acc);
    const double* Ui = tri + m * PN::TRI + PN::UINV + (int64_t)q * NB * NB;
    tile_mma_t<GTri>(Bm + kq, ld, ((int64_t)BD::per_macro - kq) * 8, Ui, NB, (int64_t)NB * NB * 8, nbq, rr, 0, acc,
                     sm);
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int r = tile_row(rr, bi, qq), c = tile_col(0, bj);
                if (r < ROWS && c < nbq) Bm[(int64_t)r * ld + kq + c] = acc[bi][bj][qq];
            }
}

// ---------------------------------------------------------------------------
// Batched FP64 MFMA product  D = C - A * Bt  on a 128 x 64 tile per workgroup.
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
    int64_t limA, limB;      // doubles of a macro's block readable from its A / Bt (reads beyond give 0)
    int lda, ldb, ldc, ldd, ldd2;
    int rows, cols, K;       // extent of the region (relative to its origin)
    int dsplit;              // first column that goes to D2 (cols if none)
    int skip_r, skip_c;      // masked corner (relative), rows/cols if none
    int tiles_c, tiles;      // column tiles, tiles per macro
    int64_t n_macro;
};

// TAG only separates the trailing-update launches (0), the Schur product (1)
// and the refinement residual (2) in profiles; the code is the same.
template <int TAG, class T>
__global__ void __launch_bounds__(T::NT, T::OCC) k_gemm(GemmArgs g) {
    __shared__ GTileSmem<T> sm;
    int64_t m;
    int tile;
    xcd_tile(g.tiles, m, tile);
    if (m >= g.n_macro) return;
    const int tr = tile / g.tiles_c, tc = tile % g.tiles_c;
    const int r0 = tr * T::TM, c0 = tc * T::TN;
    if (r0 >= g.skip_r && c0 >= g.skip_c) return;   // tile entirely in the masked corner
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / T::WN, wc = wave % T::WN;
    auto row = [&](int bi, int q) { return r0 + (wr * T::BI + bi) * 16 + (lane >> 4) + 4 * q; };
    auto col = [&](int bj) { return c0 + (wc * T::BJ + bj) * 16 + (lane & 15); };
    const double* C = g.C + m * g.sC;
    // C is fetched first and only added after the K loop, so its latency
    // overlaps the staging and the MFMA work.
    double cr[T::BI][T::BJ][4];
    auto load_c = [&]() {
#pragma unroll
        for (int bi = 0; bi < T::BI; ++bi)
#pragma unroll
            for (int bj = 0; bj < T::BJ; ++bj)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = row(bi, q), c = col(bj);
                    const bool in = r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c);
                    cr[bi][bj][q] = in ? C[(int64_t)r * g.ldc + c] : 0.0;
                }
    };
    if constexpr (!T::C_LATE) load_c();
    v4d acc[T::BI][T::BJ];
#pragma unroll
    for (int bi = 0; bi < T::BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < T::BJ; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
    tile_mma_t<T>(g.A + m * g.sA, g.lda, g.limA * 8, g.Bt + m * g.sB, g.ldb, g.limB * 8, g.K, r0, c0, acc, sm);
    if constexpr (T::C_LATE) load_c();
    double* D = g.D ? g.D + m * g.sD : nullptr;
    double* D2 = g.D2 ? g.D2 + m * g.sD2 : nullptr;
#pragma unroll
    for (int bi = 0; bi < T::BI; ++bi)
#pragma unroll
        for (int bj = 0; bj < T::BJ; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = row(bi, q), c = col(bj);
                if (r < g.rows && c < g.cols && !(r >= g.skip_r && c >= g.skip_c)) {
                    const double v = cr[bi][bj][q] - acc[bi][bj][q];
                    if (D2 && c >= g.dsplit) D2[(int64_t)r * g.ldd2 + (c - g.dsplit)] = v;
                    else if (D) D[(int64_t)r * g.ldd + c] = v;
                }
            }
}

}  // namespace mehdg
