// Back-substitution once the trace update is known (Sec. 6.2, eq. R2 then R6).
//
// After condensation the top rows of the bordered matrix hold U (upper
// factor of P S), U12 = L^-1 P (-Y) and y = L^-1 P r_V, so
//   dV = S^-1 (r_V + Y dVhat) = U^-1 (y - U12 dVhat),
// and then, with A_qq = I (x) M and the 1-D tensor structure of the lifts,
//   dQ_{lj} = -M^-1 R_Q,lj - (Lam/h_j)_axis-j dV_l + (lift of dVhat_l on the faces normal to j).
// One workgroup per macro; U and U12 are read once, row-wise and coalesced;
// dot products are reduced within a wave with DPP row permutations.
#pragma once
#include "k_condense.hpp"

namespace mehdg {

// dV = U^-1 (y - U12 dVhat) for the macro whose factored bordered matrix
// starts at Bm (dVhat in LDS dvh[NH]); the result is left in z[NV] (LDS).
// Uses the whole workgroup; U is 64 x 64 LDS scratch.
template <int P>
__device__ void back_substitute(const double* __restrict__ Bm, const double* dvh, double* z, double (*U)[65]) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int NV = D::NV, NH = D::NH, ld = BD::ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    // z = y - U12 dVhat: each wave takes RB rows at a time, lanes along the
    // rows (coalesced), and reduces the RB dot products together
    constexpr int RB = 8;
    for (int r0 = wave * RB; r0 < NV; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < NH; c += 64) {
            const double x = dvh[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < NV) s[i] += Bm[(int64_t)(r0 + i) * ld + NV + c] * x;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < NV) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            z[r0 + lane] = Bm[(int64_t)(r0 + lane) * ld + NV + NH] - si;
        }
    }
    __syncthreads();
    // U dV = z, right-looking over blocks of 64 rows from the last: wave 0
    // solves the block's 64 x 64 triangle (lane j holds row j; the solved
    // value is broadcast with a lane read), then every row above the block
    // subtracts its product with the block's solution (all waves, RB rows at
    // a time, one 64-column chunk per row)
    for (int i0 = ((NV - 1) / 64) * 64; i0 >= 0; i0 -= 64) {
        const int i1 = i0 + 64 < NV ? i0 + 64 : NV;
        const int nb = i1 - i0;
        for (int e = tid; e < 64 * 64; e += blockDim.x) {
            const int r = e >> 6, c = e & 63;
            U[r][c] = (r < nb && c < nb) ? Bm[(int64_t)(i0 + r) * ld + i0 + c] : 0.0;
        }
        __syncthreads();
        if (wave == 0) {
            double zi = (lane < nb) ? z[i0 + lane] : 0.0;
            // reciprocals of the diagonal formed up front, off the dependent chain
            const double rd = (lane < nb) ? 1.0 / U[lane][lane] : 0.0;
            for (int j = nb - 1; j >= 0; --j) {
                const double xj = read_lane_f64(zi, j) * read_lane_f64(rd, j);
                if (lane == j) zi = xj;
                else if (lane < j) zi -= U[lane][j] * xj;
            }
            if (lane < nb) z[i0 + lane] = zi;   // now holds dV for this block
        }
        __syncthreads();
        const double x = lane < nb ? z[i0 + lane] : 0.0;
        for (int r0 = wave * RB; r0 < i0; r0 += nw * RB) {
            double s[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                s[i] = (r0 + i < i0 && lane < nb) ? Bm[(int64_t)(r0 + i) * ld + i0 + lane] * x : 0.0;
#pragma unroll
            for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
            if (lane < RB && r0 + lane < i0) {
                double si = s[0];
#pragma unroll
                for (int i = 1; i < RB; ++i)
                    if (lane == i) si = s[i];
                z[r0 + lane] -= si;
            }
        }
        __syncthreads();
    }
}

// The 15 fields of dQ go through the LDS in groups of FG: all at once up to
// p = 2; three at a time at p = 3, so that two macros' LDS (79 KB each) share
// a CU; five at a time from p = 4 on, where all 15 would need 175 KB.
template <int P>
struct RecLds {
    using D = Dims<P>;
    static constexpr int FG = P >= 4 ? 5 : (P == 3 ? 3 : 15);
    double z[D::NV];
    double dvh[D::NH];
    double U[64][65];
    double a[FG * D::n], b[FG * D::n];
    Tab1D t;
};

// dV (in L.z) to dv, then dQ = A_qq^-1 (-R_Q - A_qv dV - A_qvhat dVhat) by the
// 1-D tensor structure of M and of the lifts (eq. R6).
template <int P>
__device__ void recover_dq(RecLds<P>& L, const double* __restrict__ R_q, const double* __restrict__ hs, int64_t m,
                           double* __restrict__ dv, double* __restrict__ dq) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d, n = D::n, nf = D::nf, NV = D::NV, FG = RecLds<P>::FG;
    const int tid = threadIdx.x;
    for (int i = tid; i < NV; i += blockDim.x) dv[m * NV + i] = L.z[i];
    const double h[3] = {hs[3 * m], hs[3 * m + 1], hs[3 * m + 2]};
    const double vinv = 1.0 / (h[0] * h[1] * h[2]);
    for (int g0 = 0; g0 < 15; g0 += FG) {
        // M^-1 R_Q of fields [g0, g0 + FG) by three 1-D passes
        for (int i = tid; i < FG * n; i += blockDim.x) L.a[i] = R_q[m * 15 * n + g0 * n + i];
        __syncthreads();
        double* src = L.a;
        double* dst = L.b;
        for (int axis = 0; axis < 3; ++axis) {
            const int stride = axis == 0 ? 1 : (axis == 1 ? n1d : n1d * n1d);
            for (int i = tid; i < FG * n; i += blockDim.x) {
                const int node = i % n, fld = i / n;
                const int ci = (node / stride) % n1d;
                const int base = node - ci * stride;
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < n1d; ++c) acc += L.t.Minv[ci][c] * src[fld * n + base + c * stride];
                dst[i] = acc;
            }
            __syncthreads();
            double* t = src;
            src = dst;
            dst = t;
        }
        for (int i = tid; i < FG * n; i += blockDim.x) {
            const int c = i % n, lj = g0 + i / n, l = lj / 3, j = lj % 3;
            const int ci[3] = {c % n1d, (c / n1d) % n1d, c / (n1d * n1d)};
            const int stride = j == 0 ? 1 : (j == 1 ? n1d : n1d * n1d);
            const int base = c - ci[j] * stride;
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < n1d; ++b) acc -= L.t.Lam[ci[j]][b] * L.z[l * n + base + b * stride];
            const int t1 = (j == 0) ? 1 : 0, t2 = (j == 2) ? 1 : 2;
            const int fc = ci[t1] + n1d * ci[t2];
            acc -= L.t.Minv[ci[j]][0] * L.dvh[(2 * j * 5 + l) * nf + fc];
            acc += L.t.Minv[ci[j]][n1d - 1] * L.dvh[((2 * j + 1) * 5 + l) * nf + fc];
            dq[m * 15 * n + g0 * n + i] = acc / h[j] - vinv * src[i];
        }
        __syncthreads();   // the next group overwrites a and b
    }
}

template <int P>
__global__ void __launch_bounds__(1024) k_recover(const double* __restrict__ B, const double* __restrict__ R_q,
                                                 const double* __restrict__ dvhat, const double* __restrict__ hs,
                                                 const Tab1D* __restrict__ tab, double* __restrict__ dv,
                                                 double* __restrict__ dq) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int NH = D::NH;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RecLds<P>& L = *reinterpret_cast<RecLds<P>*>(smem_raw);
    const int64_t m = blockIdx.x;
    const double* Bm = B + m * BD::per_macro;
    const int tid = threadIdx.x;
    {
        const double* src = reinterpret_cast<const double*>(tab);
        double* dst = reinterpret_cast<double*>(&L.t);
        for (int i = tid; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
    }
    for (int i = tid; i < NH; i += blockDim.x) L.dvh[i] = dvhat[m * NH + i];
    __syncthreads();
    back_substitute<P>(Bm, L.dvh, L.z, L.U);
    recover_dq<P>(L, R_q, hs, m, dv, dq);
}

// Recovery after the mixed-precision condensation, which leaves
// Z = S^-1 [-Y | r_V] in the bordered matrix (Z_Y transposed in the X rows,
// z_r in the r_V column): dV = S^-1 (r_V + Y dVhat) = z_r - Z_Y dVhat, a
// product read row by row of the X rows (coalesced over dV's index), then dQ
// as in k_recover.
template <int P>
__global__ void __launch_bounds__(1024) k_recover_z(const double* __restrict__ B, const double* __restrict__ R_q,
                                                   const double* __restrict__ dvhat, const double* __restrict__ hs,
                                                   const Tab1D* __restrict__ tab, double* __restrict__ dv,
                                                   double* __restrict__ dq) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int NV = D::NV, NH = D::NH, ld = BD::ld;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RecLds<P>& L = *reinterpret_cast<RecLds<P>*>(smem_raw);
    const int64_t m = blockIdx.x;
    const double* Bm = B + m * BD::per_macro;
    const int tid = threadIdx.x;
    {
        const double* src = reinterpret_cast<const double*>(tab);
        double* dst = reinterpret_cast<double*>(&L.t);
        for (int i = tid; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
    }
    for (int i = tid; i < NH; i += blockDim.x) L.dvh[i] = dvhat[m * NH + i];
    __syncthreads();
    for (int c = tid; c < NV; c += blockDim.x) {
        double s0 = 0.0, s1 = 0.0;
        int i = 0;
        for (; i + 2 <= NH; i += 2) {
            s0 += Bm[(int64_t)(NV + i) * ld + c] * L.dvh[i];
            s1 += Bm[(int64_t)(NV + i + 1) * ld + c] * L.dvh[i + 1];
        }
        for (; i < NH; ++i) s0 += Bm[(int64_t)(NV + i) * ld + c] * L.dvh[i];
        L.z[c] = Bm[(int64_t)c * ld + NV + NH] - (s0 + s1);
    }
    __syncthreads();
    recover_dq<P>(L, R_q, hs, m, dv, dq);
}

// New right-hand side (r_V, r_hat) for the stored factors: y = L^-1 P r_V and
// bhat = r_hat - L21 y = r_hat - X S^-1 r_V (eq. R5b); y replaces the
// right-hand-side column, so that the next k_recover gives
// dV = S^-1 (r_V + Y dVhat).  The multipliers of an outer block are stored in
// the row order after the last block of its group of delayed updates (the
// condensation moves them with the interchanges of the later blocks of the
// group, never with those of later groups), so the forward substitution
// replays the interchanges of a whole group (LAPACK order) right before the
// group's columns: width = the group's columns.  Per 64-column
// chunk: wave 0 solves the unit-lower triangle (lane j holds row j), then all
// waves update the rows below with coalesced row reads.
template <int P>
struct FsLds {
    double z[Dims<P>::NV];
    double T[64][65];
};

template <int P>
__global__ void __launch_bounds__(1024) k_fsolve(double* __restrict__ B, const int32_t* __restrict__ ipiv,
                                                const double* __restrict__ r_v, const double* __restrict__ r_h,
                                                double* __restrict__ bhat, int width) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int NV = D::NV, NH = D::NH, ld = BD::ld;
    constexpr int RB = 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    FsLds<P>& L = *reinterpret_cast<FsLds<P>*>(smem_raw);
    const int64_t m = blockIdx.x;
    double* Bm = B + m * BD::per_macro;
    const int32_t* pv = ipiv + m * NV;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int i = tid; i < NV; i += blockDim.x) L.z[i] = r_v[m * NV + i];
    __syncthreads();
    for (int kb0 = 0; kb0 < NV; kb0 += width) {
        const int w = (NV - kb0) < width ? (NV - kb0) : width;
        if (tid == 0) {
            for (int j = kb0; j < kb0 + w; ++j) {
                const int p = pv[j];
                if (p != j && p > j && p < NV) {
                    const double t = L.z[j];
                    L.z[j] = L.z[p];
                    L.z[p] = t;
                }
            }
        }
        __syncthreads();
        for (int c0 = kb0; c0 < kb0 + w; c0 += 64) {
            const int nb = (kb0 + w - c0) < 64 ? (kb0 + w - c0) : 64;
            for (int e = tid; e < 64 * 64; e += blockDim.x) {
                const int r = e >> 6, c = e & 63;
                L.T[r][c] = (r < nb && c < nb) ? Bm[(int64_t)(c0 + r) * ld + c0 + c] : 0.0;
            }
            __syncthreads();
            if (wave == 0) {
                double zi = (lane < nb) ? L.z[c0 + lane] : 0.0;
                for (int j = 0; j < nb; ++j) {
                    const double xj = read_lane_f64(zi, j);
                    if (lane > j) zi -= L.T[lane][j] * xj;
                }
                if (lane < nb) L.z[c0 + lane] = zi;
            }
            __syncthreads();
            const double x = (lane < nb) ? L.z[c0 + lane] : 0.0;
            for (int r0 = c0 + nb + wave * RB; r0 < NV; r0 += nw * RB) {
                double s[RB];
#pragma unroll
                for (int i = 0; i < RB; ++i)
                    s[i] = (lane < nb && r0 + i < NV) ? Bm[(int64_t)(r0 + i) * ld + c0 + lane] * x : 0.0;
#pragma unroll
                for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
                if (lane < RB && r0 + lane < NV) {
                    double si = s[0];
#pragma unroll
                    for (int i = 1; i < RB; ++i)
                        if (lane == i) si = s[i];
                    L.z[r0 + lane] -= si;
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < NV; i += blockDim.x) Bm[(int64_t)i * ld + NV + NH] = L.z[i];
    for (int r0 = wave * RB; r0 < NH; r0 += nw * RB) {
        double s[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = 0.0;
        for (int c = lane; c < NV; c += 64) {
            const double x = L.z[c];
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if (r0 + i < NH) s[i] += Bm[(int64_t)(NV + r0 + i) * ld + c] * x;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) s[i] = wave_sum_f64(s[i]);
        if (lane < RB && r0 + lane < NH) {
            double si = s[0];
#pragma unroll
            for (int i = 1; i < RB; ++i)
                if (lane == i) si = s[i];
            bhat[m * NH + r0 + lane] = (r_h ? r_h[m * NH + r0 + lane] : 0.0) - si;
        }
    }
}

}  // namespace mehdg
