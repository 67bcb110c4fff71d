// Residual of tetrahedral macro-elements: R_Q, R_V, R_Vhat and the face
// entropy production (Sec. 4.1 eq. s32a-c, time term of eq. C242, entropy
// integrand of Thm. EC_ES), on the red-refined P_p macro-tetrahedra of
// tet_tables.hpp.  One workgroup of 256 threads per macro-element:
//
//   1. the nodal state to LDS; the weak gradient q = M^-1 (Chat_j vhat - C_j v)
//      from the constant tables D_i = M^-1 C_i, Dh_f = M^-1 Ch_f when q is not
//      given, then R_Q = M q + C_j v - Chat_j vhat;
//   2. one thread per volume point (8 sub-tets x (p+1)^3): v, v_old, q by
//      interpolation, u(v), the Euler and viscous fluxes, stored weighted and
//      pulled back to the sub-tet's reference axes;
//   3. one thread per (sub-tet, component, sub-tet node): the point sums
//      against the sub-tet basis and its gradients, into LDS scratch; then each
//      macro node gathers its sub-tet entries (fixed order, no atomics);
//   4. one thread per face point (4 faces x 4 sub-triangles x (p+1)^2): the
//      trace state, the trace flux for the face's normal, the viscous trace
//      flux, the entropy integrand; the wall operator's integrand;
//   5. one thread per (face, sub-triangle, component, node): the point sums
//      against the trace basis; each face node gathers its sub-triangle
//      entries, giving R_Vhat, and adds them to R_V at the macro node it sits on.
//
// Every integral is a plain weighted sum over the sub-element rules; the
// tables are constant across macros (L2-resident), the per-macro geometry is
// J^-1, |det J|, and per face the outward normal and twice the area.
//
// MODE 0 is the residual.  MODE 1 is its Jacobian-vector product (with the
// pseudo-time term alpha_ps (A0 dv, w), as in the assembled Jacobian):
// phases 1, 3 and 5 are linear and run unchanged on the tangents
// (dq, dv, dvhat); phases 2 and 4 evaluate the pointwise physics in dual
// numbers seeded with the interpolated tangents and keep only the tangent
// parts.  MODE 2 writes column j = blockIdx.x of the reduced Jacobian J_r
// (the JVP in the unit direction of column j of (dv, dvhat), dq the weak
// gradient) into column j of the bordered matrix of macro m0 + blockIdx.y.
// With q the weak gradient (R_Q = 0), the bordered matrix of the condensation
// (eq. R3-R5), [[S, -Y, r_V], [X, A', r_hat]], is exactly [J_r | -R]:
//   S = A_vv - A_vq A_qq^-1 A_qv,  -Y = A_vvh - A_vq A_qq^-1 A_qvh, and so on.
// MODE 2 takes the pointwise Jacobian coefficients that k_tet_coef stores once
// per macro: the tangent at a point is the coefficient block times the unit
// direction (its value at the point, and its weak gradient there, read from
// the constant tables Phi M^-1 C_i and Phi M^-1 Ch_f), so neither the dual
// arithmetic nor the lift is repeated per column.
#pragma once
#include <type_traits>

#include "physics_n.hpp"

namespace mehdg {

template <int P>
struct TetDims {
    static constexpr int m = 2 * P;
    static constexpr int n = (m + 1) * (m + 2) * (m + 3) / 6;
    static constexpr int nf = (m + 1) * (m + 2) / 2;
    static constexpr int ns = (P + 1) * (P + 2) * (P + 3) / 6;
    static constexpr int nfs = (P + 1) * (P + 2) / 2;
    static constexpr int Gs = (P + 1) * (P + 1) * (P + 1);
    static constexpr int Ss = (P + 1) * (P + 1);
    static constexpr int G = 8 * Gs;        // volume points
    static constexpr int FP = 16 * Ss;      // face points
};

// per-macro geometry record
constexpr int TET_GEO = 32;   // invJ[9], |det J|, normals[4][3], 2 area[4]

struct TetDevTab {
    const double *phi, *dphi, *wv, *BiT, *psi, *wf, *Mt, *CT, *ChT, *DT, *DhT, *Mi;
    const int *vnode, *fnode, *tnode, *vptr, *vinc, *fptr, *finc;
};

// Pointwise Jacobian coefficients (weighted; volume flux derivatives pulled
// back to the sub-tet's reference axes e), stored coefficient-major with the
// point index fastest ([n_macro][TET_CV][G], [n_macro][TET_CF][FP]) so that
// the lanes of a wave, one point each, read contiguous memory:
//   volume point, TET_CV coefficients:
//     [5k + l]                     w (alpha_t + alpha_ps) du_k/dv_l
//     [25 + 25e + 5k + l]          w sum_i BiT_s[i][e] sum_d invJ[i][d] d(F + G)_kd/dv_l
//     [100 + 25(3e + j) + 5k + l]  w sum_i BiT_s[i][e] sum_d invJ[i][d] dG_kd/dq_lj
//   face point, TET_CF coefficients:
//     [5k + l]                     ws d(Fhat + Ghat)_k/dv_l
//     [25 + 5k + l]                ws d(Fhat + Ghat)_k/dvhat_l
//     [50 + 25j + 5k + l]          ws dGhat_k/dq_lj
constexpr int TET_CV = 325, TET_CF = 125;

// Tables of the coefficient-based columns (MODE 2).
struct TetColTab {
    const double *coefV, *coefF;      // [n_macro][TET_CV][G], [n_macro][TET_CF][FP]
    const double *ED, *EDf;           // (Phi M^-1 C_i)[point][b] as [3][n][G], [3][n][FP]
    const double *EH, *EHf;           // (Phi M^-1 Ch_f)[point][c] as [4][nf][G], [4][nf][FP]
    int64_t m0;                       // first macro of the launch (blockIdx.y counts from it)
    const int *vloc, *tloc, *fidx;    // [8][n] local index of a macro node in a sub-tet (-1: none),
                                      // [4][nf] of a face node in a sub-triangle, [4][n] face node of a macro node
};

template <int P, bool LIN>
struct TetLds {   // LIN: the tangent arrays of MODE 1
    using D = TetDims<P>;
    static constexpr int PT = (20 * D::G > 10 * D::FP) ? 20 * D::G : 10 * D::FP;
    static constexpr int SC = (8 * 5 * D::ns > 2 * 80 * D::nfs) ? 8 * 5 * D::ns : 2 * 80 * D::nfs;
    static constexpr int NL = LIN ? D::n : 1, NFL = LIN ? D::nf : 1;
    double v[5][D::n], vo[5][D::n], vh[4][5][D::nf], q[15][D::n], rv[5][D::n];
    double dv[5][NL], dvh[4][5][NFL], dq[15][NL];   // tangents (LIN)
    double pt[PT];
    double sc[SC];
    double red[4];
};

// LDS of a MODE 2 (column) workgroup: no nodal state, the sub-tet basis
// tables staged once for the test sums instead, and the volume points held
// for SB sub-tets at a time (at p = 3 two, which keeps the total under 80 KB:
// two workgroups per CU).
template <int P>
struct TetColLds {
    using D = TetDims<P>;
    static constexpr int SB = (P == 3) ? 2 : 8;
    static constexpr int PT = (20 * SB * D::Gs > 10 * D::FP) ? 20 * SB * D::Gs : 10 * D::FP;
    static constexpr int SC = TetLds<P, false>::SC;
    double rv[5][D::n];
    double pt[PT];
    double sc[SC];
    double ph[D::Gs * D::ns], dph[3 * D::Gs * D::ns];
    double red[4];
};

constexpr int TET_THREADS = 256;

// value / tangent access for the two scalar types of the point phases
template <typename S>
struct TetScalar;
template <>
struct TetScalar<double> {
    static MEHDG_HD double mk(double v, double) { return v; }
    static MEHDG_HD double val(double x) { return x; }
    static MEHDG_HD double out(double x) { return x; }
};
template <>
struct TetScalar<dual<1>> {
    static MEHDG_HD dual<1> mk(double v, double d) {
        dual<1> r;
        r.v = v;
        r.d[0] = d;
        return r;
    }
    static MEHDG_HD double val(const dual<1>& x) { return x.v; }
    static MEHDG_HD double out(const dual<1>& x) { return x.d[0]; }
};

// q = M^-1 (Chat_j vh - C_j v) from the tables D_i, Dh_f (eq. s32a with R_Q = 0).
template <int P>
__device__ void tet_lift(const TetDevTab& T, const double* gm, const double* invJ, double adet,
                         const double (*V)[TetDims<P>::n], const double (*VH)[5][TetDims<P>::nf],
                         double (*Q)[TetDims<P>::n]) {
    constexpr int n = TetDims<P>::n, nf = TetDims<P>::nf;
    for (int i = threadIdx.x; i < 5 * n; i += blockDim.x) {
        const int k = i / n, a = i - k * n;
        double dv[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; ++b) {
            const double x = V[k][b];
#pragma unroll
            for (int d = 0; d < 3; ++d) dv[d] += T.DT[(d * n + b) * n + a] * x;
        }
        double qj[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) qj[j] = -(invJ[0 * 3 + j] * dv[0] + invJ[1 * 3 + j] * dv[1] + invJ[2 * 3 + j] * dv[2]);
        for (int f = 0; f < 4; ++f) {
            double dh = 0.0;
            for (int c = 0; c < nf; ++c) dh += T.DhT[(f * nf + c) * n + a] * VH[f][k][c];
            const double s = gm[22 + f] / adet * dh;
#pragma unroll
            for (int j = 0; j < 3; ++j) qj[j] += s * gm[10 + 3 * f + j];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[3 * k + j][a] = qj[j];
    }
}

// R_Q = M q + C_j v - Chat_j vh of one macro, to global memory.
template <int P>
__device__ void tet_rq(const TetDevTab& T, const double* gm, const double* invJ, double adet,
                       const double (*V)[TetDims<P>::n], const double (*VH)[5][TetDims<P>::nf],
                       const double (*Q)[TetDims<P>::n], double* __restrict__ out) {
    constexpr int n = TetDims<P>::n, nf = TetDims<P>::nf;
    for (int i = threadIdx.x; i < 5 * n; i += blockDim.x) {
        const int k = i / n, a = i - k * n;
        double mq[3] = {0.0, 0.0, 0.0}, cv[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; ++b) {
            const double mt = T.Mt[b * n + a];
            const double x = V[k][b];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                mq[j] += mt * Q[3 * k + j][b];
                cv[j] += T.CT[(j * n + b) * n + a] * x;
            }
        }
        double r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = adet * (mq[j] + invJ[0 * 3 + j] * cv[0] + invJ[1 * 3 + j] * cv[1] + invJ[2 * 3 + j] * cv[2]);
        for (int f = 0; f < 4; ++f) {
            double ch = 0.0;
            for (int c = 0; c < nf; ++c) ch += T.ChT[(f * nf + c) * n + a] * VH[f][k][c];
#pragma unroll
            for (int j = 0; j < 3; ++j) r[j] -= gm[22 + f] * gm[10 + 3 * f + j] * ch;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) out[(k * 3 + j) * n + a] = r[j];
    }
}

// MODE 0: residual (R_q, R_v, R_vh, entropy) at (q, v, vhat) with q = qin or
// the weak gradient.  MODE 1: the tangents (JR_q, JR_v, JR_vh) in the
// direction (dq, dv, dvhat), dq = dqin or the weak gradient of (dv, dvhat);
// entropy is not written and may be null.  MODE 2: column blockIdx.x of J_r
// of macro ct.m0 + blockIdx.y into Bc (bordered matrices, ld and per_macro
// doubles apart), rows in the order V then Vhat, from the coefficients and
// tables in ct; the state arguments, R_q, R_v, R_vh and entropy are unused.
template <int P, int MODE>
__global__ void __launch_bounds__(TET_THREADS)
k_tet(const double* __restrict__ v, const double* __restrict__ vhat, const double* __restrict__ qin,
      const double* __restrict__ v_old, const double* __restrict__ dvin, const double* __restrict__ dvhin,
      const double* __restrict__ dqin, const double* __restrict__ geo, TetDevTab T, DevParams pr,
      const uint8_t* __restrict__ face_bc, double* __restrict__ R_q, double* __restrict__ R_v,
      double* __restrict__ R_vh, double* __restrict__ entropy, int32_t* __restrict__ status,
      double* __restrict__ Bc, int ld, int64_t per_macro, TetColTab ct) {
    constexpr bool LIN = MODE == 1;
    constexpr bool COL = MODE == 2;    // one column of the bordered matrix
    using D = TetDims<P>;
    using S = typename std::conditional<LIN, dual<1>, double>::type;
    using SC = TetScalar<S>;
    constexpr int n = D::n, nf = D::nf, ns = D::ns, nfs = D::nfs, Gs = D::Gs, Ss = D::Ss;
    extern __shared__ __align__(16) unsigned char smem[];
    using Lds = typename std::conditional<MODE == 2, TetColLds<P>, TetLds<P, LIN>>::type;
    Lds& L = *reinterpret_cast<Lds*>(smem);
    const int tid = threadIdx.x;
    // columns: blockIdx.x is the column, so the columns of one macro run back to back (L2 reuse)
    const int64_t m = COL ? ct.m0 + blockIdx.y : (int64_t)blockIdx.x;
    const double* gm = geo + m * TET_GEO;
    double invJ[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) invJ[i] = gm[i];
    const double adet = gm[9];
    bool bad_phys = false, bad_fin = false;

    // ---- 1. state, weak gradient, R_Q (tangents: the same linear maps)
    // (MODE 2 needs none of it: the coefficients hold the state's part)
    const int col = COL ? (int)blockIdx.x : -1;
    if constexpr (MODE != 2) {
    for (int i = tid; i < 5 * n; i += TET_THREADS) {
        (&L.v[0][0])[i] = v[m * 5 * n + i];
        if constexpr (MODE == 1) (&L.dv[0][0])[i] = dvin[m * 5 * n + i];
        else (&L.vo[0][0])[i] = v_old[m * 5 * n + i];
    }
    for (int i = tid; i < 20 * nf; i += TET_THREADS) {
        (&L.vh[0][0][0])[i] = vhat[m * 20 * nf + i];
        if constexpr (MODE == 1) (&L.dvh[0][0][0])[i] = dvhin[m * 20 * nf + i];
    }
    if (qin)
        for (int i = tid; i < 15 * n; i += TET_THREADS) (&L.q[0][0])[i] = qin[m * 15 * n + i];
    if constexpr (MODE == 1) {
        if (dqin)
            for (int i = tid; i < 15 * n; i += TET_THREADS) (&L.dq[0][0])[i] = dqin[m * 15 * n + i];
    }
    __syncthreads();
    if (!qin) tet_lift<P>(T, gm, invJ, adet, L.v, L.vh, L.q);
    if constexpr (LIN) {
        if (!dqin) tet_lift<P>(T, gm, invJ, adet, L.dv, L.dvh, L.dq);
    }
    __syncthreads();
    if constexpr (MODE == 1) tet_rq<P>(T, gm, invJ, adet, L.dv, L.dvh, L.dq, R_q + m * 15 * n);
    else if constexpr (MODE == 0) tet_rq<P>(T, gm, invJ, adet, L.v, L.vh, L.q, R_q + m * 15 * n);
    }   // MODE != 2

    // unit direction of a MODE 2 column: V column (l, b) or trace column (f0, l, c0)
    int cl = 0, cb = -1, cf0 = 0, cc0 = 0;
    const double* PHI = T.phi;     // basis tables of the test sums (staged in LDS for MODE 2)
    const double* DPHI = T.dphi;
    if constexpr (MODE == 2) {
        for (int i = tid; i < Gs * ns; i += TET_THREADS) L.ph[i] = T.phi[i];
        for (int i = tid; i < 3 * Gs * ns; i += TET_THREADS) L.dph[i] = T.dphi[i];
        PHI = L.ph;
        DPHI = L.dph;
        if (col < 5 * n) {
            cl = col / n;
            cb = col - cl * n;
        } else {
            const int r = col - 5 * n;
            cf0 = r / (5 * nf);
            cl = (r / nf) % 5;
            cc0 = r % nf;
        }
    }

    // ---- 2. volume points
    const double g = pr.gamma;
    if constexpr (MODE == 2) {
      // the points of SB sub-tets at a time, then their test sums (phase 3)
      constexpr int SB = TetColLds<P>::SB;
      for (int s0 = 0; s0 < 8; s0 += SB) {
        for (int q = tid; q < SB * Gs; q += TET_THREADS) {
            const int gp = s0 * Gs + q;
            const int s = gp / Gs, gl = gp - s * Gs;
            double dv = 0.0, dq[3];
            if (cb >= 0) {
                const int bl = ct.vloc[s * n + cb];
                if (bl >= 0) dv = T.phi[gl * ns + bl];
                double e[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) e[i] = ct.ED[((int64_t)i * n + cb) * D::G + gp];
#pragma unroll
                for (int j = 0; j < 3; ++j) dq[j] = -(invJ[0 * 3 + j] * e[0] + invJ[1 * 3 + j] * e[1] + invJ[2 * 3 + j] * e[2]);
            } else {
                const double eh = ct.EH[((int64_t)cf0 * nf + cc0) * D::G + gp] * (gm[22 + cf0] / adet);
#pragma unroll
                for (int j = 0; j < 3; ++j) dq[j] = eh * gm[10 + 3 * cf0 + j];
            }
            const double* C = ct.coefV + (int64_t)m * TET_CV * D::G + gp;   // coefficient i at C[i * G]
            double* o = L.pt + q * 20;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                o[k] = C[(5 * k + cl) * D::G] * dv;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    double x = C[(25 + 25 * e + 5 * k + cl) * D::G] * dv;
#pragma unroll
                    for (int j = 0; j < 3; ++j) x += C[(100 + 25 * (3 * e + j) + 5 * k + cl) * D::G] * dq[j];
                    o[5 + 3 * k + e] = x;
                }
                if (!isfinite(o[k]) || !isfinite(o[5 + 3 * k])) bad_fin = true;
            }
        }
        __syncthreads();
        for (int i = tid; i < SB * 5 * ns; i += TET_THREADS) {
            const int sl = i / (5 * ns), r = i - sl * 5 * ns, k = r / ns, b = r - k * ns;
            double acc = 0.0;
            for (int gl = 0; gl < Gs; ++gl) {
                const double* o = L.pt + (sl * Gs + gl) * 20;
                acc += o[k] * PHI[gl * ns + b] - o[5 + 3 * k + 0] * DPHI[(0 * Gs + gl) * ns + b] -
                       o[5 + 3 * k + 1] * DPHI[(1 * Gs + gl) * ns + b] - o[5 + 3 * k + 2] * DPHI[(2 * Gs + gl) * ns + b];
            }
            L.sc[(s0 + sl) * 5 * ns + r] = acc;
        }
        __syncthreads();
      }
    } else {
    for (int gp = tid; gp < D::G; gp += TET_THREADS) {
        const int s = gp / Gs, gl = gp - s * Gs;
        double vv0[5] = {0, 0, 0, 0, 0}, vvd[5] = {0, 0, 0, 0, 0}, vvo[5] = {0, 0, 0, 0, 0};
        double qq0[5][3] = {}, qqd[5][3] = {};
        for (int b = 0; b < ns; ++b) {
            const double ph = T.phi[gl * ns + b];
            const int a = T.vnode[s * ns + b];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vv0[k] += ph * L.v[k][a];
                if constexpr (LIN) vvd[k] += ph * L.dv[k][a];
                else vvo[k] += ph * L.vo[k][a];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    qq0[k][j] += ph * L.q[3 * k + j][a];
                    if constexpr (LIN) qqd[k][j] += ph * L.dq[3 * k + j][a];
                }
            }
        }
        S vv[5], qq[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            vv[k] = SC::mk(vv0[k], vvd[k]);
#pragma unroll
            for (int j = 0; j < 3; ++j) qq[k][j] = SC::mk(qq0[k][j], qqd[k][j]);
        }
        Prim<S> st;
        primitive(vv, g, st);
        if (!(vv0[4] < 0.0) || !(SC::val(st.rho) > 0.0)) bad_phys = true;
        S u[5];
        conservative(st, g, u);
        double tt[5];
        if constexpr (LIN) {
#pragma unroll
            for (int k = 0; k < 5; ++k) tt[k] = (pr.alpha_t + pr.alpha_ps) * SC::out(u[k]);
        } else {
            Prim<double> so;
            primitive(vvo, g, so);
            if (!(vvo[4] < 0.0) || !(so.rho > 0.0)) bad_phys = true;
            double uo[5];
            conservative(so, g, uo);
#pragma unroll
            for (int k = 0; k < 5; ++k) tt[k] = pr.alpha_t * (u[k] - uo[k]);
        }
        double F[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            S Fs[5];
            euler_flux(st, g, d, Fs);
            if (pr.viscous) {
                S Gv[5];
                viscous_flux(vv, qq, pr, d, Gv);
#pragma unroll
                for (int k = 0; k < 5; ++k) Fs[k] = Fs[k] + Gv[k];
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) F[d][k] = SC::out(Fs[k]);
        }
        const double w = T.wv[gl] * adet;
        const double* Bi = T.BiT + s * 9;
        double* o = L.pt + gp * 20;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            o[k] = w * tt[k];
            double Fx[3];   // sum_j invJ[i][j] F_kj
#pragma unroll
            for (int i = 0; i < 3; ++i) Fx[i] = invJ[i * 3 + 0] * F[0][k] + invJ[i * 3 + 1] * F[1][k] + invJ[i * 3 + 2] * F[2][k];
#pragma unroll
            for (int e = 0; e < 3; ++e) o[5 + 3 * k + e] = w * (Bi[0 * 3 + e] * Fx[0] + Bi[1 * 3 + e] * Fx[1] + Bi[2 * 3 + e] * Fx[2]);
            if (!isfinite(o[k]) || !isfinite(o[5 + 3 * k])) bad_fin = true;
        }
    }
    __syncthreads();

    // ---- 3. volume test functions
    for (int i = tid; i < 8 * 5 * ns; i += TET_THREADS) {
        const int s = i / (5 * ns), r = i - s * 5 * ns, k = r / ns, b = r - k * ns;
        double acc = 0.0;
        for (int gl = 0; gl < Gs; ++gl) {
            const double* o = L.pt + (s * Gs + gl) * 20;
            acc += o[k] * PHI[gl * ns + b] - o[5 + 3 * k + 0] * DPHI[(0 * Gs + gl) * ns + b] -
                   o[5 + 3 * k + 1] * DPHI[(1 * Gs + gl) * ns + b] - o[5 + 3 * k + 2] * DPHI[(2 * Gs + gl) * ns + b];
        }
        L.sc[i] = acc;
    }
    __syncthreads();
    }   // MODE != 2
    for (int i = tid; i < 5 * n; i += TET_THREADS) {
        const int k = i / n, a = i - k * n;
        double acc = 0.0;
        for (int e = T.vptr[a]; e < T.vptr[a + 1]; ++e) {
            const int sb = T.vinc[e], s = sb / ns, b = sb - s * ns;
            acc += L.sc[(s * 5 + k) * ns + b];
        }
        L.rv[k][a] = acc;
    }
    __syncthreads();

    // ---- 4. face points
    double ent = 0.0;
    if constexpr (MODE == 2) {
        for (int fp = tid; fp < D::FP; fp += TET_THREADS) {
            const int f = fp / (4 * Ss), r = fp - f * 4 * Ss, tr = r / Ss, sl = r - tr * Ss;
            double dv = 0.0, dvh = 0.0, dq[3];
            if (cb >= 0) {
                const int cf = ct.fidx[f * n + cb];
                if (cf >= 0) {
                    const int bl = ct.tloc[tr * nf + cf];
                    if (bl >= 0) dv = T.psi[sl * nfs + bl];
                }
                double e[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) e[i] = ct.EDf[((int64_t)i * n + cb) * D::FP + fp];
#pragma unroll
                for (int j = 0; j < 3; ++j) dq[j] = -(invJ[0 * 3 + j] * e[0] + invJ[1 * 3 + j] * e[1] + invJ[2 * 3 + j] * e[2]);
            } else {
                if (f == cf0) {
                    const int bl = ct.tloc[tr * nf + cc0];
                    if (bl >= 0) dvh = T.psi[sl * nfs + bl];
                }
                const double eh = ct.EHf[((int64_t)cf0 * nf + cc0) * D::FP + fp] * (gm[22 + cf0] / adet);
#pragma unroll
                for (int j = 0; j < 3; ++j) dq[j] = eh * gm[10 + 3 * cf0 + j];
            }
            const double* C = ct.coefF + (int64_t)m * TET_CF * D::FP + fp;   // coefficient i at C[i * FP]
            const double ws = T.wf[sl] * gm[22 + f];
            double* o = L.pt + fp * 10;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double x = C[(5 * k + cl) * D::FP] * dv + C[(25 + 5 * k + cl) * D::FP] * dvh;
#pragma unroll
                for (int j = 0; j < 3; ++j) x += C[(50 + 25 * j + 5 * k + cl) * D::FP] * dq[j];
                o[k] = x;
                o[5 + k] = (k == cl) ? ws * dvh : 0.0;
                if (!isfinite(x)) bad_fin = true;
            }
        }
    } else
    for (int fp = tid; fp < D::FP; fp += TET_THREADS) {
        const int f = fp / (4 * Ss), r = fp - f * 4 * Ss, tr = r / Ss, sl = r - tr * Ss;
        double vh0[5] = {0, 0, 0, 0, 0}, vs0[5] = {0, 0, 0, 0, 0}, qq0[5][3] = {};
        double vhd[5] = {0, 0, 0, 0, 0}, vsd[5] = {0, 0, 0, 0, 0}, qqd[5][3] = {};
        for (int b = 0; b < nfs; ++b) {
            const double ps = T.psi[sl * nfs + b];
            const int c = T.tnode[tr * nfs + b];
            const int a = T.fnode[f * nf + c];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vh0[k] += ps * L.vh[f][k][c];
                vs0[k] += ps * L.v[k][a];
                if constexpr (LIN) {
                    vhd[k] += ps * L.dvh[f][k][c];
                    vsd[k] += ps * L.dv[k][a];
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    qq0[k][j] += ps * L.q[3 * k + j][a];
                    if constexpr (LIN) qqd[k][j] += ps * L.dq[3 * k + j][a];
                }
            }
        }
        S vh[5], vs[5], qq[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            vh[k] = SC::mk(vh0[k], vhd[k]);
            vs[k] = SC::mk(vs0[k], vsd[k]);
#pragma unroll
            for (int j = 0; j < 3; ++j) qq[k][j] = SC::mk(qq0[k][j], qqd[k][j]);
        }
        const double nrm[3] = {gm[10 + 3 * f], gm[11 + 3 * f], gm[12 + 3 * f]};
        double t1[3], t2[3];
        face_frame(nrm, t1, t2);
        const double ws = T.wf[sl] * gm[22 + f];
        S Fh[5];
        trace_flux_n(vh, vs, pr, nrm, t1, t2, Fh);
        {
            Prim<double> a, b;
            primitive(vh0, g, a);
            primitive(vs0, g, b);
            if (!(vh0[4] < 0.0) || !(a.rho > 0.0)) bad_phys = true;
            if constexpr (!LIN) {
                double e = 0.0;
#pragma unroll
                for (int k = 0; k < 5; ++k) e += (vh0[k] - vs0[k]) * Fh[k];
                e -= a.rho * dot3(a.V, nrm) - b.rho * dot3(b.V, nrm);
                ent += ws * e;
            }
        }
        if (pr.viscous) {
            S Gh[5];
            viscous_trace_flux_n(vh, vs, qq, pr, nrm, Gh);
#pragma unroll
            for (int k = 0; k < 5; ++k) Fh[k] = Fh[k] + Gh[k];
        }
        double* o = L.pt + fp * 10;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            o[k] = ws * SC::out(Fh[k]);
            o[5 + k] = LIN ? ws * vhd[k] : ws * (vh0[k] + (k == 4 ? pr.gT : 0.0));
            if (!isfinite(o[k])) bad_fin = true;
        }
    }
    if constexpr (MODE == 0) {
        for (int off = 32; off > 0; off >>= 1) ent += __shfl_down(ent, off, 64);
        if ((tid & 63) == 0) L.red[tid >> 6] = ent;
    }
    __syncthreads();
    if constexpr (MODE == 0) {
        if (tid == 0) entropy[m] = L.red[0] + L.red[1] + L.red[2] + L.red[3];
    }

    // ---- 5. trace test functions
    constexpr int FS = 80 * nfs;   // (face, sub-triangle, component, node) entries
    for (int i = tid; i < FS; i += TET_THREADS) {
        const int ft = i / (5 * nfs), r = i - ft * 5 * nfs, k = r / nfs, b = r - k * nfs;
        double acc = 0.0, accw = 0.0;
        for (int sl = 0; sl < Ss; ++sl) {
            const double ps = T.psi[sl * nfs + b];
            const double* o = L.pt + (ft * Ss + sl) * 10;
            acc += ps * o[k];
            accw += ps * o[5 + k];
        }
        L.sc[i] = acc;
        L.sc[FS + i] = accw;
    }
    __syncthreads();
    for (int f = 0; f < 4; ++f) {
        const bool wall = face_bc && face_bc[m * 4 + f];
        for (int i = tid; i < 5 * nf; i += TET_THREADS) {
            const int k = i / nf, c = i - k * nf;
            double acc = 0.0, accw = 0.0;
            for (int e = T.fptr[c]; e < T.fptr[c + 1]; ++e) {
                const int tb = T.finc[e], tr = tb / nfs, b = tb - tr * nfs;
                const int idx = ((f * 4 + tr) * 5 + k) * nfs + b;
                acc += L.sc[idx];
                accw += L.sc[FS + idx];
            }
            L.rv[k][T.fnode[f * nf + c]] += acc;
            const double o = (wall && k > 0) ? accw : acc;
            if constexpr (COL) Bc[m * per_macro + (int64_t)(5 * n + (f * 5 + k) * nf + c) * ld + col] = o;
            else R_vh[((m * 4 + f) * 5 + k) * nf + c] = o;
        }
        __syncthreads();
    }
    for (int i = tid; i < 5 * n; i += TET_THREADS) {
        if constexpr (COL) Bc[m * per_macro + (int64_t)i * ld + col] = (&L.rv[0][0])[i];
        else R_v[m * 5 * n + i] = (&L.rv[0][0])[i];
    }

    // ---- status: a flagged macro's outputs are NaN
    const int flag = __syncthreads_or(bad_phys ? 1 : (bad_fin ? 2 : 0));
    if (flag) {
        const int any_phys = __syncthreads_or(bad_phys ? 1 : 0);
        const double nan = __builtin_nan("");
        if constexpr (COL) {
            for (int i = tid; i < 5 * n + 20 * nf; i += TET_THREADS) Bc[m * per_macro + (int64_t)i * ld + col] = nan;
        } else {
            for (int i = tid; i < 5 * n; i += TET_THREADS) R_v[m * 5 * n + i] = nan;
            for (int i = tid; i < 15 * n; i += TET_THREADS) R_q[m * 15 * n + i] = nan;
            for (int i = tid; i < 20 * nf; i += TET_THREADS) R_vh[m * 20 * nf + i] = nan;
        }
        if (tid == 0) {
            if (MODE == 0) entropy[m] = nan;
            // a column launch only raises a code and keeps the most basic one:
            // the coefficient kernel before it has already flagged the state
            if (status) {
                if (COL) record_status(status, m, any_phys ? ST_NONPHYSICAL : ST_NONFINITE);
                else status[m] = any_phys ? ST_NONPHYSICAL : ST_NONFINITE;
            }
        }
    } else if (!COL && tid == 0 && status) {
        status[m] = 0;   // (column launches only ever raise a flag)
    }
}

// Pointwise Jacobian coefficients of every volume and face point of a macro
// (layout at TET_CV / TET_CF above), at the state (v, vhat) with q its weak
// gradient: derivatives in v and vhat by dual numbers (dual<5>, one pass per
// seeded argument), derivatives in q by evaluating the viscous fluxes at unit
// q, since they are linear in q.  A non-physical state raises the macro's
// status (the residual launched before it has reset it).
template <int P>
__global__ void __launch_bounds__(TET_THREADS)
k_tet_coef(const double* __restrict__ v, const double* __restrict__ vhat, const double* __restrict__ geo,
           TetDevTab T, DevParams pr, double* __restrict__ coefV, double* __restrict__ coefF,
           int32_t* __restrict__ status) {
    using D = TetDims<P>;
    constexpr int n = D::n, nf = D::nf, ns = D::ns, nfs = D::nfs, Gs = D::Gs, Ss = D::Ss;
    extern __shared__ __align__(16) unsigned char smem[];
    TetLds<P, false>& L = *reinterpret_cast<TetLds<P, false>*>(smem);
    const int tid = threadIdx.x;
    const int64_t m = blockIdx.x;
    const double* gm = geo + m * TET_GEO;
    double invJ[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) invJ[i] = gm[i];
    const double adet = gm[9];
    const double g = pr.gamma;
    bool bad = false;
    for (int i = tid; i < 5 * n; i += TET_THREADS) (&L.v[0][0])[i] = v[m * 5 * n + i];
    for (int i = tid; i < 20 * nf; i += TET_THREADS) (&L.vh[0][0][0])[i] = vhat[m * 20 * nf + i];
    __syncthreads();
    tet_lift<P>(T, gm, invJ, adet, L.v, L.vh, L.q);
    __syncthreads();

    for (int gp = tid; gp < D::G; gp += TET_THREADS) {
        const int s = gp / Gs, gl = gp - s * Gs;
        double vv[5] = {0, 0, 0, 0, 0}, qq[5][3] = {};
        for (int b = 0; b < ns; ++b) {
            const double ph = T.phi[gl * ns + b];
            const int a = T.vnode[s * ns + b];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vv[k] += ph * L.v[k][a];
#pragma unroll
                for (int j = 0; j < 3; ++j) qq[k][j] += ph * L.q[3 * k + j][a];
            }
        }
        const double w = T.wv[gl] * adet;
        const double* Bi = T.BiT + s * 9;
        double K[3][3];   // K[d][e] = w sum_i BiT_s[i][e] invJ[i][d]
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 3; ++e)
                K[d][e] = w * (Bi[0 * 3 + e] * invJ[0 * 3 + d] + Bi[1 * 3 + e] * invJ[1 * 3 + d] + Bi[2 * 3 + e] * invJ[2 * 3 + d]);
        double* out = coefV + (int64_t)m * TET_CV * D::G + gp;   // coefficient i at out[i * G]
        auto put = [&](int i, double x) { out[(int64_t)i * D::G] = x; };
        dual<5> vd[5];
#pragma unroll
        for (int l = 0; l < 5; ++l) vd[l] = seed_dual<5>(vv[l], l);
        Prim<dual<5>> st;
        primitive(vd, g, st);
        if (!(vv[4] < 0.0) || !(st.rho.v > 0.0)) bad = true;
        {
            dual<5> u[5];
            conservative(st, g, u);
            const double c = (pr.alpha_t + pr.alpha_ps) * w;
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int l = 0; l < 5; ++l) put(5 * k + l, c * u[k].d[l]);
        }
        dual<5> qd[5][3];
#pragma unroll
        for (int l = 0; l < 5; ++l)
#pragma unroll
            for (int j = 0; j < 3; ++j) qd[l][j] = make_dual<5>(qq[l][j]);
        double acc[3][25];
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int i = 0; i < 25; ++i) acc[e][i] = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            dual<5> F[5];
            euler_flux(st, g, d, F);
            if (pr.viscous) {
                dual<5> Gv[5];
                viscous_flux(vd, qd, pr, d, Gv);
#pragma unroll
                for (int k = 0; k < 5; ++k) F[k] = F[k] + Gv[k];
            }
#pragma unroll
            for (int e = 0; e < 3; ++e)
#pragma unroll
                for (int k = 0; k < 5; ++k)
#pragma unroll
                    for (int l = 0; l < 5; ++l) acc[e][5 * k + l] += K[d][e] * F[k].d[l];
        }
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int i = 0; i < 25; ++i) put(25 + 25 * e + i, acc[e][i]);
        // G is linear in q: its q-derivative columns are G at unit q
        for (int l = 0; l < 5; ++l)
            for (int j = 0; j < 3; ++j) {
                double Gd[3][5] = {};
                if (pr.viscous) {
                    double qu[5][3];
#pragma unroll
                    for (int a = 0; a < 5; ++a) qu[a][0] = qu[a][1] = qu[a][2] = 0.0;
                    qu[l][j] = 1.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) viscous_flux(vv, qu, pr, d, Gd[d]);
                }
#pragma unroll
                for (int e = 0; e < 3; ++e)
#pragma unroll
                    for (int k = 0; k < 5; ++k)
                        put(100 + 25 * (3 * e + j) + 5 * k + l, K[0][e] * Gd[0][k] + K[1][e] * Gd[1][k] + K[2][e] * Gd[2][k]);
            }
    }

    for (int fp = tid; fp < D::FP; fp += TET_THREADS) {
        const int f = fp / (4 * Ss), r = fp - f * 4 * Ss, tr = r / Ss, sl = r - tr * Ss;
        double vh[5] = {0, 0, 0, 0, 0}, vs[5] = {0, 0, 0, 0, 0}, qq[5][3] = {};
        for (int b = 0; b < nfs; ++b) {
            const double ps = T.psi[sl * nfs + b];
            const int c = T.tnode[tr * nfs + b];
            const int a = T.fnode[f * nf + c];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vh[k] += ps * L.vh[f][k][c];
                vs[k] += ps * L.v[k][a];
#pragma unroll
                for (int j = 0; j < 3; ++j) qq[k][j] += ps * L.q[3 * k + j][a];
            }
        }
        const double nrm[3] = {gm[10 + 3 * f], gm[11 + 3 * f], gm[12 + 3 * f]};
        double t1[3], t2[3];
        face_frame(nrm, t1, t2);
        const double ws = T.wf[sl] * gm[22 + f];
        if (!(vh[4] < 0.0)) bad = true;
        double* out = coefF + (int64_t)m * TET_CF * D::FP + fp;   // coefficient i at out[i * FP]
        auto put = [&](int i, double x) { out[(int64_t)i * D::FP] = x; };
#pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {   // 0: d/dv, 1: d/dvhat
            dual<5> a[5], b[5], F[5];
#pragma unroll
            for (int l = 0; l < 5; ++l) {
                a[l] = (pass == 1) ? seed_dual<5>(vh[l], l) : make_dual<5>(vh[l]);
                b[l] = (pass == 0) ? seed_dual<5>(vs[l], l) : make_dual<5>(vs[l]);
            }
            trace_flux_n(a, b, pr, nrm, t1, t2, F);
            if (pr.viscous) {
                dual<5> qd[5][3], Gh[5];
#pragma unroll
                for (int l = 0; l < 5; ++l)
#pragma unroll
                    for (int j = 0; j < 3; ++j) qd[l][j] = make_dual<5>(qq[l][j]);
                viscous_trace_flux_n(a, b, qd, pr, nrm, Gh);
#pragma unroll
                for (int k = 0; k < 5; ++k) F[k] = F[k] + Gh[k];
            }
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int l = 0; l < 5; ++l) put(25 * pass + 5 * k + l, ws * F[k].d[l]);
        }
        // Ghat = G(vhat, q).n - ...: linear in q
        for (int l = 0; l < 5; ++l)
            for (int j = 0; j < 3; ++j) {
                double Gn[5] = {0, 0, 0, 0, 0};
                if (pr.viscous) {
                    double qu[5][3];
#pragma unroll
                    for (int a = 0; a < 5; ++a) qu[a][0] = qu[a][1] = qu[a][2] = 0.0;
                    qu[l][j] = 1.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        double Gd[5];
                        viscous_flux(vh, qu, pr, d, Gd);
#pragma unroll
                        for (int k = 0; k < 5; ++k) Gn[k] += nrm[d] * Gd[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < 5; ++k) put(50 + 25 * j + 5 * k + l, ws * Gn[k]);
            }
    }
    if (__syncthreads_or(bad ? 1 : 0) && tid == 0 && status) status[m] = 5;
}

// Recovery of tetrahedral macros (eq. R2, R6): dV = U^-1 (y - U12 dVhat)
// from the factored bordered matrix (the back-substitution of the hexahedral
// path), then dQ = A_qq^-1 (-R_Q - A_qv dV - A_qvh dVhat) = lift(dV, dVhat)
// - M^-1 R_Q with the weak-gradient tables.  One workgroup of 1024 threads
// per macro.
template <int P>
struct TetRecLds {
    double z[TetDims<P>::n * 5];
    double dvh[TetDims<P>::nf * 20];
    double U[64][65];
};

template <int P>
__global__ void __launch_bounds__(1024) k_tet_recover(const double* __restrict__ B, const double* __restrict__ R_q,
                                                     const double* __restrict__ dvhat, const double* __restrict__ geo,
                                                     TetDevTab T, double* __restrict__ dv, double* __restrict__ dq) {
    using D = TetDims<P>;
    constexpr int n = D::n, nf = D::nf, NV = 5 * n, NH = 20 * nf;
    static_assert(Dims<TET_TAG + P>::NV == NV && Dims<TET_TAG + P>::NH == NH, "tetrahedral sizes");
    extern __shared__ __align__(16) unsigned char smem[];
    TetRecLds<P>& L = *reinterpret_cast<TetRecLds<P>*>(smem);
    const int64_t m = blockIdx.x;
    const int tid = threadIdx.x;
    const double* gm = geo + m * TET_GEO;
    double invJ[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) invJ[i] = gm[i];
    const double adet = gm[9];
    for (int i = tid; i < NH; i += blockDim.x) L.dvh[i] = dvhat[m * NH + i];
    __syncthreads();
    back_substitute<TET_TAG + P>(B + m * Bdims<TET_TAG + P>::per_macro, L.dvh, L.z, L.U);
    __syncthreads();
    for (int i = tid; i < NV; i += blockDim.x) dv[m * NV + i] = L.z[i];
    double* out = dq + m * 15 * n;
    tet_lift<P>(T, gm, invJ, adet, reinterpret_cast<const double(*)[n]>(L.z),
                reinterpret_cast<const double(*)[5][nf]>(L.dvh), reinterpret_cast<double(*)[n]>(out));
    // the same thread owns the same (k, a) entries as in the lift
    const double* rq = R_q + m * 15 * n;
    for (int i = tid; i < 5 * n; i += blockDim.x) {
        const int k = i / n, a = i - k * n;
        double s[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; ++b) {
            const double mi = T.Mi[b * n + a];
#pragma unroll
            for (int j = 0; j < 3; ++j) s[j] += mi * rq[(3 * k + j) * n + b];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) out[(3 * k + j) * n + a] -= s[j] / adet;
    }
}

}  // namespace mehdg
