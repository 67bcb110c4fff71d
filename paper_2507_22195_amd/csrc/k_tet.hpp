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
#pragma once
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
    const double *phi, *dphi, *wv, *BiT, *psi, *wf, *Mt, *CT, *ChT, *DT, *DhT;
    const int *vnode, *fnode, *tnode, *vptr, *vinc, *fptr, *finc;
};

template <int P>
struct TetLds {
    using D = TetDims<P>;
    static constexpr int PT = (20 * D::G > 10 * D::FP) ? 20 * D::G : 10 * D::FP;
    static constexpr int SC = (8 * 5 * D::ns > 2 * 80 * D::nfs) ? 8 * 5 * D::ns : 2 * 80 * D::nfs;
    double v[5][D::n], vo[5][D::n], vh[4][5][D::nf], q[15][D::n], rv[5][D::n];
    double pt[PT];
    double sc[SC];
    double red[4];
};

constexpr int TET_THREADS = 256;

template <int P>
__global__ void __launch_bounds__(TET_THREADS)
k_tet_residual(const double* __restrict__ v, const double* __restrict__ vhat, const double* __restrict__ qin,
               const double* __restrict__ v_old, const double* __restrict__ geo, TetDevTab T, DevParams pr,
               const uint8_t* __restrict__ face_bc, double* __restrict__ R_q, double* __restrict__ R_v,
               double* __restrict__ R_vh, double* __restrict__ entropy, int32_t* __restrict__ status) {
    using D = TetDims<P>;
    constexpr int n = D::n, nf = D::nf, ns = D::ns, nfs = D::nfs, Gs = D::Gs, Ss = D::Ss;
    extern __shared__ __align__(16) unsigned char smem[];
    TetLds<P>& L = *reinterpret_cast<TetLds<P>*>(smem);
    const int tid = threadIdx.x;
    const int64_t m = blockIdx.x;
    const double* gm = geo + m * TET_GEO;
    double invJ[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) invJ[i] = gm[i];
    const double adet = gm[9];
    bool bad_phys = false, bad_fin = false;

    // ---- 1. state, weak gradient, R_Q
    for (int i = tid; i < 5 * n; i += TET_THREADS) {
        (&L.v[0][0])[i] = v[m * 5 * n + i];
        (&L.vo[0][0])[i] = v_old[m * 5 * n + i];
    }
    for (int i = tid; i < 20 * nf; i += TET_THREADS) (&L.vh[0][0][0])[i] = vhat[m * 20 * nf + i];
    if (qin)
        for (int i = tid; i < 15 * n; i += TET_THREADS) (&L.q[0][0])[i] = qin[m * 15 * n + i];
    __syncthreads();
    if (!qin) {
        for (int i = tid; i < 5 * n; i += TET_THREADS) {
            const int k = i / n, a = i - k * n;
            double dv[3] = {0.0, 0.0, 0.0};
            for (int b = 0; b < n; ++b) {
                const double x = L.v[k][b];
#pragma unroll
                for (int d = 0; d < 3; ++d) dv[d] += T.DT[(d * n + b) * n + a] * x;
            }
            double qj[3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                qj[j] = -(invJ[0 * 3 + j] * dv[0] + invJ[1 * 3 + j] * dv[1] + invJ[2 * 3 + j] * dv[2]);
            for (int f = 0; f < 4; ++f) {
                double dh = 0.0;
                for (int c = 0; c < nf; ++c) dh += T.DhT[(f * nf + c) * n + a] * L.vh[f][k][c];
                const double s = gm[22 + f] / adet * dh;
#pragma unroll
                for (int j = 0; j < 3; ++j) qj[j] += s * gm[10 + 3 * f + j];
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) L.q[3 * k + j][a] = qj[j];
        }
        __syncthreads();
    }
    for (int i = tid; i < 5 * n; i += TET_THREADS) {
        const int k = i / n, a = i - k * n;
        double mq[3] = {0.0, 0.0, 0.0}, cv[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; ++b) {
            const double mt = T.Mt[b * n + a];
            const double x = L.v[k][b];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                mq[j] += mt * L.q[3 * k + j][b];
                cv[j] += T.CT[(j * n + b) * n + a] * x;
            }
        }
        double r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = adet * (mq[j] + invJ[0 * 3 + j] * cv[0] + invJ[1 * 3 + j] * cv[1] + invJ[2 * 3 + j] * cv[2]);
        for (int f = 0; f < 4; ++f) {
            double ch = 0.0;
            for (int c = 0; c < nf; ++c) ch += T.ChT[(f * nf + c) * n + a] * L.vh[f][k][c];
#pragma unroll
            for (int j = 0; j < 3; ++j) r[j] -= gm[22 + f] * gm[10 + 3 * f + j] * ch;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) R_q[((m * 5 + k) * 3 + j) * n + a] = r[j];
    }

    // ---- 2. volume points
    const double g = pr.gamma;
    for (int gp = tid; gp < D::G; gp += TET_THREADS) {
        const int s = gp / Gs, gl = gp - s * Gs;
        double vv[5] = {0, 0, 0, 0, 0}, vvo[5] = {0, 0, 0, 0, 0}, qq[5][3] = {};
        for (int b = 0; b < ns; ++b) {
            const double ph = T.phi[gl * ns + b];
            const int a = T.vnode[s * ns + b];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                vv[k] += ph * L.v[k][a];
                vvo[k] += ph * L.vo[k][a];
#pragma unroll
                for (int j = 0; j < 3; ++j) qq[k][j] += ph * L.q[3 * k + j][a];
            }
        }
        Prim<double> st, so;
        primitive(vv, g, st);
        primitive(vvo, g, so);
        if (!(vv[4] < 0.0) || !(st.rho > 0.0) || !(vvo[4] < 0.0) || !(so.rho > 0.0)) bad_phys = true;
        double u[5], uo[5];
        conservative(st, g, u);
        conservative(so, g, uo);
        double F[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            euler_flux(st, g, d, F[d]);
            if (pr.viscous) {
                double Gv[5];
                viscous_flux(vv, qq, pr, d, Gv);
#pragma unroll
                for (int k = 0; k < 5; ++k) F[d][k] += Gv[k];
            }
        }
        const double w = T.wv[gl] * adet;
        const double* Bi = T.BiT + s * 9;
        double* o = L.pt + gp * 20;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            o[k] = w * pr.alpha_t * (u[k] - uo[k]);
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
            acc += o[k] * T.phi[gl * ns + b] - o[5 + 3 * k + 0] * T.dphi[(0 * Gs + gl) * ns + b] -
                   o[5 + 3 * k + 1] * T.dphi[(1 * Gs + gl) * ns + b] - o[5 + 3 * k + 2] * T.dphi[(2 * Gs + gl) * ns + b];
        }
        L.sc[i] = acc;
    }
    __syncthreads();
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
        double Fh[5];
        trace_flux_n(vh, vs, pr, nrm, t1, t2, Fh);
        {
            Prim<double> a, b;
            primitive(vh, g, a);
            primitive(vs, g, b);
            if (!(vh[4] < 0.0) || !(a.rho > 0.0)) bad_phys = true;
            double e = 0.0;
#pragma unroll
            for (int k = 0; k < 5; ++k) e += (vh[k] - vs[k]) * Fh[k];
            e -= a.rho * dot3(a.V, nrm) - b.rho * dot3(b.V, nrm);
            ent += ws * e;
        }
        if (pr.viscous) {
            double Gh[5];
            viscous_trace_flux_n(vh, vs, qq, pr, nrm, Gh);
#pragma unroll
            for (int k = 0; k < 5; ++k) Fh[k] += Gh[k];
        }
        double* o = L.pt + fp * 10;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            o[k] = ws * Fh[k];
            o[5 + k] = ws * (vh[k] + (k == 4 ? pr.gT : 0.0));
            if (!isfinite(Fh[k])) bad_fin = true;
        }
    }
    for (int off = 32; off > 0; off >>= 1) ent += __shfl_down(ent, off, 64);
    if ((tid & 63) == 0) L.red[tid >> 6] = ent;
    __syncthreads();
    if (tid == 0) entropy[m] = L.red[0] + L.red[1] + L.red[2] + L.red[3];

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
            R_vh[((m * 4 + f) * 5 + k) * nf + c] = (wall && k > 0) ? accw : acc;
        }
        __syncthreads();
    }
    for (int i = tid; i < 5 * n; i += TET_THREADS) R_v[m * 5 * n + i] = (&L.rv[0][0])[i];

    // ---- status: a flagged macro's outputs are NaN
    const int flag = __syncthreads_or(bad_phys ? 1 : (bad_fin ? 2 : 0));
    if (flag) {
        const int any_phys = __syncthreads_or(bad_phys ? 1 : 0);
        const double nan = __builtin_nan("");
        for (int i = tid; i < 5 * n; i += TET_THREADS) R_v[m * 5 * n + i] = nan;
        for (int i = tid; i < 15 * n; i += TET_THREADS) R_q[m * 15 * n + i] = nan;
        for (int i = tid; i < 20 * nf; i += TET_THREADS) R_vh[m * 20 * nf + i] = nan;
        if (tid == 0) {
            entropy[m] = nan;
            if (status) status[m] = any_phys ? 5 : 6;
        }
    } else if (tid == 0 && status) {
        status[m] = 0;
    }
}

}  // namespace mehdg
