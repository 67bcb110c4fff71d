// Linearised residual: Jacobian-vector (JVP) and vector-Jacobian (VJP)
// products at the state of the last assemble that stored the pointwise
// Jacobian coefficients (coefV, coefF; layouts in k_residual.hpp).
//
// The residual of Sec. 4.1 (eq. s32a-c, time term of eq. C242) is, per
// macro, quadrature of pointwise integrands tested against the basis.  Its
// derivative in a direction (dq, dv, dvhat) is the same quadrature of the
// linearised integrands: the pointwise 5x5 coefficient blocks applied to
// the direction interpolated at the Gauss points.  So the JVP runs the
// residual kernel's interpolate -> pointwise -> test structure with the
// coefficient products in place of the physics, and writes the same
// scratch and LDS fields, which test_integrands closes.  The VJP is its
// transpose: the adjoint is interpolated with the test functions, the
// transposed blocks are applied pointwise, and the result is tested with
// the trial functions.  R_Q (eq. s32a) is linear: its part needs no
// coefficients.  When dq / the q-gradient is omitted, q is the weak gradient
// of (v, vhat) (R_Q = 0), a linear map: the JVP lifts the direction, the
// VJP applies the transposed lift at the end.
//
// One workgroup of 256 threads per macro, LDS ResLds<P>, the residual's
// per-point fields reused (in LDS for p <= 2, see ResScratch).
#pragma once
#include "k_residual.hpp"

namespace mehdg {

// VJP scratch per macro: the volume adjoint sources [20][G] (5 for v, 15 for q)
// followed by the face q-sources [15][6 S].
template <int P>
struct VjpScratch {
    static constexpr int G = Dims<P>::G, S = Dims<P>::S;
    static constexpr int FACE_Q = 20 * G;
    static constexpr int total = 20 * G + 15 * 6 * S;
    static_assert(total <= RES_FIELDS * G, "VJP sources exceed the residual scratch");
};

template <int P>
__device__ __forceinline__ void stage_common(ResLds<P>& L, const Tab1D* __restrict__ tab) {
    const double* src = reinterpret_cast<const double*>(tab);
    double* dst = reinterpret_cast<double*>(&L.t);
    for (int i = threadIdx.x; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
}

template <int P>
__global__ void __launch_bounds__(256) k_jvp(const double* __restrict__ dv, const double* __restrict__ dvh,
                                             const double* __restrict__ dq, const double* __restrict__ hs,
                                             const Tab1D* __restrict__ tab, const double* __restrict__ coefV,
                                             const double* __restrict__ coefF, int viscous,
                                             const uint8_t* __restrict__ face_bc, double* __restrict__ J_q,
                                             double* __restrict__ J_v, double* __restrict__ J_vh,
                                             double* __restrict__ scratch) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, n = D::n, nf = D::nf, G = D::G, S = D::S;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ResLds<P>& L = *reinterpret_cast<ResLds<P>*>(smem_raw);
    const int64_t m = blockIdx.x;
    const int tid = threadIdx.x;

    static_assert(!ResLds<P>::QG, "the linearised products keep q in LDS (degrees 1..3)");
    stage_common<P>(L, tab);
    for (int i = tid; i < 5 * n; i += blockDim.x) (&L.v[0][0])[i] = dv[m * 5 * n + i];
    for (int i = tid; i < 30 * nf; i += blockDim.x) (&L.vh[0][0][0])[i] = dvh[m * 30 * nf + i];
    const double h[3] = {hs[3 * m], hs[3 * m + 1], hs[3 * m + 2]};
    const double hinv[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
    const double vol = h[0] * h[1] * h[2];
    __syncthreads();
    if (dq) {
        for (int i = tid; i < 15 * n; i += blockDim.x) (&L.q[0][0])[i] = dq[m * 15 * n + i];
    } else {
        lift_gradient<P>(L, hinv, &L.q[0][0]);
    }
    __syncthreads();
    double* scr = ResScratch<P>::get(smem_raw, scratch, m);

    // volume Gauss points: linearised integrands
    for (int g = tid; g < G; g += blockDim.x) {
        const int g1 = g % nq1, g2 = (g / nq1) % nq1, g3 = g / (nq1 * nq1);
        const int e1 = g1 / (P + 1), e2 = g2 / (P + 1), e3 = g3 / (P + 1);
        double vv[5] = {0, 0, 0, 0, 0}, qq[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k) qq[k][0] = qq[k][1] = qq[k][2] = 0.0;
        for (int c = 0; c <= P; ++c) {
            const int a3 = e3 * P + c;
            const double b3 = L.t.B[g3][a3];
            for (int bb = 0; bb <= P; ++bb) {
                const int a2 = e2 * P + bb;
                const double b23 = b3 * L.t.B[g2][a2];
                for (int aa = 0; aa <= P; ++aa) {
                    const int a1 = e1 * P + aa;
                    const double phi = b23 * L.t.B[g1][a1];
                    const int a = a1 + n1d * (a2 + n1d * a3);
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        vv[k] += phi * L.v[k][a];
#pragma unroll
                        for (int j = 0; j < 3; ++j) qq[k][j] += phi * L.q[3 * k + j][a];
                    }
                }
            }
        }
        const double w = vol * L.t.w[g1] * L.t.w[g2] * L.t.w[g3];
        const double* cv = coefV + (int64_t)m * G * COEF_V + g;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < 5; ++l) acc += cv[(5 * k + l) * G] * vv[l];
            scr[k * G + g] = acc;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < 5; ++l) acc += cv[(25 + 25 * i + 5 * k + l) * G] * vv[l];
                if (viscous) {
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int l = 0; l < 5; ++l) acc += cv[(100 + 25 * (3 * i + j) + 5 * k + l) * G] * qq[l][j];
                }
                scr[(5 + 5 * i + k) * G + g] = acc;
            }
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                scr[(20 + 3 * k + j) * G + g] = w * qq[k][j];
                scr[(35 + 5 * j + k) * G + g] = w * hinv[j] * vv[k];
            }
    }

    // face Gauss points: linearised total trace flux
    for (int idx = tid; idx < 6 * S; idx += blockDim.x) {
        const int f = idx / S, s = idx % S;
        const int d = face_axis(f), t1 = face_t1(f), t2 = face_t2(f);
        const double sg = face_sign(f);
        const int s1 = s % nq1, s2 = s / nq1;
        const int e1 = s1 / (P + 1), e2 = s2 / (P + 1);
        const int ad = face_side(f) ? (n1d - 1) : 0;
        double vv[5] = {0, 0, 0, 0, 0}, vh[5] = {0, 0, 0, 0, 0}, qq[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k) qq[k][0] = qq[k][1] = qq[k][2] = 0.0;
        for (int cc = 0; cc <= P; ++cc) {
            const int c2 = e2 * P + cc;
            const double bq2 = L.t.B[s2][c2];
            for (int bb = 0; bb <= P; ++bb) {
                const int c1 = e1 * P + bb;
                const double psi = bq2 * L.t.B[s1][c1];
                int ai[3];
                ai[d] = ad;
                ai[t1] = c1;
                ai[t2] = c2;
                const int a = ai[0] + n1d * (ai[1] + n1d * ai[2]);
                const int fc = c1 + n1d * c2;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    vv[k] += psi * L.v[k][a];
                    vh[k] += psi * L.vh[f][k][fc];
#pragma unroll
                    for (int j = 0; j < 3; ++j) qq[k][j] += psi * L.q[3 * k + j][a];
                }
            }
        }
        const double ws = h[t1] * h[t2] * L.t.w[s1] * L.t.w[s2];
        const double* cf = coefF + (int64_t)m * 6 * S * COEF_F + idx;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < 5; ++l)
                acc += cf[(5 * k + l) * (6 * S)] * vv[l] + cf[(25 + 5 * k + l) * (6 * S)] * vh[l];
            if (viscous) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int l = 0; l < 5; ++l) acc += cf[(50 + 25 * j + 5 * k + l) * (6 * S)] * qq[l][j];
            }
            L.fh[f][k][s] = acc;
            L.qh[f][k][s] = ws * sg * vh[k];
        }
    }
    __syncthreads();
    // the wall rows are linear in vhat: no constant term in the derivative
    test_integrands<P>(L, scr, m, face_bc ? face_bc + m * 6 : nullptr, h, 0.0, J_q, J_v, J_vh);
}

// VJP.  With g_q given (then w_q too): the gradient of
// w_q.R_Q + w_v.R_V + w_vhat.R_Vhat in (q, v, vhat).  With g_q NULL (w_q
// NULL): the gradient of w_v.R_V + w_vhat.R_Vhat in (v, vhat) with q the
// weak gradient of (v, vhat).
template <int P>
__global__ void __launch_bounds__(256) k_vjp(const double* __restrict__ wq, const double* __restrict__ wv,
                                             const double* __restrict__ wvh, const double* __restrict__ hs,
                                             const Tab1D* __restrict__ tab, const double* __restrict__ coefV,
                                             const double* __restrict__ coefF, int viscous,
                                             const uint8_t* __restrict__ face_bc, double* __restrict__ g_q,
                                             double* __restrict__ g_v, double* __restrict__ g_vh,
                                             double* __restrict__ scratch) {
    using D = Dims<P>;
    using VS = VjpScratch<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, n = D::n, nf = D::nf, G = D::G, S = D::S;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ResLds<P>& L = *reinterpret_cast<ResLds<P>*>(smem_raw);
    const int64_t m = blockIdx.x;
    const int tid = threadIdx.x;
    const bool full = g_q != nullptr;

    static_assert(!ResLds<P>::QG, "the linearised products keep q in LDS (degrees 1..3)");
    stage_common<P>(L, tab);
    for (int i = tid; i < 5 * n; i += blockDim.x) (&L.v[0][0])[i] = wv[m * 5 * n + i];
    for (int i = tid; i < 30 * nf; i += blockDim.x) (&L.vh[0][0][0])[i] = wvh[m * 30 * nf + i];
    if (full)
        for (int i = tid; i < 15 * n; i += blockDim.x) (&L.q[0][0])[i] = wq[m * 15 * n + i];
    const double h[3] = {hs[3 * m], hs[3 * m + 1], hs[3 * m + 2]};
    const double hinv[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
    const double vol = h[0] * h[1] * h[2];
    __syncthreads();
    double* scr = ResScratch<P>::get(smem_raw, scratch, m);

    // volume Gauss points: adjoint sources for v (5) and q (15)
    for (int g = tid; g < G; g += blockDim.x) {
        const int g1 = g % nq1, g2 = (g / nq1) % nq1, g3 = g / (nq1 * nq1);
        const int e1 = g1 / (P + 1), e2 = g2 / (P + 1), e3 = g3 / (P + 1);
        // mu0 = sum_a phi_a w_v, mu[i] = sum_a d_i phi_a w_v; nu, xi the same for w_q
        double mu0[5] = {0, 0, 0, 0, 0}, mu[3][5], nu[5][3], xi[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) mu[j][k] = nu[k][j] = xi[k][j] = 0.0;
        for (int c = 0; c <= P; ++c) {
            const int a3 = e3 * P + c;
            const double B3 = L.t.B[g3][a3], D3 = L.t.D[g3][a3];
            for (int bb = 0; bb <= P; ++bb) {
                const int a2 = e2 * P + bb;
                const double B2 = L.t.B[g2][a2], D2 = L.t.D[g2][a2];
                for (int aa = 0; aa <= P; ++aa) {
                    const int a1 = e1 * P + aa;
                    const double B1 = L.t.B[g1][a1], D1 = L.t.D[g1][a1];
                    const int a = a1 + n1d * (a2 + n1d * a3);
                    const double phi = B1 * B2 * B3;
                    const double dphi[3] = {D1 * B2 * B3, B1 * D2 * B3, B1 * B2 * D3};
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        const double x = L.v[k][a];
                        mu0[k] += phi * x;
#pragma unroll
                        for (int i = 0; i < 3; ++i) mu[i][k] += dphi[i] * x;
                    }
                    if (full) {
#pragma unroll
                        for (int k = 0; k < 5; ++k)
#pragma unroll
                            for (int j = 0; j < 3; ++j) {
                                const double y = L.q[3 * k + j][a];
                                nu[k][j] += phi * y;
                                xi[k][j] += dphi[j] * y;
                            }
                    }
                }
            }
        }
        const double w = vol * L.t.w[g1] * L.t.w[g2] * L.t.w[g3];
        const double* cv = coefV + (int64_t)m * G * COEF_V + g;
#pragma unroll
        for (int l = 0; l < 5; ++l) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                acc += cv[(5 * k + l) * G] * mu0[k];
#pragma unroll
                for (int i = 0; i < 3; ++i) acc += cv[(25 + 25 * i + 5 * k + l) * G] * mu[i][k];
            }
            if (full) {
#pragma unroll
                for (int j = 0; j < 3; ++j) acc += w * hinv[j] * xi[l][j];
            }
            scr[l * G + g] = acc;
        }
#pragma unroll
        for (int l = 0; l < 5; ++l)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double acc = full ? w * nu[l][j] : 0.0;
                if (viscous) {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int k = 0; k < 5; ++k) acc += cv[(100 + 25 * (3 * i + j) + 5 * k + l) * G] * mu[i][k];
                }
                scr[(5 + 3 * l + j) * G + g] = acc;
            }
    }

    // face Gauss points: rho = trace of w_v + w_vhat (on a wall face only the
    // mass row of w_vhat: rows 2..5 there are vhat_k, whose adjoint rw goes
    // straight to vhat), tau = trace of the normal component of w_q; sources
    // for v (fh), vhat (qh) and q (scratch)
    const uint8_t* bcm = face_bc ? face_bc + m * 6 : nullptr;
    for (int idx = tid; idx < 6 * S; idx += blockDim.x) {
        const int f = idx / S, s = idx % S;
        const int d = face_axis(f), t1 = face_t1(f), t2 = face_t2(f);
        const double sg = face_sign(f);
        const bool wall = bcm && bcm[f];
        const int s1 = s % nq1, s2 = s / nq1;
        const int e1 = s1 / (P + 1), e2 = s2 / (P + 1);
        const int ad = face_side(f) ? (n1d - 1) : 0;
        double rho[5] = {0, 0, 0, 0, 0}, tau[5] = {0, 0, 0, 0, 0}, rw[5] = {0, 0, 0, 0, 0};
        for (int cc = 0; cc <= P; ++cc) {
            const int c2 = e2 * P + cc;
            const double bq2 = L.t.B[s2][c2];
            for (int bb = 0; bb <= P; ++bb) {
                const int c1 = e1 * P + bb;
                const double psi = bq2 * L.t.B[s1][c1];
                int ai[3];
                ai[d] = ad;
                ai[t1] = c1;
                ai[t2] = c2;
                const int a = ai[0] + n1d * (ai[1] + n1d * ai[2]);
                const int fc = c1 + n1d * c2;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const double wh = psi * L.vh[f][k][fc];
                    rho[k] += psi * L.v[k][a];
                    if (wall && k > 0) rw[k] += wh;
                    else rho[k] += wh;
                    if (full) tau[k] += psi * L.q[3 * k + d][a];
                }
            }
        }
        const double ws = h[t1] * h[t2] * L.t.w[s1] * L.t.w[s2];
        const double* cf = coefF + (int64_t)m * 6 * S * COEF_F + idx;
#pragma unroll
        for (int l = 0; l < 5; ++l) {
            double av = 0.0, ah = 0.0;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                av += cf[(5 * k + l) * (6 * S)] * rho[k];
                ah += cf[(25 + 5 * k + l) * (6 * S)] * rho[k];
            }
            L.fh[f][l][s] = av;
            L.qh[f][l][s] = ah - ws * sg * tau[l] + ws * rw[l];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double aq = 0.0;
                if (viscous) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) aq += cf[(50 + 25 * j + 5 * k + l) * (6 * S)] * rho[k];
                }
                scr[VS::FACE_Q + (3 * l + j) * 6 * S + idx] = aq;
            }
        }
    }
    __syncthreads();

    // nodes: test the sources with the trial functions
    for (int a = tid; a < n; a += blockDim.x) {
        const int a1 = a % n1d, a2 = (a / n1d) % n1d, a3 = a / (n1d * n1d);
        int lo1, hi1, lo2, hi2, lo3, hi3;
        support_1d<P>(a1, lo1, hi1);
        support_1d<P>(a2, lo2, hi2);
        support_1d<P>(a3, lo3, hi3);
        double gv[5] = {0, 0, 0, 0, 0}, gq[15];
#pragma unroll
        for (int i = 0; i < 15; ++i) gq[i] = 0.0;
        for (int g3 = lo3 * (P + 1); g3 < (hi3 + 1) * (P + 1); ++g3) {
            const double B3 = L.t.B[g3][a3];
            for (int g2 = lo2 * (P + 1); g2 < (hi2 + 1) * (P + 1); ++g2) {
                const double B23 = B3 * L.t.B[g2][a2];
                for (int g1 = lo1 * (P + 1); g1 < (hi1 + 1) * (P + 1); ++g1) {
                    const int g = g1 + nq1 * (g2 + nq1 * g3);
                    const double phi = B23 * L.t.B[g1][a1];
#pragma unroll
                    for (int k = 0; k < 5; ++k) gv[k] += phi * scr[k * G + g];
#pragma unroll
                    for (int i = 0; i < 15; ++i) gq[i] += phi * scr[(5 + i) * G + g];
                }
            }
        }
        const int ai[3] = {a1, a2, a3};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int d = face_axis(f);
            if (ai[d] != (face_side(f) ? n1d - 1 : 0)) continue;
            const int c1 = ai[face_t1(f)], c2 = ai[face_t2(f)];
            int l1, u1, l2, u2;
            support_1d<P>(c1, l1, u1);
            support_1d<P>(c2, l2, u2);
            for (int s2 = l2 * (P + 1); s2 < (u2 + 1) * (P + 1); ++s2)
                for (int s1 = l1 * (P + 1); s1 < (u1 + 1) * (P + 1); ++s1) {
                    const int s = s1 + nq1 * s2;
                    const double psi = L.t.B[s1][c1] * L.t.B[s2][c2];
#pragma unroll
                    for (int k = 0; k < 5; ++k) gv[k] += psi * L.fh[f][k][s];
#pragma unroll
                    for (int i = 0; i < 15; ++i) gq[i] += psi * scr[VS::FACE_Q + i * 6 * S + f * S + s];
                }
        }
        if (full) {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                g_v[(m * 5 + k) * n + a] = gv[k];
#pragma unroll
                for (int j = 0; j < 3; ++j) g_q[((m * 5 + k) * 3 + j) * n + a] = gq[3 * k + j];
            }
        } else {
            // keep for the transposed weak gradient (w_v and w_q are no longer read)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                L.v[k][a] = gv[k];
#pragma unroll
                for (int j = 0; j < 3; ++j) L.q[3 * k + j][a] = gq[3 * k + j];
            }
        }
    }
    // trace nodes
    for (int idx = tid; idx < 6 * nf; idx += blockDim.x) {
        const int f = idx / nf, c = idx % nf;
        const int c1 = c % n1d, c2 = c / n1d;
        int l1, u1, l2, u2;
        support_1d<P>(c1, l1, u1);
        support_1d<P>(c2, l2, u2);
        double acc[5] = {0, 0, 0, 0, 0};
        for (int s2 = l2 * (P + 1); s2 < (u2 + 1) * (P + 1); ++s2)
            for (int s1 = l1 * (P + 1); s1 < (u1 + 1) * (P + 1); ++s1) {
                const int s = s1 + nq1 * s2;
                const double psi = L.t.B[s1][c1] * L.t.B[s2][c2];
#pragma unroll
                for (int k = 0; k < 5; ++k) acc[k] += psi * L.qh[f][k][s];
            }
        if (full) {
#pragma unroll
            for (int k = 0; k < 5; ++k) g_vh[((m * 6 + f) * 5 + k) * nf + c] = acc[k];
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) L.vh[f][k][c] = acc[k];
        }
    }
    if (full) return;
    __syncthreads();

    // transposed weak gradient: q_kj(b) = (1/h_j)[ -sum_c Lam[b_j][c] v_k(b: b_j -> c)
    //   - Minv[b_j][0] vhat_k(face 2j) + Minv[b_j][n1d-1] vhat_k(face 2j+1) ]
    for (int idx = tid; idx < 5 * n; idx += blockDim.x) {
        const int k = idx / n, a = idx % n;
        const int ai[3] = {a % n1d, (a / n1d) % n1d, a / (n1d * n1d)};
        double acc = L.v[k][a];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int stride = (j == 0) ? 1 : (j == 1 ? n1d : n1d * n1d);
            const int base = a - ai[j] * stride;
            double s = 0.0;
            for (int bj = 0; bj < n1d; ++bj) s += L.t.Lam[bj][ai[j]] * L.q[3 * k + j][base + bj * stride];
            acc -= hinv[j] * s;
        }
        g_v[(m * 5 + k) * n + a] = acc;
    }
    for (int idx = tid; idx < 30 * nf; idx += blockDim.x) {
        const int f = idx / (5 * nf), k = (idx / nf) % 5, c = idx % nf;
        const int j = face_axis(f);
        const int t1 = (j == 0) ? 1 : 0, t2 = (j == 2) ? 1 : 2;
        int bi[3];
        bi[t1] = c % n1d;
        bi[t2] = c / n1d;
        const int stride = (j == 0) ? 1 : (j == 1 ? n1d : n1d * n1d);
        bi[j] = 0;
        const int base = bi[0] + n1d * (bi[1] + n1d * bi[2]);
        double s = 0.0;
        if (face_side(f)) {
            for (int bj = 0; bj < n1d; ++bj) s += L.t.Minv[bj][n1d - 1] * L.q[3 * k + j][base + bj * stride];
        } else {
            for (int bj = 0; bj < n1d; ++bj) s -= L.t.Minv[bj][0] * L.q[3 * k + j][base + bj * stride];
        }
        g_vh[((m * 6 + f) * 5 + k) * nf + c] = L.vh[f][k][c] + hinv[j] * s;
    }
}

}  // namespace mehdg
