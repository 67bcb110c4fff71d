// Residual kernel: R_Q, R_V, R_Vhat and the face entropy production of every
// macro-element (Sec. 4.1 eq. s32a-c; stage time term of eq. C242;
// entropy integrand of Thm. EC_ES).  One workgroup per macro-element.
//
// Phases (all within the workgroup):
//  1. stage v, v_old, vhat in LDS; q from the caller, or the weak gradient
//     of (v, vhat) when q is NULL (R_Q = 0 solved with the 1-D tensor
//     structure of the mass and gradient couplings);
//  2. one thread per volume Gauss point: interpolate (only the 3^3 nodes of
//     the point's sub-element are non-zero), evaluate u(v), F, G, write
//     weighted integrands to the per-macro scratch;
//  3. one thread per face Gauss point: trace fluxes, weighted integrands in
//     LDS, entropy integrand reduced over the workgroup;
//  4. one thread per node / trace node: test the integrands against the
//     basis functions whose support contains the point.
#pragma once
#include "common.hpp"

namespace mehdg {

// volume scratch fields per Gauss point (after the flux phase)
//  [0,5)    alpha_t w (u(v) - u(v_old))_k
//  [5,20)   -(w/h_j) (F_j + G_j)_k      index 5 + 5 j + k
//  [20,35)  w q_kj                      index 20 + 3 k + j
//  [35,50)  (w/h_j) v_k                 index 35 + 5 j + k
constexpr int RES_FIELDS = 50;

// From degree 4 on, q (15 n doubles) and v_old stay out of the LDS (q in the
// per-macro global scratch, v_old read where it is interpolated), so that
// the rest fits: 101 KB at p = 4 against 217 KB with them.
template <int P>
struct ResLds {
    using D = Dims<P>;
    static constexpr bool QG = P >= 4;
    double v[5][D::n];
    double vo[QG ? 1 : 5][D::n];
    double q[QG ? 1 : 15][D::n];
    double vh[6][5][D::nf];
    double fh[6][5][D::S];      // w_s (Fhat + Ghat)_k
    double qh[6][5][D::S];      // w_s sg vhat_k (R_Q trace term)
    double red[256 / 64];
    Tab1D t;
};

// Where the per-point fields live: in the workgroup's LDS behind ResLds when
// they fit (p <= 2: RES_FIELDS x G doubles, 86 KB at p = 2), so that the test
// step reads them at LDS latency; else in the per-macro global scratch.
template <int P>
struct ResScratch {
    static constexpr size_t offset = (sizeof(ResLds<P>) + 15) / 16 * 16;
    static constexpr size_t bytes = (size_t)RES_FIELDS * Dims<P>::G * sizeof(double);
    static constexpr bool in_lds = offset + bytes <= 150 * 1024;
    static constexpr size_t lds_bytes = in_lds ? offset + bytes : sizeof(ResLds<P>);
    // doubles of the global scratch per macro: the fields when they are not
    // in LDS, then q when it is not in LDS
    static constexpr int64_t per_macro =
        (in_lds ? 0 : (int64_t)RES_FIELDS * Dims<P>::G) + (ResLds<P>::QG ? 15 * (int64_t)Dims<P>::n : 0);
    __device__ static double* get(unsigned char* smem, double* scratch, int64_t m) {
        if constexpr (in_lds) return reinterpret_cast<double*>(smem + offset);
        else return scratch + m * per_macro;
    }
    __device__ static double* q(ResLds<P>& L, double* scratch, int64_t m) {
        if constexpr (ResLds<P>::QG) return scratch + m * per_macro + (in_lds ? 0 : (int64_t)RES_FIELDS * Dims<P>::G);
        else return &L.q[0][0];
    }
};

// Pointwise Jacobian coefficients (weights and 1/h of the test derivative
// folded in).  Per volume Gauss point, COEF_V doubles, each a 5x5 [k][l]:
//   [0,25)    (alpha_t + alpha_ps) w A0,          A0 = du/dv
//   [25,100)  -(w/h_i) d(F_i + G_i)/dv,          block i
//   [100,325) -(w/h_i) dG_i/dq_{.j},             block 3 i + j
// Per face Gauss point, COEF_F doubles:
//   [0,25) w dFtot/dv, [25,50) w dFtot/dvhat, [50,125) w dGhat/dq_{.j} (block j),
// with Ftot = Fhat + Ghat the total trace flux.
// Stored coefficient-major, point index fastest: coefV [m][COEF_V][G] and
// coefF [m][COEF_F][6 S] (face points face by face), so that the lanes of a
// wave, which own consecutive points, write and read consecutive addresses.
constexpr int COEF_V = 325;
constexpr int COEF_F = 125;

__device__ __forceinline__ void volume_coefficients(const double vv[5], const double qq[5][3], double w,
                                                    const double hinv[3], const DevParams& pr,
                                                    double* __restrict__ out, int stride) {
    dual<5> vd[5];
#pragma unroll
    for (int l = 0; l < 5; ++l) vd[l] = seed_dual<5>(vv[l], l);
    Prim<dual<5>> s;
    primitive(vd, pr.gamma, s);
    {
        dual<5> u[5];
        conservative(s, pr.gamma, u);
        const double c = (pr.alpha_t + pr.alpha_ps) * w;
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int l = 0; l < 5; ++l) out[(5 * k + l) * stride] = c * u[k].d[l];
    }
    // q enters as plain values: G's v-derivative at fixed q
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        dual<5> F[5];
        euler_flux(s, pr.gamma, i, F);
        if (pr.viscous) {
            dual<5> Gv[5];
            viscous_flux(vd, qq, pr, i, Gv);
#pragma unroll
            for (int k = 0; k < 5; ++k) F[k] = F[k] + Gv[k];
        }
        const double c = -w * hinv[i];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int l = 0; l < 5; ++l) out[(25 + 25 * i + 5 * k + l) * stride] = c * F[k].d[l];
    }
    // G is linear in q: its q-derivative columns are G evaluated at unit q.
    for (int i = 0; i < 3; ++i) {
        const double c = -w * hinv[i];
        for (int l = 0; l < 5; ++l)
            for (int j = 0; j < 3; ++j) {
                double Gv[5] = {0, 0, 0, 0, 0};
                if (pr.viscous) {
                    double qu[5][3];
#pragma unroll
                    for (int a = 0; a < 5; ++a) qu[a][0] = qu[a][1] = qu[a][2] = 0.0;
                    qu[l][j] = 1.0;
                    viscous_flux(vv, qu, pr, i, Gv);
                }
#pragma unroll
                for (int k = 0; k < 5; ++k) out[(100 + 25 * (3 * i + j) + 5 * k + l) * stride] = c * Gv[k];
            }
    }
}

__device__ __forceinline__ void face_coefficients(const double vh[5], const double vv[5], const double qq[5][3],
                                                  double ws, const DevParams& pr, int d, double sg,
                                                  double* __restrict__ out, int stride) {
    // derivatives of the inviscid trace flux in v (pass 0) and vhat (pass 1)
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        dual<5> a[5], b[5], F[5];
#pragma unroll
        for (int l = 0; l < 5; ++l) {
            a[l] = (pass == 1) ? seed_dual<5>(vh[l], l) : make_dual<5>(vh[l]);
            b[l] = (pass == 0) ? seed_dual<5>(vv[l], l) : make_dual<5>(vv[l]);
        }
        trace_flux(a, b, pr, d, sg, F);
        if (pr.viscous) {
            dual<5> Gh[5];
            viscous_trace_flux(a, b, qq, pr, d, sg, Gh);
#pragma unroll
            for (int k = 0; k < 5; ++k) F[k] = F[k] + Gh[k];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int l = 0; l < 5; ++l) out[(25 * pass + 5 * k + l) * stride] = ws * F[k].d[l];
    }
    // Ghat = sg G_d(vhat, q) - ...: linear in q
    for (int l = 0; l < 5; ++l)
        for (int j = 0; j < 3; ++j) {
            double Gv[5] = {0, 0, 0, 0, 0};
            if (pr.viscous) {
                double qu[5][3];
#pragma unroll
                for (int a = 0; a < 5; ++a) qu[a][0] = qu[a][1] = qu[a][2] = 0.0;
                qu[l][j] = 1.0;
                viscous_flux(vh, qu, pr, d, Gv);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) out[(50 + 25 * j + 5 * k + l) * stride] = ws * sg * Gv[k];
        }
}

// Weak gradient at every node (R_Q = 0): q_kj = (1/h_j)[ -sum_c Lam[b_j,c] v_k(b_j -> c)
//   - Minv[b_j,0] vhat_k(face -j) + Minv[b_j,n1d-1] vhat_k(face +j) ].
template <int P>
__device__ void lift_gradient(ResLds<P>& L, const double hinv[3], double* __restrict__ Q) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d;
    for (int idx = threadIdx.x; idx < 15 * D::n; idx += blockDim.x) {
        const int b = idx % D::n;
        const int kj = idx / D::n;
        const int k = kj / 3, j = kj % 3;
        int bi[3] = {b % n1d, (b / n1d) % n1d, b / (n1d * n1d)};
        const int bj = bi[j];
        const int stride = (j == 0) ? 1 : (j == 1 ? n1d : n1d * n1d);
        const int base = b - bj * stride;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < n1d; ++c) acc -= L.t.Lam[bj][c] * L.v[k][base + c * stride];
        // tangential node index on the two faces normal to j
        const int t1 = (j == 0) ? 1 : 0, t2 = (j == 2) ? 1 : 2;
        const int fc = bi[t1] + n1d * bi[t2];
        acc -= L.t.Minv[bj][0] * L.vh[2 * j][k][fc];
        acc += L.t.Minv[bj][n1d - 1] * L.vh[2 * j + 1][k][fc];
        Q[kj * D::n + b] = acc * hinv[j];
    }
}

// Testing of the integrands against the basis functions (phase 4): volume
// fields of scr (layout above) and face fields fh, qh of the workgroup's LDS
// -> R_q, R_v, R_vh of macro m.  One thread per node, then per trace node.
// The same step closes the linearised products (k_linear.hpp).  On a wall
// face (bc[f] != 0) the trace equations 2..5 test the boundary operator
// vhat_k (+ gT for the energy row) instead of the flux: qh holds
// ws sg vhat_k, so ws vhat_k = sg qh.
template <int P>
__device__ __forceinline__ void test_integrands(const ResLds<P>& L, const double* __restrict__ scr, int64_t m,
                                                const uint8_t* __restrict__ bc, const double h[3], double gT,
                                                double* __restrict__ R_q, double* __restrict__ R_v,
                                                double* __restrict__ R_vh) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, n = D::n, nf = D::nf, G = D::G;
    const int tid = threadIdx.x;
    for (int a = tid; a < n; a += blockDim.x) {
        const int a1 = a % n1d, a2 = (a / n1d) % n1d, a3 = a / (n1d * n1d);
        int lo1, hi1, lo2, hi2, lo3, hi3;
        support_1d<P>(a1, lo1, hi1);
        support_1d<P>(a2, lo2, hi2);
        support_1d<P>(a3, lo3, hi3);
        double rv[5] = {0, 0, 0, 0, 0}, rq[5][3];
#pragma unroll
        for (int k = 0; k < 5; ++k) rq[k][0] = rq[k][1] = rq[k][2] = 0.0;
        for (int g3 = lo3 * (P + 1); g3 < (hi3 + 1) * (P + 1); ++g3) {
            const double B3 = L.t.B[g3][a3], D3 = L.t.D[g3][a3];
            for (int g2 = lo2 * (P + 1); g2 < (hi2 + 1) * (P + 1); ++g2) {
                const double B2 = L.t.B[g2][a2], D2 = L.t.D[g2][a2];
                for (int g1 = lo1 * (P + 1); g1 < (hi1 + 1) * (P + 1); ++g1) {
                    const double B1 = L.t.B[g1][a1], D1 = L.t.D[g1][a1];
                    const int g = g1 + nq1 * (g2 + nq1 * g3);
                    const double phi = B1 * B2 * B3;
                    const double dphi[3] = {D1 * B2 * B3, B1 * D2 * B3, B1 * B2 * D3};
#pragma unroll
                    for (int k = 0; k < 5; ++k) {
                        double acc = phi * scr[k * G + g];
#pragma unroll
                        for (int j = 0; j < 3; ++j) acc += dphi[j] * scr[(5 + 5 * j + k) * G + g];
                        rv[k] += acc;
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            rq[k][j] += phi * scr[(20 + 3 * k + j) * G + g] + dphi[j] * scr[(35 + 5 * j + k) * G + g];
                    }
                }
            }
        }
        // trace terms on the faces containing node a
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
                    for (int k = 0; k < 5; ++k) {
                        rv[k] += psi * L.fh[f][k][s];
                        rq[k][d] -= psi * L.qh[f][k][s];
                    }
                }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            R_v[(m * 5 + k) * n + a] = rv[k];
#pragma unroll
            for (int j = 0; j < 3; ++j) R_q[((m * 5 + k) * 3 + j) * n + a] = rq[k][j];
        }
    }
    // ---- phase 4b: test against trace basis functions
    for (int idx = tid; idx < 6 * nf; idx += blockDim.x) {
        const int f = idx / nf, c = idx % nf;
        const int c1 = c % n1d, c2 = c / n1d;
        int l1, u1, l2, u2;
        support_1d<P>(c1, l1, u1);
        support_1d<P>(c2, l2, u2);
        double acc[5] = {0, 0, 0, 0, 0};
        if (bc && bc[f]) {
            const double sg = face_sign(f), hh = h[face_t1(f)] * h[face_t2(f)];
            for (int s2 = l2 * (P + 1); s2 < (u2 + 1) * (P + 1); ++s2)
                for (int s1 = l1 * (P + 1); s1 < (u1 + 1) * (P + 1); ++s1) {
                    const int s = s1 + nq1 * s2;
                    const double psi = L.t.B[s1][c1] * L.t.B[s2][c2];
                    acc[0] += psi * L.fh[f][0][s];
#pragma unroll
                    for (int k = 1; k < 5; ++k) acc[k] += psi * sg * L.qh[f][k][s];
                    acc[4] += psi * hh * L.t.w[s1] * L.t.w[s2] * gT;
                }
        } else {
            for (int s2 = l2 * (P + 1); s2 < (u2 + 1) * (P + 1); ++s2)
                for (int s1 = l1 * (P + 1); s1 < (u1 + 1) * (P + 1); ++s1) {
                    const int s = s1 + nq1 * s2;
                    const double psi = L.t.B[s1][c1] * L.t.B[s2][c2];
#pragma unroll
                    for (int k = 0; k < 5; ++k) acc[k] += psi * L.fh[f][k][s];
                }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) R_vh[((m * 6 + f) * 5 + k) * nf + c] = acc[k];
    }
}

// The residual (and with JAC the pointwise Jacobian coefficients) of macro m
// by the whole workgroup, smem_raw the workgroup's dynamic LDS (ResScratch<P>::
// lds_bytes).  Shared by the per-degree kernel and the batch's persistent one.
template <int P, bool JAC>
__device__ __forceinline__ void residual_macro(int64_t m, unsigned char* smem_raw, const double* __restrict__ v,
                                               const double* __restrict__ vhat, const double* __restrict__ q,
                                               const double* __restrict__ v_old, const double* __restrict__ hs,
                                               const DevParams& pr, const Tab1D* __restrict__ tab,
                                               double* __restrict__ R_q, double* __restrict__ R_v,
                                               double* __restrict__ R_vh, double* __restrict__ entropy,
                                               double* __restrict__ scratch, double* __restrict__ coefV,
                                               double* __restrict__ coefF, const uint8_t* __restrict__ face_bc,
                                               int32_t* __restrict__ status) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, n = D::n, nf = D::nf, G = D::G, S = D::S;
    ResLds<P>& L = *reinterpret_cast<ResLds<P>*>(smem_raw);
    const int tid = threadIdx.x;

    // ---- phase 1: stage inputs
    {
        const double* src = reinterpret_cast<const double*>(tab);
        double* dst = reinterpret_cast<double*>(&L.t);
        for (int i = tid; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
    }
    constexpr bool QG = ResLds<P>::QG;
    for (int i = tid; i < 5 * n; i += blockDim.x) {
        (&L.v[0][0])[i] = v[m * 5 * n + i];
        if constexpr (!QG) (&L.vo[0][0])[i] = v_old[m * 5 * n + i];
    }
    for (int i = tid; i < 30 * nf; i += blockDim.x) (&L.vh[0][0][0])[i] = vhat[m * 30 * nf + i];
    double* __restrict__ Q = ResScratch<P>::q(L, scratch, m);
    const double* __restrict__ vold_m = v_old + m * 5 * n;
    const double h[3] = {hs[3 * m], hs[3 * m + 1], hs[3 * m + 2]};
    const double hinv[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
    const double vol = h[0] * h[1] * h[2];
    __syncthreads();
    if (q) {
        for (int i = tid; i < 15 * n; i += blockDim.x) Q[i] = q[m * 15 * n + i];
    } else {
        lift_gradient<P>(L, hinv, Q);
    }
    __syncthreads();

    bool bad_phys = false, bad_fin = false;
    double* scr = ResScratch<P>::get(smem_raw, scratch, m);

    // ---- phase 2: volume Gauss points
    for (int g = tid; g < G; g += blockDim.x) {
        const int g1 = g % nq1, g2 = (g / nq1) % nq1, g3 = g / (nq1 * nq1);
        const int e1 = g1 / (P + 1), e2 = g2 / (P + 1), e3 = g3 / (P + 1);
        double vv[5] = {0, 0, 0, 0, 0}, vo[5] = {0, 0, 0, 0, 0}, qq[5][3];
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
                        if constexpr (QG) vo[k] += phi * vold_m[k * n + a];
                        else vo[k] += phi * L.vo[k][a];
#pragma unroll
                        for (int j = 0; j < 3; ++j) qq[k][j] += phi * Q[(3 * k + j) * n + a];
                    }
                }
            }
        }
        const double w = vol * L.t.w[g1] * L.t.w[g2] * L.t.w[g3];
        Prim<double> s, so;
        primitive(vv, pr.gamma, s);
        primitive(vo, pr.gamma, so);
        if (!(vv[4] < 0.0) || !(s.rho > 0.0)) bad_phys = true;
        double u[5], uo[5];
        conservative(s, pr.gamma, u);
        conservative(so, pr.gamma, uo);
#pragma unroll
        for (int k = 0; k < 5; ++k) scr[k * G + g] = pr.alpha_t * w * (u[k] - uo[k]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double F[5];
            euler_flux(s, pr.gamma, j, F);
            if (pr.viscous) {
                double Gv[5];
                viscous_flux(vv, qq, pr, j, Gv);
#pragma unroll
                for (int k = 0; k < 5; ++k) F[k] += Gv[k];
            }
            const double c = -w * hinv[j];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                scr[(5 + 5 * j + k) * G + g] = c * F[k];
                if (!finite(F[k])) bad_fin = true;
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                scr[(20 + 3 * k + j) * G + g] = w * qq[k][j];
                scr[(35 + 5 * j + k) * G + g] = w * hinv[j] * vv[k];
            }
        if constexpr (JAC) volume_coefficients(vv, qq, w, hinv, pr, coefV + (int64_t)m * G * COEF_V + g, G);
    }

    // ---- phase 3: face Gauss points
    double ent = 0.0;
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
                    for (int j = 0; j < 3; ++j) qq[k][j] += psi * Q[(3 * k + j) * n + a];
                }
            }
        }
        const double ws = h[t1] * h[t2] * L.t.w[s1] * L.t.w[s2];
        double Fh[5];
        trace_flux(vh, vv, pr, d, sg, Fh);
        // entropy integrand [[v]]^T Fhat - [[Psi_n]], Psi = rho V (eq. poen)
        {
            Prim<double> a, b;
            primitive(vh, pr.gamma, a);
            primitive(vv, pr.gamma, b);
            if (!(vh[4] < 0.0) || !(a.rho > 0.0)) bad_phys = true;
            double e = 0.0;
#pragma unroll
            for (int k = 0; k < 5; ++k) e += (vh[k] - vv[k]) * Fh[k];
            e -= sg * (a.rho * a.V[d] - b.rho * b.V[d]);
            ent += ws * e;
        }
        if (pr.viscous) {
            double Gh[5];
            viscous_trace_flux(vh, vv, qq, pr, d, sg, Gh);
#pragma unroll
            for (int k = 0; k < 5; ++k) Fh[k] += Gh[k];
        }
        if constexpr (JAC)
            face_coefficients(vh, vv, qq, ws, pr, d, sg, coefF + (int64_t)m * 6 * S * COEF_F + idx, 6 * S);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            L.fh[f][k][s] = ws * Fh[k];
            L.qh[f][k][s] = ws * sg * vh[k];
            if (!finite(Fh[k])) bad_fin = true;
        }
    }
    // block reduction of the entropy production
    for (int off = 32; off > 0; off >>= 1) ent += __shfl_down(ent, off, 64);
    if ((tid & 63) == 0) L.red[tid >> 6] = ent;
    __syncthreads();
    if (tid == 0) {
        double e = 0.0;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) e += L.red[i];
        entropy[m] = e;
    }

    // ---- phase 4: test against the volume and trace basis functions
    test_integrands<P>(L, scr, m, face_bc ? face_bc + m * 6 : nullptr, h, pr.gT, R_q, R_v, R_vh);
    if (bad_phys) record_status(status, m, ST_NONPHYSICAL);
    else if (bad_fin) record_status(status, m, ST_NONFINITE);
}

template <int P, bool JAC>
__global__ void __launch_bounds__(256) k_residual(const double* __restrict__ v, const double* __restrict__ vhat,
                                                  const double* __restrict__ q, const double* __restrict__ v_old,
                                                  const double* __restrict__ hs, DevParams pr,
                                                  const Tab1D* __restrict__ tab, double* __restrict__ R_q,
                                                  double* __restrict__ R_v, double* __restrict__ R_vh,
                                                  double* __restrict__ entropy, double* __restrict__ scratch,
                                                  double* __restrict__ coefV, double* __restrict__ coefF,
                                                  const uint8_t* __restrict__ face_bc, int32_t* __restrict__ status) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    residual_macro<P, JAC>(blockIdx.x, smem_raw, v, vhat, q, v_old, hs, pr, tab, R_q, R_v, R_vh, entropy, scratch,
                           coefV, coefF, face_bc, status);
}

}  // namespace mehdg
