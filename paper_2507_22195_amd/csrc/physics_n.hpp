// Trace fluxes for a general unit normal n, device side (faces of
// tetrahedral macro-elements).  The same fluxes as physics.hpp, whose
// versions take an axis-aligned normal n = sg e_d; here n is any unit
// vector and (t1, t2) two unit tangents completing it to an orthonormal
// frame.  The dissipation operators depend on the tangents only through
// t1 t1^T + t2 t2^T, the projector onto the face, so any such pair gives
// the same flux.
#pragma once
#include "physics.hpp"

// Two unit tangents: t1 = n x e / |n x e| with e the axis of the smallest
// |n_i|, t2 = n x t1.
MEHDG_HD void face_frame(const double n[3], double t1[3], double t2[3]) {
    int a = 0;
    if (fabs(n[1]) < fabs(n[a])) a = 1;
    if (fabs(n[2]) < fabs(n[a])) a = 2;
    double e[3] = {0.0, 0.0, 0.0};
    e[a] = 1.0;
    t1[0] = n[1] * e[2] - n[2] * e[1];
    t1[1] = n[2] * e[0] - n[0] * e[2];
    t1[2] = n[0] * e[1] - n[1] * e[0];
    const double il = 1.0 / sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    t1[0] *= il;
    t1[1] *= il;
    t1[2] *= il;
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

template <typename T>
MEHDG_HD T dot3(const T a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// F.n = (rho Vn, rho Vn V + P n, Vn (rho E + P))   (eq. C5)
template <typename T>
MEHDG_HD void euler_flux_n(const Prim<T>& s, double g, const double n[3], T F[5]) {
    const T vn = dot3(s.V, n);
    const T m = s.rho * vn;
    const T H = s.P * (g / (g - 1.0)) + 0.5 * s.rho * kinetic2(s);
    F[0] = m;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[1 + i] = m * s.V[i] + s.P * n[i];
    F[4] = vn * H;
}

// Entropy-conservative KEP flux (eq. EC) along n.
template <typename T>
MEHDG_HD void ec_flux_n(const Means<T>& m, double g, const double n[3], T F[5]) {
    const T f1 = m.rho_ln * dot3(m.Vb, n);
    T f2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) f2[i] = m.Vb[i] * f1 + m.Pb * n[i];
    F[0] = f1;
    F[1] = f2[0];
    F[2] = f2[1];
    F[3] = f2[2];
    F[4] = (1.0 / (m.beta_ln * (g - 1.0)) - 0.5 * m.V2b) * f1 + m.Vb[0] * f2[0] + m.Vb[1] * f2[1] +
           m.Vb[2] * f2[2];
}

// Adds -1/2 sum_k r_k L_k T_k (r_k . jump) to F with the eigenvector columns
// for the normal n: r1,5 = (1, Vb -/+ c n, h -/+ vn c), r2 = (1, Vb, V2b/2),
// r3,4 = (0, t, Vb.t) for t = t1, t2.
template <typename T>
MEHDG_HD void eigen_dissipation_n(const T Vb[3], const T& c, const T& h, const T& V2b, const double n[3],
                                  const double t1[3], const double t2[3], const T Lw[5], const T jump[5],
                                  T F[5]) {
    const T vn = dot3(Vb, n);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double s = (w == 0) ? -1.0 : 1.0;
        T r[5];
        r[0] = cst<T>::of(1.0);
#pragma unroll
        for (int i = 0; i < 3; ++i) r[1 + i] = Vb[i] + (s * n[i]) * c;
        r[4] = h + s * (vn * c);
        const T proj = r[0] * jump[0] + r[1] * jump[1] + r[2] * jump[2] + r[3] * jump[3] + r[4] * jump[4];
        const T co = 0.5 * (Lw[w == 0 ? 0 : 4] * proj);
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = F[k] - r[k] * co;
    }
    {
        const T proj = jump[0] + Vb[0] * jump[1] + Vb[1] * jump[2] + Vb[2] * jump[3] + 0.5 * V2b * jump[4];
        const T co = 0.5 * (Lw[1] * proj);
        F[0] = F[0] - co;
        F[1] = F[1] - Vb[0] * co;
        F[2] = F[2] - Vb[1] * co;
        F[3] = F[3] - Vb[2] * co;
        F[4] = F[4] - 0.5 * V2b * co;
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double* t = (w == 0) ? t1 : t2;
        const T vt = dot3(Vb, t);
        const T proj = jump[1] * t[0] + jump[2] * t[1] + jump[3] * t[2] + vt * jump[4];
        const T co = 0.5 * (Lw[2 + w] * proj);
#pragma unroll
        for (int i = 0; i < 3; ++i) F[1 + i] = F[1 + i] - t[i] * co;
        F[4] = F[4] - vt * co;
    }
}

// KEPES flux (eq. KEPES1-KEPES5, ES) along n.
template <typename T>
MEHDG_HD void kepes_flux_n(const Prim<T>& sh, const Prim<T>& s, const T jump[5], double g, double eps,
                           const double n[3], const double t1[3], const double t2[3], T F[5]) {
    Means<T> m;
    two_point_means(sh, s, eps, m);
    ec_flux_n(m, g, n, F);
    const T c = dsqrt(g * m.Pb / m.rho_ln);
    const T h = g / (m.beta_ln * (g - 1.0)) + 0.5 * m.V2b;
    const T vn = dot3(m.Vb, n);
    const T theta = dsqrt_abs((s.P - sh.P) / (s.P + sh.P));
    const T lmax = dabs(vn) + c;
    const T ac = dabs(vn + c);
    const T av = dabs(vn);
    const T one_m = 1.0 - theta;
    const T Ta = m.rho_ln * (1.0 / (2.0 * g));
    const T Lw[5] = {(one_m * ac + theta * lmax) * Ta,
                     (one_m * av + theta * lmax) * (m.rho_ln * ((g - 1.0) / g)),
                     (one_m * av + theta * lmax) * m.Pb,
                     (one_m * av + theta * lmax) * m.Pb,
                     (one_m * ac + theta * lmax) * Ta};
    eigen_dissipation_n(m.Vb, c, h, m.V2b, n, t1, t2, Lw, jump, F);
}

// Entropy-stable flux (eq. Flux_En_Inv) along n: central average minus
// 1/2 sigma(vh) A0(vh) [[v]], sigma = |Vh.n| + c_hat.
template <typename T>
MEHDG_HD void es_flux_n(const Prim<T>& sh, const Prim<T>& s, const T jump[5], double g, const double n[3],
                        const double t1[3], const double t2[3], T F[5]) {
    T Fa[5], Fb[5];
    euler_flux_n(sh, g, n, Fa);
    euler_flux_n(s, g, n, Fb);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = 0.5 * (Fa[k] + Fb[k]);
    const T c = dsqrt(g * sh.P / sh.rho);
    const T V2 = kinetic2(sh);
    const T h = sh.P * (g / ((g - 1.0) * sh.rho)) + 0.5 * V2;
    const T sigma = dabs(dot3(sh.V, n)) + c;
    const T Ta = sh.rho * (1.0 / (2.0 * g));
    const T Lw[5] = {sigma * Ta, sigma * (sh.rho * ((g - 1.0) / g)), sigma * sh.P, sigma * sh.P, sigma * Ta};
    eigen_dissipation_n(sh.V, c, h, V2, n, t1, t2, Lw, jump, F);
}

// Inviscid trace flux Fhat(vh, v) along n, selected by pr.flux.
template <typename T>
MEHDG_HD void trace_flux_n(const T vh[5], const T v[5], const DevParams& pr, const double n[3],
                           const double t1[3], const double t2[3], T F[5]) {
    Prim<T> sh, s;
    primitive(vh, pr.gamma, sh);
    primitive(v, pr.gamma, s);
    T jump[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) jump[k] = vh[k] - v[k];
    if (pr.flux == 0) {
        Means<T> m;
        two_point_means(sh, s, pr.eps, m);
        ec_flux_n(m, pr.gamma, n, F);
    } else if (pr.flux == 1) {
        es_flux_n(sh, s, jump, pr.gamma, n, t1, t2, F);
    } else {
        kepes_flux_n(sh, s, jump, pr.gamma, pr.eps, n, t1, t2, F);
    }
}

// Viscous trace flux (eq. Flux_En_Vis) along n: G(vh, q).n - 1/2 sigma_vis [[v]].
template <typename T, typename Q>
MEHDG_HD void viscous_trace_flux_n(const T vh[5], const T v[5], const Q q[5][3], const DevParams& pr,
                                   const double n[3], T F[5]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = -(0.5 * pr.sv[k]) * (vh[k] - v[k]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T G[5];
        viscous_flux(vh, q, pr, d, G);
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = F[k] + n[d] * G[k];
    }
}
