// Pointwise physics of the entropy-variable formulation, device side.
//
// All functions are templates over the scalar T (double or dual<N>) so that
// the same source yields values and exact pointwise Jacobians.  Acoustic
// scaling: rho0 = 1, c0 = 1, gamma P = rho T.  States are entropy variables
// v = [(gamma - s)/(gamma - 1) - beta|V|^2/2, beta V, -beta], beta = rho/P
// (Sec. 2.2 eq. s222).  Trace normals are axis-aligned: n = sg * e_d.
#pragma once
#include "dual.hpp"

struct DevParams {
    double gamma, mu, kappa, lam;
    double sv[5];
    double alpha_t, alpha_ps, eps;
    double gT;             // gamma / T_wall (wall faces)
    int flux, viscous;
};

template <typename T>
struct cst;
template <>
struct cst<double> {
    static MEHDG_HD double of(double x) { return x; }
};
template <int N>
struct cst<dual<N>> {
    static MEHDG_HD dual<N> of(double x) { return make_dual<N>(x); }
};

template <typename T>
struct Prim {
    T rho, V[3], P, beta;
};

// Inverse of eq. (s222).  With beta = -v5 and |beta V|^2 = v2^2 + v3^2 + v4^2:
//   log rho = v1 + |beta V|^2 / (2 beta) - (gamma + log beta) / (gamma - 1),
// which is s = log(P / rho^gamma) solved for rho with P = rho / beta.
template <typename T>
MEHDG_HD void primitive(const T v[5], double g, Prim<T>& s) {
    s.beta = -v[4];
    const T ib = 1.0 / s.beta;
    s.V[0] = v[1] * ib;
    s.V[1] = v[2] * ib;
    s.V[2] = v[3] * ib;
    const T m2 = v[1] * v[1] + v[2] * v[2] + v[3] * v[3];
    s.rho = dexp(v[0] + 0.5 * m2 * ib - (g + dlog(s.beta)) * (1.0 / (g - 1.0)));
    s.P = s.rho * ib;
}

template <typename T>
MEHDG_HD T kinetic2(const Prim<T>& s) {
    return s.V[0] * s.V[0] + s.V[1] * s.V[1] + s.V[2] * s.V[2];
}

// u(v) = (rho, rho V, P/(gamma-1) + rho |V|^2 / 2)   (Sec. 2.1)
template <typename T>
MEHDG_HD void conservative(const Prim<T>& s, double g, T u[5]) {
    u[0] = s.rho;
    u[1] = s.rho * s.V[0];
    u[2] = s.rho * s.V[1];
    u[3] = s.rho * s.V[2];
    u[4] = s.P * (1.0 / (g - 1.0)) + 0.5 * s.rho * kinetic2(s);
}

// F_d = (rho V_d, rho V_d V + P e_d, V_d (rho E + P))   (eq. C5)
template <typename T>
MEHDG_HD void euler_flux(const Prim<T>& s, double g, int d, T F[5]) {
    const T m = s.rho * s.V[d];
    const T H = s.P * (g / (g - 1.0)) + 0.5 * s.rho * kinetic2(s);   // rho E + P
    F[0] = m;
    F[1] = m * s.V[0];
    F[2] = m * s.V[1];
    F[3] = m * s.V[2];
    F[1 + d] = F[1 + d] + s.P;
    F[4] = s.V[d] * H;
}

// Viscous flux G_d(v, q), q[l][j] ~ d v_l / d x_j  (eq. C5, C6).
// Velocity and temperature gradients by the chain rule through
// V_i = -v_{i+1}/v_5 and T = -gamma/v_5.
template <typename T, typename Q>
MEHDG_HD void viscous_flux(const T v[5], const Q q[5][3], const DevParams& pr, int d, T G[5]) {
    const T iv5 = 1.0 / v[4];
    T V[3], dV[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) V[i] = -(v[i + 1] * iv5);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dV[i][j] = -((q[i + 1][j] + V[i] * q[4][j]) * iv5);
    const T div = dV[0][0] + dV[1][1] + dV[2][2];
    T tau[3];   // tau_{i d}
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T t = dV[i][d] + dV[d][i];
        if (i == d) t = t + pr.lam * div;
        tau[i] = pr.mu * t;
    }
    const T dTd = pr.gamma * (q[4][d] * (iv5 * iv5));
    G[0] = cst<T>::of(0.0);
    G[1] = -tau[0];
    G[2] = -tau[1];
    G[3] = -tau[2];
    G[4] = -(tau[0] * V[0] + tau[1] * V[1] + tau[2] * V[2] + pr.kappa * dTd);
}

// Logarithmic mean (a_hat - a)/ln(a_hat/a) (eq. avg).  Near a = a_hat it
// uses the series of atanh(f)/f = ln(a/a_hat)/(2f), f = (a - a_hat)/(a + a_hat),
// truncated after w^3 (w = f^2), when w < eps.
template <typename T>
MEHDG_HD T log_mean(const T& a, const T& ah, double eps) {
    const T f = (a - ah) / (a + ah);
    const T w = f * f;
    T F;
    if (val(w) < eps) {
        F = 1.0 + w * (1.0 / 3.0 + w * (1.0 / 5.0 + w * (1.0 / 7.0)));
    } else {
        F = dlog(a / ah) / (2.0 * f);
    }
    return (a + ah) / (2.0 * F);
}

template <typename T>
struct Means {
    T rho_ln, beta_ln, Vb[3], Pb, V2b;
};

template <typename T>
MEHDG_HD void two_point_means(const Prim<T>& sh, const Prim<T>& s, double eps, Means<T>& m) {
    m.rho_ln = log_mean(s.rho, sh.rho, eps);
    m.beta_ln = log_mean(s.beta, sh.beta, eps);
#pragma unroll
    for (int i = 0; i < 3; ++i) m.Vb[i] = 0.5 * (s.V[i] + sh.V[i]);
    m.Pb = (s.rho + sh.rho) / (s.beta + sh.beta);   // avg(rho) / avg(beta)
    m.V2b = 0.5 * (kinetic2(s) + kinetic2(sh));
}

// Entropy-conservative KEP flux (eq. EC) for n = sg e_d.
template <typename T>
MEHDG_HD void ec_flux(const Means<T>& m, double g, int d, double sg, T F[5]) {
    const T f1 = m.rho_ln * m.Vb[d] * sg;
    T f2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) f2[i] = m.Vb[i] * f1;
    f2[d] = f2[d] + m.Pb * sg;
    F[0] = f1;
    F[1] = f2[0];
    F[2] = f2[1];
    F[3] = f2[2];
    F[4] = (1.0 / (m.beta_ln * (g - 1.0)) - 0.5 * m.V2b) * f1 + m.Vb[0] * f2[0] +
           m.Vb[1] * f2[1] + m.Vb[2] * f2[2];
}

// Adds -1/2 sum_k r_k L_k T_k (r_k . jump) to F: the matrix dissipation
// R |Lambda| T R^T of eq. (ES) with the eigenvector columns for n = sg e_d,
//   r1 = (1, Vb - c n, h - vn c), r2 = (1, Vb, V2b/2), r3,4 = (0, t, Vb.t),
//   r5 = (1, Vb + c n, h + vn c),  tangents t = e_{d+1}, e_{d+2} (mod 3).
template <typename T>
MEHDG_HD void eigen_dissipation(const T Vb[3], const T& c, const T& h, const T& V2b, int d,
                                double sg, const T Lw[5], const T jump[5], T F[5]) {
    const T vn = Vb[d] * sg;
    // wave 1 and 5 (acoustic)
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const double s = (w == 0) ? -1.0 : 1.0;
        T r[5];
        r[0] = cst<T>::of(1.0);
        r[1] = Vb[0];
        r[2] = Vb[1];
        r[3] = Vb[2];
        r[1 + d] = r[1 + d] + (s * sg) * c;
        r[4] = h + s * (vn * c);
        const T proj = r[0] * jump[0] + r[1] * jump[1] + r[2] * jump[2] + r[3] * jump[3] + r[4] * jump[4];
        const T co = 0.5 * (Lw[w == 0 ? 0 : 4] * proj);
#pragma unroll
        for (int k = 0; k < 5; ++k) F[k] = F[k] - r[k] * co;
    }
    {   // wave 2 (entropy)
        const T proj = jump[0] + Vb[0] * jump[1] + Vb[1] * jump[2] + Vb[2] * jump[3] + 0.5 * V2b * jump[4];
        const T co = 0.5 * (Lw[1] * proj);
        F[0] = F[0] - co;
        F[1] = F[1] - Vb[0] * co;
        F[2] = F[2] - Vb[1] * co;
        F[3] = F[3] - Vb[2] * co;
        F[4] = F[4] - 0.5 * V2b * co;
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {   // waves 3, 4 (shear), tangent axis t
        const int t = (d + 1 + w) % 3;
        const T proj = jump[1 + t] + Vb[t] * jump[4];
        const T co = 0.5 * (Lw[2 + w] * proj);
        F[1 + t] = F[1 + t] - co;
        F[4] = F[4] - Vb[t] * co;
    }
}

// KEPES flux (eq. KEPES1-KEPES5, ES).
template <typename T>
MEHDG_HD void kepes_flux(const Prim<T>& sh, const Prim<T>& s, const T jump[5], double g, double eps,
                         int d, double sg, T F[5]) {
    Means<T> m;
    two_point_means(sh, s, eps, m);
    ec_flux(m, g, d, sg, F);
    const T c = dsqrt(g * m.Pb / m.rho_ln);
    const T h = g / (m.beta_ln * (g - 1.0)) + 0.5 * m.V2b;
    const T vn = m.Vb[d] * sg;
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
    eigen_dissipation(m.Vb, c, h, m.V2b, d, sg, Lw, jump, F);
}

// Entropy-stable flux (eq. Flux_En_Inv): central average minus
// 1/2 sigma(vh) A0(vh) [[v]], sigma = |Vh.n| + c_hat.  A0(vh) is applied
// through its scaled eigen-decomposition at vh (eq. KEPES4 at coincident
// states): A0 = R T R^T with T = (rho/(2g), rho (g-1)/g, P, P, rho/(2g)).
template <typename T>
MEHDG_HD void es_flux(const Prim<T>& sh, const Prim<T>& s, const T jump[5], double g, int d,
                      double sg, T F[5]) {
    T Fa[5], Fb[5];
    euler_flux(sh, g, d, Fa);
    euler_flux(s, g, d, Fb);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = (0.5 * sg) * (Fa[k] + Fb[k]);
    const T c = dsqrt(g * sh.P / sh.rho);
    const T V2 = kinetic2(sh);
    const T h = sh.P * (g / ((g - 1.0) * sh.rho)) + 0.5 * V2;
    const T sigma = dabs(sh.V[d]) + c;
    const T Ta = sh.rho * (1.0 / (2.0 * g));
    const T Lw[5] = {sigma * Ta, sigma * (sh.rho * ((g - 1.0) / g)), sigma * sh.P, sigma * sh.P,
                     sigma * Ta};
    eigen_dissipation(sh.V, c, h, V2, d, sg, Lw, jump, F);
}

// Inviscid trace flux Fhat(vh, v) selected by pr.flux.
template <typename T>
MEHDG_HD void trace_flux(const T vh[5], const T v[5], const DevParams& pr, int d, double sg, T F[5]) {
    Prim<T> sh, s;
    primitive(vh, pr.gamma, sh);
    primitive(v, pr.gamma, s);
    T jump[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) jump[k] = vh[k] - v[k];
    if (pr.flux == 0) {
        Means<T> m;
        two_point_means(sh, s, pr.eps, m);
        ec_flux(m, pr.gamma, d, sg, F);
    } else if (pr.flux == 1) {
        es_flux(sh, s, jump, pr.gamma, d, sg, F);
    } else {
        kepes_flux(sh, s, jump, pr.gamma, pr.eps, d, sg, F);
    }
}

// Viscous trace flux (eq. Flux_En_Vis): G(vh, q).n - 1/2 sigma_vis [[v]].
template <typename T, typename Q>
MEHDG_HD void viscous_trace_flux(const T vh[5], const T v[5], const Q q[5][3], const DevParams& pr,
                                 int d, double sg, T F[5]) {
    T G[5];
    viscous_flux(vh, q, pr, d, G);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = sg * G[k] - (0.5 * pr.sv[k]) * (vh[k] - v[k]);
}
