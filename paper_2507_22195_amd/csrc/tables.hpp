// Host construction of the 1-D reference tables (Gauss-Lobatto nodes,
// Gauss quadrature, C0 basis on the two sub-intervals of [0,2], 1-D mass,
// its inverse and the 1-D weak-gradient operator).
#pragma once
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace mehdg {

// Legendre P_N(x) and P_{N-1}(x) by the three-term recurrence.
inline void legendre(int N, double x, double& pn, double& pnm1) {
    double p0 = 1.0, p1 = x;
    if (N == 0) {
        pn = 1.0;
        pnm1 = 0.0;
        return;
    }
    for (int k = 2; k <= N; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pnm1 = p0;
}

// Gauss-Lobatto-Legendre points on [-1,1]: zeros of (1-x^2) P_p'(x).
// Newton on r(x) = P_{p-1}(x) - x P_p(x) = (1-x^2) P_p'(x)/p, whose
// derivative is -(p+1) P_p(x) (Legendre equation).
inline void gll_points(int p, double* x) {
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double pn, pm;
            legendre(p, t, pn, pm);
            const double dt = (pm - t * pn) / ((p + 1.0) * pn);
            t += dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[i] = t;
    }
}

// Gauss-Legendre points/weights on [-1,1] with N points (Newton on P_N).
inline void gauss_rule(int N, double* x, double* w) {
    for (int i = 0; i < N; ++i) {
        double t = -std::cos(M_PI * (i + 0.75) / (N + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pn, pm;
            legendre(N, t, pn, pm);
            dp = N * (t * pn - pm) / (t * t - 1.0);
            const double dt = -pn / dp;
            t += dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double pn, pm;
        legendre(N, t, pn, pm);
        dp = N * (t * pn - pm) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// Lagrange basis on nodes[0..m) evaluated at x: value and derivative.
inline void lagrange(int m, const double* nodes, double x, double* L, double* dL) {
    for (int i = 0; i < m; ++i) {
        double prod = 1.0, dsum = 0.0;
        for (int j = 0; j < m; ++j) {
            if (j == i) continue;
            prod *= (x - nodes[j]) / (nodes[i] - nodes[j]);
        }
        // derivative: sum over k != i of 1/(x_i - x_k) prod_{j != i,k} (x - x_j)/(x_i - x_j)
        for (int k = 0; k < m; ++k) {
            if (k == i) continue;
            double t = 1.0 / (nodes[i] - nodes[k]);
            for (int j = 0; j < m; ++j) {
                if (j == i || j == k) continue;
                t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
            }
            dsum += t;
        }
        L[i] = prod;
        dL[i] = dsum;
    }
}

// Gauss-Jordan inverse with partial pivoting of an m x m matrix (host).
inline bool invert(int m, const double* A, double* Ainv) {
    double a[MEHDG_MAXN1D][2 * MEHDG_MAXN1D];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 2 * m; ++j) a[i][j] = (j < m) ? A[i * m + j] : (j - m == i ? 1.0 : 0.0);
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < 2 * m; ++j) std::swap(a[c][j], a[piv][j]);
        const double inv = 1.0 / a[c][c];
        for (int j = 0; j < 2 * m; ++j) a[c][j] *= inv;
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * m; ++j) a[r][j] -= f * a[c][j];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Ainv[i * m + j] = a[i][m + j];
    return true;
}

inline bool build_tables(int p, Tab1D& t) {
    std::memset(&t, 0, sizeof(t));
    const int n1d = 2 * p + 1, nq1 = 2 * (p + 1);
    double gll[MEHDG_MAXP + 1], gx[MEHDG_MAXP + 1], gw[MEHDG_MAXP + 1];
    gll_points(p, gll);
    gauss_rule(p + 1, gx, gw);
    double local[MEHDG_MAXP + 1];
    for (int i = 0; i <= p; ++i) local[i] = 0.5 * (gll[i] + 1.0);
    for (int e = 0; e < 2; ++e)
        for (int i = 0; i <= p; ++i) {
            const int qd = e * (p + 1) + i;
            const double xl = 0.5 * (gx[i] + 1.0);   // local coordinate in [0,1]
            double L[MEHDG_MAXP + 1], dL[MEHDG_MAXP + 1];
            lagrange(p + 1, local, xl, L, dL);
            for (int a = 0; a <= p; ++a) {
                t.B[qd][e * p + a] = L[a];
                t.D[qd][e * p + a] = dL[a];
            }
            t.w[qd] = 0.5 * gw[i];
        }
    double M1[MEHDG_MAXN1D * MEHDG_MAXN1D], C1[MEHDG_MAXN1D * MEHDG_MAXN1D], Mi[MEHDG_MAXN1D * MEHDG_MAXN1D];
    for (int a = 0; a < n1d; ++a)
        for (int b = 0; b < n1d; ++b) {
            double m = 0.0, c = 0.0;
            for (int qd = 0; qd < nq1; ++qd) {
                m += t.w[qd] * t.B[qd][a] * t.B[qd][b];
                c += t.w[qd] * t.D[qd][a] * t.B[qd][b];
            }
            M1[a * n1d + b] = m;
            C1[a * n1d + b] = c;
            t.M1[a][b] = m;
        }
    if (!invert(n1d, M1, Mi)) return false;
    for (int a = 0; a < n1d; ++a)
        for (int b = 0; b < n1d; ++b) {
            t.Minv[a][b] = Mi[a * n1d + b];
            double s = 0.0;
            for (int c = 0; c < n1d; ++c) s += Mi[a * n1d + c] * C1[c * n1d + b];
            t.Lam[a][b] = s;
        }
    return true;
}

}  // namespace mehdg
