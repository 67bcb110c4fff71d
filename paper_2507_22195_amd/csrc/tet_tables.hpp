// Reference tables of a tetrahedral macro-element, built on the host.
//
// A macro-element is a tetrahedron K resolved by the red refinement into
// eight sub-tetrahedra (Sec. 3.1, local space W_p(K), Fig. 1): the four
// corner tetrahedra at the edge midpoints and the inner octahedron split
// along the diagonal joining the midpoints of reference edges 0-2 and 1-3.
// Each sub-tetrahedron carries P_p with equispaced Lagrange nodes, so the
// macro nodes are the degree-2p lattice of K:
//   node a at xi = (i, j, k)/(2p), i + j + k <= 2p, i fastest, then j, k;
//   n = (2p+1)(2p+2)(2p+3)/6.
// Face f is opposite vertex f, with vertices (P0, P1, P2) the other three in
// increasing order; face node c sits at P0 + (i (P1-P0) + j (P2-P0))/(2p),
// i + j <= 2p, i fastest: nf = (2p+1)(2p+2)/2.  The trace space is the
// restriction of W_p(K) to the face (continuous P_p on its four
// sub-triangles), so on a face the macro basis is the trace basis.
//
// Quadrature: the collapsed Gauss-Jacobi rule with p+1 points per direction
// on every sub-tetrahedron (exact for total degree 2p+1) and the matching
// two-dimensional rule on every face sub-triangle.
//
// Besides the basis tables, the constant matrices of R_Q (eq. s32a) on the
// reference macro: M (mass), C_i (d/dxi_i phi_a, phi_b), Ch_f (phi_a, psi_c)
// on face f in face-parameter measure, and D_i = M^-1 C_i, Dh_f = M^-1 Ch_f.
// An affine macro x = X0 + J xi scales them: M_phys = |det J| M,
// C_j = |det J| sum_i (J^-1)_ij C_i, Chat_j on face f = 2 area_f n_j Ch_f.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

struct TetTab {
    int p = 0, n = 0, nf = 0, ns = 0, nfs = 0, Gs = 0, Ss = 0;
    std::vector<double> phi;    // [Gs][ns]     sub-tet basis at the sub-tet rule's points
    std::vector<double> dphi;   // [3][Gs][ns]  d/deta_e of the sub-tet basis
    std::vector<double> wv;     // [Gs]         rule weights on a sub-tet of the reference macro (x 1/8)
    std::vector<double> BiT;    // [8][3][3]    B_s^-T: grad_xi = B_s^-T grad_eta
    std::vector<double> psi;    // [Ss][nfs]    sub-triangle basis at the triangle rule's points
    std::vector<double> wf;     // [Ss]         triangle weights on a face sub-triangle (x 1/4), face-parameter measure
    std::vector<double> Mt;     // [n][n]       M (symmetric)
    std::vector<double> CT;     // [3][n][n]    CT[i][b][a] = C_i[a][b]
    std::vector<double> ChT;    // [4][nf][n]   ChT[f][c][a] = Ch_f[a][c]
    std::vector<double> DT;     // [3][n][n]    DT[i][b][a] = D_i[a][b]
    std::vector<double> DhT;    // [4][nf][n]   DhT[f][c][a] = Dh_f[a][c]
    std::vector<double> Mi;     // [n][n]       M^-1 (symmetric)
    std::vector<int> vnode;     // [8][ns]      macro node of each sub-tet node
    std::vector<int> fnode;     // [4][nf]      macro node of each face node
    std::vector<int> tnode;     // [4][nfs]     face node of each sub-triangle node
    std::vector<int> vloc;      // [8][n]       local index of a macro node in a sub-tet, or -1
    std::vector<int> tloc;      // [4][nf]      local index of a face node in a sub-triangle, or -1
    std::vector<int> fidx;      // [4][n]       face node of a macro node on face f, or -1
    // weak-gradient tables of the coefficient-based columns (point orders of the kernels:
    // volume point s*Gs + gl, face point (f*4 + tr)*Ss + sl)
    std::vector<double> ED;     // [3][n][8 Gs]   (Phi M^-1 C_i)[g][b], point index fastest
    std::vector<double> EDf;    // [3][n][16 Ss]  the same at the face points
    std::vector<double> EH;     // [4][nf][8 Gs]  (Phi M^-1 Ch_f)[g][c]
    std::vector<double> EHf;    // [4][nf][16 Ss]
    std::vector<int> vptr, vinc;   // CSR over macro nodes: entries s*ns + b with vnode[s][b] = a
    std::vector<int> fptr, finc;   // CSR over face nodes: entries t*nfs + b with tnode[t][b] = c
};

namespace tet_detail {

inline int idx3(int m, int i, int j, int k) {
    // position of (i, j, k) in the lattice order (k outer, j, i fastest)
    int off = 0;
    for (int kk = 0; kk < k; ++kk) off += (m - kk + 1) * (m - kk + 2) / 2;
    const int r = m - k;
    for (int jj = 0; jj < j; ++jj) off += r - jj + 1;
    return off + i;
}

inline int idx2(int m, int i, int j) {
    int off = 0;
    for (int jj = 0; jj < j; ++jj) off += m - jj + 1;
    return off + i;
}

// Eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations.
inline void sym_eig(int N, std::vector<double>& A, std::vector<double>& V) {
    V.assign((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) V[i * N + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) off += A[i * N + j] * A[i * N + j];
        if (off < 1e-60) break;
        for (int p = 0; p < N; ++p)
            for (int q = p + 1; q < N; ++q) {
                const double apq = A[p * N + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double th = (A[q * N + q] - A[p * N + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < N; ++k) {
                    const double akp = A[k * N + p], akq = A[k * N + q];
                    A[k * N + p] = c * akp - s * akq;
                    A[k * N + q] = s * akp + c * akq;
                }
                for (int k = 0; k < N; ++k) {
                    const double apk = A[p * N + k], aqk = A[q * N + k];
                    A[p * N + k] = c * apk - s * aqk;
                    A[q * N + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < N; ++k) {
                    const double vkp = V[k * N + p], vkq = V[k * N + q];
                    V[k * N + p] = c * vkp - s * vkq;
                    V[k * N + q] = s * vkp + c * vkq;
                }
            }
    }
}

// q-point Gauss rule on [0, 1] for the weight (1 - t)^alpha (Golub-Welsch on
// the recurrence of the Jacobi polynomials P^(alpha, 0) on [-1, 1]).
inline void gauss_jacobi01(int q, double alpha, std::vector<double>& t, std::vector<double>& w) {
    const double be = 0.0;
    std::vector<double> J((size_t)q * q, 0.0), V;
    for (int k = 0; k < q; ++k) {
        const double s = 2.0 * k + alpha + be;
        J[k * q + k] = (k == 0) ? (be - alpha) / (alpha + be + 2.0) : (be * be - alpha * alpha) / (s * (s + 2.0));
        if (k + 1 < q) {
            const double kk = k + 1.0, s1 = 2.0 * kk + alpha + be;
            const double b = 4.0 * kk * (kk + alpha) * (kk + be) * (kk + alpha + be) /
                             (s1 * s1 * (s1 + 1.0) * (s1 - 1.0));
            J[k * q + k + 1] = J[(k + 1) * q + k] = std::sqrt(b);
        }
    }
    sym_eig(q, J, V);
    std::vector<std::pair<double, double>> pw;
    for (int i = 0; i < q; ++i) pw.push_back({(1.0 + J[i * q + i]) / 2.0, V[i] * V[i] / (alpha + 1.0)});
    for (int i = 0; i < q; ++i)
        for (int j = i + 1; j < q; ++j)
            if (pw[j].first < pw[i].first) std::swap(pw[i], pw[j]);
    t.resize(q);
    w.resize(q);
    for (int i = 0; i < q; ++i) {
        t[i] = pw[i].first;
        w[i] = pw[i].second;
    }
}

// In-place inverse of a dense N x N matrix (Gauss-Jordan, partial pivoting).
inline bool invert(int N, std::vector<double>& A) {
    std::vector<double> I((size_t)N * N, 0.0);
    for (int i = 0; i < N; ++i) I[i * N + i] = 1.0;
    for (int c = 0; c < N; ++c) {
        int piv = c;
        for (int r = c + 1; r < N; ++r)
            if (std::fabs(A[r * N + c]) > std::fabs(A[piv * N + c])) piv = r;
        if (!(std::fabs(A[piv * N + c]) > 0.0)) return false;
        if (piv != c)
            for (int k = 0; k < N; ++k) {
                std::swap(A[c * N + k], A[piv * N + k]);
                std::swap(I[c * N + k], I[piv * N + k]);
            }
        const double d = 1.0 / A[c * N + c];
        for (int k = 0; k < N; ++k) {
            A[c * N + k] *= d;
            I[c * N + k] *= d;
        }
        for (int r = 0; r < N; ++r) {
            if (r == c) continue;
            const double f = A[r * N + c];
            if (f == 0.0) continue;
            for (int k = 0; k < N; ++k) {
                A[r * N + k] -= f * A[c * N + k];
                I[r * N + k] -= f * I[c * N + k];
            }
        }
    }
    A.swap(I);
    return true;
}

// Exponents of the monomials of total degree <= p in dim variables.
inline std::vector<std::vector<int>> exponents(int p, int dim) {
    std::vector<std::vector<int>> out;
    if (dim == 2) {
        for (int a = 0; a <= p; ++a)
            for (int b = 0; a + b <= p; ++b) out.push_back({a, b});
    } else {
        for (int a = 0; a <= p; ++a)
            for (int b = 0; a + b <= p; ++b)
                for (int c = 0; a + b + c <= p; ++c) out.push_back({a, b, c});
    }
    return out;
}

inline double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// Lagrange basis of degree p on the unit simplex with nodes lattice/p:
// coefficient matrix Cm [nm][nn] with phi_b(x) = sum_m mono_m(x) Cm[m][b].
inline bool lagrange_coef(int p, int dim, std::vector<double>& Cm) {
    const auto ex = exponents(p, dim);
    const int N = (int)ex.size();
    std::vector<std::vector<double>> nodes;
    if (dim == 3) {
        for (int k = 0; k <= p; ++k)
            for (int j = 0; j + k <= p; ++j)
                for (int i = 0; i + j + k <= p; ++i) nodes.push_back({(double)i / p, (double)j / p, (double)k / p});
    } else {
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i + j <= p; ++i) nodes.push_back({(double)i / p, (double)j / p});
    }
    std::vector<double> V((size_t)N * N);
    for (int r = 0; r < N; ++r)
        for (int m = 0; m < N; ++m) {
            double v = 1.0;
            for (int d = 0; d < dim; ++d) v *= ipow(nodes[r][d], ex[m][d]);
            V[r * N + m] = v;
        }
    if (!invert(N, V)) return false;   // V^-1 [m][b]
    Cm = V;
    return true;
}

// Values [nn] and gradients [dim][nn] of that basis at x.
inline void lagrange_eval(int p, int dim, const std::vector<double>& Cm, const double* x, double* val,
                          double* grad) {
    const auto ex = exponents(p, dim);
    const int N = (int)ex.size();
    for (int b = 0; b < N; ++b) {
        val[b] = 0.0;
        for (int d = 0; d < dim; ++d) grad[d * N + b] = 0.0;
    }
    for (int m = 0; m < N; ++m) {
        double mv = 1.0;
        for (int d = 0; d < dim; ++d) mv *= ipow(x[d], ex[m][d]);
        double mg[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < dim; ++d) {
            if (ex[m][d] == 0) continue;
            double g = ex[m][d] * ipow(x[d], ex[m][d] - 1);
            for (int d2 = 0; d2 < dim; ++d2)
                if (d2 != d) g *= ipow(x[d2], ex[m][d2]);
            mg[d] = g;
        }
        for (int b = 0; b < N; ++b) {
            val[b] += mv * Cm[(size_t)m * N + b];
            for (int d = 0; d < dim; ++d) grad[d * N + b] += mg[d] * Cm[(size_t)m * N + b];
        }
    }
}

}  // namespace tet_detail

// The eight sub-tetrahedra in half-units (vertex coordinates x 2).
inline void tet_subtets(int T[8][4][3]) {
    const int V[4][3] = {{0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
    auto mid = [&](int a, int b, int* o) {
        for (int d = 0; d < 3; ++d) o[d] = (V[a][d] + V[b][d]) / 2;
    };
    int m01[3], m02[3], m03[3], m12[3], m13[3], m23[3];
    mid(0, 1, m01); mid(0, 2, m02); mid(0, 3, m03); mid(1, 2, m12); mid(1, 3, m13); mid(2, 3, m23);
    const int* corner[4][4] = {{V[0], m01, m02, m03}, {m01, V[1], m12, m13}, {m02, m12, V[2], m23},
                               {m03, m13, m23, V[3]}};
    const int* ring[4] = {m01, m12, m23, m03};
    for (int s = 0; s < 4; ++s)
        for (int v = 0; v < 4; ++v)
            for (int d = 0; d < 3; ++d) T[s][v][d] = corner[s][v][d];
    for (int s = 0; s < 4; ++s) {
        const int* vs[4] = {m02, m13, ring[s], ring[(s + 1) % 4]};
        for (int v = 0; v < 4; ++v)
            for (int d = 0; d < 3; ++d) T[4 + s][v][d] = vs[v][d];
    }
}

inline bool build_tet_tables(int p, TetTab& t) {
    using namespace tet_detail;
    const int m = 2 * p;
    t.p = p;
    t.n = (m + 1) * (m + 2) * (m + 3) / 6;
    t.nf = (m + 1) * (m + 2) / 2;
    t.ns = (p + 1) * (p + 2) * (p + 3) / 6;
    t.nfs = (p + 1) * (p + 2) / 2;
    const int q = p + 1;
    t.Gs = q * q * q;
    t.Ss = q * q;
    const int n = t.n, nf = t.nf, ns = t.ns, nfs = t.nfs, Gs = t.Gs, Ss = t.Ss;

    std::vector<double> a0, w0, a1, w1, a2, w2;
    gauss_jacobi01(q, 0.0, a0, w0);
    gauss_jacobi01(q, 1.0, a1, w1);
    gauss_jacobi01(q, 2.0, a2, w2);
    std::vector<double> C3, C2;
    if (!lagrange_coef(p, 3, C3) || !lagrange_coef(p, 2, C2)) return false;

    // sub-tet rule and basis
    t.phi.assign((size_t)Gs * ns, 0.0);
    t.dphi.assign((size_t)3 * Gs * ns, 0.0);
    t.wv.assign(Gs, 0.0);
    std::vector<double> val(ns), grad(3 * ns);
    for (int k = 0; k < q; ++k)
        for (int j = 0; j < q; ++j)
            for (int i = 0; i < q; ++i) {
                const int g = i + q * (j + q * k);
                const double x[3] = {a0[i] * (1 - a1[j]) * (1 - a2[k]), a1[j] * (1 - a2[k]), a2[k]};
                t.wv[g] = w0[i] * w1[j] * w2[k] / 8.0;
                lagrange_eval(p, 3, C3, x, val.data(), grad.data());
                for (int b = 0; b < ns; ++b) {
                    t.phi[(size_t)g * ns + b] = val[b];
                    for (int e = 0; e < 3; ++e) t.dphi[((size_t)e * Gs + g) * ns + b] = grad[e * ns + b];
                }
            }
    // sub-triangle rule and basis
    t.psi.assign((size_t)Ss * nfs, 0.0);
    t.wf.assign(Ss, 0.0);
    std::vector<double> val2(nfs), grad2(2 * nfs);
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < q; ++i) {
            const int s = i + q * j;
            const double x[2] = {a0[i] * (1 - a1[j]), a1[j]};
            t.wf[s] = w0[i] * w1[j] / 4.0;
            lagrange_eval(p, 2, C2, x, val2.data(), grad2.data());
            for (int b = 0; b < nfs; ++b) t.psi[(size_t)s * nfs + b] = val2[b];
        }

    // sub-tets: node maps and gradient transforms
    int T[8][4][3];
    tet_subtets(T);
    t.vnode.assign(8 * ns, 0);
    t.BiT.assign(8 * 9, 0.0);
    for (int s = 0; s < 8; ++s) {
        int b = 0;
        for (int gk = 0; gk <= p; ++gk)
            for (int gj = 0; gj + gk <= p; ++gj)
                for (int gi = 0; gi + gj + gk <= p; ++gi, ++b) {
                    int pos[3];
                    for (int d = 0; d < 3; ++d)   // lattice units 1/(2p): vertex half-units x p
                        pos[d] = T[s][0][d] * p + gi * (T[s][1][d] - T[s][0][d]) + gj * (T[s][2][d] - T[s][0][d]) +
                                 gk * (T[s][3][d] - T[s][0][d]);
                    t.vnode[s * ns + b] = idx3(m, pos[0], pos[1], pos[2]);
                }
        std::vector<double> B(9);   // columns: sub-tet edges in xi
        for (int e = 0; e < 3; ++e)
            for (int d = 0; d < 3; ++d) B[d * 3 + e] = (T[s][e + 1][d] - T[s][0][d]) / 2.0;
        if (!invert(3, B)) return false;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) t.BiT[s * 9 + r * 3 + c] = B[c * 3 + r];
    }
    // faces: face node -> macro node; sub-triangle node -> face node
    const int FV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    const int VL[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    t.fnode.assign(4 * nf, 0);
    for (int f = 0; f < 4; ++f) {
        int c = 0;
        for (int j = 0; j <= m; ++j)
            for (int i = 0; i + j <= m; ++i, ++c) {
                int pos[3];
                for (int d = 0; d < 3; ++d)
                    pos[d] = VL[FV[f][0]][d] * m + i * (VL[FV[f][1]][d] - VL[FV[f][0]][d]) +
                             j * (VL[FV[f][2]][d] - VL[FV[f][0]][d]);
                t.fnode[f * nf + c] = idx3(m, pos[0], pos[1], pos[2]);
            }
    }
    const int TR[4][3][2] = {{{0, 0}, {1, 0}, {0, 1}}, {{1, 0}, {2, 0}, {1, 1}}, {{0, 1}, {1, 1}, {0, 2}},
                             {{1, 0}, {1, 1}, {0, 1}}};
    t.tnode.assign(4 * nfs, 0);
    for (int tr = 0; tr < 4; ++tr) {
        int b = 0;
        for (int bj = 0; bj <= p; ++bj)
            for (int bi = 0; bi + bj <= p; ++bi, ++b) {
                int pos[2];
                for (int d = 0; d < 2; ++d)
                    pos[d] = TR[tr][0][d] * p + bi * (TR[tr][1][d] - TR[tr][0][d]) + bj * (TR[tr][2][d] - TR[tr][0][d]);
                t.tnode[tr * nfs + b] = idx2(m, pos[0], pos[1]);
            }
    }
    // incidence lists
    auto csr = [](int N, int groups, int per, const std::vector<int>& map, std::vector<int>& ptr,
                  std::vector<int>& inc) {
        ptr.assign(N + 1, 0);
        for (int g = 0; g < groups; ++g)
            for (int b = 0; b < per; ++b) ptr[map[g * per + b] + 1]++;
        for (int a = 0; a < N; ++a) ptr[a + 1] += ptr[a];
        inc.assign(ptr[N], 0);
        std::vector<int> fill(ptr.begin(), ptr.end() - 1);
        for (int g = 0; g < groups; ++g)
            for (int b = 0; b < per; ++b) inc[fill[map[g * per + b]]++] = g * per + b;
    };
    csr(n, 8, ns, t.vnode, t.vptr, t.vinc);
    csr(nf, 4, nfs, t.tnode, t.fptr, t.finc);

    // constant matrices of R_Q on the reference macro
    std::vector<double> M((size_t)n * n, 0.0), C((size_t)3 * n * n, 0.0), Ch((size_t)4 * n * nf, 0.0);
    for (int s = 0; s < 8; ++s)
        for (int g = 0; g < Gs; ++g) {
            const double w = t.wv[g];
            for (int a = 0; a < ns; ++a) {
                const int A = t.vnode[s * ns + a];
                double gx[3];
                for (int i = 0; i < 3; ++i) {
                    gx[i] = 0.0;
                    for (int e = 0; e < 3; ++e) gx[i] += t.BiT[s * 9 + i * 3 + e] * t.dphi[((size_t)e * Gs + g) * ns + a];
                }
                for (int b = 0; b < ns; ++b) {
                    const int Bn = t.vnode[s * ns + b];
                    const double pb = t.phi[(size_t)g * ns + b];
                    M[(size_t)A * n + Bn] += w * t.phi[(size_t)g * ns + a] * pb;
                    for (int i = 0; i < 3; ++i) C[((size_t)i * n + A) * n + Bn] += w * gx[i] * pb;
                }
            }
        }
    for (int f = 0; f < 4; ++f)
        for (int tr = 0; tr < 4; ++tr)
            for (int s = 0; s < Ss; ++s)
                for (int a = 0; a < nfs; ++a) {
                    const int A = t.fnode[f * nf + t.tnode[tr * nfs + a]];
                    for (int b = 0; b < nfs; ++b) {
                        const int c = t.tnode[tr * nfs + b];
                        Ch[((size_t)f * n + A) * nf + c] += t.wf[s] * t.psi[(size_t)s * nfs + a] * t.psi[(size_t)s * nfs + b];
                    }
                }
    std::vector<double> Mi = M;
    if (!invert(n, Mi)) return false;
    t.Mt = M;
    t.Mi = Mi;
    t.CT.assign((size_t)3 * n * n, 0.0);
    t.DT.assign((size_t)3 * n * n, 0.0);
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                t.CT[((size_t)i * n + b) * n + a] = C[((size_t)i * n + a) * n + b];
                double d = 0.0;
                for (int c = 0; c < n; ++c) d += Mi[(size_t)a * n + c] * C[((size_t)i * n + c) * n + b];
                t.DT[((size_t)i * n + b) * n + a] = d;
            }
    // local-index maps and the weak-gradient tables at the points
    t.vloc.assign(8 * n, -1);
    for (int s = 0; s < 8; ++s)
        for (int b = 0; b < ns; ++b) t.vloc[s * n + t.vnode[s * ns + b]] = b;
    t.tloc.assign(4 * nf, -1);
    for (int tr = 0; tr < 4; ++tr)
        for (int b = 0; b < nfs; ++b) t.tloc[tr * nf + t.tnode[tr * nfs + b]] = b;
    t.fidx.assign(4 * n, -1);
    for (int f = 0; f < 4; ++f)
        for (int c = 0; c < nf; ++c) t.fidx[f * n + t.fnode[f * nf + c]] = c;
    const int G = 8 * Gs, FP = 16 * Ss;
    auto Dm = [&](int i, int a, int b) {   // (M^-1 C_i)[a][b]
        double d = 0.0;
        for (int c = 0; c < n; ++c) d += Mi[(size_t)a * n + c] * C[((size_t)i * n + c) * n + b];
        return d;
    };
    auto Dhm = [&](int f, int a, int c) {  // (M^-1 Ch_f)[a][c]
        double d = 0.0;
        for (int b = 0; b < n; ++b) d += Mi[(size_t)a * n + b] * Ch[((size_t)f * n + b) * nf + c];
        return d;
    };
    std::vector<double> Dfull((size_t)3 * n * n), Dhfull((size_t)4 * n * nf);
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) Dfull[((size_t)i * n + a) * n + b] = Dm(i, a, b);
    for (int f = 0; f < 4; ++f)
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < nf; ++c) Dhfull[((size_t)f * n + a) * nf + c] = Dhm(f, a, c);
    t.ED.assign((size_t)3 * G * n, 0.0);
    t.EH.assign((size_t)4 * G * nf, 0.0);
    for (int s = 0; s < 8; ++s)
        for (int gl = 0; gl < Gs; ++gl) {
            const int gp = s * Gs + gl;
            for (int bl = 0; bl < ns; ++bl) {
                const double ph = t.phi[(size_t)gl * ns + bl];
                const int a = t.vnode[s * ns + bl];
                for (int i = 0; i < 3; ++i)
                    for (int b = 0; b < n; ++b) t.ED[((size_t)i * n + b) * G + gp] += ph * Dfull[((size_t)i * n + a) * n + b];
                for (int f = 0; f < 4; ++f)
                    for (int c = 0; c < nf; ++c) t.EH[((size_t)f * nf + c) * G + gp] += ph * Dhfull[((size_t)f * n + a) * nf + c];
            }
        }
    t.EDf.assign((size_t)3 * FP * n, 0.0);
    t.EHf.assign((size_t)4 * FP * nf, 0.0);
    for (int f = 0; f < 4; ++f)
        for (int tr = 0; tr < 4; ++tr)
            for (int sl = 0; sl < Ss; ++sl) {
                const int fp = (f * 4 + tr) * Ss + sl;
                for (int bl = 0; bl < nfs; ++bl) {
                    const double ps = t.psi[(size_t)sl * nfs + bl];
                    const int a = t.fnode[f * nf + t.tnode[tr * nfs + bl]];
                    for (int i = 0; i < 3; ++i)
                        for (int b = 0; b < n; ++b)
                            t.EDf[((size_t)i * n + b) * FP + fp] += ps * Dfull[((size_t)i * n + a) * n + b];
                    for (int f2 = 0; f2 < 4; ++f2)
                        for (int c = 0; c < nf; ++c)
                            t.EHf[((size_t)f2 * nf + c) * FP + fp] += ps * Dhfull[((size_t)f2 * n + a) * nf + c];
                }
            }
    t.ChT.assign((size_t)4 * nf * n, 0.0);
    t.DhT.assign((size_t)4 * nf * n, 0.0);
    for (int f = 0; f < 4; ++f)
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < nf; ++c) {
                t.ChT[((size_t)f * nf + c) * n + a] = Ch[((size_t)f * n + a) * nf + c];
                double d = 0.0;
                for (int b = 0; b < n; ++b) d += Mi[(size_t)a * n + b] * Ch[((size_t)f * n + b) * nf + c];
                t.DhT[((size_t)f * nf + c) * n + a] = d;
            }
    return true;
}
