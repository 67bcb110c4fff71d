// Assembly of the bordered matrix of every macro-element (Sec. 6.2, eq. R1-R3):
//
//   B = [[ S,  -Y,  r_V  ],      S   = A_vv  - A_vq A_qq^-1 A_qv      (R3)
//        [ X,   A', r_hat]]      -Y  = A_vvh - A_vq A_qq^-1 A_qvh
//                                X   = A_hv  - A_hq A_qq^-1 A_qv
//                                A'  = A_hh  - A_hq A_qq^-1 A_qvh
//                                r_V = -R_V + A_vq A_qq^-1 R_Q,  r_hat = -R_Vhat + A_hq A_qq^-1 R_Q
//
// i.e. the Jacobian of (R_V, R_Vhat) in (V, Vhat) with Q eliminated, and the
// matching right-hand side.  Row-major, leading dimension ldB, rows
// [V rows | Vhat rows], columns [V cols | Vhat cols | rhs | padding].
//
// One workgroup owns the five rows of one test node and writes them whole
// (no atomics).  The local blocks of a row are accumulated in LDS, one
// sub-element (or sub-face) at a time, from the pointwise coefficients of
// the residual kernel.  Q is then eliminated with the tensor structure of
// A_qq = I (x) M: per axis j,
//   (M^-1 C_j)[c, b]        = Lam[c_j][b_j] / h_j   (other indices equal),
//   (M^-1 Chat_j)[c, (f,e)] = n_j Minv[c_j][i_f] / h_j  (faces normal to j),
// with Lam = M1^-1 C1 and Minv = M1^-1 the 1-D reference operators, so the
// elimination costs a 1-D contraction per entry.
#pragma once
#include "k_residual.hpp"

namespace mehdg {

__host__ __device__ constexpr int round_up8(int x) { return (x + 7) & ~7; }

template <int P>
struct Bdims {
    using D = Dims<P>;
    static constexpr int rows = D::NV + D::NH;
    static constexpr int ld = round_up8(D::NV + D::NH + 1);
    static constexpr int64_t per_macro = (int64_t)rows * ld;
};

// ---------------------------------------------------------------------------
// M^-1 R_Q per macro (A_qq^-1 R_Q without the identity factor):
// M^-1 = (Minv (x) Minv (x) Minv) / (hx hy hz).  The 15 fields are independent;
// a workgroup takes MinvRqCfg<P>::FG of them (blockIdx.y the group), so the two
// LDS copies of its fields stay within the LDS at every degree.
template <int P>
struct MinvRqCfg {
    static constexpr int FG = P >= 4 ? 5 : 15;
    static constexpr int GROUPS = 15 / FG;
};

template <int P>
__global__ void __launch_bounds__(256) k_minv_rq(const double* __restrict__ R_q, const double* __restrict__ hs,
                                                 const Tab1D* __restrict__ tab, double* __restrict__ out) {
    using D = Dims<P>;
    constexpr int n1d = D::n1d, n = D::n, FG = MinvRqCfg<P>::FG;
    __shared__ double a[FG * n], b[FG * n];
    __shared__ double Mi[n1d][n1d];
    const int64_t m = blockIdx.x;
    const int64_t f0 = (int64_t)blockIdx.y * FG * n;     // first element of the field group
    for (int i = threadIdx.x; i < n1d * n1d; i += blockDim.x) Mi[i / n1d][i % n1d] = tab->Minv[i / n1d][i % n1d];
    for (int i = threadIdx.x; i < FG * n; i += blockDim.x) a[i] = R_q[m * 15 * n + f0 + i];
    __syncthreads();
    const double s = 1.0 / (hs[3 * m] * hs[3 * m + 1] * hs[3 * m + 2]);
    double* src = a;
    double* dst = b;
    for (int axis = 0; axis < 3; ++axis) {
        const int stride = axis == 0 ? 1 : (axis == 1 ? n1d : n1d * n1d);
        for (int i = threadIdx.x; i < FG * n; i += blockDim.x) {
            const int node = i % n, field = i / n;
            const int ci = (node / stride) % n1d;
            const int base = node - ci * stride;
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < n1d; ++c) acc += Mi[ci][c] * src[field * n + base + c * stride];
            dst[i] = acc;
        }
        __syncthreads();
        double* t = src;
        src = dst;
        dst = t;
    }
    for (int i = threadIdx.x; i < FG * n; i += blockDim.x) out[m * 15 * n + f0 + i] = s * src[i];
}

// ---------------------------------------------------------------------------
// Row workgroups build the KG rows (k = 0..KG-1 of one test node) together:
// KG = 1: smaller LDS footprint, several workgroups per CU (measured faster
// than building all five rows per pass, whose accumulators fill the LDS).
// From p = 3 on the accumulators hold a CU's LDS nearly alone, so the
// workgroup grows instead (measured on the row kernel: 512 threads at p = 3,
// 1024 at p = 4 against 256).
template <int P>
struct RowCfg {
    static constexpr int KG = 1;
    static constexpr int THREADS = P >= 4 ? 1024 : (P == 3 ? 512 : 256);
};

template <int P>
struct RowLds {
    using D = Dims<P>;
    static constexpr int KG = RowCfg<P>::KG;
    static constexpr int E3 = (P + 1) * (P + 1) * (P + 1);
    static constexpr int E2 = (P + 1) * (P + 1);
    static constexpr int WS = E3 | 1;            // field stride of the volume weights (odd: no bank conflicts)
    static constexpr int WV = 20 * WS * KG;     // per trial field ([0,5) value, [5,20) q) and sub-element point
    static constexpr int WF = E2 * 25 * KG;     // per sub-face Gauss point: [0,5) v, [5,10) vhat, [10,25) q
    double av[KG][5][D::n];         // coefficient of trial v_{l,b}
    double aq[KG][15][D::n];        // coefficient of trial q_{l,j,c}  (index 3 l + j)
    double ah[KG][6][5][D::nf];     // coefficient of trial vhat_{f,l,e}
    double w[WV > WF ? WV : WF];    // work buffer of the current sub-element or sub-face
    double red[KG][RowCfg<P>::THREADS / 64];
    Tab1D t;
};

template <int P>
__device__ void row_zero(RowLds<P>& L) {
    using D = Dims<P>;
    constexpr int KG = RowLds<P>::KG;
    double* p = &L.av[0][0][0];
    for (int i = threadIdx.x; i < KG * 20 * D::n; i += blockDim.x) p[i] = 0.0;   // av and aq are contiguous
    double* h = &L.ah[0][0][0][0];
    for (int i = threadIdx.x; i < KG * 30 * D::nf; i += blockDim.x) h[i] = 0.0;
}

// Volume part of row k of node a for the sub-element (e1,e2,e3):
//   A[(a,k), (b,fld)] += sum_g W_fld(g) phi_b(g),
// W_fld(g) the test function's value and gradient at sub-element point g
// contracted with the pointwise coefficients of trial field fld (value trial l,
// or q trial (l, j)).  phi_b(g) = B(g1,b1) B(g2,b2) B(g3,b3) on the sub-element's
// Q^3 points and nodes, so the sum goes by sum factorisation: along axis 1 in
// place in the weight buffer (a thread per line), then axes 2 and 3 in
// registers (a thread per (b1, b2)): 3 Q^4 products per field instead of Q^6.
template <int P>
__device__ void row_volume(RowLds<P>& L, const double* __restrict__ coefV, int64_t m, int a1, int a2, int a3,
                           int e1, int e2, int e3, int k, bool viscous) {
    using D = Dims<P>;
    using R = RowLds<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, G = D::G, E3 = R::E3, WS = R::WS;
    constexpr int Q = P + 1;
    static_assert(R::KG == 1, "one row per pass");
    const int nfld = viscous ? 20 : 5;
    // weights: a thread per sub-element point (consecutive threads on
    // consecutive points: the coefficients are stored point index fastest),
    // its basis factors formed once for the fields it takes in turn
    const int fpp = (int)blockDim.x / E3;        // fields per pass
    if ((int)threadIdx.x < fpp * E3) {
        const int gl = threadIdx.x % E3, f0 = threadIdx.x / E3;
        const int g1 = e1 * Q + gl % Q, g2 = e2 * Q + (gl / Q) % Q, g3 = e3 * Q + gl / (Q * Q);
        const int g = g1 + nq1 * (g2 + nq1 * g3);
        const double B1 = L.t.B[g1][a1], B2 = L.t.B[g2][a2], B3 = L.t.B[g3][a3];
        const double t1 = L.t.D[g1][a1] * B2 * B3, t2 = B1 * L.t.D[g2][a2] * B3, t3 = B1 * B2 * L.t.D[g3][a3];
        const double b123 = B1 * B2 * B3;
        const double* c = coefV + (int64_t)m * G * COEF_V + g;
        for (int fld = f0; fld < nfld; fld += fpp) {
            double wv;
            if (fld < 5) {
                const int o = 5 * k + fld;
                wv = b123 * c[o * G] + t1 * c[(25 + o) * G] + t2 * c[(50 + o) * G] + t3 * c[(75 + o) * G];
            } else {
                const int j = (fld - 5) % 3, o = 5 * k + (fld - 5) / 3;
                wv = t1 * c[(100 + 25 * j + o) * G] + t2 * c[(100 + 25 * (3 + j) + o) * G] +
                     t3 * c[(100 + 25 * (6 + j) + o) * G];
            }
            L.w[fld * WS + gl] = wv;
        }
    }
    __syncthreads();
    // axis 1, in place: W[fld][g1, g2, g3] -> T[fld][b1, g2, g3]
    for (int idx = threadIdx.x; idx < nfld * Q * Q; idx += blockDim.x) {
        const int fld = idx / (Q * Q), r = idx % (Q * Q);
        double* line = L.w + fld * WS + Q * r;
        double x[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = line[i];
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) s += x[i] * L.t.B[e1 * Q + i][e1 * P + b];
            line[b] = s;
        }
    }
    __syncthreads();
    // axes 2 and 3 for one (b1, b2) per thread, added into the row's accumulators
    for (int idx = threadIdx.x; idx < nfld * Q * Q; idx += blockDim.x) {
        const int fld = idx / (Q * Q), r = idx % (Q * Q), b1l = r % Q, b2l = r / Q;
        const double* T = L.w + fld * WS;
        double t[Q];
#pragma unroll
        for (int g3l = 0; g3l < Q; ++g3l) {
            double s = 0.0;
#pragma unroll
            for (int g2l = 0; g2l < Q; ++g2l) s += T[b1l + Q * (g2l + Q * g3l)] * L.t.B[e2 * Q + g2l][e2 * P + b2l];
            t[g3l] = s;
        }
        const int b12 = (e1 * P + b1l) + n1d * (e2 * P + b2l);
        double* acc = fld < 5 ? &L.av[0][fld][0] : &L.aq[0][fld - 5][0];
#pragma unroll
        for (int b3l = 0; b3l < Q; ++b3l) {
            double s = 0.0;
#pragma unroll
            for (int g3l = 0; g3l < Q; ++g3l) s += t[g3l] * L.t.B[e3 * Q + g3l][e3 * P + b3l];
            acc[b12 + n1d * n1d * (e3 * P + b3l)] += s;
        }
    }
    __syncthreads();
}

// Face part of the rows on face f, sub-face (e1, e2); the test function on the
// face has 2-D factors at the tangential indices (c1, c2).
template <int P>
__device__ void row_face(RowLds<P>& L, const double* __restrict__ coefF, int64_t m, int f, int c1, int c2,
                         int e1, int e2, int k0, bool viscous) {
    using D = Dims<P>;
    using R = RowLds<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, S = D::S, KG = R::KG;
    constexpr int Q = P + 1;
    // one (point, trial field) pair per thread (one coefficient load each)
    const int nff = viscous ? 25 : 10;
    for (int idx = threadIdx.x; idx < R::E2 * nff * KG; idx += blockDim.x) {
        const int sl = idx % R::E2, rest = idx / R::E2;
        const int fld = rest % nff, kk = rest / nff, k = k0 + kk;
        const int s1 = e1 * Q + sl % Q, s2 = e2 * Q + sl / Q;
        const int s = s1 + nq1 * s2;
        const double* c = coefF + (int64_t)m * 6 * S * COEF_F + f * S + s;
        int off;
        if (fld < 5) off = 5 * k + fld;
        else if (fld < 10) off = 25 + 5 * k + (fld - 5);
        else off = 50 + 25 * ((fld - 10) % 3) + 5 * k + (fld - 10) / 3;
        L.w[(kk * 25 + fld) * R::E2 + sl] = L.t.B[s1][c1] * L.t.B[s2][c2] * c[off * 6 * S];
    }
    __syncthreads();
    const int d = face_axis(f), t1 = face_t1(f), t2 = face_t2(f);
    const int ad = face_side(f) ? (n1d - 1) : 0;
    const int nf_ = viscous ? 25 : 10;
    const int nent = KG * nf_ * R::E2;
    for (int idx = threadIdx.x; idx < nent; idx += blockDim.x) {
        const int bl = idx % R::E2, rest = idx / R::E2;
        const int fld = rest % nf_, kk = rest / nf_;
        const int b1 = e1 * P + bl % Q, b2 = e2 * P + bl / Q;
        const double* w = L.w + (kk * 25 + fld) * R::E2;
        double bb1[Q], bb2[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bb1[i] = L.t.B[e1 * Q + i][b1];
            bb2[i] = L.t.B[e2 * Q + i][b2];
        }
        double acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < R::E2; ++sl) acc += w[sl] * (bb1[sl % Q] * bb2[sl / Q]);
        int bi[3];
        bi[d] = ad;
        bi[t1] = b1;
        bi[t2] = b2;
        const int b = bi[0] + n1d * (bi[1] + n1d * bi[2]);
        if (fld < 5) L.av[kk][fld][b] += acc;
        else if (fld < 10) L.ah[kk][f][fld - 5][b1 + n1d * b2] += acc;
        else L.aq[kk][fld - 10][b] += acc;
    }
    __syncthreads();
}

// Eliminate Q and write the KG rows row0 + kk*rstride of B (plus their
// right-hand side entries -R + A_.q A_qq^-1 R_Q).
template <int P>
__device__ void row_write(RowLds<P>& L, double* __restrict__ Bm, int row0, int rstride,
                          const double* __restrict__ minvrq, const double* Rvals, const double hinv[3],
                          bool viscous) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int n1d = D::n1d, n = D::n, nf = D::nf, NV = D::NV, NH = D::NH, KG = RowLds<P>::KG;
    static_assert(KG == 1, "one row per pass");
    double* row = Bm + (int64_t)row0 * BD::ld;
    // V columns (l, b): an item per trial node b, whose index arithmetic and
    // lift coefficients Lam[c][b_j] serve the five fields l; Vhat columns
    // (f, l, e): an item per face node (f, e), the same for the five fields
    for (int t = threadIdx.x; t < n + 6 * nf; t += blockDim.x) {
        if (t < n) {
            const int b = t;
            const int bi[3] = {b % n1d, (b / n1d) % n1d, b / (n1d * n1d)};
            double lam[3][n1d];
            int base[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int stride = j == 0 ? 1 : (j == 1 ? n1d : n1d * n1d);
                base[j] = b - bi[j] * stride;
#pragma unroll
                for (int c = 0; c < n1d; ++c) lam[j][c] = L.t.Lam[c][bi[j]];
            }
#pragma unroll
            for (int l = 0; l < 5; ++l) {
                double val = L.av[0][l][b];
                if (viscous) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const int stride = j == 0 ? 1 : (j == 1 ? n1d : n1d * n1d);
                        const double* aq = &L.aq[0][3 * l + j][base[j]];
                        double acc = 0.0;
#pragma unroll
                        for (int c = 0; c < n1d; ++c) acc += aq[c * stride] * lam[j][c];
                        val -= hinv[j] * acc;
                    }
                }
                row[l * n + b] = val;
            }
        } else {
            const int f = (t - n) / nf, e = (t - n) % nf;
            const int d = face_axis(f);
            auto stride_of = [](int ax) { return ax == 0 ? 1 : (ax == 1 ? n1d : n1d * n1d); };
            const int iF = face_side(f) ? (n1d - 1) : 0;
            const int dstride = stride_of(d);
            // volume index of face node e with coordinate 0 along the normal
            const int cbase = (e % n1d) * stride_of(face_t1(f)) + (e / n1d) * stride_of(face_t2(f));
            double mv[n1d];
#pragma unroll
            for (int cd = 0; cd < n1d; ++cd) mv[cd] = L.t.Minv[cd][iF];
            const double sh = face_sign(f) * hinv[d];
#pragma unroll
            for (int l = 0; l < 5; ++l) {
                double val = L.ah[0][f][l][e];
                if (viscous) {
                    const double* aq = &L.aq[0][3 * l + d][cbase];
                    double acc = 0.0;
#pragma unroll
                    for (int cd = 0; cd < n1d; ++cd) acc += aq[cd * dstride] * mv[cd];
                    val += sh * acc;
                }
                row[NV + (f * 5 + l) * nf + e] = val;
            }
        }
    }
    // padding columns after the right-hand side
    for (int col = NV + NH + 1 + threadIdx.x; col < BD::ld; col += blockDim.x) row[col] = 0.0;
    // right-hand sides
    double part[KG];
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) part[kk] = 0.0;
    if (viscous)
        for (int i = threadIdx.x; i < 15 * n; i += blockDim.x) {
            const double mr = minvrq[i];
#pragma unroll
            for (int kk = 0; kk < KG; ++kk) part[kk] += (&L.aq[kk][0][0])[i] * mr;
        }
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
        double v = part[kk];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) L.red[kk][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < KG) {
        const int kk = threadIdx.x;
        double s = 0.0;
        for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += L.red[kk][i];
        Bm[(int64_t)(row0 + kk * rstride) * BD::ld + NV + NH] = -Rvals[kk] + s;
    }
    __syncthreads();
}

template <int P>
__device__ void stage_tables(RowLds<P>& L, const Tab1D* __restrict__ tab) {
    const double* src = reinterpret_cast<const double*>(tab);
    double* dst = reinterpret_cast<double*>(&L.t);
    for (int i = threadIdx.x; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
}

// Rows of the interior equations: one workgroup per (macro, node a), 5 rows;
// the workgroups of a macro share one XCD, whose L2 then serves the
// coefficient slabs they all read.
template <int P>
__global__ void __launch_bounds__(RowCfg<P>::THREADS, 4) k_rows_v(const double* __restrict__ coefV,
                                                               const double* __restrict__ coefF,
                                                               const double* __restrict__ R_v,
                                                               const double* __restrict__ minvrq,
                                                               const double* __restrict__ hs,
                                                               const Tab1D* __restrict__ tab, int viscous_i,
                                                               double* __restrict__ B, int64_t n_macro) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int n1d = D::n1d, n = D::n, KG = RowLds<P>::KG;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowLds<P>& L = *reinterpret_cast<RowLds<P>*>(smem_raw);
    int64_t m;
    int a;
    xcd_tile(n, m, a);
    if (m >= n_macro) return;
    const bool viscous = viscous_i != 0;
    const int a1 = a % n1d, a2 = (a / n1d) % n1d, a3 = a / (n1d * n1d);
    const double hinv[3] = {1.0 / hs[3 * m], 1.0 / hs[3 * m + 1], 1.0 / hs[3 * m + 2]};
    stage_tables<P>(L, tab);
    int lo[3], hi[3];
    support_1d<P>(a1, lo[0], hi[0]);
    support_1d<P>(a2, lo[1], hi[1]);
    support_1d<P>(a3, lo[2], hi[2]);
    const int ai[3] = {a1, a2, a3};
    for (int k0 = 0; k0 < 5; k0 += KG) {
        row_zero<P>(L);
        __syncthreads();
        for (int e3 = lo[2]; e3 <= hi[2]; ++e3)
            for (int e2 = lo[1]; e2 <= hi[1]; ++e2)
                for (int e1 = lo[0]; e1 <= hi[0]; ++e1)
                    row_volume<P>(L, coefV, m, a1, a2, a3, e1, e2, e3, k0, viscous);
        for (int f = 0; f < 6; ++f) {
            const int d = face_axis(f);
            if (ai[d] != (face_side(f) ? n1d - 1 : 0)) continue;
            const int c1 = ai[face_t1(f)], c2 = ai[face_t2(f)];
            int l1, u1, l2, u2;
            support_1d<P>(c1, l1, u1);
            support_1d<P>(c2, l2, u2);
            for (int e2 = l2; e2 <= u2; ++e2)
                for (int e1 = l1; e1 <= u1; ++e1) row_face<P>(L, coefF, m, f, c1, c2, e1, e2, k0, viscous);
        }
        double Rv[KG];
#pragma unroll
        for (int kk = 0; kk < KG; ++kk) Rv[kk] = R_v[(m * 5 + k0 + kk) * n + a];
        row_write<P>(L, B + m * BD::per_macro, k0 * n + a, n, minvrq + m * 15 * n, Rv, hinv, viscous);
    }
}

// Rows of the trace equations: one workgroup per (macro, face f, trace node c), 5 rows.
// The test function of such a row lives on face f, so the row couples to v and
// q only through the nf nodes of that face and to vhat only on that face: the
// accumulators are stored face-compact (index e = b_t1 + n1d b_t2 over the
// face's tangential axes), a quarter of the LDS of a volume row, so more
// workgroups share a CU.  The elimination of Q is the same as in row_write,
// with the off-face entries read as zero.
// (trace rows: 256 threads at every degree, measured fastest)
template <int P>
struct RowCfgH {
    static constexpr int THREADS = 256;
};

template <int P>
struct RowLdsH {
    using D = Dims<P>;
    static constexpr int E2 = (P + 1) * (P + 1);
    double av[5][D::nf];
    double aq[15][D::nf];
    double ah[5][D::nf];
    double w[E2 * 25];
    double red[RowCfgH<P>::THREADS / 64];
    Tab1D t;
};

template <int P>
__device__ void row_face_h(RowLdsH<P>& L, const double* __restrict__ coefF, int64_t m, int f, int c1, int c2,
                           int e1, int e2, int k, bool viscous) {
    using D = Dims<P>;
    using R = RowLdsH<P>;
    constexpr int n1d = D::n1d, nq1 = D::nq1, S = D::S;
    constexpr int Q = P + 1;
    // one (point, trial field) pair per thread (one coefficient load each)
    const int nf_ = viscous ? 25 : 10;
    for (int idx = threadIdx.x; idx < R::E2 * nf_; idx += blockDim.x) {
        const int sl = idx % R::E2, fld = idx / R::E2;
        const int s1 = e1 * Q + sl % Q, s2 = e2 * Q + sl / Q;
        const int s = s1 + nq1 * s2;
        const double* c = coefF + (int64_t)m * 6 * S * COEF_F + f * S + s;
        int off;
        if (fld < 5) off = 5 * k + fld;
        else if (fld < 10) off = 25 + 5 * k + (fld - 5);
        else off = 50 + 25 * ((fld - 10) % 3) + 5 * k + (fld - 10) / 3;
        L.w[fld * R::E2 + sl] = L.t.B[s1][c1] * L.t.B[s2][c2] * c[off * 6 * S];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nf_ * R::E2; idx += blockDim.x) {
        const int bl = idx % R::E2, fld = idx / R::E2;
        const int b1 = e1 * P + bl % Q, b2 = e2 * P + bl / Q;
        const double* w = L.w + fld * R::E2;
        double bb1[Q], bb2[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            bb1[i] = L.t.B[e1 * Q + i][b1];
            bb2[i] = L.t.B[e2 * Q + i][b2];
        }
        double acc = 0.0;
#pragma unroll
        for (int sl = 0; sl < R::E2; ++sl) acc += w[sl] * (bb1[sl % Q] * bb2[sl / Q]);
        const int e = b1 + n1d * b2;
        if (fld < 5) L.av[fld][e] += acc;
        else if (fld < 10) L.ah[fld - 5][e] += acc;
        else L.aq[fld - 10][e] += acc;
    }
    __syncthreads();
}

template <int P>
__global__ void __launch_bounds__(RowCfgH<P>::THREADS, 6) k_rows_h(const double* __restrict__ coefF,
                                                               const double* __restrict__ R_vh,
                                                               const double* __restrict__ minvrq,
                                                               const double* __restrict__ hs,
                                                               const Tab1D* __restrict__ tab, int viscous_i,
                                                               double* __restrict__ B, int64_t n_macro) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int n1d = D::n1d, n = D::n, nf = D::nf, NV = D::NV, NH = D::NH;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    RowLdsH<P>& L = *reinterpret_cast<RowLdsH<P>*>(smem_raw);
    int64_t m;
    int fc;
    xcd_tile(6 * nf, m, fc);
    if (m >= n_macro) return;
    const int f = fc / nf, c = fc % nf;
    const bool viscous = viscous_i != 0;
    const int c1 = c % n1d, c2 = c / n1d;
    const int d = face_axis(f), ft1 = face_t1(f), ft2 = face_t2(f);
    const int iF = face_side(f) ? (n1d - 1) : 0;
    const double hinv[3] = {1.0 / hs[3 * m], 1.0 / hs[3 * m + 1], 1.0 / hs[3 * m + 2]};
    {
        const double* src = reinterpret_cast<const double*>(tab);
        double* dst = reinterpret_cast<double*>(&L.t);
        for (int i = threadIdx.x; i < (int)(sizeof(Tab1D) / 8); i += blockDim.x) dst[i] = src[i];
    }
    int l1, u1, l2, u2;
    support_1d<P>(c1, l1, u1);
    support_1d<P>(c2, l2, u2);
    double* Bm = B + m * BD::per_macro;
    const double* mrq = minvrq + m * 15 * n;
    for (int k = 0; k < 5; ++k) {
        for (int i = threadIdx.x; i < 25 * nf; i += blockDim.x) (&L.av[0][0])[i] = 0.0;   // av, aq, ah
        __syncthreads();
        for (int e2 = l2; e2 <= u2; ++e2)
            for (int e1 = l1; e1 <= u1; ++e1) row_face_h<P>(L, coefF, m, f, c1, c2, e1, e2, k, viscous);
        const int64_t row = NV + (f * 5 + k) * nf + c;
        double* rowp = Bm + row * BD::ld;
        // an item per trial node b (the five V columns (l, b)) or per face node
        // (fp, e) (the five Vhat columns (fp, l, e)): index arithmetic and lift
        // coefficients once per item
        for (int t = threadIdx.x; t < n + 6 * nf; t += blockDim.x) {
            if (t < n) {
                const int b = t;
                const int bi[3] = {b % n1d, (b / n1d) % n1d, b / (n1d * n1d)};
                const int t1 = bi[ft1], t2 = bi[ft2];
                const int e = t1 + n1d * t2;
                const bool on = bi[d] == iF;
                const double lamd = L.t.Lam[iF][bi[d]];
#pragma unroll
                for (int l = 0; l < 5; ++l) {
                    double val = 0.0;
                    if (on) val = L.av[l][e];
                    if (viscous) {
                        // lift along the normal axis: the line meets the face in one node
                        val -= hinv[d] * (L.aq[3 * l + d][e] * lamd);
                        // lifts along the face: only for nodes of the face
                        if (on) {
                            double a1 = 0.0, a2 = 0.0;
#pragma unroll
                            for (int cc = 0; cc < n1d; ++cc) {
                                a1 += L.aq[3 * l + ft1][cc + n1d * t2] * L.t.Lam[cc][t1];
                                a2 += L.aq[3 * l + ft2][t1 + n1d * cc] * L.t.Lam[cc][t2];
                            }
                            val -= hinv[ft1] * a1;
                            val -= hinv[ft2] * a2;
                        }
                    }
                    rowp[l * n + b] = val;
                }
            } else {
                const int fp = (t - n) / nf, e = (t - n) % nf;
                const int dp = face_axis(fp);
                const int iFp = face_side(fp) ? (n1d - 1) : 0;
                const double sh = face_sign(fp) * hinv[dp];
                // faces of the same axis: the line along d meets face f at node e;
                // another face: the line along dp through its node e runs in face f
                // where that node lies on f, at the face-compact indices q0 + cd qs
                const int u = e % n1d, v = e / n1d;
                bool meets = false;
                int q0 = 0, qs = 1;
                if (dp != d) {
                    const bool d_is_t1 = d == face_t1(fp);
                    const int cx = d_is_t1 ? v : u;       // coordinate along the third axis
                    meets = (d_is_t1 ? u : v) == iF;
                    if (ft1 == dp) q0 = n1d * cx;
                    else {
                        q0 = cx;
                        qs = n1d;
                    }
                }
                double mv[n1d];
#pragma unroll
                for (int cd = 0; cd < n1d; ++cd) mv[cd] = L.t.Minv[cd][iFp];
                const double mff = L.t.Minv[iF][iFp];
#pragma unroll
                for (int l = 0; l < 5; ++l) {
                    double val = 0.0;
                    if (fp == f) val = L.ah[l][e];
                    if (viscous) {
                        double acc = 0.0;
                        if (dp == d) {
                            acc = L.aq[3 * l + d][e] * mff;
                        } else if (meets) {
#pragma unroll
                            for (int cd = 0; cd < n1d; ++cd) acc += L.aq[3 * l + dp][q0 + cd * qs] * mv[cd];
                        }
                        val += sh * acc;
                    }
                    rowp[NV + (fp * 5 + l) * nf + e] = val;
                }
            }
        }
        // padding columns after the right-hand side
        for (int col = NV + NH + 1 + threadIdx.x; col < BD::ld; col += blockDim.x) rowp[col] = 0.0;
        // right-hand side -R_Vhat + A_hq A_qq^-1 R_Q (only face nodes of q contribute)
        double part = 0.0;
        if (viscous)
            for (int i = threadIdx.x; i < 15 * nf; i += blockDim.x) {
                const int fld = i / nf, e = i % nf;
                int bi[3];
                bi[d] = iF;
                bi[ft1] = e % n1d;
                bi[ft2] = e / n1d;
                part += L.aq[fld][e] * mrq[fld * n + bi[0] + n1d * (bi[1] + n1d * bi[2])];
            }
        for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
        if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int i = 0; i < (int)(blockDim.x / 64); ++i) s += L.red[i];
            Bm[row * BD::ld + NV + NH] = -R_vh[((m * 6 + f) * 5 + k) * nf + c] + s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Trace rows 2..5 of the wall faces (isothermal no-slip wall: the trace
// equations there are vhat_k, plus gamma/T_wall for the energy row, tested
// against the trace basis).  Those rows depend on nothing but vhat of their
// own face and component, with the face mass matrix
//   M_f[c][c'] = h_t1 h_t2 M1[c1][c1'] M1[c2][c2']
// as coefficients; no q dependence, so no lift terms; right-hand side
// -R_vhat.  One workgroup per (macro, face); written after k_rows_h.
template <int P>
__global__ void __launch_bounds__(256) k_wall_rows(const uint8_t* __restrict__ face_bc,
                                                   const double* __restrict__ R_vh, const double* __restrict__ hs,
                                                   const Tab1D* __restrict__ tab, double* __restrict__ B) {
    using D = Dims<P>;
    using BD = Bdims<P>;
    constexpr int n1d = D::n1d, nf = D::nf, NV = D::NV, NH = D::NH, ld = BD::ld;
    const int64_t m = blockIdx.x / 6;
    const int f = blockIdx.x % 6;
    if (!face_bc[m * 6 + f]) return;
    const double hh = hs[3 * m + face_t1(f)] * hs[3 * m + face_t2(f)];
    double* Bm = B + m * BD::per_macro;
    for (int64_t e = threadIdx.x; e < (int64_t)4 * nf * ld; e += blockDim.x) {
        const int rloc = (int)(e / ld), col = (int)(e % ld);
        const int k = 1 + rloc / nf, c = rloc % nf;
        const int blk = NV + (f * 5 + k) * nf;          // this row's own (face, component) columns
        double val = 0.0;
        if (col == NV + NH) {
            val = -R_vh[((m * 6 + f) * 5 + k) * nf + c];
        } else if (col >= blk && col < blk + nf) {
            const int cp = col - blk;
            val = hh * tab->M1[c % n1d][cp % n1d] * tab->M1[c / n1d][cp / n1d];
        }
        Bm[(int64_t)(blk + c) * ld + col] = val;
    }
}

}  // namespace mehdg
