// Reference tables and index helpers shared by the kernels.
//
// A macro-element is [0,2]^3 in reference coordinates (physical x = x0 + h xi
// per axis), split into 2x2x2 sub-elements.  Along one axis the C0 space has
// n1d = 2P+1 nodes (P+1 Gauss-Lobatto points per sub-interval, the middle
// one shared) and the quadrature has nq1 = 2(P+1) Gauss points (P+1 per
// sub-interval).  Everything 3-D is a tensor product of these 1-D tables.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.hpp"

#define MEHDG_MAXP 4
#define MEHDG_MAXN1D (2 * MEHDG_MAXP + 1)
#define MEHDG_MAXNQ1 (2 * MEHDG_MAXP + 2)

struct Tab1D {
    double B[MEHDG_MAXNQ1][MEHDG_MAXN1D];   // basis at Gauss points
    double D[MEHDG_MAXNQ1][MEHDG_MAXN1D];   // d/dxi at Gauss points
    double w[MEHDG_MAXNQ1];                 // Gauss weights on [0,2]
    double M1[MEHDG_MAXN1D][MEHDG_MAXN1D];  // 1-D mass sum_q w B B
    double Minv[MEHDG_MAXN1D][MEHDG_MAXN1D];  // its inverse
    double Lam[MEHDG_MAXN1D][MEHDG_MAXN1D];   // Minv * C1, C1 = sum_q w D B
};

// status codes written by kernels (subset of mehdg_err)
#define ST_NONPHYSICAL 5
#define ST_NONFINITE 6
#define ST_SINGULAR 7
#define ST_IRNOCONV 8

template <int P>
struct Dims {
    static constexpr int n1d = 2 * P + 1;
    static constexpr int nq1 = 2 * (P + 1);
    static constexpr int n = n1d * n1d * n1d;
    static constexpr int nf = n1d * n1d;
    static constexpr int G = nq1 * nq1 * nq1;
    static constexpr int S = nq1 * nq1;    // quadrature points per macro face
    static constexpr int NV = 5 * n;
    static constexpr int NQ = 15 * n;
    static constexpr int NH = 30 * nf;
};

// Sizes of a tetrahedral macro-element of degree p under the tag P = TET_TAG + p:
// the degree-2p lattice of eight P_p sub-tetrahedra (n nodes, nf per face,
// four faces).  Only the dense condensation kernels, which see NV and NH
// alone, are instantiated with these tags.
constexpr int TET_TAG = 100;
template <int p>
struct TetSizes {
    static constexpr int n = (2 * p + 1) * (2 * p + 2) * (2 * p + 3) / 6;
    static constexpr int nf = (2 * p + 1) * (2 * p + 2) / 2;
    static constexpr int NV = 5 * n;
    static constexpr int NQ = 15 * n;
    static constexpr int NH = 20 * nf;
};
template <>
struct Dims<TET_TAG + 1> : TetSizes<1> {};
template <>
struct Dims<TET_TAG + 2> : TetSizes<2> {};
template <>
struct Dims<TET_TAG + 3> : TetSizes<3> {};

// face f: normal axis, side (0: xi = 0, outward normal -e_d; 1: xi = 2, +e_d)
__host__ __device__ __forceinline__ int face_axis(int f) { return f >> 1; }
__host__ __device__ __forceinline__ int face_side(int f) { return f & 1; }
__host__ __device__ __forceinline__ double face_sign(int f) { return (f & 1) ? 1.0 : -1.0; }
// tangential axes of a face in increasing order
__host__ __device__ __forceinline__ int face_t1(int f) { return face_axis(f) == 0 ? 1 : 0; }
__host__ __device__ __forceinline__ int face_t2(int f) { return face_axis(f) == 2 ? 1 : 2; }

// sub-interval range [lo, hi] (inclusive, in {0,1}) of the 1-D basis function i
template <int P>
__device__ __forceinline__ void support_1d(int i, int& lo, int& hi) {
    lo = (i <= P) ? 0 : 1;
    hi = (i >= P) ? 1 : 0;
}

// Per-macro status: the most basic condition is kept, i.e. the smallest
// non-zero code (non-physical before non-finite before singular), so a
// zero pivot caused by a non-physical state still reports the state.
__device__ __forceinline__ void record_status(int32_t* status, int64_t m, int code) {
    if (!status) return;
    int* p = reinterpret_cast<int*>(status + m);
    int old = atomicAdd(p, 0);
    while (old == 0 || code < old) {
        const int prev = atomicCAS(p, old, code);
        if (prev == old) break;
        old = prev;
    }
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Workgroups of one macro-element run on one XCD (and share its L2): the
// hardware deals workgroups to the eight XCDs in turn, so workgroup b is tile
// (b / 8) % tiles of macro ((b / 8) / tiles) * 8 + b % 8.  The grid has
// ceil(n / 8) * 8 * tiles workgroups; m >= n marks an idle one.
__device__ __forceinline__ void xcd_tile(int tiles, int64_t& m, int& tile) {
    const unsigned b = blockIdx.x, x = b & 7u, loc = b >> 3;
    m = (int64_t)(loc / (unsigned)tiles) * 8 + x;
    tile = (int)(loc % (unsigned)tiles);
}

inline unsigned xcd_grid(int tiles, int64_t n) { return (unsigned)(((n + 7) / 8) * 8 * tiles); }
