// Forward-mode dual numbers for device code.
//
// dual<N> carries a value and N tangents.  The pointwise physics below is
// written once as templates over the scalar type; instantiated with double it
// gives values, with dual<N> it gives exact columns of the pointwise
// Jacobians (chain rule, no finite differences).  Non-smooth points use
// d|x|/dx = sign(x) with sign(0) = 0.
#pragma once
#include <hip/hip_runtime.h>

#define MEHDG_HD __host__ __device__ __forceinline__

template <int N>
struct dual {
    double v;
    double d[N];
};

template <int N>
MEHDG_HD dual<N> make_dual(double v) {
    dual<N> r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = 0.0;
    return r;
}

template <int N>
MEHDG_HD dual<N> seed_dual(double v, int dir) {
    dual<N> r = make_dual<N>(v);
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (i == dir) ? 1.0 : 0.0;
    return r;
}

template <int N>
MEHDG_HD dual<N> operator+(const dual<N>& a, const dual<N>& b) {
    dual<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N>
MEHDG_HD dual<N> operator+(const dual<N>& a, double b) {
    dual<N> r = a;
    r.v += b;
    return r;
}
template <int N>
MEHDG_HD dual<N> operator+(double b, const dual<N>& a) { return a + b; }

template <int N>
MEHDG_HD dual<N> operator-(const dual<N>& a) {
    dual<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N>
MEHDG_HD dual<N> operator-(const dual<N>& a, const dual<N>& b) {
    dual<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N>
MEHDG_HD dual<N> operator-(const dual<N>& a, double b) {
    dual<N> r = a;
    r.v -= b;
    return r;
}
template <int N>
MEHDG_HD dual<N> operator-(double b, const dual<N>& a) {
    dual<N> r = -a;
    r.v += b;
    return r;
}

template <int N>
MEHDG_HD dual<N> operator*(const dual<N>& a, const dual<N>& b) {
    dual<N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N>
MEHDG_HD dual<N> operator*(const dual<N>& a, double b) {
    dual<N> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N>
MEHDG_HD dual<N> operator*(double b, const dual<N>& a) { return a * b; }

template <int N>
MEHDG_HD dual<N> operator/(const dual<N>& a, const dual<N>& b) {
    dual<N> r;
    const double inv = 1.0 / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
template <int N>
MEHDG_HD dual<N> operator/(const dual<N>& a, double b) {
    return a * (1.0 / b);
}
template <int N>
MEHDG_HD dual<N> operator/(double a, const dual<N>& b) {
    dual<N> r;
    const double inv = 1.0 / b.v;
    r.v = a * inv;
    const double s = -r.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = s * b.d[i];
    return r;
}

// ---- elementary functions: value overloads for double, chain rule for dual
MEHDG_HD double val(double x) { return x; }
template <int N>
MEHDG_HD double val(const dual<N>& x) { return x.v; }

MEHDG_HD double dexp(double x) { return exp(x); }
MEHDG_HD double dlog(double x) { return log(x); }
MEHDG_HD double dsqrt(double x) { return sqrt(x); }
MEHDG_HD double dabs(double x) { return fabs(x); }
MEHDG_HD double dsqrt_abs(double x) { return sqrt(fabs(x)); }

template <int N>
MEHDG_HD dual<N> dexp(const dual<N>& a) {
    dual<N> r;
    r.v = exp(a.v);
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = r.v * a.d[i];
    return r;
}
template <int N>
MEHDG_HD dual<N> dlog(const dual<N>& a) {
    dual<N> r;
    r.v = log(a.v);
    const double inv = 1.0 / a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * inv;
    return r;
}
template <int N>
MEHDG_HD dual<N> dsqrt(const dual<N>& a) {
    dual<N> r;
    r.v = sqrt(a.v);
    const double s = 0.5 / r.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <int N>
MEHDG_HD dual<N> dabs(const dual<N>& a) {
    const double s = (a.v > 0.0) ? 1.0 : ((a.v < 0.0) ? -1.0 : 0.0);
    return a * s;
}
// sqrt(|x|), derivative sign(x)/(2 sqrt|x|), taken as 0 at x = 0
template <int N>
MEHDG_HD dual<N> dsqrt_abs(const dual<N>& a) {
    dual<N> r;
    r.v = sqrt(fabs(a.v));
    const double s = (r.v > 0.0) ? ((a.v > 0.0 ? 0.5 : -0.5) / r.v) : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * s;
    return r;
}

template <typename T>
MEHDG_HD T select(bool c, const T& a, const T& b) { return c ? a : b; }

template <typename T>
MEHDG_HD T scal(double x) { return T(x); }
