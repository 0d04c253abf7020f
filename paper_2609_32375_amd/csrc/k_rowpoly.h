// k_rowpoly.h -- evaluation of the spline background B and noise map R.
//
// The background buffer stores the tensor natural spline as bicubic pieces
// (FP64).  A kernel that needs B or R along an image row first reduces the
// piece to a cubic in x for that row (FP64, once per row and piece), then
// evaluates the cubic per pixel in the working precision.  For FP32 the
// constant term is kept as an unevaluated hi+lo pair, so M = I - B keeps the
// background to ~1e-6 ADU even though B itself is ~1e3 ADU.
#pragma once
#include "k_common.h"

namespace gpk {

template <typename Real>
struct RowT;
template <>
struct RowT<float> {
    float a0h, a0l, a1, a2, a3;  // background: a0h + a0l + a1 s + a2 s^2 + a3 s^3
    float r0, r1, r2, r3;        // noise map
};
template <>
struct RowT<double> {
    double a0, a1, a2, a3;
    double r0, r1, r2, r3;
};

__device__ __forceinline__ void piece_row(const double* __restrict__ coef, int nx, int ny, int q, int ix,
                                          int jy, double u, double a[4]) {
    gdouble_t* P = (gdouble_t*)coef + (((size_t)q * (ny + 1) + jy) * (nx + 1) + ix) * 16;
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = ((P[p * 4 + 3] * u + P[p * 4 + 2]) * u + P[p * 4 + 1]) * u + P[p * 4];
}

template <typename Real>
__device__ __forceinline__ RowT<Real> make_row(const double* coef, int nx, int ny, int ix, int jy, double u);

template <>
__device__ __forceinline__ RowT<float> make_row<float>(const double* coef, int nx, int ny, int ix, int jy,
                                                       double u) {
    double a[4], r[4];
    piece_row(coef, nx, ny, 0, ix, jy, u, a);
    piece_row(coef, nx, ny, 1, ix, jy, u, r);
    RowT<float> t;
    t.a0h = (float)a[0];
    t.a0l = (float)(a[0] - (double)t.a0h);
    t.a1 = (float)a[1];
    t.a2 = (float)a[2];
    t.a3 = (float)a[3];
    t.r0 = (float)r[0];
    t.r1 = (float)r[1];
    t.r2 = (float)r[2];
    t.r3 = (float)r[3];
    return t;
}

template <>
__device__ __forceinline__ RowT<double> make_row<double>(const double* coef, int nx, int ny, int ix, int jy,
                                                         double u) {
    double a[4], r[4];
    piece_row(coef, nx, ny, 0, ix, jy, u, a);
    piece_row(coef, nx, ny, 1, ix, jy, u, r);
    RowT<double> t;
    t.a0 = a[0];
    t.a1 = a[1];
    t.a2 = a[2];
    t.a3 = a[3];
    t.r0 = r[0];
    t.r1 = r[1];
    t.r2 = r[2];
    t.r3 = r[3];
    return t;
}

// M = I - B at local coordinate s of the row's piece
__device__ __forceinline__ float eval_M(const RowT<float>& t, float s, float v) {
    float delta = fmaf(fmaf(t.a3, s, t.a2), s, t.a1) * s;
    return (v - t.a0h) - (t.a0l + delta);
}
__device__ __forceinline__ double eval_M(const RowT<double>& t, double s, double v) {
    return v - (t.a0 + ((t.a3 * s + t.a2) * s + t.a1) * s);
}
__device__ __forceinline__ float eval_R(const RowT<float>& t, float s) {
    return fmaf(fmaf(fmaf(t.r3, s, t.r2), s, t.r1), s, t.r0);
}
__device__ __forceinline__ double eval_R(const RowT<double>& t, double s) {
    return ((t.r3 * s + t.r2) * s + t.r1) * s + t.r0;
}
// background value itself (diagnostics)
__device__ __forceinline__ double eval_B(const RowT<float>& t, float s) {
    float delta = fmaf(fmaf(t.a3, s, t.a2), s, t.a1) * s;
    return (double)t.a0h + (double)(t.a0l + delta);
}
__device__ __forceinline__ double eval_B(const RowT<double>& t, double s) {
    return t.a0 + ((t.a3 * s + t.a2) * s + t.a1) * s;
}

}  // namespace gpk
