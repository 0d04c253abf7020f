// k_overlap.h -- exact area of a disk inside a pixel, without cancellation.
//
// Used by the circular apertures (arbitrary centres, FP32 or FP64) and by the
// top-hat kernels of the growth curves (FP64 taps).  The area is built from
// the clipped rectangle under the chord, the trapezoid under it and the
// circular segment between chord and arc, whose theta - sin(theta) is taken
// from a series for small angles.
#pragma once
#include "k_common.h"

namespace gpk {

// FP32: hardware reciprocal and square root (about 1 ulp; the per-pixel
// areas need no more); FP64: IEEE division and square root
__device__ __forceinline__ float ap_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double ap_div(double a, double b) { return a / b; }
__device__ __forceinline__ float ap_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double ap_sqrt(double x) { return sqrt(x); }

// theta - sin(theta) for theta = 2 asin(s) as a series in s: the derivative
// of asin(s) - s sqrt(1 - s^2) is 2 s^2 / sqrt(1 - s^2), so
//   theta - sin(theta) = 4 sum_n C(2n, n) / (4^n (2n + 3)) s^(2n + 3),
// whose terms fall by about s^2 each: for s < 1/4, 6 terms reach FP32 and 14
// terms FP64 precision.  No asin, no sin, no cancellation.
struct SegSeries {
    double a[14];
    constexpr SegSeries() : a() {
        double c = 1.0;   // C(2n, n) / 4^n
        for (int n = 0; n < 14; ++n) {
            a[n] = 4.0 * c / (2 * n + 3);
            c = c * (2 * n + 1) / (2 * n + 2);
        }
    }
};
constexpr SegSeries kSegSeries{};

template <typename Real>
__device__ __forceinline__ Real seg_series(Real s) {
    constexpr int N = (sizeof(Real) == 8) ? 14 : 6;
    const Real s2 = s * s;
    Real p = (Real)kSegSeries.a[N - 1];
#pragma unroll
    for (int n = N - 2; n >= 0; --n) p = fma(p, s2, (Real)kSegSeries.a[n]);
    return p * s2 * s;
}

// theta - sin(theta) without cancellation for small angles: theta^3/6 times
// the nested series 1 - t^2/20 (1 - t^2/42 (1 - t^2/72 (...))), denominators
// (2k)(2k+1); enough terms for the working precision at theta < 1/2
template <typename Real>
__device__ __forceinline__ Real theta_minus_sin(Real t) {
    if (t < (Real)0.5) {
        const Real t2 = t * t;
        const int nterm = (sizeof(Real) == 8) ? 8 : 5;
        Real p = (Real)1;
        for (int k = nterm; k >= 1; --k) {
            const Real den = (Real)((2 * k + 2) * (2 * k + 3));
            p = (Real)1 - t2 / den * p;
        }
        return t * t2 / (Real)6 * p;
    }
    return t - sin(t);
}

// area of the disk (centre 0, radius r) inside [a0,a1] x [b0,b1], all >= 0
template <typename Real>
__device__ __forceinline__ Real quad_area(Real a0, Real a1, Real b0, Real b1, Real r, Real r2) {
    if (a0 * a0 + b0 * b0 >= r2) return (Real)0;
    if (a1 * a1 + b1 * b1 <= r2) return (a1 - a0) * (b1 - b0);
    const Real uhi = ap_sqrt(fmax(r2 - b0 * b0, (Real)0));   // arc height == b0
    // abscissa where the arc height is b1; when b1 >= r the arc stays below b1
    const Real ulo = (b1 * b1 < r2) ? ap_sqrt(r2 - b1 * b1) : (Real)-1;
    const Real p = fmin(fmax(ulo, a0), a1);
    const Real q = fmin(uhi, a1);
    Real area = (p - a0) * (b1 - b0);
    if (q > p) {
        // arc heights above b0 at p and q: (r^2 - u^2 - b0^2) / (s(u) + b0)
        const Real sp = (p == ulo) ? b1 : ap_sqrt(fmax(r2 - p * p, (Real)0));
        const Real sq = (q == uhi) ? b0 : ap_sqrt(fmax(r2 - q * q, (Real)0));
        const Real hp = (p == ulo) ? (b1 - b0) : ap_div(fma(-p, p, fma(-b0, b0, r2)), sp + b0);
        const Real hq = (q == uhi) ? (Real)0 : ap_div(fma(-q, q, fma(-b0, b0, r2)), sq + b0);
        area += (Real)0.5 * (q - p) * (hp + hq);
        // circular segment between the chord and the arc: half chord over r
        // is the sine of half the angle it subtends
        const Real dxc = q - p, dyc = sp - sq;
        const Real chord = ap_sqrt(dxc * dxc + dyc * dyc);
        const Real sh = fmin(ap_div(chord, (Real)2 * r), (Real)1);
        const Real tms = (sh < (Real)0.25) ? seg_series<Real>(sh) : theta_minus_sin<Real>((Real)2 * asin(sh));
        area += (Real)0.5 * r2 * tms;
    }
    return area;
}

// area of disk(0, r) inside the unit pixel centred at (dx, dy)
template <typename Real>
__device__ __forceinline__ Real pixel_area(Real dx, Real dy, Real r, Real r2) {
    const Real ax = fabs(dx), ay = fabs(dy);
    const Real nx = fmax(ax - (Real)0.5, (Real)0), ny = fmax(ay - (Real)0.5, (Real)0);
    if (nx * nx + ny * ny >= r2) return (Real)0;
    const Real fx = ax + (Real)0.5, fy = ay + (Real)0.5;
    if (fx * fx + fy * fy <= r2) return (Real)1;
    const Real x0 = ax - (Real)0.5, x1 = ax + (Real)0.5;
    const Real y0 = ay - (Real)0.5, y1 = ay + (Real)0.5;
    // split at the axes (only pixels within half a pixel of the centre line)
    Real xa[2], xb[2], ya[2], yb[2];
    int nxp = 0, nyp = 0;
    if (x0 < 0) {
        xa[nxp] = 0; xb[nxp++] = -x0;
        xa[nxp] = 0; xb[nxp++] = x1;
    } else {
        xa[nxp] = x0; xb[nxp++] = x1;
    }
    if (y0 < 0) {
        ya[nyp] = 0; yb[nyp++] = -y0;
        ya[nyp] = 0; yb[nyp++] = y1;
    } else {
        ya[nyp] = y0; yb[nyp++] = y1;
    }
    Real a = 0;
    for (int i = 0; i < nxp; ++i)
        for (int j = 0; j < nyp; ++j)
            if (xb[i] > xa[i] && yb[j] > ya[j]) a += quad_area<Real>(xa[i], xb[i], ya[j], yb[j], r, r2);
    return a;
}

}  // namespace gpk
