// k_aperture.hip -- circular aperture photometry with exact pixel/disk overlap.
//
// One wavefront per catalogued object.  The object's box (every pixel the
// outer circle can touch) is walked in row bands of 16: the band's background
// and noise-map cubics are built in LDS (FP64 -> working precision), then each
// lane takes pixels of the band, forms M = I - B, and for every circle (the
// aperture radii, r_in and r_out) the exact area of the circle inside the
// pixel.  Pixels wholly inside or outside a circle take 1 or 0 directly; the
// rest use a cancellation-free formula: clipped rectangle + trapezoid under the
// chord + circular segment (theta - sin theta by series for small angles).
// Sums are compensated per lane and reduced across the wavefront in a fixed
// order, so an object's result does not depend on what else runs.
//
// The paper measures fluxes in circular apertures of several radii with the
// variance propagated through the same weights and float64 accumulation; the
// annulus background is this path's addition.
#include "k_args.h"
#include "k_rowpoly.h"

namespace gpk {

constexpr int kApBand = 16;    // rows per band
constexpr int kApNix = 12;     // x pieces a box can touch (box <= 132 px, mesh >= 16)
constexpr int kApBox = 2 * 66; // widest box (r <= 64)
constexpr int kApWaves = 4;

// make one wavefront's LDS writes visible to its other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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
    const Real uhi = sqrt(fmax(r2 - b0 * b0, (Real)0));   // arc height == b0
    // abscissa where the arc height is b1; when b1 >= r the arc stays below b1
    const Real ulo = (b1 * b1 < r2) ? sqrt(r2 - b1 * b1) : (Real)-1;
    const Real p = fmin(fmax(ulo, a0), a1);
    const Real q = fmin(uhi, a1);
    Real area = (p - a0) * (b1 - b0);
    if (q > p) {
        // arc heights above b0 at p and q: (r^2 - u^2 - b0^2) / (s(u) + b0)
        const Real sp = (p == ulo) ? b1 : sqrt(fmax(r2 - p * p, (Real)0));
        const Real sq = (q == uhi) ? b0 : sqrt(fmax(r2 - q * q, (Real)0));
        const Real hp = (p == ulo) ? (b1 - b0) : fma(-p, p, fma(-b0, b0, r2)) / (sp + b0);
        const Real hq = (q == uhi) ? (Real)0 : fma(-q, q, fma(-b0, b0, r2)) / (sq + b0);
        area += (Real)0.5 * (q - p) * (hp + hq);
        const Real dxc = q - p, dyc = sp - sq;
        const Real chord = sqrt(dxc * dxc + dyc * dyc);
        const Real th = (Real)2 * asin(fmin(chord / ((Real)2 * r), (Real)1));
        area += (Real)0.5 * r2 * theta_minus_sin(th);
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

template <typename Real>
struct Acc;
template <>
struct Acc<float> {
    F2 v;
    __device__ void zero() { v = F2{0.f, 0.f}; }
    __device__ void add(float x) { f2_acc(v, x); }
    __device__ double reduce() { return f2_d(wave_sum_f2(v)); }
};
template <>
struct Acc<double> {
    double v;
    __device__ void zero() { v = 0.0; }
    __device__ void add(double x) { v += x; }
    __device__ double reduce() { return wave_sum_d(v); }
};

template <typename Real>
struct ApShared {
    RowT<Real> tab[kApWaves][kApBand * kApNix];
    int32_t colp[kApWaves][kApBox];
    Real cols[kApWaves][kApBox];
};

template <typename Real, int NR>
__global__ __launch_bounds__(256) void k_aperture(const FrameDesc* __restrict__ desc, ApArgs a, ApCat cat,
                                                  int total_rows) {
    __shared__ ApShared<Real> sh;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int nr = NR;
    const Real rmax = (Real)a.rmax;
    const int R = (int)ceilf(a.rmax) + 1;
    const int side = 2 * R + 2;
    for (int row = blockIdx.x * kApWaves + wv; row < total_rows; row += gridDim.x * kApWaves) {
        const int f = row / a.capacity, k = row - f * a.capacity;
        const int nobj = min(cat.n_obj[f], a.capacity);
        if (k >= nobj) continue;
        const FrameDesc& d = desc[f];
        const double xc = cat.x[row], yc = cat.y[row];
        const int cxi = (int)floor(xc), cyi = (int)floor(yc);
        const Real fx = (Real)(xc - (double)cxi), fy = (Real)(yc - (double)cyi);
        const int bx0 = cxi - R, by0 = cyi - R;
        // columns of the box inside the frame and their spline pieces
        const int cx_lo = max(bx0, 0), cx_hi = min(bx0 + side - 1, d.W - 1);
        const int ixlo = (cx_lo <= cx_hi) ? piece_of(cx_lo, d.W, d.mw) : 0;
        const int nix = (cx_lo <= cx_hi) ? piece_of(cx_hi, d.W, d.mw) - ixlo + 1 : 0;
        wave_sync();
        for (int c = lane; c < side; c += 64) {
            const int px = bx0 + c;
            if (px >= 0 && px < d.W) {
                const int ix = piece_of(px, d.W, d.mw);
                sh.colp[wv][c] = ix - ixlo;
                sh.cols[wv][c] = (Real)((double)px - piece_ref(ix, d.W, d.mw));
            }
        }
        Acc<Real> sA[NR], sS[NR], sV[NR], aA, aS;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            sA[q].zero();
            sS[q].zero();
            sV[q].zero();
        }
        aA.zero();
        aS.zero();
        const Real rin = (Real)a.r_in, rout = (Real)a.r_out;
        const Real rin2 = rin * rin, rout2 = rout * rout;
        const Real inv_gain = (a.gain > 0.f) ? (Real)1 / (Real)a.gain : (Real)0;
        for (int band = 0; band < side; band += kApBand) {
            const int nb = min(kApBand, side - band);
            wave_sync();
            for (int e = lane; e < nb * nix; e += 64) {
                const int rr = e / nix, pi = e - rr * nix;
                const int py = by0 + band + rr;
                if (py < 0 || py >= d.H) continue;
                const int jy = piece_of(py, d.H, d.mh);
                const double u = (double)py - piece_ref(jy, d.H, d.mh);
                sh.tab[wv][rr * kApNix + pi] = make_row<Real>(d.coef, d.nx, d.ny, ixlo + pi, jy, u);
            }
            wave_sync();
            // pixels of the band, 8 per lane at a time with their loads in flight
            const int npx = nb * side;
            for (int e0 = 0; e0 < npx; e0 += 8 * 64) {
                float vv[8];
                int pxs[8], pys[8];
                bool use[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int e = e0 + j * 64 + lane;
                    const int rr = e / side, c = e - rr * side;
                    pxs[j] = bx0 + c;
                    pys[j] = by0 + band + rr;
                    const Real dx = (Real)(pxs[j] - cxi) - fx, dy = (Real)(pys[j] - cyi) - fy;
                    const Real ax = fmax(fabs(dx) - (Real)0.5, (Real)0), ay = fmax(fabs(dy) - (Real)0.5, (Real)0);
                    use[j] = e < npx && pxs[j] >= 0 && pxs[j] < d.W && pys[j] >= 0 && pys[j] < d.H &&
                             ax * ax + ay * ay < rmax * rmax;
                    vv[j] = use[j] ? load_px(d, pxs[j], pys[j]) : 0.0f;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (!use[j]) continue;
                    const int e = e0 + j * 64 + lane;
                    const int rr = e / side, c = e - rr * side;
                    const Real dx = (Real)(pxs[j] - cxi) - fx, dy = (Real)(pys[j] - cyi) - fy;
                    const RowT<Real>& T = sh.tab[wv][rr * kApNix + sh.colp[wv][c]];
                    const Real s = sh.cols[wv][c];
                    const Real m = eval_M(T, s, (Real)vv[j]);
                    Real var = 0;
                    if (a.want_err) {
                        const Real rr_ = eval_R(T, s);
                        var = rr_ * rr_ + ((m > (Real)0) ? m * inv_gain : (Real)0);
                    }
                    const Real wo = pixel_area<Real>(dx, dy, rout, rout2);
                    const Real wi = (rin > (Real)0) ? pixel_area<Real>(dx, dy, rin, rin2) : (Real)0;
                    const Real wa = wo - wi;
                    if (wa != (Real)0) {
                        aA.add(wa);
                        aS.add(wa * m);
                    }
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const Real rq = (Real)a.radii[q];
                        const Real w = pixel_area<Real>(dx, dy, rq, rq * rq);
                        if (w != (Real)0) {
                            sA[q].add(w);
                            sS[q].add(w * m);
                            if (a.want_err) sV[q].add(w * w * var);
                        }
                    }
                }
            }
        }
        const double Aa = aA.reduce(), Sa = aS.reduce();
        const double b = (Aa > 0.0) ? Sa / Aa : 0.0;
        // the largest circle crosses the frame boundary
        const double rm = (double)a.rmax;
        const bool any_trunc = xc - rm < -0.5 || xc + rm > (double)d.W - 0.5 || yc - rm < -0.5 ||
                               yc + rm > (double)d.H - 0.5;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const double A = sA[q].reduce(), S = sS[q].reduce();
            const double V = a.want_err ? sV[q].reduce() : 0.0;
            if (lane == 0) {
                cat.area[(size_t)row * nr + q] = A;
                cat.flux[(size_t)row * nr + q] = S - b * A;
                if (a.want_err && cat.fluxerr) cat.fluxerr[(size_t)row * nr + q] = sqrt(V);
            }
        }
        if (lane == 0) {
            cat.bkg[row] = b;
            if (any_trunc) cat.flags[row] |= kFlagTrunc;
        }
    }
}

template <typename Real>
static void launch_ap_t(const FrameDesc* desc, const ApArgs& a, const ApCat& cat, int total_rows, int blocks,
                        hipStream_t s) {
    switch (a.nr) {
        case 1: k_aperture<Real, 1><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 2: k_aperture<Real, 2><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 3: k_aperture<Real, 3><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 4: k_aperture<Real, 4><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 5: k_aperture<Real, 5><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 6: k_aperture<Real, 6><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        case 7: k_aperture<Real, 7><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
        default: k_aperture<Real, 8><<<blocks, 256, 0, s>>>(desc, a, cat, total_rows); break;
    }
}

void launch_aperture(const FrameDesc* desc, const ApArgs& a, const ApCat& cat, int total_rows, int blocks,
                     bool f64, hipStream_t s) {
    if (total_rows <= 0) return;
    if (f64) launch_ap_t<double>(desc, a, cat, total_rows, blocks, s);
    else launch_ap_t<float>(desc, a, cat, total_rows, blocks, s);
}

}  // namespace gpk
