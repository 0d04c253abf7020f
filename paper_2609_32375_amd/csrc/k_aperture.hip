// k_aperture.hip -- circular aperture photometry with exact pixel/disk overlap.
//
// One wavefront per catalogued object.  The rows of the object's box are taken
// in bands of 16: the band's background and noise-map cubics are built in LDS
// (FP64 -> working precision), the pixels the outer circle can touch are
// numbered run by run and spread over the lanes, and each lane forms M = I - B
// for its pixels and classifies them against every circle (the aperture radii,
// r_in and r_out).  Pixels wholly inside or outside a circle take weight 1 or
// 0; the rest get the exact area of the circle inside the pixel from a
// cancellation-free formula: clipped rectangle + trapezoid under the chord +
// circular segment (theta - sin theta by series for small angles).
//
// The paper measures fluxes in circular apertures of several radii with the
// variance propagated through the same weights and float64 accumulation; the
// annulus background is this path's addition.
#include "k_args.h"
#include "k_overlap.h"
#include "k_rowpoly.h"

namespace gpk {

constexpr int kApBand = 17;    // rows per band (two bands cover the 34-row box of r_max <= 15)
constexpr int kApBox = 2 * 66; // widest box (r <= 64)
constexpr int kApWaves = 4;

constexpr int kApList = 128;   // queued (pixel, circle) cuts per wavefront
constexpr int kApUnroll = 2;   // pixels per lane in flight
constexpr int kApMaxFrames = kMaxFramesPerCall;   // object-count prefix over the frames, in LDS
constexpr int kApPrefixBytes = (int)((sizeof(int32_t) * (kApMaxFrames + 1) + 15) / 16 * 16);

template <typename Real>
struct ApEntry {
    Real dx, dy, m, var;
    int32_t j;
};

// Per-wavefront LDS layout (dynamic shared memory; the host sizes it from the
// number of spline pieces a box can touch).  Bin sums are per lane, bin-major,
// so a lane's read-modify-write of its bin never conflicts with another lane.
template <typename Real, int NC>
struct ApLayout {
    int o_s, o_a, o_v, o_colp, o_cols, o_rxl, o_roff, o_tab, o_list, o_rad, bytes;
    __host__ __device__ ApLayout(int band, int nixmax) {
        int o = 0;
        auto take = [&](int n, int al) {
            o = (o + al - 1) / al * al;
            const int r = o;
            o += n;
            return r;
        };
        o_s = take(NC * 64 * 8, 16);
        o_a = take(NC * 64 * 8, 16);
        o_v = take(NC * 64 * 8, 16);
        o_colp = take(kApBox * 4, 16);
        o_cols = take(kApBox * (int)sizeof(Real), 16);
        o_rxl = take(band * 4, 16);
        o_roff = take((band + 1) * 4, 16);
        o_tab = take(band * nixmax * (int)sizeof(RowT<Real>), 16);
        o_list = take(kApList * (int)sizeof(ApEntry<Real>), 16);
        o_rad = take(NC * (int)sizeof(Real), 16);
        bytes = (o + 15) / 16 * 16;
    }
};

// Circles: the aperture radii, r_in and r_out, sorted by radius on the host
// (a.crad / a.crole).  Circles are nested, so a pixel lies wholly inside every
// circle from some index kin on, wholly outside those before kout, and only
// the circles in [kout, kin) cut it (usually none or one).  A wholly-inside
// pixel adds (M, 1, var) to bin kin; the circle sums are prefix sums over the
// bins.  A cut pixel is queued and, in a compacted lane-parallel pass, adds
// its exact weight w as (w M, w, w^2 var) to bin j and subtracts it from bin
// j + 1, so that only circle j sees it.
//
// Only the pixels the outer circle can touch are visited: each row of the box
// contributes the run of columns within half a pixel plus the chord of the
// outer circle, and the runs of a band of rows are numbered consecutively and
// spread over the lanes.  Sums are kept per lane (FP64: flux, area, variance) and
// reduced in a fixed order, so an object's result does not depend on what else
// runs.
// ONE: a one-frame call, whose descriptor comes with the launch (d1) instead
// of from the workspace table
template <typename Real, int NC, bool ONE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(Real) == 4 ? 3 : 1))) void k_aperture(const FrameDesc* __restrict__ desc, FrameDesc d1, ApArgs a, ApCat cat,
                                                  int band, int nixmax) {
    extern __shared__ __align__(16) unsigned char ap_dyn[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const ApLayout<Real, NC> L(band, nixmax);
    int32_t* fpre = reinterpret_cast<int32_t*>(ap_dyn);     // kApPrefixBytes
    unsigned char* base = ap_dyn + kApPrefixBytes + (size_t)wv * L.bytes;
    double* binS = (double*)(base + L.o_s);
    double* binA = (double*)(base + L.o_a);
    double* binV = (double*)(base + L.o_v);
    int32_t* colp = (int32_t*)(base + L.o_colp);
    Real* cols = (Real*)(base + L.o_cols);
    int32_t* rxl = (int32_t*)(base + L.o_rxl);
    int32_t* roff = (int32_t*)(base + L.o_roff);
    RowT<Real>* tab = (RowT<Real>*)(base + L.o_tab);
    ApEntry<Real>* list = (ApEntry<Real>*)(base + L.o_list);
    Real* rad = (Real*)(base + L.o_rad);
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));

    Real cr[NC], cr2[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        cr[j] = (Real)a.crad[j];
        cr2[j] = cr[j] * cr[j];
    }
    const Real rmax = cr[NC - 1], rmax2 = cr2[NC - 1];
    const int R = (int)ceilf(a.rmax) + 1;
    const int side = 2 * R + 2;
    const Real inv_gain = (a.gain > 0.f) ? (Real)1 / (Real)a.gain : (Real)0;
    // radius by circle index for the cut-pixel pass (a lane-varying index)
#pragma unroll
    for (int j = 0; j < NC; ++j)
        if (lane == j) rad[j] = cr[j];

    // The catalogued objects of all frames, numbered consecutively (frame by
    // frame, rows < n_obj only), are split into 8 contiguous ranges, one per
    // XCD: neighbouring objects, whose boxes overlap, share that XCD's L2.
    const int nf = a.nframes;
    if (wv == 0) {
        // prefix of min(n_obj, capacity) over the frames (one wavefront)
        constexpr int PER = kApMaxFrames / 64;
        int t = 0;
        for (int q = 0; q < PER; ++q) {
            const int fr = lane * PER + q;
            if (fr < nf) t += min(cat.n_obj[fr], a.capacity);
        }
        int incl = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        int run = incl - t;
        for (int q = 0; q < PER; ++q) {
            const int fr = lane * PER + q;
            fpre[fr] = run;
            if (fr < nf) run += min(cat.n_obj[fr], a.capacity);
        }
        if (lane == 63) fpre[kApMaxFrames] = incl;
    }
    __syncthreads();
    const int total = fpre[kApMaxFrames];
    const int chunk = (total + kXcds - 1) / kXcds;
    const int xcd = blockIdx.x % kXcds, per_xcd = gridDim.x / kXcds;
    const int o_end = min(total, (xcd + 1) * chunk);
    for (int o = xcd * chunk + (blockIdx.x / kXcds) * nw + wv; o < o_end; o += per_xcd * nw) {
        // frame of object o: last frame whose prefix is <= o
        int lo = 0, hi = nf - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (fpre[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        const int f = lo, k = o - fpre[f];
        const int row = f * a.capacity + k;
        const FrameDesc& d = ONE ? d1 : desc[f];
        const double xc = cat.x[row], yc = cat.y[row];
        const int cxi = (int)floor(xc), cyi = (int)floor(yc);
        const Real fx = (Real)(xc - (double)cxi), fy = (Real)(yc - (double)cyi);
        const int bx0 = cxi - R, by0 = cyi - R;
        const int cx_lo = max(bx0, 0), cx_hi = min(bx0 + side - 1, d.W - 1);
        const int ixlo = (cx_lo <= cx_hi) ? piece_of(cx_lo, d.W, d.mw) : 0;
        const int nix = (cx_lo <= cx_hi) ? min(piece_of(cx_hi, d.W, d.mw) - ixlo + 1, nixmax) : 0;
        wave_sync();
        for (int c = lane; c < side; c += 64) {
            const int px = bx0 + c;
            if (px >= 0 && px < d.W) {
                const int ix = piece_of(px, d.W, d.mw);
                colp[c] = min(ix - ixlo, nixmax - 1);
                cols[c] = (Real)((double)px - piece_ref(ix, d.W, d.mw));
            }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            binS[j * 64 + lane] = 0.0;
            binA[j * 64 + lane] = 0.0;
            binV[j * 64 + lane] = 0.0;
        }
        // queued cuts: pixels within one quadrant from the bottom of the list
        // (listn entries), pixels that straddle an axis through the centre
        // from the top (nstr entries), so that a lane-parallel round of the
        // former evaluates a single quadrant piece
        int listn = 0, nstr = 0;
        auto add_w = [&](const ApEntry<Real>& E, Real w) __attribute__((always_inline)) {
            const double ws = (double)w * (double)E.m;
            const Real wa = w, wvv = w * w * E.var;
            const int i0 = E.j * 64 + lane;
            binS[i0] += ws;
            binA[i0] += (double)wa;
            binV[i0] += (double)wvv;
            if (E.j + 1 < NC) {
                binS[i0 + 64] -= ws;
                binA[i0 + 64] -= (double)wa;
                binV[i0 + 64] -= (double)wvv;
            }
        };
        // exact weights of the queued cut pixels
        auto flush = [&]() __attribute__((always_inline)) {
            wave_sync();
            for (int e = lane; e < listn; e += 64) {
                const ApEntry<Real> E = list[e];
                const Real rj = rad[E.j];
                const Real ax = fabs(E.dx), ay = fabs(E.dy);
                const Real w = quad_area<Real>(ax - (Real)0.5, ax + (Real)0.5, ay - (Real)0.5, ay + (Real)0.5, rj,
                                               rj * rj);
                add_w(E, w);
            }
            for (int e = lane; e < nstr; e += 64) {
                const ApEntry<Real> E = list[kApList - 1 - e];
                const Real rj = rad[E.j];
                add_w(E, pixel_area<Real>(E.dx, E.dy, rj, rj * rj));
            }
            listn = 0;
            nstr = 0;
            wave_sync();
        };
        const int ry0 = max(by0, 0), ry1 = min(by0 + side - 1, d.H - 1);
        for (int band0 = ry0; band0 <= ry1; band0 += band) {
            const int nb = min(band, ry1 - band0 + 1);
            wave_sync();
            // the band's row runs: columns within half a pixel of the outer
            // circle's chord (one pixel of margin each side), clipped to the box
            int cnt = 0, xl = 0;
            if (lane < nb) {
                const int py = band0 + lane;
                const Real dy = (Real)(py - cyi) - fy;
                const Real nyd = fmax(fabs(dy) - (Real)0.5, (Real)0);
                if (nyd < rmax) {
                    const double hw = 0.5 + sqrt(fmax((double)rmax2 - (double)nyd * (double)nyd, 0.0));
                    xl = max(cx_lo, (int)floor(xc - hw) - 1);
                    const int xr = min(cx_hi, (int)ceil(xc + hw) + 1);
                    cnt = max(xr - xl + 1, 0);
                }
            }
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int total = __shfl(incl, nb - 1);
            if (lane < nb) {
                rxl[lane] = xl;
                roff[lane] = incl - cnt;
            }
            if (lane == 0) roff[nb] = total;
            for (int e = lane; e < nb * nix; e += 64) {
                const int rr = e / nix, pi = e - rr * nix;
                const int py = band0 + rr;
                const int jy = piece_of(py, d.H, d.mh);
                const double u = (double)py - piece_ref(jy, d.H, d.mh);
                tab[rr * nixmax + pi] = make_row<Real>(d.coef, d.nx, d.ny, ixlo + pi, jy, u);
            }
            wave_sync();
            // the band's row offsets in registers: a pixel's row is the number
            // of rows that end at or before it (compares, no dependent loads)
            int ro[kApBand + 1];
#pragma unroll
            for (int q = 0; q <= kApBand; ++q) ro[q] = (q <= nb) ? roff[q] : 0x7fffffff;
            for (int b0 = 0; b0 < total; b0 += 64 * kApUnroll) {
                int pxs[kApUnroll], rrs[kApUnroll];
                float iv[kApUnroll];
#pragma unroll
                for (int u = 0; u < kApUnroll; ++u) {
                    const int idx = b0 + u * 64 + lane;
                    rrs[u] = -1;
                    pxs[u] = 0;
                    iv[u] = 0.0f;
                    if (idx < total) {
                        int r = 0, start = 0;
#pragma unroll
                        for (int q = 1; q <= kApBand; ++q) {
                            const bool past = ro[q] <= idx;
                            r += past ? 1 : 0;
                            start = past ? ro[q] : start;
                        }
                        rrs[u] = r;
                        pxs[u] = rxl[r] + (idx - start);
                        iv[u] = load_px(d, pxs[u], band0 + r);
                    }
                }
#pragma unroll
                for (int u = 0; u < kApUnroll; ++u) {
                    const int r_ = rrs[u];
                    const int px = pxs[u], py = band0 + (r_ < 0 ? 0 : r_);
                    const Real dx = (Real)(px - cxi) - fx;
                    const Real dy = (Real)(py - cyi) - fy;
                    const Real ax = fabs(dx), ay = fabs(dy);
                    const Real nxd = fmax(ax - (Real)0.5, (Real)0), nyd = fmax(ay - (Real)0.5, (Real)0);
                    const Real fxd = ax + (Real)0.5, fyd = ay + (Real)0.5;
                    const Real dmin2 = nxd * nxd + nyd * nyd, dmax2 = fxd * fxd + fyd * fyd;
                    const bool use = r_ >= 0 && dmin2 < rmax2;
                    int kin = NC, kout = NC;
                    Real m = 0, var = 0;
                    if (use) {
                        const int c = px - bx0;
                        const RowT<Real> T = tab[r_ * nixmax + colp[c]];
                        const Real sx = cols[c];
                        m = eval_M(T, sx, (Real)iv[u]);
                        if (a.want_err) {
                            const Real rv = eval_R(T, sx);
                            var = rv * rv + ((m > (Real)0) ? m * inv_gain : (Real)0);
                        }
                        kin = 0;
                        kout = 0;
#pragma unroll
                        for (int j = 0; j < NC; ++j) {
                            kin += (cr2[j] < dmax2) ? 1 : 0;
                            kout += (cr2[j] <= dmin2) ? 1 : 0;
                        }
                        if (kin < NC) {
                            const int i0 = kin * 64 + lane;
                            binS[i0] += (double)m;
                            binA[i0] += 1.0;
                            binV[i0] += (double)var;
                        }
                    }
                    // circles that cut the pixel: queue (pixel, circle) pairs
                    const int ncut = kin - kout;
                    const bool str = ax < (Real)0.5 || ay < (Real)0.5;
                    for (int q = 0;; ++q) {
                        const bool has = q < ncut;
                        const uint64_t bm = __ballot(has && !str), bs = __ballot(has && str);
                        if ((bm | bs) == 0ull) break;
                        if (has) {
                            const int pos = str ? kApList - 1 - (nstr + __popcll(bs & below))
                                                : listn + __popcll(bm & below);
                            list[pos] = ApEntry<Real>{dx, dy, m, var, kout + q};
                        }
                        listn += __popcll(bm);
                        nstr += __popcll(bs);
                        if (listn + nstr > kApList - 64) flush();
                    }
                }
            }
        }
        flush();
        // circle sums: prefix over the bins in each lane (in place), then each
        // of the 3 NC totals summed over the lanes in a fixed order
        {
            double ps = 0.0, pa = 0.0, pv = 0.0;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int i0 = j * 64 + lane;
                ps += binS[i0];
                pa += binA[i0];
                pv += binV[i0];
                binS[i0] = ps;
                binA[i0] = pa;
                binV[i0] = pv;
            }
        }
        wave_sync();
        constexpr int Q = 3 * NC;
        constexpr int Q2 = (Q <= 16) ? 16 : 32;
        constexpr int G = 64 / Q2;          // lanes per total
        constexpr int SPAN = 64 / G;        // lane slots each of them sums
        double part = 0.0;
        {
            const int q = lane / G, g = lane - q * G;
            if (q < Q) {
                const int j = (q < NC) ? q : (q < 2 * NC ? q - NC : q - 2 * NC);
                const int s0 = j * 64 + g * SPAN;
                if (q < NC) {
                    for (int t = 0; t < SPAN; ++t) part += binS[s0 + t];
                } else {
                    const double* src = (q < 2 * NC) ? binA : binV;
                    for (int t = 0; t < SPAN; ++t) part += (double)src[s0 + t];
                }
            }
#pragma unroll
            for (int o = G / 2; o >= 1; o >>= 1) {
                const double w = __shfl_xor(part, o);
                part = ((lane & o) == 0) ? part + w : w + part;
            }
        }
        double S[NC], A[NC], V[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            S[j] = __shfl(part, j * G);
            A[j] = __shfl(part, (NC + j) * G);
            V[j] = a.want_err ? __shfl(part, (2 * NC + j) * G) : 0.0;
        }
        double Sin = 0, Ain = 0, Sout = 0, Aout = 0;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const int role = a.crole[j];
            if (role == kMaxRadii) {
                Sin = S[j];
                Ain = A[j];
            } else if (role == kMaxRadii + 1) {
                Sout = S[j];
                Aout = A[j];
            }
        }
        const double Aa = Aout - Ain, Sa = Sout - Sin;
        const double bk = (Aa > 0.0) ? Sa / Aa : 0.0;
        if (lane == 0) {
            const int nr = a.nr;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                const int q = a.crole[j];
                if (q < nr) {
                    cat.area[(size_t)row * nr + q] = A[j];
                    cat.flux[(size_t)row * nr + q] = S[j] - bk * A[j];
                    if (a.want_err && cat.fluxerr) cat.fluxerr[(size_t)row * nr + q] = sqrt(fmax(V[j], 0.0));
                }
            }
            cat.bkg[row] = bk;
            const double rm = (double)a.rmax;
            if (xc - rm < -0.5 || xc + rm > (double)d.W - 0.5 || yc - rm < -0.5 || yc + rm > (double)d.H - 0.5)
                cat.flags[row] |= kFlagTrunc;
        }
    }
}

template <typename Real, int NC>
static void launch_ap_nc(const FrameDesc* desc, const FrameDesc* one, const ApArgs& a, const ApCat& cat, int blocks,
                         int band, int nixmax, hipStream_t s) {
    const ApLayout<Real, NC> L(band, nixmax);
    // waves per workgroup: as many (up to kApWaves) as keep the workgroup's
    // LDS within 64 KB; the grid keeps the same number of wavefronts
    int nw = kApWaves;
    while (nw > 1 && (size_t)kApPrefixBytes + (size_t)L.bytes * nw > 64 * 1024) nw >>= 1;
    const size_t lds = (size_t)kApPrefixBytes + (size_t)L.bytes * nw;
    const int wg = blocks * (kApWaves / nw);
    const int g = kXcds * std::max(1, (wg + kXcds - 1) / kXcds);
    if (one) k_aperture<Real, NC, true><<<g, 64 * nw, lds, s>>>(desc, *one, a, cat, band, nixmax);
    else k_aperture<Real, NC, false><<<g, 64 * nw, lds, s>>>(desc, FrameDesc{}, a, cat, band, nixmax);
}

template <typename Real>
static void launch_ap_t(const FrameDesc* desc, const FrameDesc* one, const ApArgs& a, const ApCat& cat, int blocks,
                        int band, int nixmax, hipStream_t s) {
    switch (a.nr + 2) {
        case 3: launch_ap_nc<Real, 3>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 4: launch_ap_nc<Real, 4>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 5: launch_ap_nc<Real, 5>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 6: launch_ap_nc<Real, 6>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 7: launch_ap_nc<Real, 7>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 8: launch_ap_nc<Real, 8>(desc, one, a, cat, blocks, band, nixmax, s); break;
        case 9: launch_ap_nc<Real, 9>(desc, one, a, cat, blocks, band, nixmax, s); break;
        default: launch_ap_nc<Real, 10>(desc, one, a, cat, blocks, band, nixmax, s); break;
    }
}

// Pieces a box of `side` columns can touch: knots are one mesh apart except
// the last, which is at least half a mesh from its neighbour, so at most
// (side - 1) / mesh + 2 knots fall inside and the box spans one more piece.
static int ap_nixmax(int side, int mesh, int nmesh) {
    return std::max(1, std::min(nmesh + 1, (side - 1) / std::max(mesh, 1) + 3));
}

void launch_aperture(const FrameDesc* desc, const FrameDesc* one, const ApArgs& a, const ApCat& cat, int total_rows,
                     int blocks, int mesh_w, int max_nx, bool f64, hipStream_t s) {
    if (total_rows <= 0) return;
    const int R = (int)ceilf(a.rmax) + 1;
    const int side = 2 * R + 2;
    const int nixmax = ap_nixmax(side, mesh_w, max_nx);
    const int band = kApBand;
    if (f64) launch_ap_t<double>(desc, one, a, cat, blocks, band, nixmax, s);
    else launch_ap_t<float>(desc, one, a, cat, blocks, band, nixmax, s);
}

}  // namespace gpk
