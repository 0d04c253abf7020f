// k_growth.hip -- growth curves on top-hat kernels.
//
// For each integer radius r_k the aperture sum of a source is the correlation
// of M = I - B with the top-hat kernel of radius r_k, read at the pixel that
// holds the source's centroid; the noise-map variance R^2 goes through the
// same taps, and every sum is FP64 (Adaptive Aperture Photometry subsection).
// A tap is the exact area of the disk of radius r_k about the kernel's middle
// pixel centre inside the tap's pixel.  The paper evaluates each radius as one
// full-frame correlation (FFT) and keeps its values at the sources; those are
// the values computed here, directly at the sources.
//
// The kernels are nested, so a pixel offset either lies wholly inside the disk
// from some radius on (it joins the running sums there with weight 1: the
// "full" list of that radius) or is cut by one or two circles (each takes it
// with its exact area: the "cut" lists).  sum_k = sum of the full lists j <= k
// plus the cut list k.  k_growth_table builds the lists once per call (FP64
// areas, raster order within each list); k_growth copies them to LDS.
//
// One wavefront per source: it evaluates M (and R^2) over the (2R+1)^2 window
// once into LDS from per-row background cubics, then walks the lists, lane e
// mod 64 taking entry e, and reduces each radius over the lanes in a fixed
// butterfly, so a source's result does not depend on what else runs.
#include "k_args.h"
#include "k_overlap.h"
#include "k_rowpoly.h"

namespace gpk {

constexpr int kGrMaxFrames = kMaxFramesPerCall;
constexpr int kGrPrefixBytes = (int)((sizeof(int32_t) * (kGrMaxFrames + 1) + 15) / 16 * 16);

// pixel offset classes of the nested top-hat kernels (exact in FP64: the
// squared distances are multiples of 1/4)
__device__ __forceinline__ void gr_class(int dx, int dy, double& dmin2, double& dmax2) {
    const double ax = fabs((double)dx), ay = fabs((double)dy);
    const double nx = fmax(ax - 0.5, 0.0), ny = fmax(ay - 0.5, 0.0);
    dmin2 = nx * nx + ny * ny;
    dmax2 = (ax + 0.5) * (ax + 0.5) + (ay + 0.5) * (ay + 0.5);
}

// List L < nr: full list of radius L; L >= nr: cut list of radius L - nr.
// Each wavefront scans the window in raster order for its lists and appends
// with ballots, so the order inside a list is the raster order.
__global__ __launch_bounds__(512) void k_growth_table(GrowArgs a, GrowTab t) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int side = a.side, R = a.R, n2 = side * side;
    for (int L = wv; L < 2 * a.nr; L += nw) {
        const bool full = L < a.nr;
        const int k = full ? L : L - a.nr;
        const double r = (double)a.radii[k], r2 = r * r;
        const double rp2 = (k > 0) ? (double)a.radii[k - 1] * (double)a.radii[k - 1] : -1.0;
        const int beg = full ? a.full_off[k] : a.cut_off[k];
        const int end = full ? a.full_off[k + 1] : a.cut_off[k + 1];
        int run = 0;
        for (int b = 0; b < n2; b += 64) {
            const int i = b + lane;
            bool take = false;
            int wy = 0, wx = 0;
            double dmin2 = 0.0, dmax2 = 0.0;
            if (i < n2) {
                wy = i / side;
                wx = i - wy * side;
                gr_class(wx - R, wy - R, dmin2, dmax2);
                take = full ? (dmax2 <= r2 && dmax2 > rp2) : (dmin2 < r2 && r2 < dmax2);
            }
            const uint64_t bm = __ballot(take);
            const int pos = beg + run + __popcll(bm & below);
            if (take && pos < end) {
                if (full) {
                    t.full[pos] = (wy << 16) | wx;
                } else {
                    t.cut[pos] = (wy << 16) | wx;
                    t.cutw[pos] = pixel_area<double>((double)(wx - R), (double)(wy - R), r, r2);
                }
            }
            run += __popcll(bm);
        }
    }
}

template <typename Real>
struct GrLayout {
    int o_full, o_cut, o_cutw, shared;   // table (whole workgroup), after the frame prefix
    int o_m, o_v, o_tab, o_colp, o_cols, wave;   // per wavefront
    __host__ __device__ GrLayout(int nfull, int ncut, int side, int nixmax, int want_var) {
        int o = kGrPrefixBytes;
        auto take = [&](int n, int al) {
            o = (o + al - 1) / al * al;
            const int r = o;
            o += n;
            return r;
        };
        o_full = take(4 * nfull, 16);
        o_cut = take(4 * ncut, 16);
        o_cutw = take(8 * ncut, 16);
        shared = (o + 15) / 16 * 16;
        o = 0;
        o_m = take(side * side * (int)sizeof(Real), 16);
        o_v = take(want_var ? side * side * (int)sizeof(Real) : 0, 16);
        o_tab = take(side * nixmax * (int)sizeof(RowT<Real>), 16);
        o_colp = take(side * 4, 16);
        o_cols = take(side * (int)sizeof(Real), 16);
        wave = (o + 15) / 16 * 16;
    }
};

constexpr int kGrUnroll = 4;   // window pixels per lane in flight

template <typename Real, bool ONE>
__global__ __launch_bounds__(512) void k_growth(const FrameDesc* __restrict__ desc, FrameDesc d1, GrowArgs a,
                                                GrowTab t, GrowOut g) {
    extern __shared__ __align__(16) unsigned char gr_dyn[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int side = a.side, R = a.R, n2 = side * side, nixmax = a.nixmax, nr = a.nr;
    const GrLayout<Real> L(a.nfull, a.ncut, side, nixmax, a.want_var);
    int32_t* fpre = reinterpret_cast<int32_t*>(gr_dyn);
    int32_t* fl = (int32_t*)(gr_dyn + L.o_full);
    int32_t* cl = (int32_t*)(gr_dyn + L.o_cut);
    double* cw = (double*)(gr_dyn + L.o_cutw);
    unsigned char* base = gr_dyn + L.shared + (size_t)wv * L.wave;
    Real* Mw = (Real*)(base + L.o_m);
    Real* Vw = (Real*)(base + L.o_v);
    RowT<Real>* tab = (RowT<Real>*)(base + L.o_tab);
    int32_t* colp = (int32_t*)(base + L.o_colp);
    Real* cols = (Real*)(base + L.o_cols);

    for (int i = threadIdx.x; i < a.nfull; i += blockDim.x) fl[i] = t.full[i];
    for (int i = threadIdx.x; i < a.ncut; i += blockDim.x) {
        cl[i] = t.cut[i];
        cw[i] = t.cutw[i];
    }
    const int nf = a.nframes;
    if (wv == 0) {
        // prefix of min(n_obj, capacity) over the frames (one wavefront)
        constexpr int PER = kGrMaxFrames / 64;
        int tot = 0;
        for (int q = 0; q < PER; ++q) {
            const int fr = lane * PER + q;
            if (fr < nf) tot += min(g.n_obj[fr], a.capacity);
        }
        int incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        int run = incl - tot;
        for (int q = 0; q < PER; ++q) {
            const int fr = lane * PER + q;
            fpre[fr] = run;
            if (fr < nf) run += min(g.n_obj[fr], a.capacity);
        }
        if (lane == 63) fpre[kGrMaxFrames] = incl;
    }
    __syncthreads();
    const int total = fpre[kGrMaxFrames];
    // sources of all frames, numbered consecutively, in 8 contiguous ranges
    // (one per XCD): neighbouring sources, whose windows overlap, share an L2
    const int chunk = (total + kXcds - 1) / kXcds;
    const int xcd = blockIdx.x % kXcds, per_xcd = gridDim.x / kXcds;
    const int o_end = min(total, (xcd + 1) * chunk);
    for (int o = xcd * chunk + (blockIdx.x / kXcds) * nw + wv; o < o_end; o += per_xcd * nw) {
        int lo = 0, hi = nf - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (fpre[mid] <= o) lo = mid;
            else hi = mid - 1;
        }
        const int f = lo, row = f * a.capacity + (o - fpre[f]);
        const FrameDesc& d = ONE ? d1 : desc[f];
        const double fx = floor(g.x[row] + 0.5), fy = floor(g.y[row] + 0.5);
        // a pixel so far out that no tap reaches the frame (or not a number):
        // zero sums
        const bool reach = fx >= -(double)R - 1.0 && fx <= (double)d.W + R && fy >= -(double)R - 1.0 &&
                           fy <= (double)d.H + R;
        const int cx = reach ? (int)fx : 0, cy = reach ? (int)fy : 0;
        const int bx0 = cx - R, by0 = cy - R;
        // the frame inside the window, in window coordinates
        const int wx_lo = max(0, -bx0), wx_hi = min(side - 1, d.W - 1 - bx0);
        const int wy_lo = max(0, -by0), wy_hi = min(side - 1, d.H - 1 - by0);
        const bool any = reach && wx_lo <= wx_hi && wy_lo <= wy_hi;
        double my_s = 0.0, my_v = 0.0, my_a = 0.0;
        if (any) {
            const int cx_lo = bx0 + wx_lo, cx_hi = bx0 + wx_hi;
            const int ixlo = piece_of(cx_lo, d.W, d.mw);
            const int nix = min(piece_of(cx_hi, d.W, d.mw) - ixlo + 1, nixmax);
            wave_sync();
            for (int c = lane; c < side; c += 64) {
                const int px = bx0 + c;
                if (px >= 0 && px < d.W) {
                    const int ix = piece_of(px, d.W, d.mw);
                    colp[c] = min(ix - ixlo, nixmax - 1);
                    cols[c] = (Real)((double)px - piece_ref(ix, d.W, d.mw));
                }
            }
            const int nrow = wy_hi - wy_lo + 1;
            for (int e = lane; e < nrow * nix; e += 64) {
                const int rr = e / nix, pi = e - rr * nix;
                const int py = by0 + wy_lo + rr;
                const int jy = piece_of(py, d.H, d.mh);
                const double u = (double)py - piece_ref(jy, d.H, d.mh);
                tab[(wy_lo + rr) * nixmax + pi] = make_row<Real>(d.coef, d.nx, d.ny, ixlo + pi, jy, u);
            }
            wave_sync();
            // M (and R^2) over the window; zero off the frame
            for (int b = 0; b < n2; b += 64 * kGrUnroll) {
                int wi[kGrUnroll], wyv[kGrUnroll], wxv[kGrUnroll];
                bool in[kGrUnroll];
                float iv[kGrUnroll];
#pragma unroll
                for (int u = 0; u < kGrUnroll; ++u) {
                    const int i = b + u * 64 + lane;
                    wi[u] = i;
                    const int wy = (int)(((uint32_t)i * (uint32_t)a.div_magic) >> 20);
                    const int wx = i - wy * side;
                    wyv[u] = wy;
                    wxv[u] = wx;
                    in[u] = i < n2 && wx >= wx_lo && wx <= wx_hi && wy >= wy_lo && wy <= wy_hi;
                    iv[u] = in[u] ? load_px(d, bx0 + wx, by0 + wy) : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kGrUnroll; ++u) {
                    if (wi[u] >= n2) continue;
                    Real m = (Real)0, v = (Real)0;
                    if (in[u]) {
                        const RowT<Real> T = tab[wyv[u] * nixmax + colp[wxv[u]]];
                        const Real sx = cols[wxv[u]];
                        m = eval_M(T, sx, (Real)iv[u]);
                        if (a.want_var) {
                            const Real rv = eval_R(T, sx);
                            v = rv * rv;
                        }
                    }
                    Mw[wi[u]] = m;
                    if (a.want_var) Vw[wi[u]] = v;
                }
            }
            wave_sync();
            double sm = 0.0, sv = 0.0, sa = 0.0;   // this lane's share of the full lists so far
            for (int k = 0; k < nr; ++k) {
                for (int e = a.full_off[k] + lane; e < a.full_off[k + 1]; e += 64) {
                    const int pk = fl[e];
                    const int wy = pk >> 16, wx = pk & 0xffff;
                    const int w = wy * side + wx;
                    sm += (double)Mw[w];
                    if (a.want_var) sv += (double)Vw[w];
                    sa += (wx >= wx_lo && wx <= wx_hi && wy >= wy_lo && wy <= wy_hi) ? 1.0 : 0.0;
                }
                double cm = 0.0, cv = 0.0, ca = 0.0;
                for (int e = a.cut_off[k] + lane; e < a.cut_off[k + 1]; e += 64) {
                    const int pk = cl[e];
                    const double wt = cw[e];
                    const int wy = pk >> 16, wx = pk & 0xffff;
                    const int w = wy * side + wx;
                    cm += wt * (double)Mw[w];
                    if (a.want_var) cv += wt * (double)Vw[w];
                    ca += (wx >= wx_lo && wx <= wx_hi && wy >= wy_lo && wy <= wy_hi) ? wt : 0.0;
                }
                const double ts = wave_sum_d(sm + cm);
                const double tv = a.want_var ? wave_sum_d(sv + cv) : 0.0;
                const double ta = wave_sum_d(sa + ca);
                if (lane == k) {
                    my_s = ts;
                    my_v = tv;
                    my_a = ta;
                }
            }
        }
        if (lane < nr) {
            g.sum[(size_t)row * nr + lane] = my_s;
            if (g.var) g.var[(size_t)row * nr + lane] = my_v;
            g.area[(size_t)row * nr + lane] = my_a;
        }
        if (lane == 0 && g.flags) {
            const bool trunc = !reach || cx - R < 0 || cx + R >= d.W || cy - R < 0 || cy + R >= d.H;
            g.flags[row] = trunc ? kFlagTrunc : 0u;
        }
    }
}

size_t growth_lds_bytes(int nfull, int ncut, int side, int nixmax, int want_var, bool f64, int waves) {
    if (f64) {
        const GrLayout<double> L(nfull, ncut, side, nixmax, want_var);
        return (size_t)L.shared + (size_t)L.wave * waves;
    }
    const GrLayout<float> L(nfull, ncut, side, nixmax, want_var);
    return (size_t)L.shared + (size_t)L.wave * waves;
}

void launch_growth_table(const GrowArgs& a, const GrowTab& t, hipStream_t s) {
    const int nw = std::min(8, 2 * a.nr);
    k_growth_table<<<1, 64 * nw, 0, s>>>(a, t);
}

template <typename Real>
static hipError_t launch_growth_t(const FrameDesc* desc, const FrameDesc* one, const GrowArgs& a, const GrowTab& t,
                                  const GrowOut& g, int blocks, int waves, hipStream_t s) {
    const size_t lds = growth_lds_bytes(a.nfull, a.ncut, a.side, a.nixmax, a.want_var, sizeof(Real) == 8, waves);
    const int grid = kXcds * std::max(1, (blocks + kXcds - 1) / kXcds);
    if (one) {
        hipError_t e = hipFuncSetAttribute((const void*)k_growth<Real, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_growth<Real, true><<<grid, 64 * waves, lds, s>>>(desc, *one, a, t, g);
    } else {
        hipError_t e = hipFuncSetAttribute((const void*)k_growth<Real, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_growth<Real, false><<<grid, 64 * waves, lds, s>>>(desc, FrameDesc{}, a, t, g);
    }
    return hipGetLastError();
}

hipError_t launch_growth(const FrameDesc* desc, const FrameDesc* one, const GrowArgs& a, const GrowTab& t,
                         const GrowOut& g, int blocks, int waves, bool f64, hipStream_t s) {
    if (f64) return launch_growth_t<double>(desc, one, a, t, g, blocks, waves, s);
    return launch_growth_t<float>(desc, one, a, t, g, blocks, waves, s);
}

}  // namespace gpk
