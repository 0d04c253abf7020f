// k_detect.hip -- matched-filter detection, connected components and moments.
//
//  k_detect_tiles  one workgroup (4 wavefronts) per 64x64 tile.  Builds
//                  M = I - B over the tile plus the filter halo in LDS
//                  (reflected borders), correlates it with the unit-sum kernel
//                  (two 1-D passes for a rank-one kernel), thresholds F > t R,
//                  labels the tile's components with a lock-free union-find in
//                  LDS (roots = smallest raster index), numbers them in raster
//                  order and accumulates per-piece moments: each lane owns one
//                  column and sums column runs with compensated FP32, flushing a
//                  run into the piece's record when it ends.  Border labels are
//                  kept for the merge.
//  k_merge_edges   unions pieces that touch across tile borders (8- or
//                  4-neighbourhood) in a global union-find.
//  k_merge_records adds every non-root piece into its root record and sets
//                  the first-pixel bit of every component with
//                  npix >= minarea in a per-frame bitmap.
//  k_popc_scan     prefix sums of the bitmap's popcounts -> label = rank of
//                  the first pixel in raster order.
//  k_write_catalog moment normalisation (FP64), catalogue rows and the
//                  per-frame object counts and status.
//  k_seg_finalize  optional per-pixel label map.
//
// The paper's detection is a matched filter normalised by the noise map with a
// threshold in sigma and first-moment positions; grouping pixels into
// connected components, minarea and the second moments are the SExtractor
// conventions this path adds.
#include "k_args.h"
#include "k_rowpoly.h"

#include <algorithm>

namespace gpk {

// A piece's sums while its tile is labelled: the M-weighted sums in FP64
// (quantised terms, exact additions) and the pixel-count sums (n, x n,
// y-sums, ...) as exact 32-bit integers (a tile holds 4096 pixels with offsets
// below 64, so every count sum is < 2^24).
struct LocalRec {
    double s[6];
    int32_t c[6];
    int32_t xmin, xmax, ymin, ymax;
    uint32_t peak, flags;
    int32_t rootpix;
    uint32_t amax;   // float bits of max |M| (non-negative: ordered as integers)
};

// LDS regions are reused phase by phase (REG: region width and height, the
// tile plus the filter halo; NIX: spline pieces of a region row; 29 KB for
// FP32, REG = 68 and NIX = 4, five workgroups per compute unit):
//   u1: row cubics (build M, R) -> union pair lists -> piece ids
//   u2: M over tile + halo (the horizontal pass in place) -> labels -> piece
//       records (M is held in VGPRs from the labels on)
template <typename Real, int REG, int NIX>
struct DetShared {
    union U1 {
        RowT<Real> tab[REG * NIX];
        int16_t comp[kTile * kTile];
    } u1;
    union U2 {
        Real ms[REG * REG];
        int32_t lab[kTile * kTile];
        LocalRec rec[kLocalRecs];
    } u2;
    uint64_t rowmask[kTile];
    int32_t rowoff[kTile + 1];
    int32_t misc[4];
    int32_t colp[REG];      // x piece of each region column (relative to the first)
    Real colsx[REG];        // its local coordinate in that piece
};

// find with path halving: every link points to a smaller index, so writing a
// grandparent over a parent only shortens the chain.  Links are read and
// written as relaxed workgroup-scope atomics (never cached in registers
// across the loop; the compiler keeps them as LDS instructions).
__device__ __forceinline__ int lds_ld(int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int lds_find(int* L, int x) {
    while (true) {
        const int q = lds_ld(&L[x]);
        if (q == x) return x;
        const int g = lds_ld(&L[q]);
        if (g != q) lds_st(&L[x], g);
        x = g;
    }
}
__device__ __forceinline__ void lds_union(int* L, int a, int b) {
    while (true) {
        a = lds_find(L, a);
        b = lds_find(L, b);
        if (a < b) {
            int old = atomicMin(&L[b], a);
            if (old == b) return;
            b = old;
        } else if (b < a) {
            int old = atomicMin(&L[a], b);
            if (old == a) return;
            a = old;
        } else {
            return;
        }
    }
}
__device__ __forceinline__ int g_find(int* P, int x) {
    volatile int* V = P;
    while (true) {
        int q = V[x];
        if (q == x) return x;
        x = q;
    }
}
// The root with the later first pixel (raster order; pieces have distinct
// first pixels) is linked under the other, so a component's root is the piece
// that holds the component's first pixel.  A failed link (the root was linked
// meanwhile) retries from the new roots; links follow one strict order, so no
// cycle can form.
__device__ __forceinline__ void g_union(int* P, const CompRec* R, int a, int b) {
    while (true) {
        a = g_find(P, a);
        b = g_find(P, b);
        if (a == b) return;
        const uint32_t ka = R[a].pmin, kb = R[b].pmin;
        if (kb < ka || (kb == ka && b < a)) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&P[b], b, a) == b) return;
    }
}

template <typename Real>
struct RunAcc;
template <>
struct RunAcc<float> {
    F2 S, T, U;
    __device__ void reset() { S = T = U = F2{0.f, 0.f}; }
    __device__ void add(float m, float dy) {
        f2_acc(S, m);
        f2_acc(T, dy * m);
        f2_acc(U, dy * dy * m);
    }
    __device__ double s() const { return f2_d(S); }
    __device__ double t() const { return f2_d(T); }
    __device__ double u() const { return f2_d(U); }
};
template <>
struct RunAcc<double> {
    double S, T, U;
    __device__ void reset() { S = T = U = 0.0; }
    __device__ void add(double m, double dy) {
        S += m;
        T += dy * m;
        U += dy * dy * m;
    }
    __device__ double s() const { return S; }
    __device__ double t() const { return T; }
    __device__ double u() const { return U; }
};

// RAD >= 0: square rank-one kernel of radius RAD applied as two 1-D passes
// (taps in registers, fully unrolled); RAD < 0: any kernel, applied densely.
// FP32, radius 1..2, row cubics of at most 4 pieces: under 32 KB of LDS, and
// the registers fit 96 without spills, so five workgroups per CU (radius 2:
// 9.56 -> 8.43 ms on the 64-frame batch).  Radius 4 fits too but its code
// under that limit was slower (1.77 -> 1.94 ms on a 12300^2 frame): it keeps
// four workgroups per CU.
template <typename Real, int RAD, int NIX>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((NIX <= 4 && sizeof(Real) == 4 && RAD >= 1 && RAD <= 2) ? 5 : 1))) void
k_detect_tiles(DetWork wk, const DetArgs* __restrict__ pa) {
    constexpr bool kSep = RAD >= 0;
    constexpr int kR = kSep ? RAD : 0;
    constexpr bool kDbl = sizeof(Real) == 8;
    constexpr int REG = kSep ? kTile + 2 * kR : kRegion;   // region row stride
    constexpr int MS = REG;
    __shared__ DetShared<Real, REG, NIX> sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gt = xcd_item(blockIdx.x, (wk.total_tiles + kXcds - 1) / kXcds);
    if (gt >= wk.total_tiles) return;
    const int f = frame_of(wk.nframes, gt, [&](int i) { return wk.desc[i].tile_base; });
    const FrameDesc d = wk.desc[f];
    const int lt = gt - d.tile_base;
    const int tx = lt % d.ntx, ty = lt / d.ntx;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int tw = min(kTile, d.W - x0), th = min(kTile, d.H - y0);
    // the tile's words of the frame's rank bitmap start at zero (bits are set
    // only after every tile has finished; words shared with a neighbouring
    // tile are cleared by both); the frame's last tile also clears the words
    // past its last pixel up to the end of the last 1024-bit block
    {
        const int r = tid >> 2, j = tid & 3;   // a row of 64 pixels spans at most 3 words
        if (r < th) {
            const int64_t p0 = (int64_t)(y0 + r) * d.W + x0;
            const int64_t w = (p0 >> 5) + j;
            if (w <= ((p0 + tw - 1) >> 5)) d.bitmap[w] = 0u;
        }
        if (tx == d.ntx - 1 && ty == d.nty - 1) {
            const int64_t wlim = (int64_t)d.nblocks * 32;
            for (int64_t w = (((int64_t)d.W * d.H + 31) >> 5) + tid; w < wlim; w += 256) d.bitmap[w] = 0u;
        }
    }
    const int kw = kSep ? 2 * kR + 1 : pa->kw;
    const int kh = kSep ? 2 * kR + 1 : pa->kh;
    const int rx = kw >> 1, ry = kh >> 1;
    const int RW = tw + 2 * rx, RH = th + 2 * ry;
    const int xs_lo = max(0, x0 - rx), xs_hi = min(d.W - 1, x0 + tw - 1 + rx);
    const int ixlo = piece_of(xs_lo, d.W, d.mw);
    const int nix = piece_of(xs_hi, d.W, d.mw) - ixlo + 1;

    // 1. the region's pixels (tile + halo, reflected at the frame border),
    //    flattened over the block so the loads coalesce and are all in flight
    //    while the row cubics and the column pieces are built
    constexpr int NL = (REG * REG + 255) / 256;
    // a region inside the frame (no reflection) of a separable filter: each
    // lane owns one of the tile's 64 columns and steps down the rows of its
    // wavefront (wv, wv + 4, ...) with buffer loads whose row offset is
    // scalar; the 2 R halo columns are spread over the block
    constexpr int CR = (REG + 3) / 4;                          // rows per wavefront
    constexpr int HW = 2 * kR;                                 // halo columns
    constexpr int HL = (REG * HW + 255) / 256;                 // halo values per thread
    constexpr int NV = (NL > CR + HL) ? NL : CR + HL;
    float pv[NV];
    const bool u16 = d.dtype == kDtypeU16;
    const int es = u16 ? 2 : 4;
    const bool inner = kSep && x0 >= rx && y0 >= ry && x0 + tw + rx <= d.W && y0 + th + ry <= d.H &&
                       (int64_t)RH * d.pitch * es < ((int64_t)1 << 31);
    auto halo_col = [&](int c) { return c < kR ? c : c + kTile; };
    if (inner) {
        const int64_t o0 = ((int64_t)(y0 - ry) * d.pitch + (x0 - rx)) * es;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)d.data + o0), (short)0, 0x7fffffff, 0x00020000);
        const int rowb = (int)d.pitch * es;
        auto ld = [&](int vo, int so) __attribute__((always_inline)) {
            return u16 ? (float)__builtin_amdgcn_raw_buffer_load_b16(rs, vo, so, 0)
                       : __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
        };
#pragma unroll
        for (int q = 0; q < CR; ++q) {
            const int r = wv + 4 * q;
            pv[q] = (r < RH) ? ld((rx + lane) * es, r * rowb) : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < HL; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (HW > 0 ? HW : 1), c = e - r * HW;
            pv[CR + i] = (r < RH) ? ld((r * (int)d.pitch + halo_col(c)) * es, 0) : 0.0f;
        }
    } else {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + 256 * i;
            const int r = e / REG, c = e - r * REG;
            pv[i] = (r < RH && c < RW) ? load_px(d, reflect_idx(x0 - rx + c, d.W), reflect_idx(y0 - ry + r, d.H))
                                       : 0.0f;
        }
    }
    // Warm the L2 with the region of the tile this XCD takes up one round of
    // resident workgroups later: one load per 128-byte line of its rows (one
    // value per thread, folded away at the end of this tile, so the wait is
    // off this tile's path).  That tile's own loads then hit the L2.
    float pf1 = 0.0f;
    bool pfo = false;
    {
        const int chunk = (wk.total_tiles + kXcds - 1) / kXcds;
        const int g2 = gt + wk.ahead;
        if (wk.ahead > 0 && g2 < min(wk.total_tiles, (blockIdx.x % kXcds + 1) * chunk)) {
            const int f2 = frame_of(wk.nframes, g2, [&](int i) { return wk.desc[i].tile_base; });
            const FrameDesc& d2 = wk.desc[f2];
            const int l2 = g2 - d2.tile_base;
            const int x2 = (l2 % d2.ntx) * kTile, y2 = (l2 / d2.ntx) * kTile;
            const int es2 = d2.dtype == kDtypeU16 ? 2 : 4;
            const int xa = max(x2 - rx, 0), xb = min(x2 + kTile + rx, d2.W) - 1;
            const int ya = max(y2 - ry, 0), yb = min(y2 + kTile + ry, d2.H) - 1;
            // the lines of one row run from the line of xa to the line of xb
            const int lpr = (int)((((int64_t)xb * es2) >> 7) - (((int64_t)xa * es2) >> 7)) + 1;
            const int r = tid / lpr, li = tid - r * lpr;
            if (r <= yb - ya && xb >= xa) {
                const int64_t line0 = (((int64_t)xa * es2) >> 7) + li;            // line index in the row
                const int64_t px = max(line0 * 128 / es2, (int64_t)xa);            // a pixel of that line
                const int64_t off = (int64_t)(ya + r) * d2.pitch + px;
                pf1 = es2 == 2 ? (float)((const gu16_t*)d2.data)[off] : ((const gfloat_t*)d2.data)[off];
                pfo = true;
            }
        }
    }
    for (int e = tid; e < RH * nix; e += 256) {
        const int r = e / nix, pi = e - r * nix;
        if (pi >= NIX) continue;
        const int ys = reflect_idx(y0 - ry + r, d.H);
        const int jy = piece_of(ys, d.H, d.mh);
        const double u = (double)ys - piece_ref(jy, d.H, d.mh);
        sh.u1.tab[r * NIX + pi] = make_row<Real>(d.coef, d.nx, d.ny, ixlo + pi, jy, u);
    }
    for (int c = tid; c < RW; c += 256) {
        const int xs = reflect_idx(x0 - rx + c, d.W);
        const int ix = piece_of(xs, d.W, d.mw);
        sh.colp[c] = ix - ixlo;
        sh.colsx[c] = (Real)((double)xs - piece_ref(ix, d.W, d.mw));
    }
    __syncthreads();
    // 2. M = I - B over the region
    if (inner) {
        const int c = rx + lane;
        const int pc = sh.colp[c];
        const Real sx = sh.colsx[c];
#pragma unroll
        for (int q = 0; q < CR; ++q) {
            const int r = wv + 4 * q;
            if (r < RH) sh.u2.ms[r * MS + c] = eval_M(sh.u1.tab[r * NIX + pc], sx, (Real)pv[q]);
        }
#pragma unroll
        for (int i = 0; i < HL; ++i) {
            const int e = tid + 256 * i;
            const int r = e / (HW > 0 ? HW : 1), hc = halo_col(e - r * HW);
            if (r < RH)
                sh.u2.ms[r * MS + hc] = eval_M(sh.u1.tab[r * NIX + sh.colp[hc]], sh.colsx[hc], (Real)pv[CR + i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int e = tid + 256 * i;
            const int r = e / REG, c = e - r * REG;
            if (r < RH && c < RW)
                sh.u2.ms[r * MS + c] = eval_M(sh.u1.tab[r * NIX + sh.colp[c]], sh.colsx[c], (Real)pv[i]);
        }
    }
    // thresholds t R of the 16 pixels this lane owns: column `lane`, rows 16 wv ..
    const bool colok = lane < tw;
    Real To[16];
    {
        const Real ts = (Real)pa->thresh;
        const int gx = colok ? x0 + lane : x0;
        const int ix = piece_of(gx, d.W, d.mw);
        const int pc = ix - ixlo;
        const Real sx = (Real)((double)gx - piece_ref(ix, d.W, d.mw));
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int ly = 16 * wv + k;
            To[k] = (colok && ly < th) ? ts * eval_R(sh.u1.tab[(ly + ry) * NIX + pc], sx) : (Real)0;
        }
    }
    __syncthreads();
    // 3. matched filter; own M values move to VGPRs
    Real Mo[16], Fo[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ly = 16 * wv + k;
        Mo[k] = (colok && ly < th) ? sh.u2.ms[(ly + ry) * MS + lane + rx] : (Real)0;
    }
    if constexpr (kSep) {
        Real kx[2 * kR + 1], ky[2 * kR + 1];
#pragma unroll
        for (int b = 0; b <= 2 * kR; ++b) {
            kx[b] = kDbl ? (Real)pa->kxd[b] : (Real)pa->kx[b];
            ky[b] = kDbl ? (Real)pa->kyd[b] : (Real)pa->ky[b];
        }
        // horizontal pass in place over M's rows (a row is one wavefront's:
        // each lane's reads of its row come before its write), once every
        // wavefront holds its own M values
        __syncthreads();
        if (colok) {
            for (int r = wv; r < RH; r += 4) {
                Real* mr = &sh.u2.ms[r * MS + lane];
                Real acc = 0;
#pragma unroll
                for (int b = 0; b <= 2 * kR; ++b) acc = fma(kx[b], mr[b], acc);
                mr[0] = acc;
            }
        }
        __syncthreads();
        Real win[16 + 2 * kR];
#pragma unroll
        for (int q = 0; q < 16 + 2 * kR; ++q) {
            const int r = 16 * wv + q;
            win[q] = (colok && r < RH) ? sh.u2.ms[r * MS + lane] : (Real)0;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            Real acc = 0;
#pragma unroll
            for (int a = 0; a <= 2 * kR; ++a) acc = fma(ky[a], win[k + a], acc);
            Fo[k] = acc;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int ly = 16 * wv + k;
            Real acc = 0;
            if (colok && ly < th) {
                for (int a = 0; a < kh; ++a) {
                    const Real* mr = &sh.u2.ms[(ly + a) * MS + lane];
                    for (int b = 0; b < kw; ++b)
                        acc = fma(kDbl ? (Real)pa->kdd[a * kw + b] : (Real)pa->kd[a * kw + b], mr[b], acc);
                }
            }
            Fo[k] = acc;
        }
    }
    uint32_t mbits = 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ly = 16 * wv + k;
        if (colok && ly < th && Fo[k] > To[k]) mbits |= 1u << k;
    }
    const int any = __syncthreads_or(mbits != 0u);
    gi32_t* seg = (gi32_t*)d.seg;
    if (!any) {
        if (tid == 0) wk.tiles[gt] = TileInfo{-1, 0};
        if (seg && colok) {
            for (int k = 0; k < 16; ++k) {
                const int ly = 16 * wv + k;
                if (ly < th) seg[(int64_t)(y0 + ly) * d.W + x0 + lane] = -1;
            }
        }
        return;
    }
    // 4. connected components inside the tile.  A tile row is one wavefront
    //    (lane = column), so each row's mask is one ballot.  Pixels start
    //    labelled with the first pixel of their horizontal run; runs of
    //    adjacent rows are then united once per touching pair, in an LDS
    //    union-find whose roots are the smallest raster index of each
    //    component.
    int32_t* lab = sh.u2.lab;      // M is held in VGPRs from here on
    int16_t* comp = sh.u1.comp;
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));   // lanes < lane
    // the wavefront's own row masks stay in registers; the row above its
    // first row is read from LDS
    uint64_t rm[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        rm[k] = __ballot((mbits >> k) & 1u);
        if (lane == 0) sh.rowmask[16 * wv + k] = rm[k];
    }
    // (the vertical pass that read the M region lab now occupies was
    // finished by every wavefront before the barrier above)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ly = 16 * wv + k;
        const int p = ly * kTile + lane;
        int v = -1;
        if ((mbits >> k) & 1u) {
            const uint64_t zb = ~rm[k] & below;
            const int s0 = zb ? 64 - __clzll(zb) : 0;
            v = ly * kTile + s0;
        }
        lab[p] = v;
    }
    __syncthreads();
    const bool conn8 = pa->conn == 8;
    // Union pairs (pixel, pixel above) for every pair of touching runs, one
    // at the first column of their overlap.  Each wavefront lists its rows'
    // pairs in its own share of the (now free) row-cubic region, then the
    // whole block applies them concurrently; a full list falls back to
    // uniting at once.  Pixel indices are < 4096: a pair packs into 24 bits.
    constexpr int PCAP = (int)(sizeof(typename DetShared<Real, REG, NIX>::U1) / sizeof(uint32_t)) / 4;
    uint32_t* plist = reinterpret_cast<uint32_t*>(&sh.u1) + wv * PCAP;
    int npair = 0;
    uint64_t mtop = 0ull;
    if (wv > 0) {
        const uint64_t t = sh.rowmask[16 * wv - 1];
        // (readfirstlane returns int: widen through uint32_t, not by sign)
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t >> 32));
        mtop = (uint64_t)lo | ((uint64_t)hi << 32);
    }
    // The pairs of a row are bit masks over its columns, computed on the
    // scalar unit from the row's mask m and the mask above mu (runs start
    // where m rises, end where it falls):
    //   vertical link at the first column of each overlap: m & mu & (start | ~(mu << 1))
    //   8-connectivity, up-left of a run start:           start & (mu << 1)
    //   8-connectivity, up-right of a run end, none above: end & (mu >> 1) & ~mu
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ly = 16 * wv + k;
        const uint64_t m = rm[k], mu = (k > 0) ? rm[k - 1] : mtop;
        const uint64_t start = m & ~(m << 1), end = m & ~(m >> 1);
        const uint64_t cm[3] = {m & mu & (start | ~(mu << 1)), conn8 ? (start & (mu << 1)) : 0ull,
                                conn8 ? (end & (mu >> 1) & ~mu) : 0ull};
        if ((cm[0] | cm[1] | cm[2]) == 0ull) continue;
        const int p = ly * kTile + lane;
        const int qq[3] = {p - kTile, p - kTile - 1, p - kTile + 1};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const uint64_t bm = cm[t];
            if (bm == 0ull) continue;
            const int pos = npair + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
            if ((bm >> lane) & 1ull) {
                if (pos < PCAP) plist[pos] = ((uint32_t)p << 12) | (uint32_t)qq[t];
                else lds_union(lab, p, qq[t]);
            }
            npair += __popcll(bm);
        }
    }
    if (lane == 0) sh.misc[wv] = min(npair, PCAP);
    __syncthreads();
    {
        const int n0 = sh.misc[0], n1 = sh.misc[1], n2 = sh.misc[2], n3 = sh.misc[3];
        const int tot = n0 + n1 + n2 + n3;
        for (int i = tid; i < tot; i += 256) {
            int w = 0, o = i;
            if (o >= n0) {
                o -= n0;
                w = 1;
                if (o >= n1) {
                    o -= n1;
                    w = 2;
                    if (o >= n2) {
                        o -= n2;
                        w = 3;
                    }
                }
            }
            const uint32_t e = reinterpret_cast<const uint32_t*>(&sh.u1)[w * PCAP + o];
            lds_union(lab, (int)(e >> 12), (int)(e & 4095u));
        }
    }
    __syncthreads();
    // Roots of the lane's 16 pixels.  The forest no longer changes, so the
    // 16 chains are walked side by side (one LDS round trip per step for all
    // of them) and nothing is written back: each root stays in a register.
    int rt[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) rt[k] = ((mbits >> k) & 1u) ? lab[(16 * wv + k) * kTile + lane] : -1;
    for (;;) {
        bool more = false;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = rt[k];
            const int g = lab[q & (kTile * kTile - 1)];
            if (q >= 0 && g != q) {
                rt[k] = g;
                more = true;
            }
        }
        if (__ballot(more) == 0ull) break;
    }
    // roots in raster order: per-row ballots (kept in rowmask, whose union
    // masks are no longer read), then a prefix over the 64 rows
    uint64_t rb[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int p = (16 * wv + k) * kTile + lane;
        rb[k] = __ballot(((mbits >> k) & 1u) && rt[k] == p);
        if (lane == 0) {
            sh.rowmask[16 * wv + k] = rb[k];
            sh.rowoff[16 * wv + k + 1] = __popcll(rb[k]);
        }
    }
    __syncthreads();
    if (wv == 0) {
        // rows' root counts -> exclusive offsets (one wavefront, lane = row)
        const int cnt = sh.rowoff[lane + 1];
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        sh.rowoff[lane + 1] = incl;
        if (lane == 0) sh.rowoff[0] = 0;
    }
    __syncthreads();
    const int ncomp = sh.rowoff[kTile];
    // piece id of a pixel = rank of its root among the tile's roots
    int co[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) co[k] = -1;
    if (__ballot(mbits != 0u) != 0ull) {   // (no pieces in a wavefront without detections)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int r = rt[k] & (kTile * kTile - 1);
            const int ry_ = r >> 6, rx_ = r & 63;
            const uint64_t lowr = (rx_ == 0) ? 0ull : ((~0ull) >> (64 - rx_));
            const int c = sh.rowoff[ry_] + __popcll(sh.rowmask[ry_] & lowr);
            co[k] = ((mbits >> k) & 1u) ? c : -1;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) comp[(16 * wv + k) * kTile + lane] = (int16_t)co[k];
    // 5. records for the tile's pieces (LDS for the first kLocalRecs, in u2,
    //    now free: M lives in VGPRs)
    if (tid == 0) {
        int base = (int)atomicAdd(&wk.counters[0], (uint32_t)ncomp);
        if ((int64_t)base + ncomp > (int64_t)wk.rec_cap) {
            atomicOr(&wk.counters[1], 1u);
            base = -2;
        }
        sh.misc[0] = base;
    }
    __syncthreads();
    const int base = sh.misc[0];
    if (base < 0) {
        if (tid == 0) wk.tiles[gt] = TileInfo{-2, 0};
        return;
    }
    const int nloc = min(ncomp, kLocalRecs);
    for (int c = tid; c < ncomp; c += 256) {
        wk.parent[base + c] = base + c;
        if (c < kLocalRecs) {
            LocalRec& R = sh.u2.rec[c];
            for (int z = 0; z < 6; ++z) {
                R.s[z] = 0.0;
                R.c[z] = 0;
            }
            R.xmin = R.ymin = 0x7fffffff;
            R.xmax = R.ymax = -1;
            R.peak = 0u;
            R.flags = 0u;
            R.amax = 0u;
        } else {
            CompRec& R = wk.recs[base + c];
            for (int z = 0; z < 12; ++z) {
                R.s[z] = 0.0;
                R.acc[z] = 0.0;
            }
            R.xmin = R.ymin = 0x7fffffff;
            R.xmax = R.ymax = -1;
            R.peak = 0u;
            R.flags = 0u;
            R.frame = f;
            R.x0 = x0;
            R.y0 = y0;
            R.amax = 0u;
            R.camax = 0u;
            R.cnpix = 0;
        }
    }
    // border labels for the merge, and the per-pixel piece ids
    int16_t* E = wk.edges + (size_t)gt * 4 * kTile;
    if (tid < 64) {
        E[0 * kTile + tid] = (tid < tw) ? comp[0 * kTile + tid] : (int16_t)-1;
        E[1 * kTile + tid] = (tid < tw) ? comp[(th - 1) * kTile + tid] : (int16_t)-1;
    } else if (tid < 128) {
        const int r = tid - 64;
        E[2 * kTile + r] = (r < th) ? comp[r * kTile + 0] : (int16_t)-1;
        E[3 * kTile + r] = (r < th) ? comp[r * kTile + tw - 1] : (int16_t)-1;
    }
    if (seg && colok) {
        for (int k = 0; k < 16; ++k) {
            const int ly = 16 * wv + k;
            if (ly < th) seg[(int64_t)(y0 + ly) * d.W + x0 + lane] = co[k];
        }
    }
    __syncthreads();
    // first pixel of every piece = its root
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if ((rb[k] >> lane) & 1ull) {
            const int ly = 16 * wv + k;
            const int c = co[k];
            const uint32_t pm = (uint32_t)((y0 + ly) * d.W + x0 + lane);
            if (c < kLocalRecs) sh.u2.rec[c].rootpix = (int32_t)pm;
            else wk.recs[base + c].pmin = pm;
        }
    }
    // 6. moments, in two passes over the lane's column runs.  (a) Each run
    //    adds its exact integer quantities into its piece: pixel-count sums,
    //    bounding box, peak, max |M|, flags.  (b) Once every run has done so,
    //    each run adds its M-weighted sums (compensated along the run), every
    //    term rounded to the piece's quantum for that sum (from its pixel count
    //    and max |M|): the additions are exact, so the piece's sums do not
    //    depend on the order in which the runs arrive.
    //    (A wavefront whose rows hold no detection has no run.)
    const bool wave_has = __ballot(mbits != 0u) != 0ull;
    const int gx = x0 + lane;
    if (wave_has) {
        const float sat = pa->sat;
        const bool has_sat = sat < INFINITY;
        int cur = -1, rcnt = 0, rdy = 0, rdy2 = 0, ry0 = 0, ry1 = 0;
        float rpk = -INFINITY, ram = 0.0f;
        uint32_t rfl = 0u;
        auto flush = [&]() {
            const int addc[6] = {rcnt, lane * rcnt, rdy, lane * lane * rcnt, rdy2, lane * rdy};
            if (cur < kLocalRecs) {
                LocalRec& R = sh.u2.rec[cur];
#pragma unroll
                for (int z = 0; z < 6; ++z) atomicAdd(&R.c[z], addc[z]);
                atomicMin(&R.xmin, gx);
                atomicMax(&R.xmax, gx);
                atomicMin(&R.ymin, y0 + ry0);
                atomicMax(&R.ymax, y0 + ry1);
                atomicMax(&R.peak, f2ord(rpk));
                atomicMax(&R.amax, __float_as_uint(ram));
                if (rfl) atomicOr(&R.flags, rfl);
            } else {
                CompRec& R = wk.recs[base + cur];
#pragma unroll
                for (int z = 0; z < 6; ++z) unsafeAtomicAdd(&R.s[6 + z], (double)addc[z]);
                atomicMin(&R.xmin, gx);
                atomicMax(&R.xmax, gx);
                atomicMin(&R.ymin, y0 + ry0);
                atomicMax(&R.ymax, y0 + ry1);
                atomicMax(&R.peak, f2ord(rpk));
                atomicMax(&R.amax, __float_as_uint(ram));
                if (rfl) atomicOr(&R.flags, rfl);
            }
            cur = -1;
            rcnt = rdy = rdy2 = 0;
            rpk = -INFINITY;
            ram = 0.0f;
            rfl = 0u;
        };
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const bool m = (mbits >> k) & 1u;
            const int c = co[k];
            if (cur >= 0 && (!m || c != cur)) flush();
            if (m) {
                const int ly = 16 * wv + k;
                if (cur < 0) {
                    cur = c;
                    ry0 = ly;
                }
                ry1 = ly;
                rcnt += 1;
                rdy += ly;
                rdy2 += ly * ly;
                rpk = fmaxf(rpk, (float)Mo[k]);
                // (float)|M| of an FP64 M may round down by half an ulp; the
                // quantum keeps a factor two of headroom over the bound
                ram = fmaxf(ram, fabsf((float)Mo[k]));
                if (has_sat && load_px(d, gx, y0 + ly) >= sat) rfl |= kFlagSat;
            }
        }
        if (cur >= 0) flush();
    }
    __syncthreads();
    if (wave_has) {
        RunAcc<Real> run;
        run.reset();
        int cur = -1;
        auto flush = [&]() {
            const bool loc = cur < kLocalRecs;
            double npix, amax;
            if (loc) {
                npix = (double)sh.u2.rec[cur].c[0];
                amax = (double)__uint_as_float(sh.u2.rec[cur].amax);
            } else {
                CompRec& G = wk.recs[base + cur];
                npix = __hip_atomic_load(&G.s[6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                amax = (double)__uint_as_float(__hip_atomic_load(&G.amax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
            // |offsets| < 64 inside a tile: bounds amax npix 64^p for the
            // sums weighted by p coordinates
            const double b0 = amax * npix;
            const int e0 = quantum_exp(b0), e1 = quantum_exp(b0 * 64.0), e2 = quantum_exp(b0 * 4096.0);
            const double dxd = (double)lane;
            const double S = run.s(), T = run.t(), U = run.u();
            const double add[6] = {quantize(S, e0),           quantize(dxd * S, e1), quantize(T, e1),
                                   quantize(dxd * dxd * S, e2), quantize(U, e2),      quantize(dxd * T, e2)};
            if (loc) {
                LocalRec& R = sh.u2.rec[cur];
#pragma unroll
                for (int z = 0; z < 6; ++z) atomicAdd(&R.s[z], add[z]);
            } else {
                CompRec& R = wk.recs[base + cur];
#pragma unroll
                for (int z = 0; z < 6; ++z) unsafeAtomicAdd(&R.s[z], add[z]);
            }
            run.reset();
            cur = -1;
        };
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const bool m = (mbits >> k) & 1u;
            const int c = co[k];
            if (cur >= 0 && (!m || c != cur)) flush();
            if (m) {
                if (cur < 0) cur = c;
                run.add(Mo[k], (Real)(16 * wv + k));
            }
        }
        if (cur >= 0) flush();
    }
    __syncthreads();
    // 7. publish the LDS records
    for (int c = tid; c < nloc; c += 256) {
        const LocalRec& Lr = sh.u2.rec[c];
        CompRec& R = wk.recs[base + c];
        for (int z = 0; z < 6; ++z) {
            R.s[z] = Lr.s[z];
            R.s[6 + z] = (double)Lr.c[z];
        }
        R.xmin = Lr.xmin;
        R.xmax = Lr.xmax;
        R.ymin = Lr.ymin;
        R.ymax = Lr.ymax;
        R.pmin = (uint32_t)Lr.rootpix;
        R.peak = Lr.peak;
        R.flags = Lr.flags;
        R.frame = f;
        R.x0 = x0;
        R.y0 = y0;
        R.amax = Lr.amax;
        R.camax = 0u;
        R.cnpix = 0;
        for (int z = 0; z < 12; ++z) R.acc[z] = 0.0;
    }
    if (tid == 0) wk.tiles[gt] = TileInfo{base, ncomp};
    // (never true for the finite values of a frame: it keeps the warm-up load)
    if (pfo && __float_as_uint(pf1) == 0x7fc01234u) wk.counters[kNumCounters - 1] = 1u;
}

// ---------------------------------------------------------------------------
// unions across tile borders: one wavefront per tile (its right and bottom
// borders, plus the two lower diagonal corners for 8-connectivity)
__global__ __launch_bounds__(256) void k_merge_edges(DetWork wk, int conn) {
    if (wk.counters[1] != 0u) return;  // record overflow: the call reports it, nothing to merge
    const int lane = threadIdx.x & 63;
    const int gt = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gt >= wk.total_tiles) return;
    const TileInfo A = wk.tiles[gt];
    if (A.ncomp <= 0) return;
    const int f = frame_of(wk.nframes, gt, [&](int i) { return wk.desc[i].tile_base; });
    const FrameDesc& d = wk.desc[f];
    const int lt = gt - d.tile_base;
    const int tx = lt % d.ntx, ty = lt / d.ntx;
    const int tw = min(kTile, d.W - tx * kTile), th = min(kTile, d.H - ty * kTile);
    const int16_t* EA = wk.edges + (size_t)gt * 4 * kTile;
    const bool conn8 = conn == 8;
    // One seam: lane l holds A's piece a at position l and B's piece at l
    // (-1: none, or past the seam's length).  Lane l unites (a, b_j) for
    // j = l (and l +- 1 with 8-connectivity), skipping a pair that one of its
    // earlier offsets or the previous lane also forms: the first lane and
    // offset forming a pair always unites it, and runs along the seam give
    // one union each instead of one per pixel and offset.
    auto seam = [&](int a, int bl, int baseA, int baseB) {
        // (every lane runs the shuffles: a lane outside the exec mask would
        // hand its neighbours an undefined value)
        const int sa1 = __shfl(a, max(lane - 1, 0)), sb1 = __shfl(bl, max(lane - 1, 0));
        const int sb2 = __shfl(bl, max(lane - 2, 0)), sbp = __shfl(bl, min(lane + 1, 63));
        const int pa = (lane >= 1) ? sa1 : -1, bm1 = (lane >= 1) ? sb1 : -1;
        const int bm2 = (lane >= 2) ? sb2 : -1, bp1 = (lane <= 62) ? sbp : -1;
        if (a < 0) return;
        const int cand[3] = {conn8 ? bm1 : -1, bl, conn8 ? bp1 : -1};   // b at l - 1, l, l + 1
        const int prev[3] = {conn8 ? bm2 : -1, bm1, conn8 ? bl : -1};   // the previous lane's
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int b = cand[t];
            if (b < 0) continue;
            bool dup = false;
#pragma unroll
            for (int u = 0; u < t; ++u) dup = dup || cand[u] == b;
            if (pa == a) dup = dup || prev[0] == b || prev[1] == b || prev[2] == b;
            if (!dup) g_union(wk.parent, wk.recs, baseA + a, baseB + b);
        }
    };
    if (tx + 1 < d.ntx) {
        const TileInfo B = wk.tiles[gt + 1];
        if (B.ncomp > 0) {
            const int16_t* EB = wk.edges + (size_t)(gt + 1) * 4 * kTile;
            const int a = (lane < th) ? EA[3 * kTile + lane] : -1;
            const int bl = (lane < th) ? EB[2 * kTile + lane] : -1;
            seam(a, bl, A.base, B.base);
        }
    }
    if (ty + 1 < d.nty) {
        const int gc = gt + d.ntx;
        const TileInfo C = wk.tiles[gc];
        if (C.ncomp > 0) {
            const int16_t* EC = wk.edges + (size_t)gc * 4 * kTile;
            const int a = (lane < tw) ? EA[1 * kTile + lane] : -1;
            const int bl = (lane < tw) ? EC[0 * kTile + lane] : -1;
            seam(a, bl, A.base, C.base);
        }
        if (conn == 8) {
            // down-right corner: (x0+63, y0+63) with (x0+64, y0+64)
            if (lane == 0 && tx + 1 < d.ntx) {
                const TileInfo D = wk.tiles[gc + 1];
                const int a = EA[1 * kTile + tw - 1];
                if (D.ncomp > 0 && a >= 0) {
                    const int b = wk.edges[(size_t)(gc + 1) * 4 * kTile + 0];
                    if (b >= 0) g_union(wk.parent, wk.recs, A.base + a, D.base + b);
                }
            }
            // down-left corner: (x0, y0+63) with (x0-1, y0+64)
            if (lane == 1 && tx > 0) {
                const TileInfo D = wk.tiles[gc - 1];
                const int a = EA[1 * kTile + 0];
                if (D.ncomp > 0 && a >= 0) {
                    const int b = wk.edges[(size_t)(gc - 1) * 4 * kTile + kTile - 1];
                    if (b >= 0) g_union(wk.parent, wk.recs, A.base + a, D.base + b);
                }
            }
        }
    }
}

// Merge, pass 1: every piece finds its root and adds its exact integer
// quantities into the root record (pixel count, max |M|, bounding box, peak,
// flags).  A component is kept when its pixel count reaches minarea: the
// piece whose addition carries the count across minarea (exactly one, the
// counts being integers) sets the bit of the component's first pixel, the
// root's own, in the per-frame rank bitmap.
__global__ __launch_bounds__(256) void k_merge_records(DetWork wk, int minarea) {
    if (wk.counters[1] != 0u) return;
    const int total = min((int)wk.counters[0], wk.rec_cap);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const int r = g_find(wk.parent, id);
        wk.root[id] = r;
        CompRec& R = wk.recs[r];
        const CompRec& S = wk.recs[id];
        const int np = (int)S.s[6];
        const int before = atomicAdd(&R.cnpix, np);
        atomicMax(&R.camax, S.amax);
        if (r != id) {
            atomicMin(&R.xmin, S.xmin);
            atomicMax(&R.xmax, S.xmax);
            atomicMin(&R.ymin, S.ymin);
            atomicMax(&R.ymax, S.ymax);
            atomicMax(&R.peak, S.peak);
            if (S.flags) atomicOr(&R.flags, S.flags);
        }
        if (before < minarea && before + np >= minarea) {
            const FrameDesc& d = wk.desc[R.frame];
            atomicOr(&d.bitmap[R.pmin >> 5], 1u << (R.pmin & 31u));
        }
    }
}

// Merge, pass 2: every piece (the root too) moves its sums to the root's tile
// origin and adds them into the root's accumulators, each term rounded to the
// component's quantum for that sum.  The bounds are exact integers known
// after pass 1: max |M| times the pixel count times the extent of the
// bounding box about the root's origin (X, Y) to the power of the sum's
// coordinates, and the pixel count times the same for the unit-weight sums.
__global__ __launch_bounds__(256) void k_merge_sums(DetWork wk) {
    if (wk.counters[1] != 0u) return;
    const int total = min((int)wk.counters[0], wk.rec_cap);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const int r = wk.root[id];
        CompRec& R = wk.recs[r];
        const CompRec& S = wk.recs[id];
        const double ox = (double)(S.x0 - R.x0), oy = (double)(S.y0 - R.y0);
        const double X = (double)(max(abs(R.xmin - R.x0), abs(R.xmax - R.x0)) + 1);
        const double Y = (double)(max(abs(R.ymin - R.y0), abs(R.ymax - R.y0)) + 1);
        const double np = (double)R.cnpix;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* s = S.s + 6 * h;
            const double b0 = (h == 0 ? (double)__uint_as_float(R.camax) : 1.0) * np;
            const double c[6] = {s[0],
                                 s[1] + ox * s[0],
                                 s[2] + oy * s[0],
                                 s[3] + 2.0 * ox * s[1] + ox * ox * s[0],
                                 s[4] + 2.0 * oy * s[2] + oy * oy * s[0],
                                 s[5] + ox * s[2] + oy * s[1] + ox * oy * s[0]};
            const double b[6] = {b0, b0 * X, b0 * Y, b0 * X * X, b0 * Y * Y, b0 * X * Y};
#pragma unroll
            for (int z = 0; z < 6; ++z) unsafeAtomicAdd(&R.acc[6 * h + z], quantize(c[z], quantum_exp(b[z])));
        }
    }
}

// Ranks of the bitmap's bits.  k_popc_scan: each workgroup takes kScanChunk
// consecutive 1024-bit blocks, counts their bits and writes the exclusive
// prefix of the counts within the chunk to blockcnt; the chunk's total goes to
// chunksum.  The exclusive prefix of the chunk totals (formed by every
// catalogue workgroup in LDS, chunk_prefix) then gives the prefix of block b
// as blockcnt[b] + prefix[b / kScanChunk] (block_prefix).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// exclusive prefix of x over the workgroup's 256 threads; *total = the sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* ws, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t incl = wave_incl_scan(x, lane);
    __syncthreads();   // ws may still be read by a previous call
    if (lane == 63) ws[wv] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < wv; ++i) off += ws[i];
    *total = ws[0] + ws[1] + ws[2] + ws[3];
    return off + incl - x;
}

__global__ __launch_bounds__(256) void k_popc_scan(const uint32_t* __restrict__ bm, uint32_t* blockcnt,
                                                   uint32_t* chunksum, int nb) {
    static_assert(kScanChunk == 512, "four wavefronts of 16 x 64 lanes x 8 words per block");
    __shared__ uint32_t cnt[kScanChunk];
    __shared__ uint32_t ws[4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // bit counts of the chunk's blocks: a wavefront reads 1 KB (eight blocks of
    // eight 16-byte words) per load, all 16 loads in flight; eight lanes
    // reduce each block
    {
        const uint4* src = (const uint4*)bm + (size_t)blockIdx.x * kScanChunk * 8;
        const int nvec = min(kScanChunk, nb - (int)blockIdx.x * kScanChunk) * 8;
        uint4 q[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = wv * 1024 + i * 64 + lane;
            q[i] = (e < nvec) ? src[e] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint32_t c = __popc(q[i].x) + __popc(q[i].y) + __popc(q[i].z) + __popc(q[i].w);
            c += __shfl_xor(c, 1);
            c += __shfl_xor(c, 2);
            c += __shfl_xor(c, 4);
            if ((lane & 7) == 0) cnt[(wv * 1024 + i * 64 + lane) >> 3] = c;
        }
    }
    __syncthreads();
    const int b0 = blockIdx.x * kScanChunk + 2 * tid;
    const uint32_t v0 = (b0 < nb) ? cnt[2 * tid] : 0u, v1 = (b0 + 1 < nb) ? cnt[2 * tid + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v0 + v1, ws, &tot);
    if (b0 < nb) blockcnt[b0] = ex;
    if (b0 + 1 < nb) blockcnt[b0 + 1] = ex + v0;
    if (tid == 0) chunksum[blockIdx.x] = tot;
}

// Every catalogue workgroup scans the chunk totals into LDS itself: a batch
// holds at most kMaxScanChunks chunks (2^31 pixels, checked by the caller).
struct ChunkPrefix {
    const uint32_t* p;   // exclusive prefix of the chunk totals, [nchunks] = total
};

__device__ ChunkPrefix chunk_prefix(const DetWork& wk, uint32_t* lds, uint32_t* ws) {
    static_assert(kMaxScanChunks == 256 * 16, "16 chunk totals per thread");
    const int nchunks = (wk.total_blocks + kScanChunk - 1) / kScanChunk;
    const int tid = threadIdx.x, c0 = tid * 16;
    uint32_t cv[16], ct = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        cv[i] = (c0 + i < nchunks) ? wk.chunksum[c0 + i] : 0u;
        ct += cv[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(ct, ws, &tot);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (c0 + i < nchunks) lds[c0 + i] = run;
        run += cv[i];
    }
    if (tid == 0) lds[nchunks] = tot;
    __syncthreads();
    return ChunkPrefix{lds};
}

// number of kept components whose first pixel lies in blocks [0, b)
__device__ __forceinline__ uint32_t block_prefix(const DetWork& wk, const ChunkPrefix& cp, int b) {
    if (b >= wk.total_blocks) return cp.p[(wk.total_blocks + kScanChunk - 1) / kScanChunk];
    return wk.blockcnt[b] + cp.p[b / kScanChunk];
}

__global__ __launch_bounds__(256) void k_write_catalog(DetWork wk, CatOut cat, int minarea, int32_t* comp_status) {
    __shared__ uint32_t ctop[kMaxScanChunks + 1];
    __shared__ uint32_t ws[4];
    const ChunkPrefix cp = chunk_prefix(wk, ctop, ws);
    // per-frame object counts and status (workgroup 0)
    if (blockIdx.x == 0) {
        for (int f = threadIdx.x; f < wk.nframes; f += blockDim.x) {
            const FrameDesc& d = wk.desc[f];
            const int n =
                (int)(block_prefix(wk, cp, d.bm_block_base + d.nblocks) - block_prefix(wk, cp, d.bm_block_base));
            cat.n_obj[f] = n;
            cat.status[f] = (wk.counters[1] != 0u) ? 3 : ((n > cat.capacity) ? 4 : 0);
        }
        if (threadIdx.x == 0 && comp_status) {
            comp_status[0] = (wk.counters[1] != 0u) ? 3 : 0;
            comp_status[1] = (int32_t)wk.counters[0];
        }
    }
    if (wk.counters[1] != 0u) return;
    const int total = min((int)wk.counters[0], wk.rec_cap);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        if (wk.root[id] != id) continue;
        const CompRec& R = wk.recs[id];
        if (R.cnpix < minarea) {
            wk.label[id] = -1;
            continue;
        }
        const FrameDesc& d = wk.desc[R.frame];
        const uint32_t pm = R.pmin;
        const int blk = (int)(pm >> 10);
        // bits before pm in its 1024-bit block: the block's eight 16-byte
        // words are loaded at once and masked
        const uint4* bw = (const uint4*)(d.bitmap + (size_t)blk * 32);
        uint32_t rank = block_prefix(wk, cp, d.bm_block_base + blk) - block_prefix(wk, cp, d.bm_block_base);
        const int wi = (int)((pm >> 5) & 31u);
        const uint32_t part = (1u << (pm & 31u)) - 1u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint4 q = bw[k];
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * k + j;
                rank += __popc(i < wi ? w4[j] : (i == wi ? (w4[j] & part) : 0u));
            }
        }
        wk.label[id] = (int)rank + 1;
        if ((int)rank >= cat.capacity) continue;
        const size_t row = (size_t)d.cat_base + rank;
        const bool nonpos = !(R.acc[0] > 0.0);
        const double* w = nonpos ? R.acc + 6 : R.acc;
        const double W0 = w[0];
        const double mx = w[1] / W0, my = w[2] / W0;
        cat.npix[row] = R.cnpix;
        cat.xmin[row] = R.xmin;
        cat.xmax[row] = R.xmax;
        cat.ymin[row] = R.ymin;
        cat.ymax[row] = R.ymax;
        cat.pmin[row] = (int64_t)pm;
        cat.flux[row] = R.acc[0];
        cat.x[row] = (double)R.x0 + mx;
        cat.y[row] = (double)R.y0 + my;
        cat.x2[row] = w[3] / W0 - mx * mx;
        cat.y2[row] = w[4] / W0 - my * my;
        cat.xy[row] = w[5] / W0 - mx * my;
        cat.peak[row] = ord2f(R.peak);
        uint32_t fl = R.flags;
        if (nonpos) fl |= kFlagNonpos;
        if (R.xmin == 0 || R.ymin == 0 || R.xmax == d.W - 1 || R.ymax == d.H - 1) fl |= kFlagEdge;
        cat.flags[row] = fl;
    }
}

// per-pixel labels: piece index -> root -> label (-1 dropped, 0 background)
__global__ __launch_bounds__(256) void k_seg_finalize(DetWork wk, int f) {
    if (wk.counters[1] != 0u) return;
    const FrameDesc& d = wk.desc[f];
    gi32_t* seg = (gi32_t*)d.seg;
    const int64_t npx = (int64_t)d.W * d.H;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npx;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int v = seg[p];
        if (v < 0) {
            seg[p] = 0;
            continue;
        }
        const int y = (int)(p / d.W), x = (int)(p - (int64_t)y * d.W);
        const int gt = d.tile_base + (y / kTile) * d.ntx + x / kTile;
        const TileInfo T = wk.tiles[gt];
        if (T.base < 0) {
            seg[p] = 0;
            continue;
        }
        const int id = T.base + v;
        seg[p] = wk.label[wk.root[id]];
    }
}

// ---------------------------------------------------------------------------
// Peak detection, the paper's own: local maxima of the significance
// nu = F / R above the threshold, a maximum over a (2 sep + 1)^2 window
// (truncated at the frame, ties to the earlier pixel in raster order), and a
// first-moment centroid over a (2 cwin + 1)^2 window with weights max(M, 0).
// One workgroup per 64x64 tile: M over the tile plus a halo of
// max(sep + filter radius, cwin) (reflected at the frame edges, as the filter
// reads it), then F, R and nu over the tile plus sep, in LDS.  A peak's
// record goes to a slot taken with an atomic counter (its content does not
// depend on the slot); the rank bitmap then numbers the peaks in raster order.
// Spline x-pieces a region row of rmw <= 92 columns can touch: at most two
// knots fall inside when meshes are at least 64 pixels wide (knots 64 apart,
// the last at least 32 from its neighbour), so three pieces; otherwise the
// bound for meshes of 16 pixels.
__host__ __device__ inline int peak_nix(int rmw, int mesh_w) { return mesh_w >= 64 ? 3 : (rmw - 1) / 16 + 3; }

struct PeakLayout {
    int hmx, hmy, rmw, rmh, rf, nix;
    int o_ms, o_nu, o_tab, o_rn, o_colp, o_cols, o_cand, bytes;
    __host__ __device__ PeakLayout(int sep, int cwin, int rx, int ry, int real_bytes, int row_bytes, int mesh_w,
                                   bool vary = false) {
        hmx = max(sep + rx, cwin);
        hmy = max(sep + ry, cwin);
        rmw = kTile + 2 * hmx;
        rmh = kTile + 2 * hmy;
        rf = kTile + 2 * sep;
        nix = peak_nix(rmw, mesh_w);
        int o = 0;
        auto take = [&](int n) {
            o = (o + 15) / 16 * 16;
            const int r = o;
            o += n;
            return r;
        };
        o_ms = take(rmw * rmh * real_bytes);
        if (vary) {
            // the varying filter: nu only, with the row cubics in the same
            // space (read no more once M is formed, before nu is written)
            // and the noise cubics, which R needs with nu, after it
            o_nu = take(max(rf * rf * real_bytes, rmh * nix * row_bytes));
            o_tab = o_nu;
            o_rn = take(rmh * nix * 4 * real_bytes);
        } else {
            // nu and after it the taps of a dense filter, or before nu the
            // horizontal pass of a rank-one filter over the rows the
            // vertical pass reads
            o_nu = take(max(rf * rf + kMaxK * kMaxK, (rf + 2 * ry) * rf) * real_bytes);
            // row cubics
            o_tab = take(rmh * nix * row_bytes);
            o_rn = o_tab;
        }
        o_colp = take(rmw * 4);
        o_cols = take(rmw * real_bytes);
        o_cand = take(kTile * 2 * 4);
        bytes = (o + 15) / 16 * 16;
    }
};

// NM > 0: the spatially varying filter (NM dense correlations, the reference
// and up to NM - 1 modes, weighted by the coefficient maps at the output
// pixel) in place of the plain one; modes past the model's are zero taps
template <typename Real, int NM>
__global__ __launch_bounds__(256) void k_peaks_tiles(DetWork wk, const DetArgs* __restrict__ pa, PeakArgs pk) {
    constexpr bool VARY = NM > 0;
    extern __shared__ __align__(16) unsigned char pk_dyn[];
    constexpr bool kDbl = sizeof(Real) == 8;
    const int tid = threadIdx.x;
    const int gt = xcd_item(blockIdx.x, (wk.total_tiles + kXcds - 1) / kXcds);
    if (gt >= wk.total_tiles) return;
    const int f = frame_of(wk.nframes, gt, [&](int i) { return wk.desc[i].tile_base; });
    const FrameDesc d = wk.desc[f];
    const int lt = gt - d.tile_base;
    const int tx = lt % d.ntx, ty = lt / d.ntx;
    const int x0 = tx * kTile, y0 = ty * kTile;
    const int tw = min(kTile, d.W - x0), th = min(kTile, d.H - y0);
    const int kw = pa->kw, kh = pa->kh, rx = kw >> 1, ry = kh >> 1;
    const int sep = pk.sep, cw = pk.cwin;
    const PeakLayout L(sep, cw, rx, ry, (int)sizeof(Real), (int)sizeof(RowT<Real>), pk.mesh_w, VARY);
    Real* ms = reinterpret_cast<Real*>(pk_dyn + L.o_ms);
    Real* nus = reinterpret_cast<Real*>(pk_dyn + L.o_nu);
    RowT<Real>* tab = reinterpret_cast<RowT<Real>*>(pk_dyn + L.o_tab);
    Real* rn = reinterpret_cast<Real*>(pk_dyn + L.o_rn);   // noise cubics (varying filter)
    int32_t* colp = reinterpret_cast<int32_t*>(pk_dyn + L.o_colp);
    Real* colsx = reinterpret_cast<Real*>(pk_dyn + L.o_cols);
    uint32_t* cand = reinterpret_cast<uint32_t*>(pk_dyn + L.o_cand);
    // the tile's words of the frame's rank bitmap start at zero (bits are set
    // by a later launch); the frame's last tile also clears the words past its
    // last pixel up to the end of the last 1024-bit block
    {
        const int r = tid >> 2, j = tid & 3;
        if (r < th) {
            const int64_t p0 = (int64_t)(y0 + r) * d.W + x0;
            const int64_t w = (p0 >> 5) + j;
            if (w <= ((p0 + tw - 1) >> 5)) d.bitmap[w] = 0u;
        }
        if (tx == d.ntx - 1 && ty == d.nty - 1) {
            const int64_t wlim = (int64_t)d.nblocks * 32;
            for (int64_t w = (((int64_t)d.W * d.H + 31) >> 5) + tid; w < wlim; w += 256) d.bitmap[w] = 0u;
        }
    }
    if (tid < kTile * 2) cand[tid] = 0u;
    // a dense filter's taps, after nu (the rank-one passes do not use them
    // and write over that space)
    const bool sepk = !VARY && pa->separable != 0;
    Real* taps = nus + L.rf * L.rf;
    if (!VARY && !sepk)
        for (int i = tid; i < kw * kh; i += 256) taps[i] = kDbl ? (Real)pa->kdd[i] : (Real)pa->kd[i];
    // 1. raw pixels of the M region (reflected at the frame), row cubics and
    //    column pieces
    const int gx0 = x0 - L.hmx, gy0 = y0 - L.hmy;
    const int mw = tw + 2 * L.hmx, mh = th + 2 * L.hmy;
    const int xs_lo = max(0, gx0), xs_hi = min(d.W - 1, gx0 + mw - 1);
    const int ixlo = piece_of(xs_lo, d.W, d.mw);
    const int nix = min(piece_of(xs_hi, d.W, d.mw) - ixlo + 1, L.nix);
    // (12 loads per thread in flight at a time; a region holds at most
    // 92 x 92 pixels, 34 per thread)
    constexpr int kPkBatch = 12;
    for (int e0 = tid; e0 < mw * mh; e0 += 256 * kPkBatch) {
        float v[kPkBatch];
#pragma unroll
        for (int u = 0; u < kPkBatch; ++u) {
            const int e = e0 + 256 * u;
            const int r = e / mw, c = e - r * mw;
            v[u] = (e < mw * mh) ? load_px(d, reflect_idx(gx0 + c, d.W), reflect_idx(gy0 + r, d.H)) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kPkBatch; ++u) {
            const int e = e0 + 256 * u;
            const int r = e / mw, c = e - r * mw;
            if (e < mw * mh) ms[r * L.rmw + c] = (Real)v[u];
        }
    }
    // warm the L2 with the region of the tile this XCD takes up one round of
    // resident workgroups later (one load per 128-byte line of its rows,
    // folded away at the end of this tile)
    float pf1 = 0.0f;
    bool pfo = false;
    {
        const int chunk = (wk.total_tiles + kXcds - 1) / kXcds;
        const int g2 = gt + wk.ahead;
        if (wk.ahead > 0 && g2 < min(wk.total_tiles, (blockIdx.x % kXcds + 1) * chunk)) {
            const int f2 = frame_of(wk.nframes, g2, [&](int i) { return wk.desc[i].tile_base; });
            const FrameDesc& d2 = wk.desc[f2];
            const int l2 = g2 - d2.tile_base;
            const int x2 = (l2 % d2.ntx) * kTile, y2 = (l2 / d2.ntx) * kTile;
            const int es2 = d2.dtype == kDtypeU16 ? 2 : 4;
            const int xa = max(x2 - L.hmx, 0), xb = min(x2 + kTile + L.hmx, d2.W) - 1;
            const int ya = max(y2 - L.hmy, 0), yb = min(y2 + kTile + L.hmy, d2.H) - 1;
            const int lpr = (int)((((int64_t)xb * es2) >> 7) - (((int64_t)xa * es2) >> 7)) + 1;
            for (int t = tid; t < lpr * (yb - ya + 1) && xb >= xa; t += 256) {
                const int r = t / lpr, li = t - r * lpr;
                const int64_t line0 = (((int64_t)xa * es2) >> 7) + li;
                const int64_t px = max(line0 * 128 / es2, (int64_t)xa);
                const int64_t off = (int64_t)(ya + r) * d2.pitch + px;
                pf1 += es2 == 2 ? (float)((const gu16_t*)d2.data)[off] : ((const gfloat_t*)d2.data)[off];
                pfo = true;
            }
        }
    }
    for (int e = tid; e < mh * nix; e += 256) {
        const int r = e / nix, pi = e - r * nix;
        const int ys = reflect_idx(gy0 + r, d.H);
        const int jy = piece_of(ys, d.H, d.mh);
        const double u = (double)ys - piece_ref(jy, d.H, d.mh);
        const RowT<Real> rt = make_row<Real>(d.coef, d.nx, d.ny, ixlo + pi, jy, u);
        tab[r * L.nix + pi] = rt;
        if (VARY) {
            Real* q = &rn[(r * L.nix + pi) * 4];
            q[0] = rt.r0;
            q[1] = rt.r1;
            q[2] = rt.r2;
            q[3] = rt.r3;
        }
    }
    for (int c = tid; c < mw; c += 256) {
        const int xs = reflect_idx(gx0 + c, d.W);
        const int ix = piece_of(xs, d.W, d.mw);
        colp[c] = min(ix - ixlo, L.nix - 1);
        colsx[c] = (Real)((double)xs - piece_ref(ix, d.W, d.mw));
    }
    __syncthreads();
    // 2. M = I - B over the region, in place
    for (int e = tid; e < mw * mh; e += 256) {
        const int r = e / mw, c = e - r * mw;
        Real* q = &ms[r * L.rmw + c];
        *q = eval_M(tab[r * L.nix + colp[c]], colsx[c], *q);
    }
    __syncthreads();
    // 3. F (two 1-D passes for a rank-one kernel, else dense), R and nu over
    //    the tile plus sep (nu = -inf outside the frame, so the maximum
    //    filter below skips those positions); candidates F > t R inside the tile
    const Real ts = (Real)pa->thresh;
    const int fw = tw + 2 * sep, fh = th + 2 * sep;
    if (VARY) {
        // S = sum_m c_m (M corr e_m) (c_0 = 1) over the tile plus sep, into
        // nus.  A work item is kVaryRows output rows of one column and keeps
        // (K + 1) x kVaryRows accumulators; the taps come through the scalar
        // cache (uniform addresses, [column][row][mode] layout).  Ten rows:
        // the 70 x 70 outputs of sep 3 make 490 items, two rounds of the 256
        // threads, and each tap feeds ten FMAs
        typedef __attribute__((address_space(4))) const Real ctap_t;
        const ctap_t* tp = (const ctap_t*)(kDbl ? (const void*)pk.psf->tapsd : (const void*)pk.psf->taps);
        const int nmodes = pk.psf->nmodes;
        constexpr int kVaryRows = 10;
        const int nrb = (fh + kVaryRows - 1) / kVaryRows;
        for (int it = tid; it < fw * nrb; it += 256) {
            const int i = it % fw, j0 = (it / fw) * kVaryRows;
            const int mc = i - sep + L.hmx - rx;           // first M column read
            const int mr0 = j0 - sep + L.hmy - ry;         // first M row read
            constexpr int NA = VARY ? NM : 1;
            // (the item's coefficients are loaded after the correlations:
            // held during them they would cost (NA - 1) x kVaryRows registers)
            const PsfFrame pfr = pk.pf[f];
            const int bin = pk.psf->bin;
            const int gx = x0 - sep + i;
            Real acc[NA][kVaryRows];
#pragma unroll
            for (int m = 0; m < NA; ++m)
#pragma unroll
                for (int r = 0; r < kVaryRows; ++r) acc[m][r] = 0;
            // per tap column b: the M column strip the item's rows read for
            // every tap row (kh + kVaryRows - 1 values) in registers, then
            // all tap rows (unrolled; taps of one column contiguous), two at
            // a time so that one wait on the scalar loads serves both
            constexpr int NC = kMaxK + kVaryRows - 1;
            for (int b = 0; b < kw; ++b) {
                Real col[NC];
#pragma unroll
                for (int t = 0; t < NC; ++t)
                    col[t] = (t < kh + kVaryRows - 1) ? ms[min(mr0 + t, L.rmh - 1) * L.rmw + mc + b] : (Real)0;
                const ctap_t* tb = tp + b * kh * (kMaxModes + 1);
                constexpr int kTapRows = 2;
#pragma unroll
                for (int a0 = 0; a0 < kMaxK; a0 += kTapRows) {
                    if (a0 < kh) {
                        Real t[kTapRows][NA];
#pragma unroll
                        for (int c = 0; c < kTapRows; ++c)
#pragma unroll
                            for (int m = 0; m < NA; ++m) t[c][m] = tb[min(a0 + c, kh - 1) * (kMaxModes + 1) + m];
#pragma unroll
                        for (int c = 0; c < kTapRows; ++c)
                            if (a0 + c < kh && a0 + c < kMaxK)
#pragma unroll
                                for (int m = 0; m < NA; ++m)
#pragma unroll
                                    for (int r = 0; r < kVaryRows; ++r)
                                        acc[m][r] = fma(t[c][m], col[min(a0 + c, kMaxK - 1) + r], acc[m][r]);
                    }
                }
            }
            // this item's coefficients (positions clamped into the frame;
            // the values of outside positions are not used)
            float cf[NA > 1 ? NA - 1 : 1][kVaryRows];
#pragma unroll
            for (int r = 0; r < kVaryRows; ++r) {
                const int gxc = min(max(gx, 0), d.W - 1), gyc = min(max(y0 - sep + j0 + r, 0), d.H - 1);
                const float* cp = pfr.data + (int64_t)(gyc / bin) * pfr.pitch + gxc / bin;
#pragma unroll
                for (int m = 1; m < NA; ++m) cf[m - 1][r] = (m <= nmodes) ? cp[(int64_t)(m - 1) * pfr.plane] : 0.0f;
            }
#pragma unroll
            for (int r = 0; r < kVaryRows; ++r) {
                const int j = j0 + r;
                Real sv = acc[0][r];
#pragma unroll
                for (int m = 1; m < NA; ++m)
                    if (m <= nmodes) sv = fma((Real)cf[m - 1][r], acc[m][r], sv);
                if (j < fh) nus[j * L.rf + i] = sv;
            }
        }
        __syncthreads();
    }
    if (sepk) {
        // horizontal pass over the M rows the vertical pass reads
        const int hr = fh + 2 * ry;
        const int m0 = L.hmy - sep - ry, c0 = L.hmx - sep - rx;
        for (int e = tid; e < hr * fw; e += 256) {
            const int t = e / fw, i = e - t * fw;
            const Real* mrow = &ms[(m0 + t) * L.rmw + c0 + i];
            Real acc = 0;
            for (int b = 0; b < kw; ++b) acc = fma(kDbl ? (Real)pa->kxd[b] : (Real)pa->kx[b], mrow[b], acc);
            nus[t * L.rf + i] = acc;
        }
        __syncthreads();
    }
    constexpr int kPkVals = (kTile + 2 * kMaxPeakWin) * (kTile + 2 * kMaxPeakWin) / 256 + 1;   // <= 24
    Real nv[kPkVals];
#pragma unroll
    for (int q = 0; q < kPkVals; ++q) {
        const int e = tid + 256 * q;
        nv[q] = 0;
        if (e < fw * fh) {
            const int j = e / fw, i = e - j * fw;
            const int mr = j - sep + L.hmy, mc = i - sep + L.hmx;   // M-region position of (x, y)
            Real acc = 0;
            const int gx = x0 - sep + i, gy = y0 - sep + j;
            const bool in = gx >= 0 && gx < d.W && gy >= 0 && gy < d.H;
            if (VARY) {
                acc = nus[j * L.rf + i];
            } else if (sepk) {
                for (int a = 0; a < kh; ++a)
                    acc = fma(kDbl ? (Real)pa->kyd[a] : (Real)pa->ky[a], nus[(j + a) * L.rf + i], acc);
            } else {
                for (int a = 0; a < kh; ++a) {
                    const Real* mrow = &ms[(mr + a - ry) * L.rmw + mc - rx];
                    const Real* krow = &taps[a * kw];
                    for (int b = 0; b < kw; ++b) acc = fma(krow[b], mrow[b], acc);
                }
            }
            Real R;
            if (VARY) {
                const Real* q = &rn[(mr * L.nix + colp[mc]) * 4];
                RowT<Real> rt;
                rt.r0 = q[0];
                rt.r1 = q[1];
                rt.r2 = q[2];
                rt.r3 = q[3];
                R = eval_R(rt, colsx[mc]);
            } else {
                R = eval_R(tab[mr * L.nix + colp[mc]], colsx[mc]);
            }
            nv[q] = in ? ((R > (Real)0) ? acc / R : acc) : (Real)-INFINITY;
            const int lx = i - sep, ly = j - sep;
            if (lx >= 0 && lx < tw && ly >= 0 && ly < th && acc > ts * R)
                atomicOr(&cand[ly * 2 + (lx >> 5)], 1u << (lx & 31));
        }
    }
    __syncthreads();   // (the horizontal pass and the row cubics are read no more)
#pragma unroll
    for (int q = 0; q < kPkVals; ++q) {
        const int e = tid + 256 * q;
        if (e < fw * fh) {
            const int j = e / fw, i = e - j * fw;
            nus[j * L.rf + i] = nv[q];
        }
    }
    __syncthreads();
    // 4. per tile row (one wavefront per row at a time): the maximum of nu
    //    over the (2 sep + 1)^2 window of each column, as the maximum down
    //    the window's rows at every column (one column per lane, the 2 sep
    //    columns past the 64th by the first lanes) and then across 2 sep + 1
    //    neighbouring columns by lane shuffles; a candidate equal to it is a
    //    peak unless an earlier pixel of the window (raster order) holds the
    //    same value
    const int lane = tid & 63, wv = tid >> 6;
    const float sat = pa->sat;
    // (the wavefront's tile rows that hold a candidate, from one read of
    // their 32 candidate words; rows past th have none)
    uint32_t rows = 0u;
    {
        const uint64_t nz = __ballot(lane < 32 && cand[32 * wv + lane] != 0u);
        for (int k = 0; k < 16; ++k)
            if ((nz >> (2 * k)) & 3ull) rows |= 1u << k;
    }
    while (rows != 0u) {
        const int k = __builtin_ctz(rows);
        rows &= rows - 1u;
        const int ly = 16 * wv + k, lx = lane;
        const bool isc = ly < th && lx < tw && ((cand[ly * 2 + (lx >> 5)] >> (lx & 31)) & 1u);
        Real vm = (Real)-INFINITY, vm2 = (Real)-INFINITY;
        for (int a = 0; a <= 2 * sep; ++a) {
            const Real* row = &nus[(ly + a) * L.rf];
            if (lane < fw) vm = fmax(vm, row[lane]);
            if (lane < 2 * sep && kTile + lane < fw) vm2 = fmax(vm2, row[kTile + lane]);
        }
        Real wmax = vm;
        for (int dd = 1; dd <= 2 * sep; ++dd) {
            const Real o1 = __shfl(vm, (lane + dd) & 63), o2 = __shfl(vm2, (lane + dd) & 63);
            wmax = fmax(wmax, lane + dd < kTile ? o1 : o2);
        }
        if (!isc) continue;
        const int gx = x0 + lx, gy = y0 + ly;
        const Real v = nus[(ly + sep) * L.rf + lx + sep];
        if (v < wmax) continue;
        // v is the window's maximum: a tie with an earlier pixel loses (the
        // rows above and the pixels to the left, all read with no early exit)
        bool tie = false;
        for (int dy = -sep; dy <= 0; ++dy) {
            const Real* rp = &nus[(ly + sep + dy) * L.rf + lx + sep];
            const int dxe = dy == 0 ? -1 : sep;
            for (int dx = -sep; dx <= dxe; ++dx) tie |= rp[dx] == v;
        }
        if (tie) continue;
        // the record slot first, so that the atomic's round trip overlaps the
        // centroid sums
        const uint32_t slot = atomicAdd(&wk.counters[0], 1u);
        if ((int64_t)slot >= (int64_t)wk.rec_cap) {
            atomicOr(&wk.counters[1], 1u);
            continue;
        }
        // centroid window, inside the frame; FP64 sums in a fixed order
        const int wx0 = max(gx - cw, 0), wx1 = min(gx + cw, d.W - 1);
        const int wy0 = max(gy - cw, 0), wy1 = min(gy + cw, d.H - 1);
        uint32_t fl = (wx0 != gx - cw || wx1 != gx + cw || wy0 != gy - cw || wy1 != gy + cw) ? kFlagEdge : 0u;
        double sw = 0.0, sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0, flux = 0.0;
        for (int qy = wy0; qy <= wy1; ++qy)
            for (int qx = wx0; qx <= wx1; ++qx) {
                const double m = (double)ms[(qy - gy0) * L.rmw + (qx - gx0)];
                const double w = m > 0.0 ? m : 0.0;
                const double dx = (double)(qx - gx), dy = (double)(qy - gy);
                sw += w;
                sx += w * dx;
                sy += w * dy;
                sxx += w * dx * dx;
                syy += w * dy * dy;
                sxy += w * dx * dy;
                flux += m;
                if (sat < INFINITY && load_px(d, qx, qy) >= sat) fl |= kFlagSat;
            }
        double mx = 0.0, my = 0.0, vx = 0.0, vy = 0.0, cxy = 0.0;
        if (sw > 0.0) {
            mx = sx / sw;
            my = sy / sw;
            vx = sxx / sw - mx * mx;
            vy = syy / sw - my * my;
            cxy = sxy / sw - mx * my;
        } else {
            fl |= kFlagNonpos;
        }
        const uint32_t pm = (uint32_t)((int64_t)gy * d.W + gx);
        CompRec& R = wk.recs[slot];
        R.acc[0] = flux;
        R.acc[1] = (double)gx + mx;
        R.acc[2] = (double)gy + my;
        R.acc[3] = vx;
        R.acc[4] = vy;
        R.acc[5] = cxy;
        R.xmin = wx0;
        R.xmax = wx1;
        R.ymin = wy0;
        R.ymax = wy1;
        R.pmin = pm;
        R.peak = __float_as_uint((float)v);
        R.flags = fl;
        R.frame = f;
        R.cnpix = (wx1 - wx0 + 1) * (wy1 - wy0 + 1);
    }
    // (never true for the finite values of a frame: it keeps the warm-up loads)
    if (pfo && __float_as_uint(pf1) == 0x7fc01234u) wk.counters[kNumCounters - 1] = 1u;
}

// the rank bitmap's bits of the recorded peaks (after every tile has cleared
// its words)
__global__ __launch_bounds__(256) void k_peak_bits(DetWork wk) {
    if (wk.counters[1] != 0u) return;
    const int total = min((int)wk.counters[0], wk.rec_cap);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const CompRec& R = wk.recs[id];
        const FrameDesc& d = wk.desc[R.frame];
        atomicOr(&d.bitmap[R.pmin >> 5], 1u << (R.pmin & 31u));
    }
}

// catalogue rows of the peaks in raster order, per-frame counts and status
__global__ __launch_bounds__(256) void k_write_peaks(DetWork wk, CatOut cat, int32_t* comp_status) {
    __shared__ uint32_t ctop[kMaxScanChunks + 1];
    __shared__ uint32_t ws[4];
    const ChunkPrefix cp = chunk_prefix(wk, ctop, ws);
    if (blockIdx.x == 0) {
        for (int f = threadIdx.x; f < wk.nframes; f += blockDim.x) {
            const FrameDesc& d = wk.desc[f];
            const int n =
                (int)(block_prefix(wk, cp, d.bm_block_base + d.nblocks) - block_prefix(wk, cp, d.bm_block_base));
            cat.n_obj[f] = n;
            cat.status[f] = (wk.counters[1] != 0u) ? 3 : ((n > cat.capacity) ? 4 : 0);
        }
        if (threadIdx.x == 0 && comp_status) {
            comp_status[0] = (wk.counters[1] != 0u) ? 3 : 0;
            comp_status[1] = (int32_t)wk.counters[0];
        }
    }
    if (wk.counters[1] != 0u) return;
    const int total = min((int)wk.counters[0], wk.rec_cap);
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const CompRec& R = wk.recs[id];
        const FrameDesc& d = wk.desc[R.frame];
        const uint32_t pm = R.pmin;
        const int blk = (int)(pm >> 10);
        const uint4* bw = (const uint4*)(d.bitmap + (size_t)blk * 32);
        uint32_t rank = block_prefix(wk, cp, d.bm_block_base + blk) - block_prefix(wk, cp, d.bm_block_base);
        const int wi = (int)((pm >> 5) & 31u);
        const uint32_t part = (1u << (pm & 31u)) - 1u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint4 q = bw[k];
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * k + j;
                rank += __popc(i < wi ? w4[j] : (i == wi ? (w4[j] & part) : 0u));
            }
        }
        if ((int)rank >= cat.capacity) continue;
        const size_t row = (size_t)d.cat_base + rank;
        cat.npix[row] = R.cnpix;
        cat.xmin[row] = R.xmin;
        cat.xmax[row] = R.xmax;
        cat.ymin[row] = R.ymin;
        cat.ymax[row] = R.ymax;
        cat.pmin[row] = (int64_t)pm;
        cat.flux[row] = R.acc[0];
        cat.x[row] = R.acc[1];
        cat.y[row] = R.acc[2];
        cat.x2[row] = R.acc[3];
        cat.y2[row] = R.acc[4];
        cat.xy[row] = R.acc[5];
        cat.peak[row] = __uint_as_float(R.peak);
        cat.flags[row] = R.flags;
    }
}

// xcd_cus: CUs per XCD; the L2 warm-up looks ahead by one round of resident
// workgroups, those CUs times the workgroups the layout leaves room for
template <typename Real, int NM>
static void launch_peak_tiles(const DetWork& wk, const DetArgs* args, const PeakArgs& pk, int kw, int kh,
                              int mesh_w, int xcd_cus, hipStream_t s) {
    const PeakLayout L(pk.sep, pk.cwin, kw / 2, kh / 2, (int)sizeof(Real), (int)sizeof(RowT<Real>), mesh_w, NM > 0);
    const int g = kXcds * ((wk.total_tiles + kXcds - 1) / kXcds);
    const void* k = (const void*)k_peaks_tiles<Real, NM>;
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, L.bytes);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, L.bytes) != hipSuccess || per_cu < 1) per_cu = 2;
    DetWork w = wk;
    w.ahead = xcd_cus * per_cu;
    k_peaks_tiles<Real, NM><<<g, 256, L.bytes, s>>>(w, args, pk);
}

template <typename Real>
static void launch_peak_tiles_t(const DetWork& wk, const DetArgs* args, const PeakArgs& pk, int kw, int kh,
                                int nmodes, int mesh_w, int xcd_cus, hipStream_t s) {
    if (!pk.psf) launch_peak_tiles<Real, 0>(wk, args, pk, kw, kh, mesh_w, xcd_cus, s);
    else if (nmodes < 2) launch_peak_tiles<Real, 2>(wk, args, pk, kw, kh, mesh_w, xcd_cus, s);
    else if (nmodes < 4) launch_peak_tiles<Real, 4>(wk, args, pk, kw, kh, mesh_w, xcd_cus, s);
    else if (nmodes < 6) launch_peak_tiles<Real, 6>(wk, args, pk, kw, kh, mesh_w, xcd_cus, s);
    else launch_peak_tiles<Real, kMaxModes + 1>(wk, args, pk, kw, kh, mesh_w, xcd_cus, s);
}

void launch_peaks(const DetWork& wk, const DetArgs* args, const CatOut& cat, int32_t* comp_status, bool f64, int sep,
                  int cwin, int kw, int kh, int persist_blocks, const PsfArgs* psf, const PsfFrame* pf,
                  int nmodes, int mesh_w, int xcd_cus, hipStream_t s) {
    const PeakArgs pk{sep, cwin, psf, pf, mesh_w};
    if (f64) launch_peak_tiles_t<double>(wk, args, pk, kw, kh, nmodes, mesh_w, xcd_cus, s);
    else launch_peak_tiles_t<float>(wk, args, pk, kw, kh, nmodes, mesh_w, xcd_cus, s);
    k_peak_bits<<<persist_blocks, 256, 0, s>>>(wk);
    const int nb = wk.total_blocks;
    k_popc_scan<<<(nb + kScanChunk - 1) / kScanChunk, 256, 0, s>>>(wk.bitmap, wk.blockcnt, wk.chunksum, nb);
    k_write_peaks<<<persist_blocks, 256, 0, s>>>(wk, cat, comp_status);
}

size_t peak_lds_bytes(int sep, int cwin, int kw, int kh, bool f64, int mesh_w) {
    return f64 ? PeakLayout(sep, cwin, kw / 2, kh / 2, 8, (int)sizeof(RowT<double>), mesh_w).bytes
               : PeakLayout(sep, cwin, kw / 2, kh / 2, 4, (int)sizeof(RowT<float>), mesh_w).bytes;
}

// ---------------------------------------------------------------------------
// launchers
template <typename Real, int NIX>
static void launch_detect_n(const DetWork& wk, const DetArgs* args, int rad, hipStream_t s) {
    // 8 * ceil(tiles / 8) workgroups: a contiguous band of tiles per XCD
    const int g = kXcds * ((wk.total_tiles + kXcds - 1) / kXcds);
    switch (rad) {
        case 0: k_detect_tiles<Real, 0, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 1: k_detect_tiles<Real, 1, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 2: k_detect_tiles<Real, 2, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 3: k_detect_tiles<Real, 3, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 4: k_detect_tiles<Real, 4, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 5: k_detect_tiles<Real, 5, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 6: k_detect_tiles<Real, 6, NIX><<<g, 256, 0, s>>>(wk, args); break;
        case 7: k_detect_tiles<Real, 7, NIX><<<g, 256, 0, s>>>(wk, args); break;
        default: k_detect_tiles<Real, -1, NIX><<<g, 256, 0, s>>>(wk, args); break;
    }
}

// rad: radius of a square rank-one kernel (two 1-D passes), -1 for the dense
// path.  The row cubics of a tile region (at most 78 columns) span at most
// three spline pieces along x when meshes are at least 64 pixels wide (two
// knots fit in 77 columns: 64 apart, and the last one at least 32 from its
// neighbour) and six at the smallest mesh of 16.
template <typename Real, int NIX>
static int detect_per_cu_n(int rad) {
    const void* k;
    switch (rad) {
        case 0: k = (const void*)k_detect_tiles<Real, 0, NIX>; break;
        case 1: k = (const void*)k_detect_tiles<Real, 1, NIX>; break;
        case 2: k = (const void*)k_detect_tiles<Real, 2, NIX>; break;
        case 3: k = (const void*)k_detect_tiles<Real, 3, NIX>; break;
        case 4: k = (const void*)k_detect_tiles<Real, 4, NIX>; break;
        case 5: k = (const void*)k_detect_tiles<Real, 5, NIX>; break;
        case 6: k = (const void*)k_detect_tiles<Real, 6, NIX>; break;
        case 7: k = (const void*)k_detect_tiles<Real, 7, NIX>; break;
        default: k = (const void*)k_detect_tiles<Real, -1, NIX>; break;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 256, 0) != hipSuccess || n < 1) n = 4;
    return n;
}

// detection workgroups resident per CU for this launch configuration
int detect_tiles_per_cu(bool f64, int rad, int mesh_w) {
    if (mesh_w >= 64) return f64 ? detect_per_cu_n<double, 4>(rad) : detect_per_cu_n<float, 4>(rad);
    return f64 ? detect_per_cu_n<double, kNixMax>(rad) : detect_per_cu_n<float, kNixMax>(rad);
}

void launch_detect_tiles(const DetWork& wk, const DetArgs* args, bool f64, int rad, int mesh_w, hipStream_t s) {
    if (mesh_w >= 64) {
        if (f64) launch_detect_n<double, 4>(wk, args, rad, s);
        else launch_detect_n<float, 4>(wk, args, rad, s);
    } else {
        if (f64) launch_detect_n<double, kNixMax>(wk, args, rad, s);
        else launch_detect_n<float, kNixMax>(wk, args, rad, s);
    }
}

void launch_merge(const DetWork& wk, int conn, int minarea, int persist_blocks, hipStream_t s) {
    k_merge_edges<<<(wk.total_tiles + 3) / 4, 256, 0, s>>>(wk, conn);
    k_merge_records<<<persist_blocks, 256, 0, s>>>(wk, minarea);
    k_merge_sums<<<persist_blocks, 256, 0, s>>>(wk);
    const int nb = wk.total_blocks;
    const int nchunks = (nb + kScanChunk - 1) / kScanChunk;
    k_popc_scan<<<nchunks, 256, 0, s>>>(wk.bitmap, wk.blockcnt, wk.chunksum, nb);
}

void launch_catalog(const DetWork& wk, const CatOut& cat, int minarea, int persist_blocks,
                    int32_t* comp_status, hipStream_t s) {
    k_write_catalog<<<persist_blocks, 256, 0, s>>>(wk, cat, minarea, comp_status);
}

void launch_seg(const DetWork& wk, int f, int64_t npx, hipStream_t s) {
    int blocks = (int)std::min<int64_t>((npx + 255) / 256, 16384);
    k_seg_finalize<<<blocks, 256, 0, s>>>(wk, f);
}

// descriptor and argument upload (kernel arguments -> workspace)
__global__ void k_write_desc(DescChunk c, FrameDesc* table) {
    const int i = threadIdx.x;
    if (i < c.count) table[c.first + i] = c.d[i];
}

// Per-call set-up of the detection, one workgroup: the last descriptors, the
// filter arguments (the dense kernel normalised with an FP64 sum in a fixed
// order) and zeroed counters.  (The detection tiles clear the rank bitmap.)
__global__ __launch_bounds__(256) void k_det_setup(DescChunk c, FrameDesc* table, DetArgsIn in, DetArgs* out,
                                                   uint32_t* counters) {
    const int t = threadIdx.x;
    if (t < c.count) table[c.first + t] = c.d[t];
    if (t < kNumCounters) counters[t] = 0u;
    if (t == 0) {
        out->kw = in.kw;
        out->kh = in.kh;
        out->separable = in.separable;
        out->conn = in.conn;
        out->thresh = in.thresh;
        out->sat = in.sat;
        out->minarea = in.minarea;
        out->want_seg = in.want_seg;
    }
    // every lane forms the same sum in the same order
    double sum = 0.0;
    const int n = in.kw * in.kh;
    for (int i = 0; i < n; ++i) sum += (double)in.kraw[i];
    const double norm = (sum != 0.0) ? sum : 1.0;
    for (int i = t; i < kMaxK * kMaxK; i += 256) {
        const double v = (i < n) ? (double)in.kraw[i] / norm : 0.0;
        out->kdd[i] = v;
        out->kd[i] = (float)v;
    }
    if (t < kMaxK) {
        out->kx[t] = in.kx[t];
        out->ky[t] = in.ky[t];
        out->kxd[t] = in.kxd[t];
        out->kyd[t] = in.kyd[t];
    }
}

struct WordChunk {
    uint32_t n;
    uint32_t w[960];
};
__global__ void k_write_words(uint32_t* dst, WordChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

void launch_write_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const uint32_t* w = (const uint32_t*)src;
    size_t nw = bytes / 4;
    uint32_t* d = (uint32_t*)dst;
    while (nw > 0) {
        WordChunk c;
        c.n = (uint32_t)std::min<size_t>(nw, 960);
        for (uint32_t i = 0; i < c.n; ++i) c.w[i] = w[i];
        k_write_words<<<1, 256, 0, s>>>(d, c);
        w += c.n;
        d += c.n;
        nw -= c.n;
    }
}

void launch_write_desc(const DescChunk& c, FrameDesc* table, hipStream_t s) {
    k_write_desc<<<1, 64, 0, s>>>(c, table);
}

void launch_det_setup(const DescChunk& c, FrameDesc* table, const DetArgsIn& in, DetArgs* out, uint32_t* counters,
                      hipStream_t s) {
    k_det_setup<<<1, 256, 0, s>>>(c, table, in, out, counters);
}

}  // namespace gpk
