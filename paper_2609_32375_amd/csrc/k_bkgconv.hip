// k_bkgconv.hip -- local background by convolution, with invalid pixels
// filled from their valid neighbours and a per-pixel noise map.
//
// B = K corr I' for a separable unit-sum kernel K = ky kx^T with half-sample
// reflected borders, where I' is the frame with every invalid pixel (mask
// set, or raw value >= sat) replaced by N = (K corr vI) / (K corr v), the
// kernel-weighted mean of the valid pixels around it (v = 1 valid, 0
// invalid).  Since I' = vI + (1 - v) N,
//   B = A + K corr ((1 - v) N),   A = K corr vI,
// so the path is two rounds of separable passes:
//   1. horizontal pass of vI -> hA; per row, one flag per 64-column band:
//      "an invalid pixel lies here"
//   2. vertical pass -> A; in the 64 x 64 tiles that hold an invalid pixel,
//      C = K corr v from the validity of the tile's neighbourhood (staged as
//      bits, both 1-D passes inside the tile) and the fill image
//      G = (1 - v) A / C -> A, G
//   3. horizontal pass of G -> hG, in the rows with an invalid pixel within
//      the kernel's reach only
//   4. vertical pass of hG, B = A + (K corr G), noise map R from B
// Everywhere else C is never read and K corr G is exactly +0 (a sum of zero
// products), so those sums are skipped: the results are those of the four
// full passes, bit for bit.
// Sums accumulate in FP64 from values stored in the working precision, with
// the unit-sum FP64 taps read as uniform kernel arguments (zero-padded to a
// multiple of 8: a zero tap adds an exact zero).  Each pass stages its rows
// (or a column band) in LDS with the reflection applied on load, and every
// thread keeps a block of 8 consecutive outputs in registers, sliding a
// 16-value window through the staged data: one LDS read per 8 FMAs per
// channel.  Each output's sum runs over the taps in order.  Each pass is one
// launch over every frame of the call: a frame table in the workspace gives
// each frame's slices of the planes and flags and its first workgroup of
// each pass.  Noise map for a dark-subtracted frame in ADU:
//   R^2 = (g max(B, 0) + rn^2 + dark texp) / g^2.
#include "k_args.h"

namespace gpk {

constexpr int kCvT = 8;                     // outputs per thread (register block)
constexpr int kCvThreads = 256;
constexpr int kCvSeg = kCvThreads * kCvT;   // outputs per horizontal workgroup
constexpr int kCvCols = 64;                 // columns per vertical workgroup
constexpr int kCvRows = 64;                 // output rows per vertical workgroup (4 groups x 2 blocks)
static_assert(kCvSeg == kCvSegPx && kCvCols == kCvTilePx && kCvRows == kCvTilePx, "workgroup shapes");

// the frame of a flattened workgroup index: base[] ascending from 0, so the
// bases <= item form a prefix (one ballot per 64 frames; all lanes active)
__device__ __forceinline__ int cv_frame_of(const int32_t* __restrict__ base, int n, int item) {
    const int lane = threadIdx.x & 63;
    int f = -1;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const uint64_t m = __ballot(i < n && base[i] <= item);
        f += __popcll(m);
        if (m != ~0ull) break;
    }
    return f;
}

__device__ __forceinline__ FrameDesc cv_desc(const CvFrame& F) {
    FrameDesc d{};
    d.data = F.data;
    d.pitch = F.pitch;
    d.W = F.W;
    d.H = F.H;
    d.dtype = F.dtype;
    return d;
}

// 64-bit words of validity bits per staged row in a tile: columns
// xc0 - hx + 0 .. 63 + padded taps + 7
constexpr int kCvBitWords = (kCvCols + kConvTapsPad + kCvT + 63) / 64;

__host__ __device__ __forceinline__ int cv_pad(int n) { return (n + kCvT - 1) / kCvT * kCvT; }
__host__ __device__ __forceinline__ size_t conv_v_band_bytes(int ly, bool f64) {
    return (size_t)(kCvRows + cv_pad(ly)) * kCvCols * (f64 ? 8 : 4);
}

__device__ __forceinline__ bool cv_valid(const FrameDesc& d, const uint8_t* mask, int x, int y, float sat, float& v) {
    v = load_px(d, x, y);
    return !(mask && mask[(int64_t)y * d.pitch + x]) && v < sat;
}

// acc[j] += sum_b k[b] w(j + b) over the padded taps, w(i) = src[i * step]:
// the window w[0..15] holds w(c + 0..15) for the 8-tap block at c
template <typename Real>
__device__ __forceinline__ void cv_block(const Real* src, int step, const double* k, int np, double* acc) {
    double w[2 * kCvT];
#pragma unroll
    for (int q = 0; q < kCvT; ++q) w[q] = (double)src[q * step];
    for (int c = 0; c < np; c += kCvT) {
#pragma unroll
        for (int q = 0; q < kCvT; ++q) w[kCvT + q] = (double)src[(c + kCvT + q) * step];
#pragma unroll
        for (int b = 0; b < kCvT; ++b) {
            const double kb = k[c + b];
#pragma unroll
            for (int j = 0; j < kCvT; ++j) acc[j] = fma(kb, w[j + b], acc[j]);
        }
#pragma unroll
        for (int q = 0; q < kCvT; ++q) w[q] = w[kCvT + q];
    }
}

// The columns (or rows) that reads of [a, b] with half-sample reflection at
// the borders of [0, n) can touch lie in [lo, hi] (a superset; monotone in
// [a, b], so a sub-range never reaches beyond its range's reach).
__device__ __forceinline__ void cv_reach(int a, int b, int n, int& lo, int& hi) {
    if (a >= 0 && b < n) {
        lo = a;
        hi = b;
    } else if (a < 0 && b >= n) {
        lo = 0;
        hi = n - 1;
    } else if (a < 0) {
        lo = 0;
        hi = min(n - 1, max(b, -a - 1));
    } else {
        lo = max(0, min(a, 2 * n - 1 - b));
        hi = n - 1;
    }
}

// A horizontal workgroup's staging: position i = tid + 256 k of the row
// segment plus halo, every load issued before the first store (the loads of
// positions past n repeat position n - 1 and are discarded).  FIRST: vI from
// the frame (T: its pixel type) and the band flags; else G where the row's
// band flag fr says it was written, zero elsewhere.
constexpr int kHStage = (kCvSeg + kConvTapsPad + kCvThreads - 1) / kCvThreads;

// half-sample reflection into [0, n) for -n <= i < 2n (one reflection), as selects
__device__ __forceinline__ int reflect1(int i, int n) {
    i = i < 0 ? -i - 1 : i;
    return i >= n ? 2 * n - 1 - i : i;
}

// ONE: the frame is at least half a kernel wide, so one reflection reaches
// every staged position; the loads then have no branch between them
template <typename Real, bool FIRST, typename T, bool ONE>
__device__ __forceinline__ void cv_stage_h(const FrameDesc& d, const uint8_t* __restrict__ mask, float sat,
                                           const Real* __restrict__ src, const uint8_t* fr, int x0, int hx, int n,
                                           int nseg, int span, int y, Real* s0, int* bfl) {
    typedef __attribute__((address_space(1))) const T gT;
    Real pv[kHStage];
    uint8_t mv[kHStage];
    const int64_t row = FIRST ? (int64_t)y * d.pitch : (int64_t)y * d.W;
    // without a mask, read the frame's first byte in its place (ignored)
    const uint8_t* mp = mask ? mask + row : (const uint8_t*)d.data;
    const int mstep = mask ? 1 : 0;
#pragma unroll
    for (int k = 0; k < kHStage; ++k) {
        const int i = min((int)threadIdx.x + k * kCvThreads, n - 1);
        const int xs = ONE ? reflect1(x0 - hx + i, d.W) : reflect_idx(x0 - hx + i, d.W);
        if (FIRST) {
            pv[k] = (Real)((gT*)d.data)[row + xs];
            mv[k] = mp[xs * mstep];
        } else {
            pv[k] = src[row + xs];
            mv[k] = fr[xs / kCvCols];
        }
    }
#pragma unroll
    for (int k = 0; k < kHStage; ++k) {
        const int i = threadIdx.x + k * kCvThreads;
        if (i < span) {
            Real v0 = (Real)0;
            if (i < n) {
                if (FIRST) {
                    if (!(mstep && mv[k]) && (float)pv[k] < sat) v0 = pv[k];
                    else if (i >= hx && i < hx + nseg) bfl[(i - hx) / kCvCols] = 1;
                } else if (mv[k]) {
                    v0 = pv[k];
                }
            }
            s0[i] = v0;
        }
    }
}

template <typename Real, bool FIRST, typename T>
__device__ __forceinline__ void cv_stage_h(const FrameDesc& d, const uint8_t* __restrict__ mask, float sat,
                                           const Real* __restrict__ src, const uint8_t* fr, int x0, int hx, int n,
                                           int nseg, int span, int y, Real* s0, int* bfl) {
    if (d.W >= hx) cv_stage_h<Real, FIRST, T, true>(d, mask, sat, src, fr, x0, hx, n, nseg, span, y, s0, bfl);
    else cv_stage_h<Real, FIRST, T, false>(d, mask, sat, src, fr, x0, hx, n, nseg, span, y, s0, bfl);
}

// FIRST: vI from the frame, and the invalid-pixel flags of the segment's
// bands; else G from src in the rows whose reach holds an invalid pixel
template <typename Real, bool FIRST>
__global__ __launch_bounds__(kCvThreads) void k_conv_h(CvWork w, int nframes, int total, CvArgs a) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    __shared__ int bfl[kCvSeg / kCvCols];
    const int item = xcd_item(blockIdx.x, (total + kXcds - 1) / kXcds);
    if (item >= total) return;
    const int f = cv_frame_of(w.hbase, nframes, item);
    int* flag = w.fflag + f;
    if (!FIRST && flag[0] == 0) return;   // nothing to fill in this frame
    const CvFrame F = w.tab[f];
    const FrameDesc d = cv_desc(F);
    const uint8_t* mask = F.mask;
    const float sat = a.sat;
    const Real* src = (const Real*)w.G + F.plane;
    Real* out = (Real*)w.hA + F.plane;
    uint8_t* inval = w.flags + F.flags;
    const int nsegs = (d.W + kCvSeg - 1) / kCvSeg, local = item - w.hbase[f];
    const int np = cv_pad(a.lx), span = kCvSeg + np;
    Real* s0 = reinterpret_cast<Real*>(cv_dyn);
    const int y = local / nsegs, x0 = (local - y * nsegs) * kCvSeg, hx = a.lx >> 1;
    const int nb = (d.W + kCvCols - 1) / kCvCols;
    const int nseg = min(kCvSeg, d.W - x0);
    const int n = nseg + a.lx - 1;   // staged values any written output reads
    uint8_t* fr = inval + (int64_t)y * nb;
    if (FIRST) {
        if (threadIdx.x < kCvSeg / kCvCols) bfl[threadIdx.x] = 0;
        __syncthreads();
    } else {
        int lo, hi;
        cv_reach(x0 - hx, x0 + nseg - 1 + hx, d.W, lo, hi);
        bool any = false;
        for (int b = lo / kCvCols + (int)threadIdx.x; b <= hi / kCvCols; b += kCvThreads) any |= fr[b] != 0;
        if (!__syncthreads_or(any)) return;   // G is zero wherever this row segment reads it
    }
    if (FIRST) {
        if (d.dtype == kDtypeU16)
            cv_stage_h<Real, true, uint16_t>(d, mask, sat, src, fr, x0, hx, n, nseg, span, y, s0, bfl);
        else
            cv_stage_h<Real, true, float>(d, mask, sat, src, fr, x0, hx, n, nseg, span, y, s0, bfl);
    } else {
        cv_stage_h<Real, false, float>(d, mask, sat, src, fr, x0, hx, n, nseg, span, y, s0, bfl);
    }
    __syncthreads();
    if (FIRST && threadIdx.x < kCvSeg / kCvCols) {
        // every band of every row is written once: no clearing between frames
        const int b = x0 / kCvCols + threadIdx.x;
        if (b < nb) {
            fr[b] = (uint8_t)bfl[threadIdx.x];
            if (bfl[threadIdx.x]) atomicOr(flag, 1);
        }
    }
    const int i0 = threadIdx.x * kCvT;
    if (i0 >= nseg) return;
    double a0[kCvT];
#pragma unroll
    for (int j = 0; j < kCvT; ++j) a0[j] = 0.0;
    cv_block(s0 + i0, 1, a.kx, np, a0);
    Real* o0 = out + (int64_t)y * d.W + x0 + i0;
    const int m = min(kCvT, nseg - i0);
#pragma unroll
    for (int j = 0; j < kCvT; ++j)
        if (j < m) o0[j] = (Real)a0[j];
}

// rows y0 - hy + r, r < nrows, of a 64-column band (columns clamped to the
// frame; the values are only read for columns inside it); zero beyond nrows
// and, with act, in the rows act marks as zero.  Thread (c, g) stages column
// c of rows g, g + 4, ..., kVStage loads in flight before their stores.
constexpr int kVStage = 16;
template <typename Real>
__device__ __forceinline__ void cv_stage(const Real* __restrict__ src, const FrameDesc& d, int xc0, int y0, int hy,
                                         int nrows, int rows, const uint8_t* act, Real* band) {
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const Real* col = src + min(xc0 + c, d.W - 1);
    for (int r0 = g; r0 < rows; r0 += 4 * kVStage) {
        Real v[kVStage];
#pragma unroll
        for (int k = 0; k < kVStage; ++k) {
            const int r = r0 + 4 * k;
            v[k] = (Real)0;
            if (r < nrows && (!act || act[r])) v[k] = col[(int64_t)reflect_idx(y0 - hy + r, d.H) * d.W];
        }
#pragma unroll
        for (int k = 0; k < kVStage; ++k) {
            const int r = r0 + 4 * k;
            if (r < rows) band[r * kCvCols + c] = v[k];
        }
    }
}

// The same band of FP32 rows loaded straight into LDS (global_load_lds: no
// register round trip, every row's load in flight at once); rows past nrows
// repeat row nrows - 1, finite values that only the zero-padded taps and the
// discarded outputs below the tile read.  Each wavefront waits for its own
// loads; the caller's barrier then publishes the band.
__device__ __forceinline__ void cv_stage_direct(const float* __restrict__ src, const FrameDesc& d, int xc0, int y0,
                                                int hy, int nrows, int rows, float* band) {
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const float* col = src + min(xc0 + c, d.W - 1);
    for (int r = g; r < rows; r += kCvThreads / kCvCols) {
        const float* p = col + (int64_t)reflect_idx(y0 - hy + min(r, nrows - 1), d.H) * d.W;
        __builtin_amdgcn_global_load_lds((const void*)p, (void __attribute__((address_space(3)))*)&band[r * kCvCols],
                                         4, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// the vertical sums of one channel for this thread's column and its two
// blocks of 8 rows, g * 16 + 0..7 and g * 16 + 8..15 (blocks wholly below
// the last output row are skipped)
template <typename Real>
__device__ __forceinline__ void cv_vsum(const Real* band, const double* k, int np, int c, int g, int nr,
                                        double* acc) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r0 = g * 2 * kCvT + h * kCvT;
#pragma unroll
        for (int j = 0; j < kCvT; ++j) acc[h * kCvT + j] = 0.0;
        if (r0 < nr) cv_block(band + r0 * kCvCols + c, kCvCols, k, np, acc + h * kCvT);
    }
}

// Horizontal pass of the validity v inside a tile: band[r][c] = sum_j kx[j]
// v(xc0 - hx + c + j, row r) for the staged rows, from bits[r] (bit cc of a
// row: column xc0 - hx + cc, reflected, is valid).  The same sums, in the
// same order and stored in the same precision, as a full horizontal pass of v.
template <typename Real>
__device__ __forceinline__ void cv_hbits(const uint64_t* bits, const double* k, int np, int rows, Real* band) {
    for (int it = threadIdx.x; it < rows * (kCvCols / kCvT); it += blockDim.x) {
        const int r = it / (kCvCols / kCvT), c0 = (it - r * (kCvCols / kCvT)) * kCvT;
        const uint8_t* by = reinterpret_cast<const uint8_t*>(bits + r * kCvBitWords);
        double acc[kCvT], w[2 * kCvT];
#pragma unroll
        for (int j = 0; j < kCvT; ++j) acc[j] = 0.0;
        unsigned b8 = by[c0 / 8];
#pragma unroll
        for (int q = 0; q < kCvT; ++q) w[q] = (b8 >> q) & 1u ? 1.0 : 0.0;
        for (int c = 0; c < np; c += kCvT) {
            b8 = by[(c0 + c) / 8 + 1];
#pragma unroll
            for (int q = 0; q < kCvT; ++q) w[kCvT + q] = (b8 >> q) & 1u ? 1.0 : 0.0;
#pragma unroll
            for (int b = 0; b < kCvT; ++b) {
                const double kb = k[c + b];
#pragma unroll
                for (int j = 0; j < kCvT; ++j) acc[j] = fma(kb, w[j + b], acc[j]);
            }
#pragma unroll
            for (int q = 0; q < kCvT; ++q) w[q] = w[kCvT + q];
        }
#pragma unroll
        for (int j = 0; j < kCvT; ++j) band[r * kCvCols + c0 + j] = (Real)acc[j];
    }
}

// noise map of a dark-subtracted frame in ADU from B.  FP64 maps: the
// formula as written, in FP64.  FP32 maps: R^2 = max(B, 0) / g + (rn^2 +
// dark t) / g^2 from the host's FP64 constants, rounded to FP32, and its
// correctly rounded FP32 square root (within 1.25 ulp of R).
template <typename Real>
__device__ __forceinline__ Real cv_noise(double b, const CvArgs& a) {
    const double sky = b > 0.0 ? b : 0.0;
    if (sizeof(Real) == 4) return (Real)sqrtf((float)fma(a.nm_c1, sky, a.nm_c0));
    const double var_e =
        fma((double)a.gain, sky, fma((double)a.read_noise, (double)a.read_noise, (double)a.dark * (double)a.exptime));
    return (Real)sqrt(var_e / ((double)a.gain * (double)a.gain));
}

// FIRST: A from hA; B and R where the fill round adds nothing; in tiles with
// an invalid pixel, C, the fill image G and the unfilled count.  Else, in the
// tiles the fill round reaches: B = A + (K corr G) and the noise map.
template <typename Real, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_v(CvWork w, int nframes, int total, CvArgs a) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    __shared__ uint8_t act[kCvRows + kConvTapsPad];
    const int item = xcd_item(blockIdx.x, (total + kXcds - 1) / kXcds);
    if (item >= total) return;
    const int f = cv_frame_of(w.vbase, nframes, item);
    const int local = item - w.vbase[f];
    const CvFrame F = w.tab[f];
    uint8_t* late_tile = w.tiles + F.tiles;
    if (!FIRST && late_tile[local] == 0) return;   // B and R were written by the first vertical pass
    const FrameDesc d = cv_desc(F);
    const uint8_t* mask = F.mask;
    const float sat = a.sat;
    const Real* in0 = (const Real*)w.hA + F.plane;
    Real* outG = (Real*)w.G + F.plane;
    Real* back = (Real*)F.back;   // also A until the fill round adds to it
    Real* outA = back;
    Real* rms = (Real*)F.rms;
    const uint8_t* inval = w.flags + F.flags;
    int* flag = w.fflag + f;
    int64_t* unfilled = w.unfilled + f;
    const int ntx = (d.W + kCvCols - 1) / kCvCols, ty = local / ntx, tx = local - ty * ntx;
    const int np = cv_pad(a.ly), rows = kCvRows + np;
    Real* band = reinterpret_cast<Real*>(cv_dyn);
    const int xc0 = tx * kCvCols, y0 = ty * kCvRows, hy = a.ly >> 1, hx = a.lx >> 1;
    const int nr = min(kCvRows, d.H - y0), nrows = nr + a.ly - 1;
    const int nb = (d.W + kCvCols - 1) / kCvCols;
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const int x = xc0 + c;
    double s0[2 * kCvT], s1[2 * kCvT];
    // late: K corr G may be non-zero in this tile (some staged row's reach
    // along x holds an invalid pixel; act marks those rows).  Known from the
    // flags of the first horizontal pass, so the first vertical pass already
    // finishes B and R where it is not.
    bool late = false;
    if (flag[0] != 0) {
        int lo, hi;
        cv_reach(xc0 - hx, min(xc0 + kCvCols, d.W) - 1 + hx, d.W, lo, hi);
        bool mine = false;
        for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
            const uint8_t* fr = inval + (int64_t)reflect_idx(y0 - hy + r, d.H) * nb;
            bool on = false;
            for (int b = lo / kCvCols; b <= hi / kCvCols; ++b) on |= fr[b] != 0;
            act[r] = on;
            mine |= on;
        }
        late = __syncthreads_or(mine);
    }
    if (FIRST && threadIdx.x == 0) late_tile[local] = late;
    bool fill;   // FIRST: the tile holds an invalid pixel
    if (FIRST) {
        const bool mine = (int)threadIdx.x < nr && inval[(int64_t)(y0 + threadIdx.x) * nb + tx] != 0;
        fill = __syncthreads_or(mine);
    } else {
        fill = true;
    }
    if constexpr (FIRST && sizeof(Real) == 4)
        cv_stage_direct(reinterpret_cast<const float*>(in0), d, xc0, y0, hy, nrows, rows,
                        reinterpret_cast<float*>(band));
    else
        cv_stage(in0, d, xc0, y0, hy, nrows, rows, FIRST ? nullptr : act, band);
    __syncthreads();
    cv_vsum(band, a.ky, np, c, g, nr, s0);
    if (FIRST && fill) {
        // C over the tile: validity bits of its neighbourhood, then both passes
        uint64_t* bits = reinterpret_cast<uint64_t*>(cv_dyn + conv_v_band_bytes(a.ly, sizeof(Real) == 8));
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int k = wv; k < rows * kCvBitWords; k += blockDim.x / 64) {
            const int r = k / kCvBitWords, cc = (k - r * kCvBitWords) * 64 + lane;
            bool ok = false;
            if (r < nrows && cc < kCvCols + a.lx - 1) {
                float v;
                ok = cv_valid(d, mask, reflect_idx(xc0 - hx + cc, d.W), reflect_idx(y0 - hy + r, d.H), sat, v);
            }
            const uint64_t m = __ballot(ok);
            if (lane == 0) bits[k] = m;
        }
        __syncthreads();   // bits staged; every wave is done with the band of A
        cv_hbits(bits, a.kx, cv_pad(a.lx), rows, band);
        __syncthreads();
        cv_vsum(band, a.ky, np, c, g, nr, s1);
    }
    if (x >= d.W) return;
    int64_t nun = 0;
    double av[2 * kCvT];   // A of this thread's outputs, all loaded before back (its own plane) is written
    if (!FIRST) {
#pragma unroll
        for (int q = 0; q < 2 * kCvT; ++q) {
            const int r = g * 2 * kCvT + q;
            av[q] = r < nr ? (double)outA[(int64_t)(y0 + r) * d.W + x] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 2 * kCvT; ++q) {
        const int r = g * 2 * kCvT + q;
        if (r >= nr) break;
        const int y = y0 + r;
        const int64_t o = (int64_t)y * d.W + x;
        if (FIRST) {
            const Real ar = (Real)s0[q];
            if (late) {
                outA[o] = ar;   // finished by the fill round
            } else {
                const double b = (double)ar + 0.0;   // B = A + (K corr G), the latter an exact +0 here
                back[o] = (Real)b;
                rms[o] = cv_noise<Real>(b, a);
            }
            if (fill) {
                float v;
                const bool ok = cv_valid(d, mask, x, y, sat, v);
                double gv = 0.0;
                if (!ok) {
                    if (s1[q] != 0.0) gv = s0[q] / s1[q];
                    else ++nun;
                }
                outG[o] = (Real)gv;
            }
        } else {
            const double b = av[q] + s0[q];
            back[o] = (Real)b;
            rms[o] = cv_noise<Real>(b, a);
        }
    }
    if (FIRST && nun) atomicAdd((unsigned long long*)unfilled, (unsigned long long)nun);
}

// the frame records and workgroup bases of one chunk; the per-frame flags
// and unfilled counts start at zero
__global__ void k_conv_setup(CvChunk c, CvWork w) {
    const int i = threadIdx.x;
    if (i < c.count) {
        w.tab[c.first + i] = c.f[i];
        w.hbase[c.first + i] = c.hbase[i];
        w.vbase[c.first + i] = c.vbase[i];
        w.fflag[c.first + i] = 0;
        w.unfilled[c.first + i] = 0;
    }
}

size_t conv_h_lds(int lx, bool f64) { return (size_t)(kCvSeg + cv_pad(lx)) * (f64 ? 8 : 4); }
size_t conv_v_lds(int ly, bool f64) {
    return conv_v_band_bytes(ly, f64) + (size_t)(kCvRows + cv_pad(ly)) * kCvBitWords * 8;
}

template <typename Real>
static hipError_t conv_t(int nframes, int htotal, int vtotal, const CvArgs& a, const CvWork& w, hipStream_t s) {
    const size_t lh = conv_h_lds(a.lx, sizeof(Real) == 8), lv = conv_v_lds(a.ly, sizeof(Real) == 8);
    hipError_t e;
    const void* hk[2] = {(const void*)k_conv_h<Real, true>, (const void*)k_conv_h<Real, false>};
    const void* vk[2] = {(const void*)k_conv_v<Real, true>, (const void*)k_conv_v<Real, false>};
    for (int i = 0; i < 2; ++i) {
        if ((e = hipFuncSetAttribute(hk[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lh)) != hipSuccess)
            return e;
        if ((e = hipFuncSetAttribute(vk[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lv)) != hipSuccess)
            return e;
    }
    // grids of whole XCD chunks over every frame's workgroups
    const unsigned gh = (unsigned)((htotal + kXcds - 1) / kXcds) * kXcds;
    const unsigned gv = (unsigned)((vtotal + kXcds - 1) / kXcds) * kXcds;
    // 1. horizontal: vI -> hA, invalid-pixel flags
    k_conv_h<Real, true><<<gh, kCvThreads, lh, s>>>(w, nframes, htotal, a);
    // 2. vertical: A -> back (B and R where step 4 adds nothing); C and the
    //    fill image G in flagged tiles
    k_conv_v<Real, true><<<gv, 256, lv, s>>>(w, nframes, vtotal, a);
    // 3. horizontal pass of G into hA, rows within reach of an invalid pixel
    k_conv_h<Real, false><<<gh, kCvThreads, lh, s>>>(w, nframes, htotal, a);
    // 4. B = A + vertical pass of it and the noise map, in the tiles it reaches
    k_conv_v<Real, false><<<gv, 256, lv, s>>>(w, nframes, vtotal, a);
    return hipGetLastError();
}

hipError_t launch_conv(const CvChunk* chunks, int nchunks, int nframes, int htotal, int vtotal, const CvArgs& a,
                       const CvWork& w, bool f64, hipStream_t s) {
    for (int i = 0; i < nchunks; ++i) k_conv_setup<<<1, 64, 0, s>>>(chunks[i], w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return f64 ? conv_t<double>(nframes, htotal, vtotal, a, w, s) : conv_t<float>(nframes, htotal, vtotal, a, w, s);
}

}  // namespace gpk
