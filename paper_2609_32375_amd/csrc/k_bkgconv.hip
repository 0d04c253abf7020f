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
// channel.  Each output's sum runs over the taps in order.  Noise map for a
// dark-subtracted frame in ADU:
//   R^2 = (g max(B, 0) + rn^2 + dark texp) / g^2.
#include "k_args.h"

namespace gpk {

constexpr int kCvT = 8;                     // outputs per thread (register block)
constexpr int kCvThreads = 256;
constexpr int kCvSeg = kCvThreads * kCvT;   // outputs per horizontal workgroup
constexpr int kCvCols = 64;                 // columns per vertical workgroup
constexpr int kCvRows = 64;                 // output rows per vertical workgroup (4 groups x 2 blocks)

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

// FIRST: vI from the frame, and the invalid-pixel flags of the segment's
// bands; else G from src in the rows whose reach holds an invalid pixel
template <typename Real, bool FIRST>
__global__ __launch_bounds__(kCvThreads) void k_conv_h(FrameDesc d, const uint8_t* __restrict__ mask, float sat,
                                                       const Real* __restrict__ src, Real* __restrict__ out,
                                                       uint8_t* __restrict__ inval, CvArgs a,
                                                       int* __restrict__ flag) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    __shared__ int bfl[kCvSeg / kCvCols];
    if (!FIRST && flag[0] == 0) return;   // nothing to fill in this frame
    const int np = cv_pad(a.lx), span = kCvSeg + np;
    Real* s0 = reinterpret_cast<Real*>(cv_dyn);
    const int y = blockIdx.y, x0 = blockIdx.x * kCvSeg, hx = a.lx >> 1;
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
    for (int i = threadIdx.x; i < span; i += kCvThreads) {
        Real v0 = (Real)0;
        if (i < n) {
            const int xs = reflect_idx(x0 - hx + i, d.W);
            if (FIRST) {
                float v;
                if (cv_valid(d, mask, xs, y, sat, v)) v0 = (Real)v;
                else if (i >= hx && i < hx + nseg) bfl[(i - hx) / kCvCols] = 1;
            } else if (fr[xs / kCvCols]) {
                v0 = src[(int64_t)y * d.W + xs];
            }
        }
        s0[i] = v0;
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

// rows y0 - hy + i, i < nrows, of a 64-column band (columns clamped to the
// frame; the values are only read for columns inside it); zero beyond nrows
// and, with act, in the rows act marks as zero
template <typename Real>
__device__ __forceinline__ void cv_stage(const Real* __restrict__ src, const FrameDesc& d, int xc0, int y0, int hy,
                                         int nrows, int rows, const uint8_t* act, Real* band) {
    for (int i = threadIdx.x; i < rows * kCvCols; i += blockDim.x) {
        const int r = i / kCvCols, c = i - r * kCvCols;
        const int x = min(xc0 + c, d.W - 1);
        band[i] = r < nrows && (!act || act[r]) ? src[(int64_t)reflect_idx(y0 - hy + r, d.H) * d.W + x] : (Real)0;
    }
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

// FIRST: A from hA; in tiles with an invalid pixel, C, the fill image G and
// the unfilled count.  Else: B = A + (K corr G) and the noise map.
template <typename Real, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_v(FrameDesc d, const uint8_t* __restrict__ mask, float sat,
                                                const Real* __restrict__ in0, Real* outA, Real* outG, Real* back,
                                                Real* rms, const uint8_t* __restrict__ inval, CvArgs a,
                                                int* __restrict__ flag, int64_t* __restrict__ unfilled) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    __shared__ uint8_t act[kCvRows + kConvTapsPad];
    const int np = cv_pad(a.ly), rows = kCvRows + np;
    Real* band = reinterpret_cast<Real*>(cv_dyn);
    const int xc0 = blockIdx.x * kCvCols, y0 = blockIdx.y * kCvRows, hy = a.ly >> 1, hx = a.lx >> 1;
    const int nr = min(kCvRows, d.H - y0), nrows = nr + a.ly - 1;
    const int nb = (d.W + kCvCols - 1) / kCvCols;
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const int x = xc0 + c;
    double s0[2 * kCvT], s1[2 * kCvT];
    bool fill;   // FIRST: the tile holds an invalid pixel; else: K corr G may be non-zero here
    if (FIRST) {
        const bool mine = (int)threadIdx.x < nr && inval[(int64_t)(y0 + threadIdx.x) * nb + blockIdx.x] != 0;
        fill = __syncthreads_or(mine);
    } else {
        if (flag[0] == 0) {
            fill = false;
        } else {
            // staged rows whose reach along x holds an invalid pixel
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
            fill = __syncthreads_or(mine);
        }
    }
    if (FIRST || fill) {
        cv_stage(in0, d, xc0, y0, hy, nrows, rows, FIRST ? nullptr : act, band);
        __syncthreads();
        cv_vsum(band, a.ky, np, c, g, nr, s0);
    } else {
#pragma unroll
        for (int q = 0; q < 2 * kCvT; ++q) s0[q] = 0.0;
    }
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
#pragma unroll
    for (int q = 0; q < 2 * kCvT; ++q) {
        const int r = g * 2 * kCvT + q;
        if (r >= nr) break;
        const int y = y0 + r;
        const int64_t o = (int64_t)y * d.W + x;
        if (FIRST) {
            outA[o] = (Real)s0[q];
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
            const double b = (double)outA[o] + s0[q];
            back[o] = (Real)b;
            const double sky = b > 0.0 ? b : 0.0;
            const double var_e = fma((double)a.gain, sky, fma((double)a.read_noise, (double)a.read_noise,
                                                                (double)a.dark * (double)a.exptime));
            rms[o] = (Real)sqrt(var_e / ((double)a.gain * (double)a.gain));
        }
    }
    if (FIRST && nun) atomicAdd((unsigned long long*)unfilled, (unsigned long long)nun);
}

__global__ void k_conv_clear(int* flag, int64_t* unfilled) {
    if (threadIdx.x == 0) {
        flag[0] = 0;
        if (unfilled) unfilled[0] = 0;
    }
}

size_t conv_h_lds(int lx, bool f64) { return (size_t)(kCvSeg + cv_pad(lx)) * (f64 ? 8 : 4); }
size_t conv_v_lds(int ly, bool f64) {
    return conv_v_band_bytes(ly, f64) + (size_t)(kCvRows + cv_pad(ly)) * kCvBitWords * 8;
}

template <typename Real>
static hipError_t conv_frame_t(const FrameDesc& d, const uint8_t* mask, float sat, const CvArgs& a, Real* hA,
                               uint8_t* inval, Real* G, Real* back, Real* rms, int* flag, int64_t* unfilled,
                               hipStream_t s) {
    const size_t lh = conv_h_lds(a.lx, sizeof(Real) == 8), lv = conv_v_lds(a.ly, sizeof(Real) == 8);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_h<Real, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lh)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_h<Real, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lh)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_v<Real, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lv)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_v<Real, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lv)) != hipSuccess)
        return e;
    const dim3 gh((d.W + kCvSeg - 1) / kCvSeg, d.H), gv((d.W + kCvCols - 1) / kCvCols, (d.H + kCvRows - 1) / kCvRows);
    k_conv_clear<<<1, 64, 0, s>>>(flag, unfilled);
    // 1. horizontal: vI -> hA, invalid-pixel flags
    k_conv_h<Real, true><<<gh, kCvThreads, lh, s>>>(d, mask, sat, nullptr, hA, inval, a, flag);
    // 2. vertical: A -> back (kept until step 4); C and the fill image G in flagged tiles
    k_conv_v<Real, true><<<gv, 256, lv, s>>>(d, mask, sat, hA, back, G, nullptr, nullptr, inval, a, flag, unfilled);
    // 3. horizontal pass of G into hA, rows within reach of an invalid pixel
    k_conv_h<Real, false><<<gh, kCvThreads, lh, s>>>(d, mask, sat, G, hA, inval, a, flag);
    // 4. B = A + vertical pass of it; noise map
    k_conv_v<Real, false><<<gv, 256, lv, s>>>(d, mask, sat, hA, back, nullptr, back, rms, inval, a, flag, nullptr);
    return hipGetLastError();
}

hipError_t launch_conv_frame(const FrameDesc& d, const uint8_t* mask, float sat, const CvArgs& a, void* hA,
                             void* inval, void* G, void* back, void* rms, int* flag, int64_t* unfilled, bool f64,
                             hipStream_t s) {
    if (f64)
        return conv_frame_t<double>(d, mask, sat, a, (double*)hA, (uint8_t*)inval, (double*)G, (double*)back,
                                    (double*)rms, flag, unfilled, s);
    return conv_frame_t<float>(d, mask, sat, a, (float*)hA, (uint8_t*)inval, (float*)G, (float*)back, (float*)rms,
                               flag, unfilled, s);
}

}  // namespace gpk
