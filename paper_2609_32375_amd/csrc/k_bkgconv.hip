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
//   1. horizontal pass of vI and v                        -> hA, hC
//   2. vertical pass: A, C; fill image G = (1 - v) A / C  -> A, G
//   3. horizontal pass of G (only if the frame has invalid pixels) -> hG
//   4. vertical pass of hG, B = A + (K corr G), noise map R from B
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

__host__ __device__ __forceinline__ int cv_pad(int n) { return (n + kCvT - 1) / kCvT * kCvT; }

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

// FIRST: the two channels vI and v from the frame; else one channel from src
template <typename Real, bool FIRST>
__global__ __launch_bounds__(kCvThreads) void k_conv_h(FrameDesc d, const uint8_t* __restrict__ mask, float sat,
                                                       const Real* __restrict__ src, Real* __restrict__ out0,
                                                       Real* __restrict__ out1, CvArgs a, int* __restrict__ flag) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    if (!FIRST && flag[0] == 0) return;   // nothing to fill in this frame
    const int np = cv_pad(a.lx), span = kCvSeg + np;
    Real* s0 = reinterpret_cast<Real*>(cv_dyn);
    Real* s1 = s0 + span;
    const int y = blockIdx.y, x0 = blockIdx.x * kCvSeg, hx = a.lx >> 1;
    const int n = min(kCvSeg, d.W - x0) + a.lx - 1;   // staged values any written output reads
    for (int i = threadIdx.x; i < span; i += kCvThreads) {
        Real v0 = (Real)0, v1 = (Real)0;
        if (i < n) {
            const int xs = reflect_idx(x0 - hx + i, d.W);
            if (FIRST) {
                float v;
                if (cv_valid(d, mask, xs, y, sat, v)) {
                    v0 = (Real)v;
                    v1 = (Real)1;
                }
            } else {
                v0 = src[(int64_t)y * d.W + xs];
            }
        }
        s0[i] = v0;
        if (FIRST) s1[i] = v1;
    }
    __syncthreads();
    const int i0 = threadIdx.x * kCvT;
    if (x0 + i0 >= d.W) return;
    double a0[kCvT], a1[kCvT];
#pragma unroll
    for (int j = 0; j < kCvT; ++j) a0[j] = a1[j] = 0.0;
    cv_block(s0 + i0, 1, a.kx, np, a0);
    if (FIRST) cv_block(s1 + i0, 1, a.kx, np, a1);
    Real* o0 = out0 + (int64_t)y * d.W + x0 + i0;
    Real* o1 = FIRST ? out1 + (int64_t)y * d.W + x0 + i0 : nullptr;
    const int m = min(kCvT, d.W - x0 - i0);
#pragma unroll
    for (int j = 0; j < kCvT; ++j)
        if (j < m) {
            o0[j] = (Real)a0[j];
            if (FIRST) o1[j] = (Real)a1[j];
        }
}

// rows y0 - hy + i, i < nrows, of a 64-column band (columns clamped to the
// frame; the values are only read for columns inside it), zero beyond nrows
template <typename Real>
__device__ __forceinline__ void cv_stage(const Real* __restrict__ src, const FrameDesc& d, int xc0, int y0, int hy,
                                         int nrows, int rows, Real* band) {
    for (int i = threadIdx.x; i < rows * kCvCols; i += blockDim.x) {
        const int r = i / kCvCols, c = i - r * kCvCols;
        const int x = min(xc0 + c, d.W - 1);
        band[i] = r < nrows ? src[(int64_t)reflect_idx(y0 - hy + r, d.H) * d.W + x] : (Real)0;
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

// FIRST: A and C from hA, hC; the fill image G and the unfilled count.
// Else: B = A + (K corr G) and the noise map.
template <typename Real, bool FIRST>
__global__ __launch_bounds__(256) void k_conv_v(FrameDesc d, const uint8_t* __restrict__ mask, float sat,
                                                const Real* __restrict__ in0, const Real* __restrict__ in1,
                                                Real* outA, Real* outG, Real* back, Real* rms, CvArgs a,
                                                int* __restrict__ flag, int64_t* __restrict__ unfilled) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    Real* band = reinterpret_cast<Real*>(cv_dyn);
    const int np = cv_pad(a.ly), rows = kCvRows + np;
    const int xc0 = blockIdx.x * kCvCols, y0 = blockIdx.y * kCvRows, hy = a.ly >> 1;
    const int nr = min(kCvRows, d.H - y0), nrows = nr + a.ly - 1;
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const int x = xc0 + c;
    double s0[2 * kCvT], s1[2 * kCvT];
    const bool fill = FIRST || flag[0] != 0;
    if (fill) {
        cv_stage(in0, d, xc0, y0, hy, nrows, rows, band);
        __syncthreads();
        cv_vsum(band, a.ky, np, c, g, nr, s0);
    }
    if (FIRST) {
        __syncthreads();
        cv_stage(in1, d, xc0, y0, hy, nrows, rows, band);
        __syncthreads();
        cv_vsum(band, a.ky, np, c, g, nr, s1);
    }
    if (x >= d.W) return;
    int64_t nun = 0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < 2 * kCvT; ++q) {
        const int r = g * 2 * kCvT + q;
        if (r >= nr) break;
        const int y = y0 + r;
        const int64_t o = (int64_t)y * d.W + x;
        if (FIRST) {
            float v;
            const bool ok = cv_valid(d, mask, x, y, sat, v);
            outA[o] = (Real)s0[q];
            double gv = 0.0;
            if (!ok) {
                any = true;
                if (s1[q] != 0.0) gv = s0[q] / s1[q];
                else ++nun;
            }
            outG[o] = (Real)gv;
        } else {
            const double b = (double)outA[o] + (fill ? s0[q] : 0.0);
            back[o] = (Real)b;
            const double sky = b > 0.0 ? b : 0.0;
            const double var_e = fma((double)a.gain, sky, fma((double)a.read_noise, (double)a.read_noise,
                                                                (double)a.dark * (double)a.exptime));
            rms[o] = (Real)sqrt(var_e / ((double)a.gain * (double)a.gain));
        }
    }
    if (FIRST) {
        if (any) atomicOr(flag, 1);
        if (nun) atomicAdd((unsigned long long*)unfilled, (unsigned long long)nun);
    }
}

__global__ void k_conv_clear(int* flag, int64_t* unfilled) {
    if (threadIdx.x == 0) {
        flag[0] = 0;
        if (unfilled) unfilled[0] = 0;
    }
}

size_t conv_h_lds(int lx, bool f64) { return 2 * (size_t)(kCvSeg + cv_pad(lx)) * (f64 ? 8 : 4); }
size_t conv_v_lds(int ly, bool f64) { return (size_t)(kCvRows + cv_pad(ly)) * kCvCols * (f64 ? 8 : 4); }

template <typename Real>
static hipError_t conv_frame_t(const FrameDesc& d, const uint8_t* mask, float sat, const CvArgs& a, Real* hA,
                               Real* hC, Real* G, Real* back, Real* rms, int* flag, int64_t* unfilled,
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
    // 1. horizontal: vI -> hA, v -> hC
    k_conv_h<Real, true><<<gh, kCvThreads, lh, s>>>(d, mask, sat, nullptr, hA, hC, a, flag);
    // 2. vertical: A -> back (kept until step 4), fill image -> G
    k_conv_v<Real, true><<<gv, 256, lv, s>>>(d, mask, sat, hA, hC, back, G, nullptr, nullptr, a, flag, unfilled);
    // 3. horizontal pass of G into hA (skipped without invalid pixels)
    k_conv_h<Real, false><<<gh, kCvThreads, lh, s>>>(d, mask, sat, G, hA, nullptr, a, flag);
    // 4. B = A + vertical pass of it; noise map
    k_conv_v<Real, false><<<gv, 256, lv, s>>>(d, mask, sat, hA, nullptr, back, nullptr, back, rms, a, flag, nullptr);
    return hipGetLastError();
}

hipError_t launch_conv_frame(const FrameDesc& d, const uint8_t* mask, float sat, const CvArgs& a, void* hA, void* hC,
                             void* G, void* back, void* rms, int* flag, int64_t* unfilled, bool f64,
                             hipStream_t s) {
    if (f64)
        return conv_frame_t<double>(d, mask, sat, a, (double*)hA, (double*)hC, (double*)G, (double*)back,
                                    (double*)rms, flag, unfilled, s);
    return conv_frame_t<float>(d, mask, sat, a, (float*)hA, (float*)hC, (float*)G, (float*)back, (float*)rms, flag,
                               unfilled, s);
}

}  // namespace gpk
