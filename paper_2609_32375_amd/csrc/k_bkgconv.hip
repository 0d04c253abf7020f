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
// Sums accumulate in FP64 from values stored in the working precision; each
// pass stages its rows (or a column band) in LDS with the reflection applied
// on load.  Noise map for a dark-subtracted frame in ADU:
//   R^2 = (g max(B, 0) + rn^2 + dark texp) / g^2.
#include "k_args.h"

namespace gpk {

constexpr int kCvSeg = 256;    // outputs per horizontal workgroup
constexpr int kCvCols = 64;    // columns per vertical workgroup
constexpr int kCvRows = 64;    // output rows per vertical workgroup

// normalised taps in LDS (every thread forms the same FP64 sum in one order)
__device__ __forceinline__ void cv_taps(const float* raw, int n, double* out) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += (double)raw[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = (double)raw[i] / s;
}

__device__ __forceinline__ bool cv_valid(const FrameDesc& d, const uint8_t* mask, int x, int y, float sat, float& v) {
    v = load_px(d, x, y);
    return !(mask && mask[(int64_t)y * d.pitch + x]) && v < sat;
}

// FIRST: the two channels vI and v from the frame; else one channel from src
template <typename Real, bool FIRST>
__global__ __launch_bounds__(kCvSeg) void k_conv_h(FrameDesc d, const uint8_t* __restrict__ mask, float sat,
                                                   const Real* __restrict__ src, Real* __restrict__ out0,
                                                   Real* __restrict__ out1, CvArgs a, int* __restrict__ flag) {
    extern __shared__ __align__(16) unsigned char cv_dyn[];
    if (!FIRST && flag[0] == 0) return;   // nothing to fill in this frame
    double* kx = reinterpret_cast<double*>(cv_dyn);
    Real* s0 = reinterpret_cast<Real*>(cv_dyn + sizeof(double) * kMaxConvTaps);
    Real* s1 = s0 + (kCvSeg + kMaxConvTaps);
    cv_taps(a.kx, a.lx, kx);
    const int y = blockIdx.y, x0 = blockIdx.x * kCvSeg, hx = a.lx >> 1;
    const int n = min(kCvSeg, d.W - x0) + a.lx - 1;
    for (int i = threadIdx.x; i < n; i += kCvSeg) {
        const int xs = reflect_idx(x0 - hx + i, d.W);
        if (FIRST) {
            float v;
            const bool ok = cv_valid(d, mask, xs, y, sat, v);
            s0[i] = ok ? (Real)v : (Real)0;
            s1[i] = ok ? (Real)1 : (Real)0;
        } else {
            s0[i] = src[(int64_t)y * d.W + xs];
        }
    }
    __syncthreads();
    const int x = x0 + threadIdx.x;
    if (x >= d.W) return;
    double a0 = 0.0, a1 = 0.0;
    for (int b = 0; b < a.lx; ++b) {
        a0 = fma(kx[b], (double)s0[threadIdx.x + b], a0);
        if (FIRST) a1 = fma(kx[b], (double)s1[threadIdx.x + b], a1);
    }
    out0[(int64_t)y * d.W + x] = (Real)a0;
    if (FIRST) out1[(int64_t)y * d.W + x] = (Real)a1;
}

// vertical sum of one channel over the staged band: out[r] for this thread's
// column, rows r0, r0 + 4, ... (4 row groups of the 256 threads)
template <typename Real>
__device__ __forceinline__ void cv_vsum(const Real* band, const double* ky, int ly, int c, int g, int nr,
                                        double* acc) {
#pragma unroll
    for (int q = 0; q < kCvRows / 4; ++q) {
        const int r = g + 4 * q;
        double s = 0.0;
        if (r < nr)
            for (int t = 0; t < ly; ++t) s = fma(ky[t], (double)band[(r + t) * kCvCols + c], s);
        acc[q] = s;
    }
}

template <typename Real>
__device__ __forceinline__ void cv_stage(const Real* __restrict__ src, const FrameDesc& d, int xc0, int y0, int hy,
                                         int nrows, Real* band) {
    for (int i = threadIdx.x; i < nrows * kCvCols; i += blockDim.x) {
        const int r = i / kCvCols, c = i - r * kCvCols;
        const int x = min(xc0 + c, d.W - 1);
        band[i] = src[(int64_t)reflect_idx(y0 - hy + r, d.H) * d.W + x];
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
    double* ky = reinterpret_cast<double*>(cv_dyn);
    Real* band = reinterpret_cast<Real*>(cv_dyn + sizeof(double) * kMaxConvTaps);
    cv_taps(a.ky, a.ly, ky);
    const int xc0 = blockIdx.x * kCvCols, y0 = blockIdx.y * kCvRows, hy = a.ly >> 1;
    const int nr = min(kCvRows, d.H - y0), nrows = nr + a.ly - 1;
    const int c = threadIdx.x & (kCvCols - 1), g = threadIdx.x / kCvCols;
    const int x = xc0 + c;
    double s0[kCvRows / 4], s1[kCvRows / 4];
    const bool fill = FIRST || flag[0] != 0;
    if (FIRST || fill) {
        cv_stage(in0, d, xc0, y0, hy, nrows, band);
        __syncthreads();
        cv_vsum(band, ky, a.ly, c, g, nr, s0);
    }
    if (FIRST) {
        __syncthreads();
        cv_stage(in1, d, xc0, y0, hy, nrows, band);
        __syncthreads();
        cv_vsum(band, ky, a.ly, c, g, nr, s1);
    }
    if (x >= d.W) return;
    int64_t nun = 0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < kCvRows / 4; ++q) {
        const int r = g + 4 * q;
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

size_t conv_h_lds(bool f64) { return sizeof(double) * kMaxConvTaps + 2 * (kCvSeg + kMaxConvTaps) * (f64 ? 8 : 4); }
size_t conv_v_lds(int ly, bool f64) {
    return sizeof(double) * kMaxConvTaps + (size_t)(kCvRows + ly - 1) * kCvCols * (f64 ? 8 : 4);
}

template <typename Real>
static hipError_t conv_frame_t(const FrameDesc& d, const uint8_t* mask, float sat, const CvArgs& a, Real* hA,
                               Real* hC, Real* G, Real* back, Real* rms, int* flag, int64_t* unfilled,
                               hipStream_t s) {
    const size_t lh = conv_h_lds(sizeof(Real) == 8), lv = conv_v_lds(a.ly, sizeof(Real) == 8);
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_v<Real, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lv)) != hipSuccess)
        return e;
    if ((e = hipFuncSetAttribute((const void*)k_conv_v<Real, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lv)) != hipSuccess)
        return e;
    const dim3 gh((d.W + kCvSeg - 1) / kCvSeg, d.H), gv((d.W + kCvCols - 1) / kCvCols, (d.H + kCvRows - 1) / kCvRows);
    k_conv_clear<<<1, 64, 0, s>>>(flag, unfilled);
    // 1. horizontal: vI -> hA, v -> hC
    k_conv_h<Real, true><<<gh, kCvSeg, lh, s>>>(d, mask, sat, nullptr, hA, hC, a, flag);
    // 2. vertical: A -> back (kept until step 4), fill image -> G
    k_conv_v<Real, true><<<gv, 256, lv, s>>>(d, mask, sat, hA, hC, back, G, nullptr, nullptr, a, flag, unfilled);
    // 3. horizontal pass of G into hA (skipped without invalid pixels)
    k_conv_h<Real, false><<<gh, kCvSeg, lh, s>>>(d, mask, sat, G, hA, nullptr, a, flag);
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
