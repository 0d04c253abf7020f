// k_common.h -- device-side descriptors and helpers shared by the gfx950 kernels.
//
// Frames of a batch are described by FrameDesc records that live in the
// workspace; every stage kernel works on a flattened index space (meshes,
// tiles, objects) over all frames and finds its frame by a binary search over
// per-frame prefix offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpk {

constexpr int kTile = 64;          // detection tile edge; equals the wavefront width
constexpr int kMaxK = 15;          // largest filter edge
constexpr int kMaxR = kMaxK / 2;   // largest filter half-width
constexpr int kNixMax = 6;         // spline x-pieces a tile region (<= 78 columns) can touch (mesh >= 16)
constexpr int kRegion = kTile + 2 * kMaxR;  // 78: tile plus filter halo
constexpr int kLocalRecs = 160;    // components per tile accumulated in LDS
constexpr int kMaxRadii = 8;
constexpr int kDescChunk = 8;      // descriptors written per init launch
constexpr int kNumCounters = 64;   // detection counters (zeroed per call)
constexpr int kScanChunk = 512;    // rank bitmap: 1024-bit blocks per scan workgroup
constexpr int kMaxScanChunks = 4096;   // scan workgroups of one batch (2^31 pixels)

enum : int { kDtypeU16 = 1, kDtypeF32 = 2 };
enum : uint32_t { kFlagSat = 1u, kFlagEdge = 2u, kFlagNonpos = 4u, kFlagTrunc = 8u };

struct FrameDesc {
    const void* data;
    int64_t pitch;
    int32_t W, H, dtype, pad0;
    int32_t mw, mh, nx, ny;
    double* back_raw;     // [ny][nx]
    double* rms_raw;
    double* back;         // filtered
    double* rms;
    double* coef;         // [2][ny+1][nx+1][16]
    int32_t* iters;       // [ny][nx]
    double* ycoef;        // workspace: [2][ny+1][nx][4]
    double* scratch;      // workspace: Thomas sweeps of the y and x splines
    int32_t mesh_base;    // first flattened mesh of this frame
    int32_t tile_base;    // first flattened detection tile
    int32_t ntx, nty;     // detection tiles per row / column
    uint32_t* bitmap;     // first-pixel bitmap of this frame (1024-bit blocks)
    int32_t bm_block_base, nblocks;
    int32_t cat_base;     // first catalogue row of this frame
    int32_t pad1;
    int32_t* seg;         // nullable segmentation map (int32 [H][W])
};

struct DescChunk {
    int32_t first, count;
    FrameDesc d[kDescChunk];
};

// Per-component partial record (one per connected piece inside one tile).
// Sums are taken about the reference (x0, y0) = origin of the tile that
// produced the piece:
//   s[0..5]  = sum M, M dx, M dy, M dx^2, M dy^2, M dx dy
//   s[6..11] = the same with unit weights (n, dx, dy, ...)
// Every term added into s[] or acc[] is first rounded to a multiple of a power
// of two (quantum) chosen from exact integer bounds of the sum, so that every
// partial sum is an exact multiple of the quantum within the double range and
// the result does not depend on the order of the additions.  After the merge
// the component's root record holds in acc[] the sums of all its pieces about
// the root's tile origin, in cnpix its pixel count and in camax its max |M|.
struct CompRec {
    double s[12];
    double acc[12];
    int32_t xmin, xmax, ymin, ymax;  // frame coordinates (the component's, at the root)
    uint32_t pmin;                   // raster index of the first pixel in the frame
    uint32_t peak;                   // order-preserving bits of max M
    uint32_t flags;
    int32_t frame;
    int32_t x0, y0;
    uint32_t amax;                   // float bits of the piece's max |M|
    uint32_t camax;                  // float bits of the component's max |M| (root)
    int32_t cnpix;                   // pixels of the component (root)
    int32_t pad[3];
};

// Quantum of a sum bounded by `bound` (sum of |terms| <= bound): 2^e with
// bound < 2^(e + 51), so that the sum of the rounded terms stays an exact
// multiple of 2^e below 2^53 2^e.  Zero bound: every term is zero.
__device__ __forceinline__ int quantum_exp(double bound) {
    if (!(bound > 0.0)) return 0;
    int ex;
    (void)frexp(bound, &ex);   // bound < 2^ex
    return ex - 51;
}
__device__ __forceinline__ double quantize(double v, int e) { return ldexp(rint(ldexp(v, -e)), e); }

struct TileInfo {
    int32_t base;   // first record id (-1 when the tile holds no component)
    int32_t ncomp;
};

// Workspace pointers used by the detection kernels.
struct DetWork {
    FrameDesc* desc;
    int32_t nframes;
    int32_t total_tiles;
    uint32_t* counters;    // [0] records used, [1] overflow flag
    TileInfo* tiles;       // [total_tiles]
    int16_t* edges;        // [total_tiles][4][64]: top, bottom, left, right
    CompRec* recs;         // [rec_cap]
    int32_t* parent;       // [rec_cap]
    int32_t* root;         // [rec_cap]
    int32_t* label;        // [rec_cap]
    uint32_t* blockcnt;    // [total_blocks + 1] bitmap popcounts -> exclusive prefix
    uint32_t* chunksum;    // scan helper
    uint32_t* bitmap;      // all frames' first-pixel bitmaps
    int32_t rec_cap;
    int32_t total_blocks;
    int32_t ahead;         // tiles an XCD's resident workgroups span (the L2 warm-up distance)
    int32_t pad;
};

// ---------------------------------------------------------------------------
// order-preserving float bits (monotone uint32 image of IEEE float)
__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// ---------------------------------------------------------------------------
// compensated FP32 arithmetic (Knuth two-sum)
struct F2 {
    float hi, lo;
};
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
    float s, e;
    two_sum(a.hi, b.hi, s, e);
    e += a.lo + b.lo;
    float h = s + e;
    return F2{h, e - (h - s)};
}
// running compensated sum of single values
__device__ __forceinline__ void f2_acc(F2& a, float v) {
    float s, e;
    two_sum(a.hi, v, s, e);
    a.hi = s;
    a.lo += e;
}
// Workgroups are handed to the 8 XCDs (each with its own L2) in turn.  With a
// grid of 8 * chunk workgroups, item (blockIdx mod 8) * chunk + blockIdx / 8
// gives each XCD a contiguous run of items, so neighbours that share data
// (tile halos, overlapping apertures) meet in the same L2.  Items >= n: none.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int block, int chunk) { return (block % kXcds) * chunk + block / kXcds; }

// make one wavefront's LDS writes visible to its other lanes
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double f2_d(F2 a) { return (double)a.hi + (double)a.lo; }

// deterministic wavefront reductions (fixed butterfly order)
__device__ __forceinline__ F2 wave_sum_f2(F2 v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        F2 w{__shfl_xor(v.hi, o), __shfl_xor(v.lo, o)};
        // order the operands by lane so both partners compute the same value
        v = ((threadIdx.x & o) == 0) ? f2_add(v, w) : f2_add(w, v);
    }
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        double w = __shfl_xor(v, o);
        v = ((threadIdx.x & o) == 0) ? v + w : w + v;
    }
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// ---------------------------------------------------------------------------
// frame lookup by flattened index: the last frame whose base <= idx
template <typename Get>
__device__ __forceinline__ int frame_of(int nframes, int idx, Get base) {
    int lo = 0, hi = nframes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base(mid) <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// half-sample symmetric reflection into [0, n)
__device__ __forceinline__ int reflect_idx(int i, int n) {
    if (i >= 0 && i < n) return i;
    int p = 2 * n;
    int r = i % p;
    if (r < 0) r += p;
    return (r < n) ? r : (p - 1 - r);
}

// frames live in global memory: address them as such (global_load rather
// than the generic flat path)
typedef __attribute__((address_space(1))) const float gfloat_t;
typedef __attribute__((address_space(1))) const uint16_t gu16_t;
typedef __attribute__((address_space(1))) const double gdouble_t;
typedef __attribute__((address_space(1))) int32_t gi32_t;

__device__ __forceinline__ float load_px(const FrameDesc& d, int x, int y) {
    int64_t off = (int64_t)y * d.pitch + x;
    if (d.dtype == kDtypeU16) return (float)((gu16_t*)d.data)[off];
    return ((gfloat_t*)d.data)[off];
}

// mesh centre ("knot") along an axis and the spline piece holding a pixel:
// piece k spans [c_{k-1}, c_k); piece 0 and piece n extend to the frame edges
__device__ __forceinline__ double knot_at(int k, int n, int m) {
    int a = k * m;
    int b = min(a + m, n);
    return 0.5 * (double)(a + b - 1);
}
__device__ __forceinline__ int piece_of(int p, int n, int m) {
    int k0 = p / m;
    int a = k0 * m;
    int b = min(a + m, n);
    // c_{k0} = (a + b - 1) / 2 ; p >= c_{k0}  <=>  2p >= a + b - 1
    return k0 + ((2 * p >= a + b - 1) ? 1 : 0);
}
__device__ __forceinline__ double piece_ref(int piece, int n, int m) {
    return knot_at(piece > 0 ? piece - 1 : 0, n, m);
}

}  // namespace gpk
