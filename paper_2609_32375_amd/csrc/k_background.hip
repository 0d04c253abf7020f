// k_background.hip -- mesh background for gfx950.
//
//  k_mesh_stats   one workgroup per mesh.  The mesh's pixels stay in VGPRs for
//                 the whole kappa-sigma loop.  Each clipping pass tests every
//                 surviving pixel against |v - med| <= kappa*sigma, accumulates
//                 the shifted sums of the new set (compensated) and bins it into
//                 an LDS histogram over the clip window; the exact median is the
//                 order statistic found through the histogram's prefix sums and
//                 a gather of the (few) pixels in the target bin.  All float
//                 reductions run in a fixed order, so a mesh gives bit-identical
//                 results wherever it is scheduled.
//  k_spline_y_pcr, k_spline_x_pcr (and the *_blk variants)
//                 grids of at most 127 knots per axis: the f x f median over
//                 the mesh grid (truncated at the edges) and the natural cubic
//                 splines through the mesh centres, one wavefront per spline up
//                 to 63 knots on the solved axis, one 128-thread workgroup up to
//                 127, solved in FP64 by parallel cyclic reduction and turned
//                 into bicubic pieces per mesh cell.
//  k_grid_filter, k_spline_*
//                 the same for larger grids: one thread per mesh for the
//                 filter, one per spline for the FP64 Thomas solve.
//
// The statistics follow the SExtractor method the paper cites for local
// background estimation; the paper's background subsection fixes the output
// role: a per-pixel background and a per-pixel noise map (here the clipped
// rms, interpolated like the background).
#include "k_args.h"
#include "k_rowpoly.h"

namespace gpk {

constexpr int kBins = 4096;
constexpr int kMaxWaves = 16;     // up to 1024 threads per mesh

constexpr int kBuf = 4096;        // sorted window of ranks around the median
constexpr int kHalf = 512;        // half-width of that window, in ranks
constexpr int kRankSmall = 16;    // first-level bins up to this size are ordered by rank counting
constexpr int kRankMax = 256;     // second-level bins beyond this size go to the merge sort

template <int NB>
struct MeshShared {
    static constexpr int kNB = NB;
    union {
        uint32_t hist[NB];
        float buf2[kBuf];     // second buffer of the window sort
    };
    float buf[kBuf];
    double pd[2][kMaxWaves][2];                // block_stats partials, double-buffered
    int32_t pi[2][kMaxWaves][2];
    float pmin[2][kMaxWaves], pmax[2][kMaxWaves];
    uint32_t wsum[kMaxWaves];
    uint32_t maxnb, wmin, wmax;
    int32_t sel_bin[2];
    uint32_t sel_cum[2];
    uint32_t cnt, kmin, kmax;
    int32_t ucnt[kMaxWaves];
};

template <int NB>
__device__ __forceinline__ int bin_of(float v, float lo, float scale) {
    float t = (v - lo) * scale;
    t = fminf(fmaxf(t, 0.0f), (float)(NB - 1));
    return (int)t;
}

template <int NB>
__device__ __forceinline__ float bin_scale(float lo, float hi) { return (hi > lo) ? (float)NB / (hi - lo) : 0.0f; }

// exclusive scan of one uint32 per thread over the block
template <int NT, typename SH>
__device__ __forceinline__ uint32_t block_exscan(uint32_t x, SH& sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) sh.wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int i = 0; i < w; ++i) off += sh.wsum[i];
    __syncthreads();
    return off + incl - x;
}

template <int NT, typename SH>
__device__ int block_sum_i(int x, SH& sh) {
    constexpr int NW = NT / 64;
    x = wave_sum_i(x);
    if ((threadIdx.x & 63) == 0) sh.ucnt[threadIdx.x >> 6] = x;
    __syncthreads();
    int s = 0;
    for (int i = 0; i < NW; ++i) s += sh.ucnt[i];
    __syncthreads();
    return s;
}

// deterministic block reduction of two FP64 sums, two counts and min/max
// (wavefront butterflies, then the wavefront partials in wavefront order).
// The partials alternate between two LDS sets (par flips on every call), so
// one barrier per call suffices: a set is written again only two calls later,
// after every thread has passed the barrier of the call in between.
template <int NT, typename SH>
__device__ __forceinline__ void block_stats(double& a, double& b, int& n, int& n2, float& mn, float& mx, int& par,
                                            SH& sh) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    const int P = par;
    par ^= 1;
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    n = wave_sum_i(n);
    n2 = wave_sum_i(n2);
    mn = wave_min(mn);
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) {
        sh.pd[P][w][0] = a;
        sh.pd[P][w][1] = b;
        sh.pi[P][w][0] = n;
        sh.pi[P][w][1] = n2;
        sh.pmin[P][w] = mn;
        sh.pmax[P][w] = mx;
    }
    __syncthreads();
    a = sh.pd[P][0][0];
    b = sh.pd[P][0][1];
    n = sh.pi[P][0][0];
    n2 = sh.pi[P][0][1];
    mn = sh.pmin[P][0];
    mx = sh.pmax[P][0];
    // all partials loaded at once up to 8 wavefronts; 16 would spill
#pragma unroll(NW > 8 ? 4 : 8)
    for (int i = 1; i < NW; ++i) {
        a += sh.pd[P][i][0];
        b += sh.pd[P][i][1];
        n += sh.pi[P][i][0];
        n2 += sh.pi[P][i][1];
        mn = fminf(mn, sh.pmin[P][i]);
        mx = fmaxf(mx, sh.pmax[P][i]);
    }
}

// Ascending bitonic sort of the SEG = 64 E values a wavefront holds, E per
// lane (lane l holds positions l E .. l E + E - 1): partners closer than E sit
// in the same lane, the others are exchanged with a lane shuffle.
template <int E>
__device__ __forceinline__ void wave_sort(float (&x)[E], int lane) {
#pragma unroll
    for (int k = 2; k <= 64 * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int g = e ^ j;
                    if (g > e) {
                        const bool up = ((lane * E + e) & k) == 0;
                        const float a = x[e], b = x[g];
                        x[e] = up ? fminf(a, b) : fmaxf(a, b);
                        x[g] = up ? fmaxf(a, b) : fminf(a, b);
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const float o = __shfl_xor(x[e], j / E);
                    const int i = lane * E + e;
                    const bool up = (i & k) == 0, lower = (i & j) == 0;
                    x[e] = (lower == up) ? fminf(x[e], o) : fmaxf(x[e], o);
                }
            }
        }
    }
}

template <int E>
__device__ __forceinline__ void wave_sort_segment(float* buf, int w, int lane) {
    float x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = buf[w * 64 * E + lane * E + e];
    wave_sort<E>(x, lane);
#pragma unroll
    for (int e = 0; e < E; ++e) buf[w * 64 * E + lane * E + e] = x[e];
}

// Ascending sort of a[0, P) (P a power of two, 64 <= P <= 64 * 16 * waves)
// using b[0, P) as scratch: each wavefront sorts a segment of SEG values in
// registers, then segments are merged pairwise, every value finding its place
// by a binary search in the partner segment (ties: the left segment first).
// Returns the buffer that holds the result.
template <int NT>
__device__ __forceinline__ float* sort_window(float* a, float* b, int P) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nseg = min(NW, P / 64);
    const int SEG = P / nseg;
    __syncthreads();
    if (w < nseg) {
        // values per lane: SEG / 64 <= kBuf / NT (only those shapes exist)
        constexpr int EMAX = kBuf / NT;
        const int E = SEG / 64;
        if (E == 1) wave_sort_segment<1>(a, w, lane);
        else if (E == 2) wave_sort_segment<2>(a, w, lane);
        else if (E == 4 || EMAX < 8) wave_sort_segment<(EMAX < 4 ? EMAX : 4)>(a, w, lane);
        else if (E == 8 || EMAX < 16) wave_sort_segment<(EMAX < 8 ? EMAX : 8)>(a, w, lane);
        else wave_sort_segment<(EMAX < 16 ? EMAX : 16)>(a, w, lane);
    }
    __syncthreads();
    // merge rounds (merge path): thread t writes outputs [t E, t E + E) of the
    // merged pair; it finds how many of them come from the left segment by a
    // binary search along that output diagonal (ties: the left segment
    // first), then merges its E outputs sequentially
    const int E = max(1, P / NT);
    for (int len = SEG; len < P; len <<= 1) {
        const int o0 = threadIdx.x * E;
        if (o0 < P) {
            const int pair = o0 / (2 * len);
            const float* A = a + pair * 2 * len;
            const float* B = A + len;
            const int dg = o0 - pair * 2 * len;
            int lo = max(0, dg - len), hi = min(dg, len);
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (A[mid] <= B[dg - mid - 1]) lo = mid + 1;
                else hi = mid;
            }
            int i = lo, j = dg - lo;
            float va = (i < len) ? A[i] : INFINITY, vb = (j < len) ? B[j] : INFINITY;
            float* out = b + pair * 2 * len + dg;
            for (int e = 0; e < E; ++e) {
                const bool ta = (j >= len) || (i < len && va <= vb);
                out[e] = ta ? va : vb;
                if (ta) {
                    ++i;
                    va = (i < len) ? A[i] : INFINITY;
                } else {
                    ++j;
                    vb = (j < len) ? B[j] : INFINITY;
                }
            }
        }
        __syncthreads();
        float* t = a;
        a = b;
        b = t;
    }
    return a;
}


// Bin b of a histogram is stored at slot hist_slot(b): the low bits are
// XORed with a function of the thread b / per that owns the bin in the scan,
// so that the threads of a wavefront reading their own bins side by side hit
// 64 different LDS banks.
template <int NT, int NB>
__device__ __forceinline__ int hist_slot(int b) {
    constexpr int per = NB / NT;   // a power of two <= 64
    constexpr int G = (64 / per) > 0 ? 64 / per : 1;
    return b ^ (((b / per) / G) & (per - 1));
}

// bins narrower than 0.99 units hold one integer value each (edge bins also
// collect the clamped values outside the range)
template <int NB>
__device__ __forceinline__ bool single_value_bin(bool int_vals, float scale, int b) {
    return int_vals && scale >= 1.01f && b != 0 && b != NB - 1;
}

struct Placed {
    int b1, b2;       // first and last bin of the selected ranks
    uint32_t base;    // values in bins below b1
    int m;            // values in bins b1 .. b2
    uint32_t maxnb;   // largest of those bins that may hold different values
};

// Histogram of the values each(f) visits over [lo, lo + NB / scale), the bins
// holding ranks ra and rb, and the first slot of every bin in [b1, b2]
// relative to b1 (left in the histogram for the caller's placement).
// first: also resets the window's value range (read by the caller between a
// first-level and a second-level call, so only the first one may reset it).
template <int NT, typename SH, typename Each>
__device__ __forceinline__ Placed place_bins(Each&& each, float lo, float scale, bool int_vals, int ra, int rb,
                                             bool first, SH& sh) {
    constexpr int NB = SH::kNB;
    constexpr int per = NB / NT;
    const int tid = threadIdx.x;
    for (int b = tid; b < NB; b += NT) sh.hist[b] = 0u;
    if (tid == 0) {
        sh.maxnb = 0u;
        if (first) {
            sh.wmin = 0xffffffffu;
            sh.wmax = 0u;
        }
    }
    __syncthreads();
    each([&](float x) { atomicAdd(&sh.hist[hist_slot<NT, NB>(bin_of<NB>(x, lo, scale))], 1u); });
    __syncthreads();
    uint32_t c[per];
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
        c[q] = sh.hist[hist_slot<NT, NB>(tid * per + q)];
        tot += c[q];
    }
    const uint32_t pre = block_exscan<NT>(tot, sh);
    const int rr[2] = {ra, rb};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const uint32_t r = (uint32_t)rr[t];
        if (pre <= r && r < pre + tot) {
            uint32_t cum = pre;
            for (int q = 0; q < per; ++q) {
                if (r < cum + c[q]) {
                    sh.sel_bin[t] = tid * per + q;
                    sh.sel_cum[t] = cum;
                    break;
                }
                cum += c[q];
            }
        }
    }
    __syncthreads();
    Placed P;
    P.b1 = sh.sel_bin[0];
    P.b2 = sh.sel_bin[1];
    P.base = sh.sel_cum[0];
    {
        uint32_t cum = pre, big = 0u;
#pragma unroll
        for (int q = 0; q < per; ++q) {
            const int b = tid * per + q;
            if (b >= P.b1 && b <= P.b2) {
                sh.hist[hist_slot<NT, NB>(b)] = cum - P.base;
                if (!single_value_bin<NB>(int_vals, scale, b)) big = max(big, c[q]);
            }
            if (b == P.b2) sh.cnt = cum + c[q] - P.base;
            cum += c[q];
        }
        if (big > 1u) atomicMax(&sh.maxnb, big);
    }
    __syncthreads();
    P.m = (int)sh.cnt;
    P.maxnb = sh.maxnb;
    return P;
}

// Copies src[0, m), grouped by bin (bin slices ending at the histogram's
// entries), to dst in ascending order: each value's place is its slice start
// plus the smaller values of its slice (and the equal ones before it).
template <int NT, typename SH>
__device__ __forceinline__ void rank_place(const float* src, float* dst, int m, float lo, float scale, bool int_vals,
                                           const Placed& P, SH& sh) {
    constexpr int NB = SH::kNB;
    for (int j = threadIdx.x; j < m; j += NT) {
        const float x = src[j];
        const int b = bin_of<NB>(x, lo, scale);
        int r = j;   // a bin of equal values keeps its order
        if (!single_value_bin<NB>(int_vals, scale, b)) {
            const int s0 = (b == P.b1) ? 0 : (int)sh.hist[hist_slot<NT, NB>(b - 1)];
            const int e = (int)sh.hist[hist_slot<NT, NB>(b)];
            r = s0;
            for (int i = s0; i < e; i += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ii = i + u;
                    const float y = src[min(ii, e - 1)];
                    r += (ii < e && (y < x || (y == x && ii < j))) ? 1 : 0;
                }
            }
        }
        dst[r] = x;
    }
}

// Sort the values of ranks [ra, rb] (0-based, within the alive set) and their
// bin-mates into a window; returns the rank of its first value (-1 when the
// gathered bins exceed the buffer), its count in m and its storage in win.
// each(f) calls f on every alive value of the thread; each2(f1, f2) calls f1
// on all of them, then f2(f1's result, value) where that result is >= 0.  The
// histogram window [wlo, whi] only steers the binning (bins are clamped).
// The window is gathered grouped by bin (each bin's slice found from the
// histogram's prefix sums).  Small bins are then ordered directly by rank
// counting; otherwise a second histogram over the window's own value range
// spreads it over fine bins, it is regrouped by those and ordered by rank
// counting.  A window over half the buffer, or a fine bin of more than
// kRankMax different values, goes through the merge sort instead.
// int_vals: the values are integers.
template <int NT, typename Each, typename Each2, typename SH>
__device__ __forceinline__ int build_window(Each&& each, Each2&& each2, float wlo, float whi, int ra, int rb,
                                            bool int_vals, int& m, const float*& win, SH& sh) {
    constexpr int NB = SH::kNB;
    const int tid = threadIdx.x, lane = tid & 63;
    const float scale = bin_scale<NB>(wlo, whi);
    const Placed P1 = place_bins<NT>(each, wlo, scale, int_vals, ra, rb, true, sh);
    m = P1.m;
    if (m > kBuf) return -1;
    // gather: all slots are claimed before any value is stored
    float gmn = INFINITY, gmx = -INFINITY;
    each2(
        [&](float x) {
            const int b = bin_of<NB>(x, wlo, scale);
            return (b >= P1.b1 && b <= P1.b2) ? (int)atomicAdd(&sh.hist[hist_slot<NT, NB>(b)], 1u) : -1;
        },
        [&](int slot, float x) {
            sh.buf[slot] = x;
            gmn = fminf(gmn, x);
            gmx = fmaxf(gmx, x);
        });
    gmn = wave_min(gmn);
    gmx = wave_max(gmx);
    if (lane == 0 && gmn <= gmx) {
        atomicMin(&sh.wmin, f2ord(gmn));
        atomicMax(&sh.wmax, f2ord(gmx));
    }
    __syncthreads();
    float* out = sh.buf + kBuf / 2;
    if (m <= kBuf / 2 && P1.maxnb <= (uint32_t)kRankSmall) {
        rank_place<NT>(sh.buf, out, m, wlo, scale, int_vals, P1, sh);
        __syncthreads();
        win = out;
        return (int)P1.base;
    }
    if (m <= kBuf / 2) {
        const float lo2 = ord2f(sh.wmin), hi2 = ord2f(sh.wmax);
        const float scale2 = bin_scale<NB>(lo2, hi2);
        if (!(scale2 > 0.0f)) {
            win = sh.buf;   // one value only
            return (int)P1.base;
        }
        auto each_buf = [&](auto&& f) __attribute__((always_inline)) {
            for (int j = tid; j < m; j += NT) f(sh.buf[j]);
        };
        const Placed P2 = place_bins<NT>(each_buf, lo2, scale2, int_vals, 0, m - 1, false, sh);
        if (P2.maxnb <= (uint32_t)kRankMax) {
            constexpr int MAXJ = (kBuf / 2 + NT - 1) / NT;
            int sl[MAXJ];
            float xv[MAXJ];
#pragma unroll
            for (int i = 0; i < MAXJ; ++i) {
                const int j = tid + i * NT;
                xv[i] = (j < m) ? sh.buf[j] : 0.0f;
                sl[i] = (j < m) ? (int)atomicAdd(&sh.hist[hist_slot<NT, NB>(bin_of<NB>(xv[i], lo2, scale2))], 1u)
                                : -1;
            }
#pragma unroll
            for (int i = 0; i < MAXJ; ++i)
                if (sl[i] >= 0) out[sl[i]] = xv[i];
            __syncthreads();
            rank_place<NT>(out, sh.buf, m, lo2, scale2, int_vals, P2, sh);
            __syncthreads();
            win = sh.buf;
            return (int)P1.base;
        }
    }
    int Pn = 64;
    while (Pn < m) Pn <<= 1;
    for (int i = m + tid; i < Pn; i += NT) sh.buf[i] = INFINITY;
    win = sort_window<NT>(sh.buf, sh.buf2, Pn);
    return (int)P1.base;
}

// Values of ranks r1 <= r2 of the alive set by bisection on the
// order-preserving keys; count_le(x) gives the thread's alive values <= x.
// For windows the buffer cannot hold.
template <int NT, typename SH, typename CountLe>
__device__ void bisect_pair(CountLe&& count_le, float lmn, float lmx, int r1, int r2, float& o1, float& o2,
                            SH& sh) {
    auto kth = [&](int k) {
        uint32_t a = f2ord(lmn), z = f2ord(lmx);
        while (a < z) {
            const uint32_t mid = a + ((z - a) >> 1);
            const int cnt = block_sum_i<NT>(count_le(ord2f(mid)), sh);
            if (cnt > k) z = mid;
            else a = mid + 1;
        }
        return ord2f(a);
    };
    o1 = kth(r1);
    o2 = (r2 == r1) ? o1 : kth(r2);
}

// One workgroup per mesh; the mesh's pixels stay in registers (PPT per
// thread) for the whole clipping loop, a clipped value being replaced by NaN
// (pixel values are finite).  Pass 0 gives sigma0 of all pixels.  A clipping
// pass tests every alive value against the interval, taking the dropped
// values off the thread's FP64 sums.  The median comes from a sorted window of
// ranks around it (built through a histogram of the alive values), which
// stays valid while the ranks removed below keep the median inside it.  With
// no pixel array in LDS, several meshes share a compute unit.
// waves per SIMD the register budget is set for: two 8-wave or four 4-wave
// workgroups per compute unit
template <int NT, int PPT>
constexpr int mesh_waves_per_eu() { return 4; }

// ONE: a one-frame call, whose descriptor comes with the launch (d1);
// workgroup 0 stores it in the table for the launches that follow
template <int NT, int PPT, bool ONE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(mesh_waves_per_eu<NT, PPT>())))
void k_mesh_stats(FrameDesc* __restrict__ desc, FrameDesc d1, int nframes, BkgArgs a) {
    __shared__ MeshShared<kBins> sh;
    const int tid = threadIdx.x;
    const int gm = blockIdx.x;
    if (ONE && gm == 0 && tid == 0) desc[0] = d1;
    const int f = ONE ? 0 : frame_of(nframes, gm, [&](int i) { return desc[i].mesh_base; });
    const FrameDesc d = ONE ? d1 : desc[f];
    if (a.skip_u16 && d.dtype == kDtypeU16) return;
    const int lm = gm - d.mesh_base;
    const int mi = lm % d.nx, mj = lm / d.nx;
    const int x0 = mi * d.mw, y0 = mj * d.mh;
    const int w = min(d.mw, d.W - x0), h = min(d.mh, d.H - y0);
    const int n = w * h;
    const bool int_vals = d.dtype == kDtypeU16;

    float v[PPT];
    int cnt_t = 0;
    {
        // pixel k * NT + tid of the mesh.  A full mesh whose width divides NT
        // puts every thread's k-th pixel dy = NT / w rows below its previous
        // one: buffer loads with the row step as a scalar offset.  Other
        // meshes step by NT without divisions.
        const int dy = NT / w, dx = NT - dy * w;
        int yy = tid / w, xx = tid - yy * w;
        const bool u16 = d.dtype == kDtypeU16;
        const int es = u16 ? 2 : 4;
        // (byte offsets within the mesh must fit the 32-bit buffer offsets)
        if (n == NT * PPT && dx == 0 && (int64_t)h * d.pitch * es < ((int64_t)1 << 31)) {
            const int64_t o0 = ((int64_t)y0 * d.pitch + x0) * es;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)d.data + o0), (short)0, 0x7fffffff, 0x00020000);
            const int vo = (yy * (int)d.pitch + xx) * es;
            const int so = dy * (int)d.pitch * es;
            if (u16) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) v[k] = (float)__builtin_amdgcn_raw_buffer_load_b16(rs, vo, k * so, 0);
            } else {
#pragma unroll
                for (int k = 0; k < PPT; ++k)
                    v[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, k * so, 0));
            }
            cnt_t = PPT;
        } else {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                v[k] = NAN;
                if (k * NT + tid < n) {
                    v[k] = load_px(d, x0 + xx, y0 + yy);
                    ++cnt_t;
                }
                xx += dx;
                yy += dy;
                if (xx >= w) {
                    xx -= w;
                    ++yy;
                }
            }
        }
    }
    // pass 0: sigma0 of all pixels (FP64 sums shifted by the first pixel)
    const double c0 = (double)load_px(d, x0, y0);
    double s1 = 0.0, s2 = 0.0;
    float mn = INFINITY, mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (k < cnt_t) {
            const double dd = (double)v[k] - c0;
            s1 += dd;
            s2 = fma(dd, dd, s2);
            mn = fminf(mn, v[k]);
            mx = fmaxf(mx, v[k]);
        }
    }
    int cnt = 0, unused = 0, par = 0;
    block_stats<NT>(s1, s2, cnt, unused, mn, mx, par, sh);
    const int out_idx = mj * d.nx + mi;
    if (mn == mx) {
        if (tid == 0) {
            d.back_raw[out_idx] = (double)mn;
            d.rms_raw[out_idx] = 0.0;
            d.iters[out_idx] = 0;
        }
        return;
    }
    const double nd0 = (double)n;
    const double m1 = s1 / nd0;
    const double var0 = s2 / nd0 - m1 * m1;
    const double sig0 = sqrt(var0 > 0.0 ? var0 : 0.0);
    double mean = c0 + m1;
    double sig = sig0;

    int ncur = n;
    int R0 = -1, bm = 0;      // rank of win[0] in the alive set (-1: no window)
    const float* win = sh.buf;
    float med_h, med_l;
    float lmn = mn, lmx = mx;
    // every alive value of the thread (NaN marks the padding and clipped ones);
    // each2 claims all results of f1 (in groups of 16) before calling f2
    auto each_alive = [&](auto&& f) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < PPT; ++k)
            if (v[k] == v[k]) f(v[k]);
    };
    auto each2_alive = [&](auto&& f1, auto&& f2) __attribute__((always_inline)) {
        constexpr int C = PPT < 16 ? PPT : 16;
#pragma unroll
        for (int k0 = 0; k0 < PPT; k0 += C) {
            int r[C];
#pragma unroll
            for (int k = 0; k < C; ++k) r[k] = (v[k0 + k] == v[k0 + k]) ? f1(v[k0 + k]) : -1;
#pragma unroll
            for (int k = 0; k < C; ++k)
                if (r[k] >= 0) f2(r[k], v[k0 + k]);
        }
    };
    auto count_le = [&](float x) {
        int c = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) c += (v[k] <= x) ? 1 : 0;   // false for NaN
        return c;
    };
    // exact median (an unevaluated pair when the count is even) of the alive
    // set, from the window, rebuilding it when the median has left it
    auto median = [&](float wlo, float whi) __attribute__((always_inline)) {
        const int r2 = ncur / 2;
        const int r1 = (ncur & 1) ? r2 : r2 - 1;
        float o1, o2;
        if (R0 < 0 || r1 - R0 < 0 || r2 - R0 >= bm) {
            R0 = build_window<NT>(each_alive, each2_alive, wlo, whi, max(r1 - kHalf, 0), min(r2 + kHalf, ncur - 1),
                                  int_vals, bm, win, sh);
            if (R0 < 0) R0 = build_window<NT>(each_alive, each2_alive, wlo, whi, r1, r2, int_vals, bm, win, sh);
        }
        if (R0 >= 0) {
            o1 = win[r1 - R0];
            o2 = win[r2 - R0];
        } else {
            bisect_pair<NT>(count_le, lmn, lmx, r1, r2, o1, o2, sh);
        }
        if (r1 == r2) {
            med_h = o1;
            med_l = 0.0f;
        } else {
            // (o1 + o2) / 2 as an unevaluated pair: exact
            float s, e;
            two_sum(o1, o2, s, e);
            med_h = 0.5f * s;
            med_l = 0.5f * e;
        }
    };
    // the median of all pixels lies within one sigma of their mean
    median((float)(mean - sig0), (float)(mean + sig0));
    // the alive set's FP64 sums, shifted by a float near the mean (so every
    // shifted value is exact)
    const double cs = (double)(float)mean;
    double t1 = 0.0, t2 = 0.0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (k < cnt_t) {
            const double e = (double)v[k] - cs;
            t1 += e;
            t2 = fma(e, e, t2);
        }
    }

    int iters = 0, na = cnt_t;   // alive values of the thread
    for (int it = 0; it < a.max_iter; ++it) {
        const float thr = (float)((double)a.clip * sig);
        // clipping pass: every alive value outside the interval is dropped;
        // only those below it shift the ranks of the survivors.  A NaN (dead)
        // value compares false, and fminf / fmaxf pass over it.
        int nrem = 0;
        float tmn = INFINITY, tmx = -INFINITY;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const float x = v[k];
            const float dx = (x - med_h) - med_l;
            if (fabsf(dx) > thr) {
                const double e = (double)x - cs;
                t1 -= e;
                t2 = fma(-e, e, t2);
                nrem += (dx < -thr) ? 1 : 0;
                --na;
                v[k] = NAN;
            }
            tmn = fminf(tmn, v[k]);
            tmx = fmaxf(tmx, v[k]);
        }
        int nn = na;
        double q1s = t1, q2s = t2;
        block_stats<NT>(q1s, q2s, nn, nrem, tmn, tmx, par, sh);
        ++iters;
        if (nn == ncur || nn == 0) break;
        ncur = nn;
        if (R0 >= 0) R0 -= nrem;
        lmn = tmn;
        lmx = tmx;
        const double nd = (double)nn;
        const double q1 = q1s / nd;
        const double vv = q2s / nd - q1 * q1;
        mean = cs + q1;
        sig = (lmn == lmx) ? 0.0 : sqrt(vv > 0.0 ? vv : 0.0);
        median(lmn, lmx);
    }
    if (tid == 0) {
        const double med = (double)med_h + (double)med_l;
        const double dsig = fabs(sig - sig0);
        const double back = (dsig < (double)a.crowd * sig0) ? mean
                                                             : ((double)a.mode_a * med - (double)a.mode_b * mean);
        d.back_raw[out_idx] = back;
        d.rms_raw[out_idx] = sig;
        d.iters[out_idx] = iters;
    }
}


// ---------------------------------------------------------------------------
// uint16 frames: exact integer statistics.  Each clipping pass keeps the
// values within k sigma of the current median, so the surviving set is
// always every pixel value inside an interval [L, H] of integers.  With one
// LDS histogram of the mesh's values (1-ADU bins over a 4096-value window
// around the median; a bright star that stretches the range first gets a
// coarse histogram that locates that window) the counts, sums and exact
// median of every pass come from the histogram's prefix, and all sums are
// exact integers: no per-pixel work after the histogram, unless an interval
// or a median leaves the window (then exact passes over the registers).
// The clip decisions are taken in FP64 on exact statistics, like the FP64
// definition.
constexpr int kU16Bins = 1024;            // 64 lanes x 16 bins
constexpr int kU16Per = kU16Bins / 64;

// The window's prefix sums: p0[b] = pixels in bins [0, b), p1[b] and p2[b]
// their sums of (bin) and (bin)^2; index kU16Bins holds the totals.
struct MeshU16Shared {
    uint32_t p0[kU16Bins + 1];          // histogram, then its prefix
    uint32_t p1[kU16Bins + 1];
    uint64_t p2[kU16Bins + 1];
    uint64_t pa[2][kMaxWaves][2];       // block partials, double-buffered
    uint32_t pc[2][kMaxWaves][4];
    uint64_t ws[kMaxWaves][2];          // wavefront totals of the scan
    uint32_t wc[kMaxWaves];
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o) {
    const uint32_t lo = __shfl_xor((uint32_t)v, o), hi = __shfl_xor((uint32_t)(v >> 32), o);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int o) {
    const uint32_t lo = __shfl_up((uint32_t)v, o), hi = __shfl_up((uint32_t)(v >> 32), o);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// exact block sums: two counts, two 64-bit sums, min and max (integers: the
// order of the additions does not matter)
template <int NT>
__device__ __forceinline__ void block_u16(uint32_t& c0, uint32_t& c1, uint64_t& s1, uint64_t& s2, uint32_t& mn,
                                          uint32_t& mx, int& par, MeshU16Shared& sh) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    const int P = par;
    par ^= 1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        c0 += __shfl_xor(c0, o);
        c1 += __shfl_xor(c1, o);
        s1 += shfl_xor_u64(s1, o);
        s2 += shfl_xor_u64(s2, o);
        mn = min(mn, (uint32_t)__shfl_xor(mn, o));
        mx = max(mx, (uint32_t)__shfl_xor(mx, o));
    }
    if ((threadIdx.x & 63) == 0) {
        sh.pc[P][w][0] = c0;
        sh.pc[P][w][1] = c1;
        sh.pc[P][w][2] = mn;
        sh.pc[P][w][3] = mx;
        sh.pa[P][w][0] = s1;
        sh.pa[P][w][1] = s2;
    }
    __syncthreads();
    c0 = c1 = 0u;
    s1 = s2 = 0ull;
    mn = 0xffffffffu;
    mx = 0u;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        c0 += sh.pc[P][i][0];
        c1 += sh.pc[P][i][1];
        mn = min(mn, sh.pc[P][i][2]);
        mx = max(mx, sh.pc[P][i][3]);
        s1 += sh.pa[P][i][0];
        s2 += sh.pa[P][i][1];
    }
}

// histogram in p0 -> exclusive prefix sums p0, p1, p2 (bins split evenly
// over the block, each thread a contiguous run)
template <int NT>
__device__ __forceinline__ void u16_prefix(MeshU16Shared& sh) {
    constexpr int PER = kU16Bins / NT;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t c[PER], tc = 0, t1 = 0;
    uint64_t t2 = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const uint32_t b = (uint32_t)(t * PER + i);
        c[i] = sh.p0[b];
        tc += c[i];
        t1 += c[i] * b;
        t2 += (uint64_t)c[i] * b * b;
    }
    uint32_t ic = tc, i1 = t1;
    uint64_t i2 = t2;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t yc = __shfl_up(ic, o), y1 = __shfl_up(i1, o);
        const uint64_t y2 = shfl_up_u64(i2, o);
        if (lane >= o) {
            ic += yc;
            i1 += y1;
            i2 += y2;
        }
    }
    if (lane == 63) {
        sh.wc[w] = ic;
        sh.ws[w][0] = i1;
        sh.ws[w][1] = i2;
    }
    __syncthreads();
    uint32_t rc = ic - tc, r1 = i1 - t1;
    uint64_t r2 = i2 - t2;
    for (int i = 0; i < w; ++i) {
        rc += sh.wc[i];
        r1 += (uint32_t)sh.ws[i][0];
        r2 += sh.ws[i][1];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const uint32_t b = (uint32_t)(t * PER + i);
        sh.p0[b] = rc;
        sh.p1[b] = r1;
        sh.p2[b] = r2;
        rc += c[i];
        r1 += c[i] * b;
        r2 += (uint64_t)c[i] * b * b;
    }
    if (t == NT - 1) {
        sh.p0[kU16Bins] = rc;
        sh.p1[kU16Bins] = r1;
        sh.p2[kU16Bins] = r2;
    }
    __syncthreads();
}

// largest bin b with p0[b] <= g (0 <= g < total): two LDS reads and ballots
// per wavefront, no barrier
__device__ __forceinline__ int u16_find(const MeshU16Shared& sh, uint32_t g) {
    const int lane = threadIdx.x & 63;
    const int c = __popcll(__ballot(sh.p0[lane * kU16Per] <= g)) - 1;
    const bool le = lane < kU16Per && sh.p0[c * kU16Per + lane] <= g;
    return c * kU16Per + __popcll(__ballot(le)) - 1;
}

template <int NT, int PPT, bool ONE>
__global__ __launch_bounds__(NT) void k_mesh_stats_u16(FrameDesc* __restrict__ desc, FrameDesc d1, int nframes,
                                                       BkgArgs a) {
    __shared__ MeshU16Shared sh;
    constexpr uint32_t kNone = 0xffffffffu;   // padding / not a pixel
    const int tid = threadIdx.x, lane = tid & 63;
    const int gm = blockIdx.x;
    if (ONE && gm == 0 && tid == 0) desc[0] = d1;
    const int f = ONE ? 0 : frame_of(nframes, gm, [&](int i) { return desc[i].mesh_base; });
    const FrameDesc d = ONE ? d1 : desc[f];
    if (d.dtype != kDtypeU16) return;   // float32 frames of a mixed batch: the float kernel
    const int lm = gm - d.mesh_base;
    const int mi = lm % d.nx, mj = lm / d.nx;
    const int x0 = mi * d.mw, y0 = mj * d.mh;
    const int w = min(d.mw, d.W - x0), h = min(d.mh, d.H - y0);
    const int n = w * h;
    const int out_idx = mj * d.nx + mi;

    // 1. the mesh's pixels into registers (pixel k * NT + tid of the mesh)
    uint32_t u[PPT];
    {
        const int dy = NT / w, dx = NT - dy * w;
        int yy = tid / w, xx = tid - yy * w;
        if (n == NT * PPT && dx == 0 && (int64_t)h * d.pitch * 2 < ((int64_t)1 << 31)) {
            const int64_t o0 = ((int64_t)y0 * d.pitch + x0) * 2;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)d.data + o0), (short)0, 0x7fffffff, 0x00020000);
            const int vo = (yy * (int)d.pitch + xx) * 2;
            const int so = dy * (int)d.pitch * 2;
#pragma unroll
            for (int k = 0; k < PPT; ++k) u[k] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, vo, k * so, 0);
        } else {
            const gu16_t* src = (const gu16_t*)d.data;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                u[k] = kNone;
                if (k * NT + tid < n) u[k] = (uint32_t)src[(int64_t)(y0 + yy) * d.pitch + x0 + xx];
                xx += dx;
                yy += dy;
                if (xx >= w) {
                    xx -= w;
                    ++yy;
                }
            }
        }
    }
    // 2. count, min, max and the exact sums of (v - c0), (v - c0)^2 about the
    //    mesh's first pixel c0 (then re-centred on the minimum), one barrier
    const uint32_t c0 = (uint32_t)((const gu16_t*)d.data)[(int64_t)y0 * d.pitch + x0];
    uint32_t na = 0u, unused = 0u, mn = 0xffffffffu, mx = 0u;
    uint64_t t1 = 0ull, t2 = 0ull;   // (v - c0) as two's complement, (v - c0)^2
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint32_t v = u[k];
        if (v != kNone) {
            const int64_t e = (int64_t)v - (int64_t)c0;
            ++na;
            t1 += (uint64_t)e;
            t2 += (uint64_t)(e * e);
            mn = min(mn, v);
            mx = max(mx, v);
        }
    }
    int par = 0;
    block_u16<NT>(na, unused, t1, t2, mn, mx, par, sh);
    if (mn == mx) {
        if (tid == 0) {
            d.back_raw[out_idx] = (double)mn;
            d.rms_raw[out_idx] = 0.0;
            d.iters[out_idx] = 0;
        }
        return;
    }
    {
        // about the minimum: S1' = S1 + n (c0 - mn), S2' = S2 + 2 (c0 - mn) S1 + n (c0 - mn)^2
        const int64_t sh0 = (int64_t)c0 - (int64_t)mn;
        const int64_t s1 = (int64_t)t1;
        t2 = (uint64_t)((int64_t)t2 + 2 * sh0 * s1 + (int64_t)na * sh0 * sh0);
        t1 = (uint64_t)(s1 + (int64_t)na * sh0);
    }
    // exact statistics of the pixels in [lo, hi] from the registers (all
    // wavefronts, one barrier): count, count below lo, sums of (v - mn)^p
    auto reg_stats = [&](uint32_t lo, uint32_t hi, uint32_t& c, uint32_t& below, uint64_t& s1, uint64_t& s2) {
        c = below = 0u;
        s1 = s2 = 0ull;
        uint32_t z0 = 0xffffffffu, z1 = 0u;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint32_t v = u[k];
            const bool in = v != kNone && v >= lo && v <= hi;
            const uint64_t dd = (uint64_t)(v - mn);
            c += in ? 1u : 0u;
            below += (v < lo) ? 1u : 0u;
            s1 += in ? dd : 0ull;
            s2 += in ? dd * dd : 0ull;
        }
        block_u16<NT>(c, below, s1, s2, z0, z1, par, sh);
    };
    // 3. histogram window: 1-ADU bins over [wlo, wlo + NB) holding the
    //    median, with prefix sums; cbw = pixels below it
    int sft = 0;
    while (((mx - mn) >> sft) >= (uint32_t)kU16Bins) ++sft;
    for (int b = tid; b < kU16Bins; b += NT) sh.p0[b] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (u[k] != kNone) atomicAdd(&sh.p0[(u[k] - mn) >> sft], 1u);
    __syncthreads();
    u16_prefix<NT>(sh);
    uint32_t wlo = mn, cbw = 0u;
    if (sft > 0) {
        // the coarse bin of the lower median; the window starts half a window
        // below it, on a coarse-bin boundary
        const int bm = u16_find(sh, (na - 1) / 2);
        const int b0 = max(0, bm - ((kU16Bins / 2) >> sft));
        cbw = sh.p0[b0];
        wlo = mn + ((uint32_t)b0 << sft);
        __syncthreads();
        for (int b = tid; b < kU16Bins; b += NT) sh.p0[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint32_t r = u[k] - wlo;   // (kNone and values below wlo wrap above NB)
            if (u[k] != kNone && r < (uint32_t)kU16Bins) atomicAdd(&sh.p0[r], 1u);
        }
        __syncthreads();
        u16_prefix<NT>(sh);
    }
    const uint32_t wtot = sh.p0[kU16Bins];
    const uint32_t whi = wlo + (uint32_t)kU16Bins - 1u;   // last value inside the window
    // From here every wavefront runs the clipping loop by itself on the same
    // data (uniform results, no barrier), except for the rare intervals or
    // ranks outside the window, which take block-wide register passes.
    auto stats = [&](uint32_t lo, uint32_t hi, uint32_t& c, uint32_t& below, uint64_t& s1, uint64_t& s2) {
        if (lo >= wlo && hi <= whi) {
            const uint32_t a0 = lo - wlo, a1 = hi - wlo + 1;
            c = sh.p0[a1] - sh.p0[a0];
            const uint64_t q1 = (uint64_t)(sh.p1[a1] - sh.p1[a0]);
            const uint64_t q2 = sh.p2[a1] - sh.p2[a0];
            // sums of (v - mn) = (bin + off)
            const uint64_t off = (uint64_t)(wlo - mn);
            s1 = q1 + off * c;
            s2 = q2 + 2ull * off * q1 + off * off * c;
            below = cbw + sh.p0[a0];
        } else {
            reg_stats(lo, hi, c, below, s1, s2);
        }
    };
    // value of global rank g (0-based over all the mesh's pixels) within [lo, hi]
    auto value_at = [&](uint32_t g, uint32_t lo, uint32_t hi) -> uint32_t {
        if (g >= cbw && g < cbw + wtot) return wlo + (uint32_t)u16_find(sh, g - cbw);
        // outside the window: bisection on the smallest x with #(v <= x) > g
        uint32_t zl = lo, zh = hi;
        while (zl < zh) {
            const uint32_t mid = zl + ((zh - zl) >> 1);
            uint32_t c, bl;
            uint64_t s1, s2;
            reg_stats(0u, mid, c, bl, s1, s2);
            if (c > g) zh = mid;
            else zl = mid + 1;
        }
        return zl;
    };
    auto sigma_of = [&](uint32_t c, uint64_t s1, uint64_t s2) {
        // n^2 var = n S2 - S1^2, exact in 64-bit integers (< 2^61)
        const uint64_t num = (uint64_t)c * s2 - s1 * s1;
        const double nd = (double)c;
        return sqrt((double)num / (nd * nd));
    };
    const double sig0 = sigma_of(na, t1, t2);
    double sig = sig0;
    double mean = (double)mn + (double)t1 / (double)na;
    uint32_t L = mn, H = mx, below = 0u;
    auto median = [&]() {
        const uint32_t r2 = na / 2, r1 = (na & 1) ? r2 : r2 - 1;
        const uint32_t v1 = value_at(below + r1, L, H);
        const uint32_t v2 = (r2 == r1) ? v1 : value_at(below + r2, L, H);
        return 0.5 * ((double)v1 + (double)v2);
    };
    double med = median();
    const double clip = (double)a.clip;
    int iters = 0;
    for (int it = 0; it < a.max_iter; ++it) {
        const double lim = clip * sig;
        // the new interval: every integer v of [L, H] with |v - med| <= lim
        // (the differences are exact; the bounds from FP64 are nudged to the
        // exact decision)
        double cl = ceil(med - lim), ch = floor(med + lim);
        while (cl - 1.0 >= (double)L && med - (cl - 1.0) <= lim) cl -= 1.0;
        while (cl <= (double)H && med - cl > lim) cl += 1.0;
        while (ch + 1.0 <= (double)H && (ch + 1.0) - med <= lim) ch += 1.0;
        while (ch >= (double)L && ch - med > lim) ch -= 1.0;
        const uint32_t Ln = (uint32_t)fmax(cl, (double)L), Hn = (uint32_t)fmin(ch, (double)H);
        uint32_t c = 0u, bl = 0u;
        uint64_t s1 = 0ull, s2 = 0ull;
        if (Ln <= Hn) stats(Ln, Hn, c, bl, s1, s2);
        ++iters;
        if (c == na || c == 0u) break;
        L = Ln;
        H = Hn;
        na = c;
        below = bl;
        sig = (L == H) ? 0.0 : sigma_of(c, s1, s2);
        mean = (double)mn + (double)s1 / (double)c;
        med = median();
    }
    if (tid == 0) {
        const double dsig = fabs(sig - sig0);
        const double back = (dsig < (double)a.crowd * sig0) ? mean
                                                             : ((double)a.mode_a * med - (double)a.mode_b * mean);
        d.back_raw[out_idx] = back;
        d.rms_raw[out_idx] = sig;
        d.iters[out_idx] = iters;
    }
}

// ---------------------------------------------------------------------------
// f x f median over the mesh grid, back and rms separately
// median of w[0], w[S], ..., w[(n-1) S] (insertion sort in place)
__device__ double median_small(double* w, int n, int S) {
    for (int i = 1; i < n; ++i) {
        const double x = w[i * S];
        int j = i - 1;
        while (j >= 0 && w[j * S] > x) {
            w[(j + 1) * S] = w[j * S];
            --j;
        }
        w[(j + 1) * S] = x;
    }
    return (n & 1) ? w[(n / 2) * S] : 0.5 * (w[(n / 2 - 1) * S] + w[(n / 2) * S]);
}

// median of the first n of w[0, N) (the rest +inf) by rank counting: the value
// of rank k has k smaller values (equal ones ranked by position)
template <int N>
__device__ __forceinline__ double median_regs(const double (&w)[N], int n) {
    const int k1 = (n - 1) / 2, k2 = n / 2;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        int r = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) r += (w[j] < w[i] || (w[j] == w[i] && j < i)) ? 1 : 0;
        a = (r == k1) ? w[i] : a;
        b = (r == k2) ? w[i] : b;
    }
    return (n & 1) ? a : 0.5 * (a + b);
}

// one thread per mesh.  F > 0: the F x F window in registers (all loads in
// flight); F == 0: any size, the window in the thread's own LDS column
constexpr int kGridThreads = 64;
template <int F>
__global__ __launch_bounds__(kGridThreads) void k_grid_filter(const FrameDesc* __restrict__ desc, int nframes,
                                                              int total, int fsize) {
    __shared__ double w[(F > 0) ? 1 : 49 * kGridThreads];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int f = frame_of(nframes, g, [&](int i) { return desc[i].mesh_base; });
    const FrameDesc& d = desc[f];
    const int lm = g - d.mesh_base;
    const int i = lm % d.nx, j = lm / d.nx;
    const int hh = (F > 0) ? F / 2 : fsize / 2;
    if constexpr (F > 0) {
        double wb[F * F], wr[F * F];
        int n = 0;
#pragma unroll
        for (int e = 0; e < F * F; ++e) {
            const int b = j - hh + e / F, c = i - hh + e % F;
            const bool in = b >= 0 && b < d.ny && c >= 0 && c < d.nx;
            wb[e] = in ? d.back_raw[b * d.nx + c] : INFINITY;
            wr[e] = in ? d.rms_raw[b * d.nx + c] : INFINITY;
            n += in ? 1 : 0;
        }
        d.back[lm] = median_regs(wb, n);
        d.rms[lm] = median_regs(wr, n);
    } else {
        double* wt = w + threadIdx.x;
        for (int q = 0; q < 2; ++q) {
            const double* src = q ? d.rms_raw : d.back_raw;
            double* dst = q ? d.rms : d.back;
            int n = 0;
            for (int b = j - hh; b <= j + hh; ++b)
                for (int c = i - hh; c <= i + hh; ++c)
                    if (b >= 0 && b < d.ny && c >= 0 && c < d.nx) wt[(n++) * kGridThreads] = src[b * d.nx + c];
            dst[lm] = median_small(wt, n, kGridThreads);
        }
    }
}

// ---------------------------------------------------------------------------
// Natural spline second derivatives through (t_k, f_k), k < n, by Thomas
// elimination.  The elimination factors depend on the knots only, so a block
// computes them once into LDS (spline_factor) and every column then runs a
// single dependent chain (spline_solve), its right-hand sides loaded ahead.
__device__ void spline_factor(int n, const double* t, double* c, double* den) {
    double cp = 0.0;
    for (int k = 1; k <= n - 2; ++k) {
        const double h0 = t[k] - t[k - 1], h1 = t[k + 1] - t[k];
        const double b = 2.0 * (h0 + h1);
        const double dk = (k == 1) ? b : b - h0 * cp;
        den[k] = dk;
        cp = h1 / dk;
        c[k] = cp;
    }
}

// f at stride fs; r (work) and m (result) at stride ms
__device__ void spline_solve(int n, const double* t, const double* c, const double* den,
                             const double* __restrict__ f, int fs, double* __restrict__ r,
                             double* __restrict__ m, int ms) {
    m[0] = 0.0;
    if (n > 1) m[(n - 1) * ms] = 0.0;
    if (n < 3) return;
    double rp = 0.0;
    double f0 = f[0], f1 = f[fs];
#pragma unroll 4
    for (int k = 1; k <= n - 2; ++k) {
        const double f2 = f[(k + 1) * fs];
        const double h0 = t[k] - t[k - 1], h1 = t[k + 1] - t[k];
        const double rhs = 6.0 * ((f2 - f1) / h1 - (f1 - f0) / h0);
        rp = (k == 1) ? rhs / den[k] : (rhs - h0 * rp) / den[k];
        r[k * ms] = rp;
        f0 = f1;
        f1 = f2;
    }
    double mk = rp;
    m[(n - 2) * ms] = mk;
#pragma unroll 4
    for (int k = n - 3; k >= 1; --k) {
        mk = r[k * ms] - c[k] * mk;
        m[k * ms] = mk;
    }
}

// cubic of one spline piece in local coordinate s = t - ref:
// piece 0 (t < t_0) and piece n (t >= t_{n-1}) are the end tangents,
// piece j in [1, n-1] spans [t_{j-1}, t_j)
__device__ void piece_poly(int n, const double* t, const double* f, int fs, const double* m, int ms,
                           int piece, double out[4]) {
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (n == 1) {
        out[0] = f[0];
        return;
    }
    if (piece == 0) {
        double h = t[1] - t[0];
        out[0] = f[0];
        out[1] = (f[fs] - f[0]) / h - h * (2.0 * m[0] + m[ms]) / 6.0;
        return;
    }
    if (piece == n) {
        double h = t[n - 1] - t[n - 2];
        out[0] = f[(n - 1) * fs];
        out[1] = (f[(n - 1) * fs] - f[(n - 2) * fs]) / h + h * (m[(n - 2) * ms] + 2.0 * m[(n - 1) * ms]) / 6.0;
        return;
    }
    int j = piece - 1;
    double h = t[j + 1] - t[j];
    double mj = m[j * ms], mj1 = m[(j + 1) * ms];
    out[0] = f[j * fs];
    out[1] = (f[(j + 1) * fs] - f[j * fs]) / h - h * (2.0 * mj + mj1) / 6.0;
    out[2] = 0.5 * mj;
    out[3] = (mj1 - mj) / (6.0 * h);
}

constexpr int kSplThreads = 256;
constexpr int kSplCols = 64;       // small grids: columns per workgroup (one wavefront)
constexpr int kSplSmallN = 100;    // small grids: knots per axis held in LDS

// The same elimination with reciprocals: ih[k] = 1 / (t_{k+1} - t_k) (every
// thread computes its share before the call), c[k] and iden[k] = 1 / den[k]
// (one thread), so the column solves are chains of FMAs.
__device__ __forceinline__ void spline_factor_inv(int n, const double* t, double* c, double* iden) {
    double cp = 0.0;
    for (int k = 1; k <= n - 2; ++k) {
        const double h0 = t[k] - t[k - 1], h1 = t[k + 1] - t[k];
        const double b = 2.0 * (h0 + h1);
        const double id = 1.0 / ((k == 1) ? b : b - h0 * cp);
        iden[k] = id;
        cp = h1 * id;
        c[k] = cp;
    }
}

// second derivatives m (stride ms) of the column f (stride fs); m holds the
// forward sweep's values until the back sweep overwrites them in place
__device__ __forceinline__ void spline_solve_inv(int n, const double* t, const double* c, const double* iden,
                                                 const double* ih, const double* f, int fs, double* m, int ms) {
    m[0] = 0.0;
    if (n > 1) m[(n - 1) * ms] = 0.0;
    if (n < 3) return;
    double rp = 0.0;
    double f0 = f[0], f1 = f[fs];
#pragma unroll 4
    for (int k = 1; k <= n - 2; ++k) {
        const double f2 = f[(k + 1) * fs];
        const double rhs = 6.0 * ((f2 - f1) * ih[k] - (f1 - f0) * ih[k - 1]);
        rp = (rhs - (t[k] - t[k - 1]) * rp) * iden[k];
        m[k * ms] = rp;
        f0 = f1;
        f1 = f2;
    }
    double mk = rp;
#pragma unroll 4
    for (int k = n - 3; k >= 1; --k) {
        mk = m[k * ms] - c[k] * mk;
        m[k * ms] = mk;
    }
}

// piece_poly with the reciprocal spacings
__device__ __forceinline__ void piece_poly_inv(int n, const double* t, const double* ih, const double* f, int fs,
                                               const double* m, int ms, int piece, double out[4]) {
    constexpr double kSixth = 1.0 / 6.0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (n == 1) {
        out[0] = f[0];
        return;
    }
    if (piece == 0) {
        const double h = t[1] - t[0];
        out[0] = f[0];
        out[1] = (f[fs] - f[0]) * ih[0] - h * (2.0 * m[0] + m[ms]) * kSixth;
        return;
    }
    if (piece == n) {
        const double h = t[n - 1] - t[n - 2];
        out[0] = f[(n - 1) * fs];
        out[1] = (f[(n - 1) * fs] - f[(n - 2) * fs]) * ih[n - 2] + h * (m[(n - 2) * ms] + 2.0 * m[(n - 1) * ms]) * kSixth;
        return;
    }
    const int j = piece - 1;
    const double h = t[j + 1] - t[j];
    const double mj = m[j * ms], mj1 = m[(j + 1) * ms];
    out[0] = f[j * fs];
    out[1] = (f[(j + 1) * fs] - f[j * fs]) * ih[j] - h * (2.0 * mj + mj1) * kSixth;
    out[2] = 0.5 * mj;
    out[3] = (mj1 - mj) * ih[j] * kSixth;
}

// A column of n values (stride s) into the LDS column `lane` of fl.  The
// first kSplPre loads are issued by prefetch_column and waited for only in
// store_column, so the knot factorisation runs while they are in flight; the
// rest follow 16 at a time.  Indices are clamped to the column, so no load
// needs a branch.
constexpr int kSplPre = 64;

__device__ __forceinline__ void prefetch_column(double (&x)[kSplPre], const double* v, int s, int n) {
    const gdouble_t* g = (const gdouble_t*)v;   // global loads: they do not hold up LDS waits
#pragma unroll
    for (int j = 0; j < kSplPre; ++j) x[j] = g[(size_t)min(j, n - 1) * s];
}

__device__ __forceinline__ void store_column(double* fl, int lane, const double (&x)[kSplPre], const double* v,
                                             int s, int n) {
#pragma unroll
    for (int j = 0; j < kSplPre; ++j)
        if (j < n) fl[j * kSplCols + lane] = x[j];
    const gdouble_t* g = (const gdouble_t*)v;
    for (int k0 = kSplPre; k0 < n; k0 += 16) {
        double y[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) y[j] = g[(size_t)min(k0 + j, n - 1) * s];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (k0 + j < n) fl[(k0 + j) * kSplCols + lane] = y[j];
    }
}

// Small grids (at most kSplSmallN knots on the solved axis): a wavefront takes
// 64 columns; their values are loaded into LDS at once (all loads in flight),
// solved and cut into pieces there, and only the pieces go to global memory.
// blockIdx.y = frame.  Y: one column per (quantity, mesh column).
__global__ __launch_bounds__(kSplCols) void k_spline_y_small(const FrameDesc* __restrict__ desc) {
    __shared__ double tk[kSplSmallN], cf[kSplSmallN], idn[kSplSmallN], ih[kSplSmallN];
    __shared__ double fl[kSplSmallN * kSplCols], ml[kSplSmallN * kSplCols];
    const FrameDesc& d = desc[blockIdx.y];
    const int ny = d.ny, nx = d.nx, lane = threadIdx.x;
    if ((int)blockIdx.x * kSplCols >= 2 * nx) return;
    const int g = blockIdx.x * kSplCols + lane;
    const bool on = g < 2 * nx;
    const int q = on ? g / nx : 0, i = on ? g - q * nx : 0;
    const double* col = (q ? d.rms : d.back) + i;
    for (int k = lane; k < ny; k += kSplCols) tk[k] = knot_at(k, d.H, d.mh);
    __syncthreads();
    double x[kSplPre];
    prefetch_column(x, col, nx, ny);
    for (int k = lane; k + 1 < ny; k += kSplCols) ih[k] = 1.0 / (tk[k + 1] - tk[k]);
    if (lane == 0) spline_factor_inv(ny, tk, cf, idn);
    store_column(fl, lane, x, col, nx, ny);
    __syncthreads();
    if (!on) return;
    spline_solve_inv(ny, tk, cf, idn, ih, fl + lane, kSplCols, ml + lane, kSplCols);
#pragma unroll 4
    for (int jy = 0; jy <= ny; ++jy) {
        double c[4];
        piece_poly_inv(ny, tk, ih, fl + lane, kSplCols, ml + lane, kSplCols, jy, c);
        double* o = d.ycoef + (((size_t)q * (ny + 1) + jy) * nx + i) * 4;
        o[0] = c[0];
        o[1] = c[1];
        o[2] = c[2];
        o[3] = c[3];
    }
}

// X: one column per (quantity, y piece, power of u), as k_spline_x
__global__ __launch_bounds__(kSplCols) void k_spline_x_small(const FrameDesc* __restrict__ desc) {
    __shared__ double tk[kSplSmallN], cf[kSplSmallN], idn[kSplSmallN], ih[kSplSmallN];
    __shared__ double fl[kSplSmallN * kSplCols], ml[kSplSmallN * kSplCols];
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny, lane = threadIdx.x;
    const int G = 8 * (ny + 1);
    if ((int)blockIdx.x * kSplCols >= G) return;
    const int g = blockIdx.x * kSplCols + lane;
    const bool on = g < G;
    const int r = g & 3;
    const int jy = on ? (g >> 2) % (ny + 1) : 0;
    const int q = on ? (g >> 2) / (ny + 1) : 0;
    const double* vals = d.ycoef + (((size_t)q * (ny + 1) + jy) * nx) * 4 + r;  // stride 4
    for (int k = lane; k < nx; k += kSplCols) tk[k] = knot_at(k, d.W, d.mw);
    __syncthreads();
    double x[kSplPre];
    prefetch_column(x, vals, 4, nx);
    for (int k = lane; k + 1 < nx; k += kSplCols) ih[k] = 1.0 / (tk[k + 1] - tk[k]);
    if (lane == 0) spline_factor_inv(nx, tk, cf, idn);
    store_column(fl, lane, x, vals, 4, nx);
    __syncthreads();
    if (!on) return;
    spline_solve_inv(nx, tk, cf, idn, ih, fl + lane, kSplCols, ml + lane, kSplCols);
#pragma unroll 4
    for (int ix = 0; ix <= nx; ++ix) {
        double c[4];
        piece_poly_inv(nx, tk, ih, fl + lane, kSplCols, ml + lane, kSplCols, ix, c);
        double* o = d.coef + (((size_t)q * (ny + 1) + jy) * (nx + 1) + ix) * 16;
        for (int p = 0; p < 4; ++p) o[p * 4 + r] = c[p];
    }
}

// ---------------------------------------------------------------------------
// Grids of at most kPcrMax knots per axis: one wavefront per spline, lane k =
// knot k.  The tridiagonal system of the natural spline's second derivatives
// (interior rows h_{k-1} m_{k-1} + 2 (h_{k-1} + h_k) m_k + h_k m_{k+1} =
// 6 (f_{k+1} - f_k) / h_k - 6 (f_k - f_{k-1}) / h_{k-1}, m_0 = m_{n-1} = 0)
// is solved by parallel cyclic reduction: six rounds, each eliminating the
// couplings to the rows at distance 1, 2, ..., 32 (fetched by lane shuffles;
// rows outside the spline are identity rows).  The matrix is strictly
// diagonally dominant, so the reduction is stable.  Lane p then forms piece p
// from the values of lanes clamp(p - 1, 0, n - 2) and the next one.  The
// y splines also apply the mesh filter (lane k takes mesh (k, i)).
constexpr int kPcrMax = 63;   // knots: the n + 1 pieces fit one wavefront

// second derivatives at the knots; t0 = t_{k-1}, t1 = t_k, t2 = t_{k+1}
__device__ __forceinline__ double pcr_second_derivs(int n, int lane, double t0, double t1, double t2, double fm,
                                                    double f, double fp) {
    const bool row = lane >= 1 && lane <= n - 2;
    const double h0 = t1 - t0, h1 = t2 - t1;
    double a = row ? h0 : 0.0, b = row ? 2.0 * (h0 + h1) : 1.0, c = row ? h1 : 0.0;
    double d = row ? 6.0 * ((fp - f) / h1 - (f - fm) / h0) : 0.0;
#pragma unroll
    for (int st = 1; st < 64; st <<= 1) {
        const double rb = 1.0 / b;
        const bool okl = lane >= st, okh = lane + st < 64;
        const int sl = okl ? lane - st : lane, sh = okh ? lane + st : lane;
        const double al = __shfl(a, sl), cl = __shfl(c, sl), dl = __shfl(d, sl), rl = __shfl(rb, sl);
        const double ah = __shfl(a, sh), ch = __shfl(c, sh), dh = __shfl(d, sh), rh = __shfl(rb, sh);
        const double al_ = okl ? al : 0.0, cl_ = okl ? cl : 0.0, dl_ = okl ? dl : 0.0, rl_ = okl ? rl : 1.0;
        const double ah_ = okh ? ah : 0.0, ch_ = okh ? ch : 0.0, dh_ = okh ? dh : 0.0, rh_ = okh ? rh : 1.0;
        const double alpha = -a * rl_, gamma = -c * rh_;
        b = b + alpha * cl_ + gamma * ah_;
        d = d + alpha * dl_ + gamma * dh_;
        a = alpha * al_;
        c = gamma * ch_;
    }
    return d / b;
}

// piece p of the spline through n knots from the values at knots A =
// clamp(p - 1, 0, n - 2) and A + 1 and their spacing hA; out[r] = coefficient
// of u^r, u = position - reference knot
__device__ __forceinline__ void spline_piece(int n, int p, double fA, double fB, double mA, double mB, double hA,
                                             double out[4]) {
    constexpr double kSixth = 1.0 / 6.0;
    const double ih = 1.0 / hA;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (n == 1) {
        out[0] = fA;
    } else if (p == 0) {
        out[0] = fA;
        out[1] = (fB - fA) * ih - hA * (2.0 * mA + mB) * kSixth;
    } else if (p == n) {
        out[0] = fB;
        out[1] = (fB - fA) * ih + hA * (mA + 2.0 * mB) * kSixth;
    } else {
        out[0] = fA;
        out[1] = (fB - fA) * ih - hA * (2.0 * mA + mB) * kSixth;
        out[2] = 0.5 * mA;
        out[3] = (mB - mA) * ih * kSixth;
    }
}

// piece p = lane, the values of knots A and A + 1 fetched by lane shuffles
__device__ __forceinline__ void pcr_piece(int n, int lane, double f, double m, double h, double out[4]) {
    const int A = min(max(lane - 1, 0), max(n - 2, 0));
    const double fA = __shfl(f, A), fB = __shfl(f, A + 1), mA = __shfl(m, A), mB = __shfl(m, A + 1);
    const double hA = __shfl(h, A);
    spline_piece(n, lane, fA, fB, mA, mB, hA, out);
}

// Grids of 64 to kPcrBlkMax knots on the solved axis: the same reduction over
// a workgroup of 128 threads (thread = knot), seven rounds, the rows exchanged
// through LDS (s*: 128 doubles each)
constexpr int kPcrBlkMax = 127;

__device__ double pcr_second_derivs_blk(int n, int k, double t0, double t1, double t2, double fm, double f,
                                        double fp, double* sa, double* sc, double* sd, double* sr) {
    const bool row = k >= 1 && k <= n - 2;
    const double h0 = t1 - t0, h1 = t2 - t1;
    double a = row ? h0 : 0.0, b = row ? 2.0 * (h0 + h1) : 1.0, c = row ? h1 : 0.0;
    double d = row ? 6.0 * ((fp - f) / h1 - (f - fm) / h0) : 0.0;
    for (int st = 1; st < 128; st <<= 1) {
        sa[k] = a;
        sc[k] = c;
        sd[k] = d;
        sr[k] = 1.0 / b;
        __syncthreads();
        const bool okl = k >= st, okh = k + st < 128;
        const double al = okl ? sa[k - st] : 0.0, cl = okl ? sc[k - st] : 0.0, dl = okl ? sd[k - st] : 0.0;
        const double rl = okl ? sr[k - st] : 1.0;
        const double ah = okh ? sa[k + st] : 0.0, ch = okh ? sc[k + st] : 0.0, dh = okh ? sd[k + st] : 0.0;
        const double rh = okh ? sr[k + st] : 1.0;
        __syncthreads();
        const double alpha = -a * rl, gamma = -c * rh;
        b = b + alpha * cl + gamma * ah;
        d = d + alpha * dl + gamma * dh;
        a = alpha * al;
        c = gamma * ch;
    }
    return d / b;
}

// y splines (and the mesh filter when F > 0), one workgroup per (quantity,
// mesh column); blockIdx.y = frame
template <int F>
__global__ __launch_bounds__(128) void k_spline_y_pcr_blk(const FrameDesc* __restrict__ desc) {
    __shared__ double sa[128], sc[128], sd[128], sr[128];
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny, t = threadIdx.x;
    const int g = blockIdx.x;
    if (g >= 2 * nx) return;
    const int q = g / nx, i = g - q * nx;
    const int k = min(t, ny - 1);
    double f;
    if constexpr (F > 0) {
        constexpr int hh = F / 2;
        const gdouble_t* raw = (const gdouble_t*)(q ? d.rms_raw : d.back_raw);
        double w[F * F];
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < F * F; ++e) {
            const int b = k - hh + e / F, c = i - hh + e % F;
            const bool in = b >= 0 && b < ny && c >= 0 && c < nx;
            w[e] = in ? raw[b * nx + c] : INFINITY;
            cnt += in ? 1 : 0;
        }
        f = median_regs(w, cnt);
        if (t < ny) (q ? d.rms : d.back)[k * nx + i] = f;
    } else {
        f = ((const gdouble_t*)(q ? d.rms : d.back))[k * nx + i];
    }
    const double t0 = knot_at(max(k - 1, 0), d.H, d.mh), t1 = knot_at(k, d.H, d.mh);
    const double t2 = knot_at(min(k + 1, ny - 1), d.H, d.mh);
    sd[t] = f;
    __syncthreads();
    const double fm = sd[max(t - 1, 0)], fp = sd[min(t + 1, 127)];
    __syncthreads();
    const double m = pcr_second_derivs_blk(ny, t, t0, t1, t2, fm, f, fp, sa, sc, sd, sr);
    sa[t] = f;
    sc[t] = m;
    sd[t] = t2 - t1;
    __syncthreads();
    if (t <= ny) {
        const int A = min(max(t - 1, 0), max(ny - 2, 0));
        double cf[4];
        spline_piece(ny, t, sa[A], sa[A + 1], sc[A], sc[A + 1], sd[A], cf);
        double* o = d.ycoef + (((size_t)q * (ny + 1) + t) * nx + i) * 4;
        o[0] = cf[0];
        o[1] = cf[1];
        o[2] = cf[2];
        o[3] = cf[3];
    }
}

// x splines, one workgroup per (quantity, y piece, power of u); blockIdx.y = frame
__global__ __launch_bounds__(128) void k_spline_x_pcr_blk(const FrameDesc* __restrict__ desc) {
    __shared__ double sa[128], sc[128], sd[128], sr[128];
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny, t = threadIdx.x;
    const int g = blockIdx.x;
    if (g >= 8 * (ny + 1)) return;
    const int b = g >> 2, r = g & 3;   // b = q (ny + 1) + jy
    const int k = min(t, nx - 1);
    const double f = ((const gdouble_t*)d.ycoef)[((size_t)b * nx + k) * 4 + r];
    const double t0 = knot_at(max(k - 1, 0), d.W, d.mw), t1 = knot_at(k, d.W, d.mw);
    const double t2 = knot_at(min(k + 1, nx - 1), d.W, d.mw);
    sd[t] = f;
    __syncthreads();
    const double fm = sd[max(t - 1, 0)], fp = sd[min(t + 1, 127)];
    __syncthreads();
    const double m = pcr_second_derivs_blk(nx, t, t0, t1, t2, fm, f, fp, sa, sc, sd, sr);
    sa[t] = f;
    sc[t] = m;
    sd[t] = t2 - t1;
    __syncthreads();
    if (t <= nx) {
        const int A = min(max(t - 1, 0), max(nx - 2, 0));
        double cf[4];
        spline_piece(nx, t, sa[A], sa[A + 1], sc[A], sc[A + 1], sd[A], cf);
        double* o = d.coef + ((size_t)b * (nx + 1) + t) * 16;
        for (int pp = 0; pp < 4; ++pp) o[pp * 4 + r] = cf[pp];
    }
}

// y splines (and the mesh filter when F > 0): blockIdx.y = frame, one
// wavefront per (quantity, mesh column), four per workgroup
template <int F>
__global__ __launch_bounds__(256) void k_spline_y_pcr(const FrameDesc* __restrict__ desc) {
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny, lane = threadIdx.x & 63;
    const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= 2 * nx) return;
    const int q = g / nx, i = g - q * nx;
    const int k = min(lane, ny - 1);
    double f;
    if constexpr (F > 0) {
        constexpr int hh = F / 2;
        const gdouble_t* raw = (const gdouble_t*)(q ? d.rms_raw : d.back_raw);
        double w[F * F];
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < F * F; ++e) {
            const int b = k - hh + e / F, c = i - hh + e % F;
            const bool in = b >= 0 && b < ny && c >= 0 && c < nx;
            w[e] = in ? raw[b * nx + c] : INFINITY;
            cnt += in ? 1 : 0;
        }
        f = median_regs(w, cnt);
        if (lane < ny) (q ? d.rms : d.back)[k * nx + i] = f;
    } else {
        f = ((const gdouble_t*)(q ? d.rms : d.back))[k * nx + i];
    }
    const double t0 = knot_at(max(k - 1, 0), d.H, d.mh), t1 = knot_at(k, d.H, d.mh);
    const double t2 = knot_at(min(k + 1, ny - 1), d.H, d.mh);
    const double fm = __shfl(f, max(lane - 1, 0)), fp = __shfl(f, min(lane + 1, 63));
    const double m = pcr_second_derivs(ny, lane, t0, t1, t2, fm, f, fp);
    double c[4];
    pcr_piece(ny, lane, f, m, t2 - t1, c);
    if (lane <= ny) {
        double* o = d.ycoef + (((size_t)q * (ny + 1) + lane) * nx + i) * 4;
        o[0] = c[0];
        o[1] = c[1];
        o[2] = c[2];
        o[3] = c[3];
    }
}

// x splines: blockIdx.y = frame; workgroup = (quantity, y piece), its four
// wavefronts the four powers of u
__global__ __launch_bounds__(256) void k_spline_x_pcr(const FrameDesc* __restrict__ desc) {
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny, lane = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int b = blockIdx.x;
    if (b >= 2 * (ny + 1)) return;
    const int k = min(lane, nx - 1);
    const double f = ((const gdouble_t*)d.ycoef)[((size_t)b * nx + k) * 4 + r];   // b = q (ny + 1) + jy
    const double t0 = knot_at(max(k - 1, 0), d.W, d.mw), t1 = knot_at(k, d.W, d.mw);
    const double t2 = knot_at(min(k + 1, nx - 1), d.W, d.mw);
    const double fm = __shfl(f, max(lane - 1, 0)), fp = __shfl(f, min(lane + 1, 63));
    const double m = pcr_second_derivs(nx, lane, t0, t1, t2, fm, f, fp);
    double c[4];
    pcr_piece(nx, lane, f, m, t2 - t1, c);
    if (lane <= nx) {
        double* o = d.coef + ((size_t)b * (nx + 1) + lane) * 16;
        for (int p = 0; p < 4; ++p) o[p * 4 + r] = c[p];
    }
}

// Larger grids: y-splines, blockIdx.y = frame; one thread per (quantity, mesh column)
__global__ __launch_bounds__(kSplThreads) void k_spline_y(const FrameDesc* __restrict__ desc) {
    __shared__ double tk[kSplineMaxKnots], cf[kSplineMaxKnots], dn[kSplineMaxKnots];
    const FrameDesc& d = desc[blockIdx.y];
    const int ny = d.ny, nx = d.nx;
    if ((int)blockIdx.x * kSplThreads >= 2 * nx) return;
    for (int k = threadIdx.x; k < ny; k += kSplThreads) tk[k] = knot_at(k, d.H, d.mh);
    __syncthreads();
    if (threadIdx.x == 0) spline_factor(ny, tk, cf, dn);
    __syncthreads();
    const int g = blockIdx.x * kSplThreads + threadIdx.x;
    if (g >= 2 * nx) return;
    const int q = g / nx, i = g - q * nx;
    const double* col = (q ? d.rms : d.back) + i;
    // scratch [k][g]: work then second derivatives, 2 nx columns each
    double* r = d.scratch + g;
    double* mm = d.scratch + (size_t)2 * nx * ny + g;
    spline_solve(ny, tk, cf, dn, col, nx, r, mm, 2 * nx);
#pragma unroll 4
    for (int jy = 0; jy <= ny; ++jy) {
        double c[4];
        piece_poly(ny, tk, col, nx, mm, 2 * nx, jy, c);
        double* o = d.ycoef + (((size_t)q * (ny + 1) + jy) * nx + i) * 4;
        o[0] = c[0];
        o[1] = c[1];
        o[2] = c[2];
        o[3] = c[3];
    }
}

// x-splines: the tensor spline's row cubic on y piece jy is a cubic in u whose
// four coefficients are linear in the column values, so the x spline of each
// coefficient vector (one natural spline per (quantity, jy, power of u)) gives
// the bicubic pieces directly: coef[q][jy][ix][p*4+r] = x-piece p coefficient
// of the spline through (ycoef[q][jy][k][r])_k.  Exact on constant grids.
// blockIdx.y = frame; one thread per (quantity, jy, power).
__global__ __launch_bounds__(kSplThreads) void k_spline_x(const FrameDesc* __restrict__ desc) {
    __shared__ double tk[kSplineMaxKnots], cf[kSplineMaxKnots], dn[kSplineMaxKnots];
    const FrameDesc& d = desc[blockIdx.y];
    const int nx = d.nx, ny = d.ny;
    const int G = 8 * (ny + 1);
    if ((int)blockIdx.x * kSplThreads >= G) return;
    for (int k = threadIdx.x; k < nx; k += kSplThreads) tk[k] = knot_at(k, d.W, d.mw);
    __syncthreads();
    if (threadIdx.x == 0) spline_factor(nx, tk, cf, dn);
    __syncthreads();
    const int g = blockIdx.x * kSplThreads + threadIdx.x;
    if (g >= G) return;
    const int r = g & 3;
    const int jy = (g >> 2) % (ny + 1);
    const int q = (g >> 2) / (ny + 1);
    double* base = d.scratch + (size_t)8 * nx * ny;   // after the y-spline scratch
    double* w = base + g;                               // [k][g], G columns
    double* mm = base + (size_t)G * nx + g;
    const double* vals = d.ycoef + (((size_t)q * (ny + 1) + jy) * nx) * 4 + r;  // stride 4
    spline_solve(nx, tk, cf, dn, vals, 4, w, mm, G);
#pragma unroll 4
    for (int ix = 0; ix <= nx; ++ix) {
        double c[4];
        piece_poly(nx, tk, vals, 4, mm, G, ix, c);
        double* o = d.coef + (((size_t)q * (ny + 1) + jy) * (nx + 1) + ix) * 16;
        for (int p = 0; p < 4; ++p) o[p * 4 + r] = c[p];
    }
}

// ---------------------------------------------------------------------------
// launchers
// cfg: 0 = automatic, 1 = 256 x 16, 2 = 512 x 16, 3 = 512 x 32, 4 = 1024 x 16
// (threads x pixels per thread; the product must cover the largest mesh)
template <int NT, int PPT>
static void launch_mesh_nt(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, BkgArgs a,
                           hipStream_t s) {
    if (one) k_mesh_stats<NT, PPT, true><<<total_meshes, NT, 0, s>>>(desc, *one, nframes, a);
    else k_mesh_stats<NT, PPT, false><<<total_meshes, NT, 0, s>>>(desc, FrameDesc{}, nframes, a);
}

template <int NT, int PPT>
static void launch_mesh_u16_nt(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, BkgArgs a,
                               hipStream_t s) {
    if (one) k_mesh_stats_u16<NT, PPT, true><<<total_meshes, NT, 0, s>>>(desc, *one, nframes, a);
    else k_mesh_stats_u16<NT, PPT, false><<<total_meshes, NT, 0, s>>>(desc, FrameDesc{}, nframes, a);
}

// uint16 meshes; cfg as for the float kernel (threads x pixels per thread)
void launch_mesh_stats_u16(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, int max_area,
                           BkgArgs a, int cfg, hipStream_t s) {
    if (cfg == 0) cfg = (max_area <= 4096) ? 1 : (max_area <= 8192) ? 2 : 3;
    if (cfg == 1 && max_area > 4096) cfg = 3;
    if (cfg == 2 && max_area > 8192) cfg = 3;
    switch (cfg) {
        case 1: launch_mesh_u16_nt<256, 16>(desc, one, nframes, total_meshes, a, s); break;
        case 2: launch_mesh_u16_nt<512, 16>(desc, one, nframes, total_meshes, a, s); break;
        case 4: launch_mesh_u16_nt<1024, 16>(desc, one, nframes, total_meshes, a, s); break;
        default: launch_mesh_u16_nt<512, 32>(desc, one, nframes, total_meshes, a, s); break;
    }
}

void launch_mesh_stats(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, int max_area, BkgArgs a,
                       int cfg, hipStream_t s) {
    if (cfg == 0) cfg = (max_area <= 4096) ? 1 : (max_area <= 8192) ? 2 : 3;
    if (cfg == 1 && max_area > 4096) cfg = 3;
    if (cfg == 2 && max_area > 8192) cfg = 3;
    switch (cfg) {
        case 1: launch_mesh_nt<256, 16>(desc, one, nframes, total_meshes, a, s); break;
        case 2: launch_mesh_nt<512, 16>(desc, one, nframes, total_meshes, a, s); break;
        case 4: launch_mesh_nt<1024, 16>(desc, one, nframes, total_meshes, a, s); break;
        default: launch_mesh_nt<512, 32>(desc, one, nframes, total_meshes, a, s); break;
    }
}

void launch_grid_filter(const FrameDesc* desc, int nframes, int total_meshes, int fsize, hipStream_t s) {
    const int blocks = (total_meshes + kGridThreads - 1) / kGridThreads;
    switch (fsize) {
        case 1: k_grid_filter<1><<<blocks, kGridThreads, 0, s>>>(desc, nframes, total_meshes, fsize); break;
        case 3: k_grid_filter<3><<<blocks, kGridThreads, 0, s>>>(desc, nframes, total_meshes, fsize); break;
        case 5: k_grid_filter<5><<<blocks, kGridThreads, 0, s>>>(desc, nframes, total_meshes, fsize); break;
        default: k_grid_filter<0><<<blocks, kGridThreads, 0, s>>>(desc, nframes, total_meshes, fsize); break;
    }
}

// mesh filter of size fsize (0: none, the grids are given) and the splines
// in two launches, for grids of at most kPcrMax knots per axis and filters of
// at most 5 x 5 (filter_spline_fits)
bool filter_spline_fits(int max_nx, int max_ny, int fsize) {
    return max_nx <= kPcrBlkMax && max_ny <= kPcrBlkMax && fsize <= 5;
}

// each axis by its own knot count: up to kPcrMax one wavefront per spline,
// up to kPcrBlkMax one 128-thread workgroup
void launch_filter_spline(const FrameDesc* desc, int nframes, int max_nx, int max_ny, int fsize, hipStream_t s) {
    if (max_ny <= kPcrMax) {
        const dim3 gy((2 * max_nx + 3) / 4, nframes);
        switch (fsize) {
            case 0: k_spline_y_pcr<0><<<gy, 256, 0, s>>>(desc); break;
            case 1: k_spline_y_pcr<1><<<gy, 256, 0, s>>>(desc); break;
            case 3: k_spline_y_pcr<3><<<gy, 256, 0, s>>>(desc); break;
            default: k_spline_y_pcr<5><<<gy, 256, 0, s>>>(desc); break;
        }
    } else {
        const dim3 gy(2 * max_nx, nframes);
        switch (fsize) {
            case 0: k_spline_y_pcr_blk<0><<<gy, 128, 0, s>>>(desc); break;
            case 1: k_spline_y_pcr_blk<1><<<gy, 128, 0, s>>>(desc); break;
            case 3: k_spline_y_pcr_blk<3><<<gy, 128, 0, s>>>(desc); break;
            default: k_spline_y_pcr_blk<5><<<gy, 128, 0, s>>>(desc); break;
        }
    }
    if (max_nx <= kPcrMax) k_spline_x_pcr<<<dim3(2 * (max_ny + 1), nframes), 256, 0, s>>>(desc);
    else k_spline_x_pcr_blk<<<dim3(8 * (max_ny + 1), nframes), 128, 0, s>>>(desc);
}

void launch_spline(const FrameDesc* desc, int nframes, int max_nx, int max_ny, hipStream_t s) {
    if (max_ny <= kSplSmallN)
        k_spline_y_small<<<dim3((2 * max_nx + kSplCols - 1) / kSplCols, nframes), kSplCols, 0, s>>>(desc);
    else
        k_spline_y<<<dim3((2 * max_nx + kSplThreads - 1) / kSplThreads, nframes), kSplThreads, 0, s>>>(desc);
    if (max_nx <= kSplSmallN)
        k_spline_x_small<<<dim3((8 * (max_ny + 1) + kSplCols - 1) / kSplCols, nframes), kSplCols, 0, s>>>(desc);
    else
        k_spline_x<<<dim3((8 * (max_ny + 1) + kSplThreads - 1) / kSplThreads, nframes), kSplThreads, 0, s>>>(desc);
}

// ---------------------------------------------------------------------------
// full-resolution background and noise maps of one frame (diagnostic output;
// the same per-row cubic and per-pixel evaluation as the detection kernel)
template <typename Real>
__global__ __launch_bounds__(256) void k_bkg_map(FrameDesc d, double* bmap, double* rmap) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= d.W) return;
    for (int y = blockIdx.y; y < d.H; y += gridDim.y) {
    const int jy = piece_of(y, d.H, d.mh);
    const double u = (double)y - piece_ref(jy, d.H, d.mh);
    const int ix = piece_of(x, d.W, d.mw);
    const RowT<Real> t = make_row<Real>(d.coef, d.nx, d.ny, ix, jy, u);
    const Real s = (Real)((double)x - piece_ref(ix, d.W, d.mw));
    const size_t o = (size_t)y * d.W + x;
    if (bmap) bmap[o] = eval_B(t, s);
    if (rmap) rmap[o] = (double)eval_R(t, s);
    }
}

void launch_bkg_map(const FrameDesc& d, double* bmap, double* rmap, bool f64, hipStream_t s) {
    dim3 grid((d.W + 255) / 256, d.H < 32768 ? d.H : 32768);
    if (f64) k_bkg_map<double><<<grid, 256, 0, s>>>(d, bmap, rmap);
    else k_bkg_map<float><<<grid, 256, 0, s>>>(d, bmap, rmap);
}

}  // namespace gpk
