// runtime.hip -- host side of the C ABI declared in include/gp.h.
//
// Responsibilities: argument validation (synchronous errors), the layout of
// the background buffer and of the workspace for a batch of frames, frame
// descriptors (written into the workspace by small kernels so that the whole
// call sequence can be captured into a HIP graph), kernel launches on the
// caller's stream, and optional per-kernel timing with HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gp.h"
#include "k_args.h"

using namespace gpk;

// ---------------------------------------------------------------------------
// errors
static thread_local std::string g_err;

static gp_status fail(gp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(GP_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char* gp_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Static device scratch for gp_detect_noalloc: each device the library runs
// on holds one copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it only stands for the symbol): the
// device address of each device's copy is looked up once, with that device
// current, when a context is created on it, and kept per device.
constexpr size_t kStaticScratchBytes = GP_DETECT_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// the calling thread's current device is `device` on entry
static hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    return e;
}

static void* scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}
extern "C" const char* gp_version(void) { return "gpphot 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// context
struct ProfPair {
    std::string name;
    hipEvent_t a, b;
};

struct gp_ctx {
    int device = 0;
    int cus = 256;
    bool profiling = false;
    std::mutex mu;
    std::vector<ProfPair> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, int64_t>> totals;
    std::string tune_path;
    int mesh_cfg = 0;     // launch shape of the mesh-statistics kernel (0 = automatic)
    bool tuning = false;  // time the candidates of a shape class not yet in `tuned`
    std::map<std::string, int> tuned;   // shape class -> chosen launch shape
};

namespace {
struct ProfScope {
    gp_ctx* c;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr;
    // enable = false: never record (a call that must create nothing)
    ProfScope(gp_ctx* c_, hipStream_t s_, const char* n, bool enable = true) : c(c_), s(s_), name(n) {
        if (!enable || !c->profiling) return;
        std::lock_guard<std::mutex> g(c->mu);
        a = take();
        (void)hipEventRecord(a, s);
    }
    hipEvent_t take() {
        if (c->pool.empty()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            return e;
        }
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    ~ProfScope() {
        if (!a) return;
        std::lock_guard<std::mutex> g(c->mu);
        hipEvent_t b = take();
        (void)hipEventRecord(b, s);
        c->pending.push_back(ProfPair{name, a, b});
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct FramePlan {
    int nx, ny, ntx, nty;
    int64_t meshes, tiles, nblocks;
    size_t bkg_off;  // frame block offset in the background buffer
    size_t back_raw, rms_raw, back, rms, coef, iters, bkg_bytes;  // relative to block
    size_t spl_off;  // workspace offset of this frame's spline scratch
    size_t ycoef_n, scr_n;  // doubles
};

struct Plan {
    std::vector<FramePlan> fr;
    int64_t total_meshes = 0, total_tiles = 0, total_blocks = 0, total_ycols = 0, total_xrows = 0,
            total_px = 0;
    int max_area = 0;
    int max_nx = 0, max_ny = 0;
    size_t bkg_bytes = 0;
    // workspace sections
    size_t o_desc = 0, o_detargs = 0, o_counters = 0, o_tiles = 0, o_edges = 0, o_recs = 0, o_parent = 0,
           o_root = 0, o_label = 0, o_bitmap = 0, o_blockcnt = 0, o_chunks = 0, o_spline = 0, o_psf = 0,
           ws_bytes = 0;
    int64_t rec_cap = 0;
};

gp_status check_frames(const gp_frame* frames, int32_t nframes) {
    if (!frames) return fail(GP_ERR_INVALID_ARG, "frames is NULL");
    if (nframes < 1) return fail(GP_ERR_INVALID_ARG, "nframes must be >= 1 (got %d)", nframes);
    if (nframes > kMaxFramesPerCall)
        return fail(GP_ERR_UNSUPPORTED, "at most %d frames per call (got %d)", kMaxFramesPerCall, nframes);
    for (int f = 0; f < nframes; ++f) {
        const gp_frame& F = frames[f];
        if (!F.data) return fail(GP_ERR_INVALID_ARG, "frame %d: data is NULL", f);
        if (F.width < 1 || F.height < 1)
            return fail(GP_ERR_INVALID_ARG, "frame %d: bad size %dx%d", f, F.width, F.height);
        if (F.pitch < F.width) return fail(GP_ERR_INVALID_ARG, "frame %d: pitch < width", f);
        if (F.dtype != GP_U16 && F.dtype != GP_F32)
            return fail(GP_ERR_INVALID_ARG, "frame %d: unknown dtype %d", f, F.dtype);
        if (F.pitch * F.height >= (int64_t)1 << 31)
            return fail(GP_ERR_UNSUPPORTED, "frame %d: pitch * height >= 2^31 elements", f);
    }
    return GP_OK;
}

gp_status check_bkg(const gp_bkg_params* bp, const gp_frame* frames, int32_t nframes) {
    if (!bp) return fail(GP_ERR_INVALID_ARG, "background parameters are NULL");
    if (bp->mesh_w < 16 || bp->mesh_h < 16)
        return fail(GP_ERR_UNSUPPORTED, "mesh %dx%d: meshes must be at least 16 pixels", bp->mesh_w, bp->mesh_h);
    if ((int64_t)bp->mesh_w * bp->mesh_h > 16384)
        return fail(GP_ERR_UNSUPPORTED, "mesh %dx%d: at most 16384 pixels per mesh", bp->mesh_w, bp->mesh_h);
    if (bp->filter_size < 1 || bp->filter_size > 7 || !(bp->filter_size & 1))
        return fail(GP_ERR_INVALID_ARG, "filter_size must be odd in [1, 7] (got %d)", bp->filter_size);
    if (!(bp->clip_sigma > 0.f) || !std::isfinite(bp->clip_sigma))
        return fail(GP_ERR_INVALID_ARG, "clip_sigma must be positive");
    if (!std::isfinite(bp->crowd_tol) || !std::isfinite(bp->mode_a) || !std::isfinite(bp->mode_b))
        return fail(GP_ERR_INVALID_ARG, "non-finite background parameter");
    if (bp->max_iter < 0) return fail(GP_ERR_INVALID_ARG, "max_iter must be >= 0");
    for (int f = 0; f < nframes; ++f) {
        const int64_t nx = ceil_div((int64_t)frames[f].width, bp->mesh_w);
        const int64_t ny = ceil_div((int64_t)frames[f].height, bp->mesh_h);
        if (nx > kSplineMaxKnots || ny > kSplineMaxKnots)
            return fail(GP_ERR_UNSUPPORTED, "frame %d: %lldx%lld meshes, at most %d per axis", f, (long long)nx,
                        (long long)ny, kSplineMaxKnots);
    }
    return GP_OK;
}

gp_status check_det(const gp_det_params* dp) {
    if (!dp) return fail(GP_ERR_INVALID_ARG, "detection parameters are NULL");
    if (!dp->kernel) return fail(GP_ERR_INVALID_ARG, "filter kernel is NULL");
    if (dp->kw < 1 || dp->kh < 1 || dp->kw > kMaxK || dp->kh > kMaxK || !(dp->kw & 1) || !(dp->kh & 1))
        return fail(GP_ERR_INVALID_ARG, "kernel must be odd and at most 15 per side (got %dx%d)", dp->kw, dp->kh);
    for (int i = 0; i < dp->kw * dp->kh; ++i)
        if (!std::isfinite(dp->kernel[i])) return fail(GP_ERR_INVALID_ARG, "kernel has a non-finite tap");
    if (!std::isfinite(dp->thresh)) return fail(GP_ERR_INVALID_ARG, "thresh must be finite");
    if (dp->minarea < 1) return fail(GP_ERR_INVALID_ARG, "minarea must be >= 1");
    if (dp->connectivity != 4 && dp->connectivity != 8)
        return fail(GP_ERR_INVALID_ARG, "connectivity must be 4 or 8");
    if (std::isnan(dp->sat_level)) return fail(GP_ERR_INVALID_ARG, "sat_level is NaN");
    if (dp->precision != GP_PREC_F32 && dp->precision != GP_PREC_F64)
        return fail(GP_ERR_INVALID_ARG, "unknown precision %d", dp->precision);
    return GP_OK;
}

gp_status check_ap(const gp_ap_params* ap) {
    if (!ap) return fail(GP_ERR_INVALID_ARG, "aperture parameters are NULL");
    if (ap->nr < 1 || ap->nr > kMaxRadii) return fail(GP_ERR_INVALID_ARG, "nr must be in [1, 8]");
    if (!ap->radii) return fail(GP_ERR_INVALID_ARG, "radii is NULL");
    for (int i = 0; i < ap->nr; ++i)
        if (!(ap->radii[i] > 0.f) || ap->radii[i] > 64.f)
            return fail(GP_ERR_INVALID_ARG, "radius %d must be in (0, 64]", i);
    if (!(ap->r_in >= 0.f) || !(ap->r_out > ap->r_in) || ap->r_out > 64.f)
        return fail(GP_ERR_INVALID_ARG, "annulus must satisfy 0 <= r_in < r_out <= 64");
    if (!std::isfinite(ap->gain)) return fail(GP_ERR_INVALID_ARG, "gain must be finite");
    if (ap->precision != GP_PREC_F32 && ap->precision != GP_PREC_F64)
        return fail(GP_ERR_INVALID_ARG, "unknown precision %d", ap->precision);
    return GP_OK;
}

// background layout (independent of the workspace)
void plan_bkg(const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp, Plan& P) {
    P.fr.resize(nframes);
    size_t off = 0;
    for (int f = 0; f < nframes; ++f) {
        FramePlan& F = P.fr[f];
        const int W = frames[f].width, H = frames[f].height;
        F.nx = (int)ceil_div(W, bp->mesh_w);
        F.ny = (int)ceil_div(H, bp->mesh_h);
        F.meshes = (int64_t)F.nx * F.ny;
        size_t g = align256(sizeof(double) * F.meshes);
        F.back_raw = 0;
        F.rms_raw = g;
        F.back = 2 * g;
        F.rms = 3 * g;
        F.coef = 4 * g;
        size_t cb = align256(sizeof(double) * 2 * (F.nx + 1) * (F.ny + 1) * 16);
        F.iters = F.coef + cb;
        F.bkg_bytes = F.iters + align256(sizeof(int32_t) * F.meshes);
        F.bkg_off = off;
        off += F.bkg_bytes;
        P.total_meshes += F.meshes;
        P.total_ycols += 2 * F.nx;
        P.total_xrows += 2 * (int64_t)(F.ny + 1) * 4;
        P.max_nx = std::max(P.max_nx, F.nx);
        P.max_ny = std::max(P.max_ny, F.ny);
        const int mw = std::min(bp->mesh_w, W), mh = std::min(bp->mesh_h, H);
        P.max_area = std::max(P.max_area, mw * mh);
        F.ntx = (int)ceil_div(W, kTile);
        F.nty = (int)ceil_div(H, kTile);
        F.tiles = (int64_t)F.ntx * F.nty;
        F.nblocks = ceil_div((int64_t)W * H, 1024);
        P.total_tiles += F.tiles;
        P.total_blocks += F.nblocks;
        P.total_px += (int64_t)W * H;
        F.ycoef_n = (size_t)2 * (F.ny + 1) * F.nx * 4;
        // Thomas sweeps: 4 ny per y-spline (2 nx of them), 4 nx per x-spline (8 (ny+1))
        F.scr_n = (size_t)8 * F.nx * F.ny + (size_t)32 * F.nx * (F.ny + 1);
    }
    P.bkg_bytes = off;
}

// Workspace: fixed sections first (their offsets depend only on the batch),
// then the component-record arrays, whose capacity is whatever fits.
void plan_fixed(int32_t nframes, Plan& P) {
    size_t o = 0;
    auto sec = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    P.o_desc = sec(sizeof(FrameDesc) * nframes);
    P.o_detargs = sec(sizeof(DetArgs));
    P.o_counters = sec(kNumCounters * sizeof(uint32_t));
    P.o_tiles = sec(sizeof(TileInfo) * P.total_tiles);
    P.o_edges = sec(sizeof(int16_t) * 4 * kTile * P.total_tiles);
    P.o_bitmap = sec(128 * (size_t)P.total_blocks);
    P.o_blockcnt = sec(sizeof(uint32_t) * (P.total_blocks + 1));
    P.o_chunks = sec(sizeof(uint32_t) * (ceil_div(P.total_blocks, kScanChunk) + 1));
    P.o_psf = sec(sizeof(PsfArgs) + sizeof(PsfFrame) * nframes);
    P.o_spline = o;
    for (int f = 0; f < nframes; ++f) {
        FramePlan& F = P.fr[f];
        F.spl_off = o;
        o += align256(sizeof(double) * (F.ycoef_n + F.scr_n));
    }
    P.o_recs = o;
}

size_t rec_bytes(int64_t cap) {
    return align256(sizeof(CompRec) * cap) + 3 * align256(sizeof(int32_t) * cap);
}

void plan_recs(int64_t cap, Plan& P) {
    P.rec_cap = cap;
    P.o_parent = P.o_recs + align256(sizeof(CompRec) * cap);
    P.o_root = P.o_parent + align256(sizeof(int32_t) * cap);
    P.o_label = P.o_root + align256(sizeof(int32_t) * cap);
    P.ws_bytes = P.o_recs + rec_bytes(cap);
}

int64_t default_rec_cap(const Plan& P) { return std::max<int64_t>(65536, P.total_px / 64); }

// largest record capacity a workspace of ws_bytes holds (0 if none)
int64_t cap_for(const Plan& P, size_t ws_bytes) {
    if (ws_bytes < P.o_recs + rec_bytes(1)) return 0;
    int64_t lo = 1, hi = ((int64_t)1 << 31) - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (P.o_recs + rec_bytes(mid) <= ws_bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// descriptors -> workspace table, kDescChunk per launch; with `tail` the last
// chunk is returned instead, for the caller's own set-up launch
gp_status upload_desc(const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp, const Plan& P,
                      const void* bkg, void* ws, int32_t cat_capacity, int32_t* const* seg, hipStream_t s,
                      DescChunk* tail = nullptr) {
    char* W = (char*)ws;
    char* B = (char*)bkg;
    FrameDesc* table = (FrameDesc*)(W + P.o_desc);
    int64_t mesh_base = 0, tile_base = 0, blk_base = 0;
    DescChunk ch{};
    for (int f = 0; f < nframes; ++f) {
        const FramePlan& F = P.fr[f];
        FrameDesc d{};
        d.data = frames[f].data;
        d.pitch = frames[f].pitch;
        d.W = frames[f].width;
        d.H = frames[f].height;
        d.dtype = frames[f].dtype;
        d.mw = bp->mesh_w;
        d.mh = bp->mesh_h;
        d.nx = F.nx;
        d.ny = F.ny;
        char* fb = B + F.bkg_off;
        d.back_raw = (double*)(fb + F.back_raw);
        d.rms_raw = (double*)(fb + F.rms_raw);
        d.back = (double*)(fb + F.back);
        d.rms = (double*)(fb + F.rms);
        d.coef = (double*)(fb + F.coef);
        d.iters = (int32_t*)(fb + F.iters);
        double* sp = (double*)(W + F.spl_off);
        d.ycoef = sp;
        d.scratch = sp + F.ycoef_n;
        d.mesh_base = (int32_t)mesh_base;
        d.tile_base = (int32_t)tile_base;
        d.ntx = F.ntx;
        d.nty = F.nty;
        d.bitmap = (uint32_t*)(W + P.o_bitmap) + blk_base * 32;
        d.bm_block_base = (int32_t)blk_base;
        d.nblocks = (int32_t)F.nblocks;
        d.cat_base = f * cat_capacity;
        d.seg = seg ? seg[f] : nullptr;
        mesh_base += F.meshes;
        tile_base += F.tiles;
        blk_base += F.nblocks;
        if (ch.count == 0) ch.first = f;
        ch.d[ch.count++] = d;
        if (tail && f == nframes - 1) {
            *tail = ch;
        } else if (ch.count == kDescChunk || f == nframes - 1) {
            launch_write_desc(ch, table, s);
            HIP_TRY(hipGetLastError());
            ch = DescChunk{};
        }
    }
    return GP_OK;
}

// rank-one test of the filter kernel; on success fills normalised factors.
// The kernel counts as rank one only when every tap equals the product of
// the factors (the tap's column through the peak times its row through the
// peak, over the peak) to within 4 float32 rounding units of the tap itself:
// the two 1-D passes then apply the given kernel up to the rounding already in
// its float taps.  Anything else is applied densely.
bool separable_factors(const gp_det_params* dp, double* kx, double* ky) {
    const int kw = dp->kw, kh = dp->kh;
    const float* K = dp->kernel;
    int am = 0, bm = 0;
    double vmax = 0.0;
    for (int a = 0; a < kh; ++a)
        for (int b = 0; b < kw; ++b)
            if (std::fabs((double)K[a * kw + b]) > vmax) {
                vmax = std::fabs((double)K[a * kw + b]);
                am = a;
                bm = b;
            }
    if (vmax == 0.0) return false;
    std::vector<double> u(kh), v(kw);
    for (int a = 0; a < kh; ++a) u[a] = K[a * kw + bm];
    for (int b = 0; b < kw; ++b) v[b] = (double)K[am * kw + b] / (double)K[am * kw + bm];
    for (int a = 0; a < kh; ++a)
        for (int b = 0; b < kw; ++b)
            if (std::fabs((double)K[a * kw + b] - u[a] * v[b]) > 4.0 * 0x1p-24 * std::fabs((double)K[a * kw + b]))
                return false;
    double su = 0.0, sv = 0.0;
    for (double x : u) su += x;
    for (double x : v) sv += x;
    if (su == 0.0 || sv == 0.0) return false;
    for (int a = 0; a < kh; ++a) ky[a] = u[a] / su;
    for (int b = 0; b < kw; ++b) kx[b] = v[b] / sv;
    return true;
}

// filter arguments of a detection call (the dense kernel is normalised on the
// device; a rank-one kernel also gets its normalised factors)
DetArgsIn det_in(const gp_det_params* dp) {
    DetArgsIn in{};
    in.kw = dp->kw;
    in.kh = dp->kh;
    in.conn = dp->connectivity;
    in.thresh = dp->thresh;
    in.sat = dp->sat_level;
    in.minarea = dp->minarea;
    in.want_seg = 0;
    for (int i = 0; i < dp->kw * dp->kh; ++i) in.kraw[i] = dp->kernel[i];
    double kx[kMaxK] = {0}, ky[kMaxK] = {0};
    in.separable = separable_factors(dp, kx, ky) ? 1 : 0;
    for (int i = 0; i < kMaxK; ++i) {
        in.kx[i] = (float)kx[i];
        in.ky[i] = (float)ky[i];
        in.kxd[i] = kx[i];
        in.kyd[i] = ky[i];
    }
    return in;
}

gp_status check_ws(const Plan& P, void* ws, size_t ws_bytes) {
    if (!ws) return fail(GP_ERR_INVALID_ARG, "workspace is NULL");
    if (ws_bytes < P.ws_bytes)
        return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, P.ws_bytes);
    return GP_OK;
}

}  // namespace

namespace {
// The tune cache is a flat JSON object {"<shape class>": <choice>, ...}.
void tune_load(gp_ctx* c) {
    FILE* fh = std::fopen(c->tune_path.c_str(), "r");
    if (!fh) return;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, fh)) > 0) txt.append(buf, n);
    std::fclose(fh);
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = txt.substr(i + 1, j - i - 1);
        size_t k = txt.find(':', j);
        if (k == std::string::npos) break;
        c->tuned[key] = (int)std::strtol(txt.c_str() + k + 1, nullptr, 10);
        i = txt.find_first_of(",}", k);
        if (i == std::string::npos) break;
    }
}

void tune_save(gp_ctx* c) {
    if (c->tune_path.empty()) return;
    const std::string tmp = c->tune_path + ".tmp";
    FILE* fh = std::fopen(tmp.c_str(), "w");
    if (!fh) return;
    std::fputs("{", fh);
    bool first = true;
    for (const auto& kv : c->tuned) {
        std::fprintf(fh, "%s\n \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    std::fputs("\n}\n", fh);
    std::fclose(fh);
    std::rename(tmp.c_str(), c->tune_path.c_str());
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// The choice for a shape class: the cached one, else (tuning on, not under
// graph capture) the fastest candidate, each timed on the call's stream after
// a warm-up launch, else `fallback`.
template <typename Launch>
int choose(gp_ctx* c, const std::string& key, const std::vector<int>& cands, int fallback, hipStream_t s,
           Launch&& launch) {
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) return it->second;
    if (!c->tuning || cands.size() < 2 || capturing(s)) return fallback;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fallback;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fallback;
    }
    int best = fallback;
    float best_ms = 1e30f;
    for (int cand : cands) {
        launch(cand);
        (void)hipEventRecord(e0, s);
        launch(cand);
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[key] = best;
    tune_save(c);
    return best;
}
}  // namespace

extern "C" gp_status gp_ctx_set_tuning(gp_ctx* ctx, int32_t on) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "ctx is NULL");
    ctx->tuning = on != 0;
    return GP_OK;
}

extern "C" gp_status gp_ctx_create(int device, const char* tune_cache, gp_ctx** out) {
    if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(GP_ERR_INVALID_ARG, "device %d of %d", device, n);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GP_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    {
        // the static scratch's address on this device (the previous current
        // device is restored)
        int prev = 0;
        HIP_TRY(hipGetDevice(&prev));
        HIP_TRY(hipSetDevice(device));
        const hipError_t e = scratch_setup(device);
        HIP_TRY(hipSetDevice(prev));
        if (e != hipSuccess)
            return fail(GP_ERR_HIP, "device %d: address of the static scratch: %s", device, hipGetErrorString(e));
    }
    gp_ctx* c = new gp_ctx;
    c->device = device;
    c->cus = prop.multiProcessorCount;
    if (tune_cache) {
        c->tune_path = tune_cache;
        tune_load(c);
    }
    *out = c;
    return GP_OK;
}

extern "C" void gp_ctx_destroy(gp_ctx* c) {
    if (!c) return;
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

extern "C" gp_status gp_background_layout(const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                                          gp_bkg_layout* layouts, size_t* bytes) {
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    if (layouts)
        for (int f = 0; f < nframes; ++f) {
            const FramePlan& F = P.fr[f];
            gp_bkg_layout& L = layouts[f];
            L.nx = F.nx;
            L.ny = F.ny;
            L.back_raw = (int64_t)(F.bkg_off + F.back_raw);
            L.rms_raw = (int64_t)(F.bkg_off + F.rms_raw);
            L.back = (int64_t)(F.bkg_off + F.back);
            L.rms = (int64_t)(F.bkg_off + F.rms);
            L.coef = (int64_t)(F.bkg_off + F.coef);
            L.iters = (int64_t)(F.bkg_off + F.iters);
            L.bytes = (int64_t)F.bkg_bytes;
        }
    if (bytes) *bytes = P.bkg_bytes;
    return GP_OK;
}

extern "C" gp_status gp_workspace_size(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                                       const gp_bkg_params* bp, const gp_det_params* dp, const gp_ap_params* ap,
                                       int32_t cat_capacity, int64_t comp_capacity, size_t* bytes) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    if (!bytes) return fail(GP_ERR_INVALID_ARG, "bytes is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if (dp && (st = check_det(dp)) != GP_OK) return st;
    if (ap && (st = check_ap(ap)) != GP_OK) return st;
    if (cat_capacity < 0) return fail(GP_ERR_INVALID_ARG, "cat_capacity < 0");
    if (comp_capacity < 0 || comp_capacity >= ((int64_t)1 << 31))
        return fail(GP_ERR_INVALID_ARG, "comp_capacity out of range");
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    plan_recs(comp_capacity > 0 ? comp_capacity : default_rec_cap(P), P);
    *bytes = P.ws_bytes;
    return GP_OK;
}

extern "C" gp_status gp_background(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                                   void* bkg, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    P.ws_bytes = P.o_recs;  // the record arrays are not used here
    if ((st = check_ws(P, ws, ws_bytes)) != GP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    // a one-frame call passes its descriptor with the mesh-statistics launch,
    // which stores it in the table for the launches that follow
    const bool one = nframes == 1 && !(bp->flags & GP_BKG_GRID_GIVEN);
    DescChunk tail{};
    if ((st = upload_desc(frames, nframes, bp, P, bkg, ws, 0, nullptr, s, one ? &tail : nullptr)) != GP_OK) return st;
    FrameDesc* desc = (FrameDesc*)((char*)ws + P.o_desc);
    if (!(bp->flags & GP_BKG_GRID_GIVEN)) {
        bool any_u16 = false, any_f32 = false;
        for (int f = 0; f < nframes; ++f) (frames[f].dtype == GP_U16 ? any_u16 : any_f32) = true;
        BkgArgs a{bp->clip_sigma, bp->crowd_tol, bp->mode_a, bp->mode_b, bp->max_iter, bp->filter_size,
                  any_u16 ? 1 : 0};
        {
            ProfScope ps(ctx, s, "mesh_stats");
            std::vector<int> cands;
            if (P.max_area <= 4096) cands.push_back(1);
            if (P.max_area <= 8192) cands.push_back(2);
            cands.push_back(3);
            cands.push_back(4);
            const FrameDesc* d1 = one ? &tail.d[0] : nullptr;
            if (any_u16) {
                // uint16 frames: exact integer statistics
                const int cfg = ctx->mesh_cfg ? ctx->mesh_cfg
                                              : choose(ctx, "mesh_stats_u16:" + std::to_string(P.max_area), cands, 0,
                                                       s, [&](int k) {
                                                           launch_mesh_stats_u16(desc, d1, nframes, (int)P.total_meshes,
                                                                                 P.max_area, a, k, s);
                                                       });
                launch_mesh_stats_u16(desc, d1, nframes, (int)P.total_meshes, P.max_area, a, cfg, s);
            }
            if (any_f32) {
                const int cfg = ctx->mesh_cfg ? ctx->mesh_cfg
                                              : choose(ctx, "mesh_stats:" + std::to_string(P.max_area), cands, 0, s,
                                                       [&](int k) {
                                                           launch_mesh_stats(desc, d1, nframes, (int)P.total_meshes,
                                                                             P.max_area, a, k, s);
                                                       });
                launch_mesh_stats(desc, d1, nframes, (int)P.total_meshes, P.max_area, a, cfg, s);
            }
        }
        HIP_TRY(hipGetLastError());
    }
    // small grids: the filter inside the y-spline launch
    const bool given = (bp->flags & GP_BKG_GRID_GIVEN) != 0;
    const int fsize = given ? 0 : bp->filter_size;
    if (filter_spline_fits(P.max_nx, P.max_ny, fsize)) {
        ProfScope ps(ctx, s, "filter_spline");
        launch_filter_spline(desc, nframes, P.max_nx, P.max_ny, fsize, s);
        HIP_TRY(hipGetLastError());
        return GP_OK;
    }
    if (!given) {
        ProfScope ps(ctx, s, "grid_filter");
        launch_grid_filter(desc, nframes, (int)P.total_meshes, bp->filter_size, s);
    }
    HIP_TRY(hipGetLastError());
    {
        ProfScope ps(ctx, s, "spline");
        launch_spline(desc, nframes, P.max_nx, P.max_ny, s);
    }
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

extern "C" gp_status gp_background_map(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                                       const gp_bkg_params* bp, const void* bkg, int32_t index, int32_t precision,
                                       double* back_map, double* rms_map, void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    if (index < 0 || index >= nframes) return fail(GP_ERR_INVALID_ARG, "frame index %d of %d", index, nframes);
    if (precision != GP_PREC_F32 && precision != GP_PREC_F64)
        return fail(GP_ERR_INVALID_ARG, "unknown precision %d", precision);
    if (!back_map && !rms_map) return GP_OK;
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    const FramePlan& F = P.fr[index];
    FrameDesc d{};
    d.data = frames[index].data;
    d.pitch = frames[index].pitch;
    d.W = frames[index].width;
    d.H = frames[index].height;
    d.dtype = frames[index].dtype;
    d.mw = bp->mesh_w;
    d.mh = bp->mesh_h;
    d.nx = F.nx;
    d.ny = F.ny;
    d.coef = (double*)((char*)bkg + F.bkg_off + F.coef);
    HIP_TRY(hipSetDevice(ctx->device));
    launch_bkg_map(d, back_map, rms_map, precision == GP_PREC_F64, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

static gp_status check_cat(const gp_catalog* cat, bool need_moments) {
    if (!cat) return fail(GP_ERR_INVALID_ARG, "catalogue is NULL");
    if (cat->capacity < 0) return fail(GP_ERR_INVALID_ARG, "catalogue capacity < 0");
    if (!cat->n_obj || !cat->status) return fail(GP_ERR_INVALID_ARG, "catalogue n_obj/status is NULL");
    if (!cat->x || !cat->y || !cat->flags) return fail(GP_ERR_INVALID_ARG, "catalogue x/y/flags is NULL");
    if (need_moments && (!cat->npix || !cat->xmin || !cat->xmax || !cat->ymin || !cat->ymax || !cat->pmin ||
                         !cat->flux || !cat->x2 || !cat->y2 || !cat->xy || !cat->peak))
        return fail(GP_ERR_INVALID_ARG, "a catalogue column is NULL");
    return GP_OK;
}

// prof = false: no timing events (nothing is created during the call)
static gp_status detect_run(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                            const void* bkg, const gp_det_params* dp, gp_catalog* cat, int32_t* const* seg,
                            int32_t* comp_status, void* ws, size_t ws_bytes, void* stream, bool prof) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if ((st = check_det(dp)) != GP_OK) return st;
    if ((st = check_cat(cat, true)) != GP_OK) return st;
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    plan_recs(1, P);
    if ((st = check_ws(P, ws, ws_bytes)) != GP_OK) return st;
    plan_recs(cap_for(P, ws_bytes), P);
    if (P.total_tiles >= ((int64_t)1 << 31)) return fail(GP_ERR_UNSUPPORTED, "too many tiles in one batch");
    if (ceil_div(P.total_blocks, kScanChunk) > kMaxScanChunks)
        return fail(GP_ERR_UNSUPPORTED, "a detection batch holds at most 2^31 pixels (1024-pixel blocks per frame)");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    DescChunk tail{};
    if ((st = upload_desc(frames, nframes, bp, P, bkg, ws, cat->capacity, seg, s, &tail)) != GP_OK) return st;
    char* W = (char*)ws;
    // filter arguments
    DetArgsIn in = det_in(dp);
    in.want_seg = seg ? 1 : 0;
    DetArgs* dargs = (DetArgs*)(W + P.o_detargs);
    DetWork wk{};
    wk.desc = (FrameDesc*)(W + P.o_desc);
    wk.nframes = nframes;
    wk.total_tiles = (int32_t)P.total_tiles;
    wk.counters = (uint32_t*)(W + P.o_counters);
    wk.tiles = (TileInfo*)(W + P.o_tiles);
    wk.edges = (int16_t*)(W + P.o_edges);
    wk.recs = (CompRec*)(W + P.o_recs);
    wk.parent = (int32_t*)(W + P.o_parent);
    wk.root = (int32_t*)(W + P.o_root);
    wk.label = (int32_t*)(W + P.o_label);
    wk.blockcnt = (uint32_t*)(W + P.o_blockcnt);
    wk.chunksum = (uint32_t*)(W + P.o_chunks);
    wk.bitmap = (uint32_t*)(W + P.o_bitmap);
    wk.rec_cap = (int32_t)P.rec_cap;
    wk.total_blocks = (int32_t)P.total_blocks;
    const bool f64 = dp->precision == GP_PREC_F64;
    const int rad = (in.separable && dp->kw == dp->kh) ? dp->kw / 2 : -1;
    // tiles an XCD holds in flight (its CUs times the detection workgroups
    // resident per CU)
    wk.ahead = std::max(0, ctx->cus / kXcds) * detect_tiles_per_cu(f64, rad, bp->mesh_w);
    {
        ProfScope ps(ctx, s, "setup", prof);
        launch_det_setup(tail, (FrameDesc*)(W + P.o_desc), in, dargs, wk.counters, s);
    }
    HIP_TRY(hipGetLastError());
    {
        ProfScope ps(ctx, s, "detect_tiles", prof);
        launch_detect_tiles(wk, dargs, f64, rad, bp->mesh_w, s);
    }
    HIP_TRY(hipGetLastError());
    const int persist = ctx->cus * 4;
    {
        ProfScope ps(ctx, s, "merge", prof);
        launch_merge(wk, dp->connectivity, dp->minarea, persist, s);
    }
    HIP_TRY(hipGetLastError());
    CatOut co{cat->capacity, cat->n_obj, cat->status, cat->npix, cat->xmin, cat->xmax, cat->ymin, cat->ymax,
              cat->pmin, cat->flux, cat->x, cat->y, cat->x2, cat->y2, cat->xy, cat->peak, cat->flags};
    {
        ProfScope ps(ctx, s, "catalog", prof);
        launch_catalog(wk, co, dp->minarea, persist, comp_status, s);
    }
    HIP_TRY(hipGetLastError());
    if (seg) {
        ProfScope ps(ctx, s, "seg", prof);
        for (int f = 0; f < nframes; ++f)
            if (seg[f]) launch_seg(wk, f, (int64_t)frames[f].width * frames[f].height, s);
    }
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

extern "C" gp_status gp_detect(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                               const void* bkg, const gp_det_params* dp, gp_catalog* cat, int32_t* const* seg,
                               int32_t* comp_status, void* ws, size_t ws_bytes, void* stream) {
    return detect_run(ctx, frames, nframes, bp, bkg, dp, cat, seg, comp_status, ws, ws_bytes, stream, true);
}

extern "C" gp_status gp_detect_noalloc(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                                       const gp_bkg_params* bp, const void* bkg, const gp_det_params* dp,
                                       gp_catalog* cat, int32_t* const* seg, int32_t* comp_status, void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    plan_recs(1, P);
    if (P.ws_bytes > kStaticScratchBytes)
        return fail(GP_ERR_UNSUPPORTED,
                    "batch too large for the static scratch: its detection needs at least %zu bytes, the scratch "
                    "holds %zu (use gp_detect with a workspace)",
                    P.ws_bytes, kStaticScratchBytes);
    void* ws = scratch_of(ctx->device);
    if (!ws) return fail(GP_ERR_HIP, "no static scratch address for device %d", ctx->device);
    return detect_run(ctx, frames, nframes, bp, bkg, dp, cat, seg, comp_status, ws, kStaticScratchBytes, stream,
                      false);
}

// gp_peaks and gp_peaks_psf (psf null: the plain filter of dp)
static gp_status peaks_run(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                           const void* bkg, const gp_det_params* dp, const gp_peak_params* pp,
                           const gp_psf_model* psf, gp_catalog* cat, int32_t* comp_status, void* ws, size_t ws_bytes,
                           void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if (psf) {
        if (!dp) return fail(GP_ERR_INVALID_ARG, "detection parameters are NULL");
        if (!std::isfinite(dp->thresh)) return fail(GP_ERR_INVALID_ARG, "thresh must be finite");
        if (std::isnan(dp->sat_level)) return fail(GP_ERR_INVALID_ARG, "sat_level is NaN");
        if (dp->precision != GP_PREC_F32 && dp->precision != GP_PREC_F64)
            return fail(GP_ERR_INVALID_ARG, "unknown precision %d", dp->precision);
        if (!psf->kernels) return fail(GP_ERR_INVALID_ARG, "PSF kernels are NULL");
        if (psf->kw < 1 || psf->kh < 1 || psf->kw > kMaxK || psf->kh > kMaxK || !(psf->kw & 1) || !(psf->kh & 1))
            return fail(GP_ERR_INVALID_ARG, "PSF kernels must be odd and at most 15 per side (got %dx%d)", psf->kw,
                        psf->kh);
        if (psf->nmodes < 0 || psf->nmodes > kMaxModes)
            return fail(GP_ERR_INVALID_ARG, "nmodes must be in [0, %d]", kMaxModes);
        if (psf->bin < 1) return fail(GP_ERR_INVALID_ARG, "coefficient-map bin must be >= 1");
        for (int i = 0; i < (psf->nmodes + 1) * psf->kw * psf->kh; ++i)
            if (!std::isfinite(psf->kernels[i])) return fail(GP_ERR_INVALID_ARG, "PSF kernel has a non-finite tap");
        if (psf->nmodes > 0) {
            if (!psf->maps) return fail(GP_ERR_INVALID_ARG, "coefficient maps are NULL");
            for (int f = 0; f < nframes; ++f) {
                const gp_coef_maps& m = psf->maps[f];
                const int64_t mx = ceil_div(frames[f].width, psf->bin), my = ceil_div(frames[f].height, psf->bin);
                if (!m.data) return fail(GP_ERR_INVALID_ARG, "coefficient maps of frame %d are NULL", f);
                if (m.pitch < mx || (psf->nmodes > 1 && m.plane < m.pitch * my) || m.plane < 0)
                    return fail(GP_ERR_INVALID_ARG, "coefficient maps of frame %d: pitch or plane too small", f);
            }
        }
    } else if ((st = check_det(dp)) != GP_OK) {
        return st;
    }
    if (!pp) return fail(GP_ERR_INVALID_ARG, "peak parameters are NULL");
    if (pp->sep < 0 || pp->sep > kMaxPeakWin || pp->cwin < 0 || pp->cwin > kMaxPeakWin)
        return fail(GP_ERR_INVALID_ARG, "sep and cwin must be in [0, %d] (got %d, %d)", kMaxPeakWin, pp->sep, pp->cwin);
    if ((st = check_cat(cat, true)) != GP_OK) return st;
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    const int kw = psf ? psf->kw : dp->kw, kh = psf ? psf->kh : dp->kh;
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    plan_recs(1, P);
    if ((st = check_ws(P, ws, ws_bytes)) != GP_OK) return st;
    plan_recs(cap_for(P, ws_bytes), P);
    if (P.total_tiles >= ((int64_t)1 << 31)) return fail(GP_ERR_UNSUPPORTED, "too many tiles in one batch");
    if (ceil_div(P.total_blocks, kScanChunk) > kMaxScanChunks)
        return fail(GP_ERR_UNSUPPORTED, "a detection batch holds at most 2^31 pixels (1024-pixel blocks per frame)");
    const bool f64 = dp->precision == GP_PREC_F64;
    if (peak_lds_bytes(pp->sep, pp->cwin, kw, kh, f64, bp->mesh_w) > 160 * 1024)
        return fail(GP_ERR_UNSUPPORTED, "peak windows and filter too large for one tile's LDS");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    DescChunk tail{};
    if ((st = upload_desc(frames, nframes, bp, P, bkg, ws, cat->capacity, nullptr, s, &tail)) != GP_OK) return st;
    char* W = (char*)ws;
    DetArgsIn in{};
    if (psf) {
        // the plain-filter fields are unused: a dense reference tap keeps the
        // device normalisation finite
        in.kw = kw;
        in.kh = kh;
        in.conn = 8;
        in.thresh = dp->thresh;
        in.sat = dp->sat_level;
        in.minarea = 1;
        in.kraw[(kh / 2) * kw + kw / 2] = 1.0f;
    } else {
        in = det_in(dp);
    }
    DetArgs* dargs = (DetArgs*)(W + P.o_detargs);
    DetWork wk{};
    wk.desc = (FrameDesc*)(W + P.o_desc);
    wk.nframes = nframes;
    wk.total_tiles = (int32_t)P.total_tiles;
    wk.counters = (uint32_t*)(W + P.o_counters);
    wk.tiles = (TileInfo*)(W + P.o_tiles);
    wk.edges = (int16_t*)(W + P.o_edges);
    wk.recs = (CompRec*)(W + P.o_recs);
    wk.parent = (int32_t*)(W + P.o_parent);
    wk.root = (int32_t*)(W + P.o_root);
    wk.label = (int32_t*)(W + P.o_label);
    wk.blockcnt = (uint32_t*)(W + P.o_blockcnt);
    wk.chunksum = (uint32_t*)(W + P.o_chunks);
    wk.bitmap = (uint32_t*)(W + P.o_bitmap);
    wk.rec_cap = (int32_t)P.rec_cap;
    wk.total_blocks = (int32_t)P.total_blocks;
    // tiles an XCD holds in flight (two peak workgroups per CU)
    wk.ahead = std::max(0, ctx->cus / kXcds) * 2;
    PsfArgs* pargs = nullptr;
    PsfFrame* pframes = nullptr;
    {
        ProfScope ps(ctx, s, "setup");
        launch_det_setup(tail, (FrameDesc*)(W + P.o_desc), in, dargs, wk.counters, s);
        if (psf) {
            // the model's header and taps (FP32 as given and their exact FP64
            // values), then the frames' map descriptors
            pargs = (PsfArgs*)(W + P.o_psf);
            pframes = (PsfFrame*)(W + P.o_psf + sizeof(PsfArgs));
            // taps as [column][row][mode], modes padded to kMaxModes + 1
            const int nt = kw * kh * (kMaxModes + 1);
            std::vector<float> tf(nt, 0.0f);
            std::vector<double> td(nt, 0.0);
            for (int m = 0; m <= psf->nmodes; ++m)
                for (int a = 0; a < kh; ++a)
                    for (int b = 0; b < kw; ++b) {
                        const float v = psf->kernels[(m * kh + a) * kw + b];
                        tf[(b * kh + a) * (kMaxModes + 1) + m] = v;
                        td[(b * kh + a) * (kMaxModes + 1) + m] = (double)v;
                    }
            const int32_t hdr[4] = {psf->nmodes, psf->bin, kw, kh};
            launch_write_bytes(pargs, hdr, sizeof(hdr), s);
            launch_write_bytes(pargs->taps, tf.data(), tf.size() * 4, s);
            launch_write_bytes(pargs->tapsd, td.data(), td.size() * 8, s);
            std::vector<PsfFrame> pf(nframes);
            for (int f = 0; f < nframes; ++f)
                pf[f] = psf->nmodes > 0 ? PsfFrame{psf->maps[f].data, psf->maps[f].pitch, psf->maps[f].plane}
                                        : PsfFrame{nullptr, 0, 0};
            launch_write_bytes(pframes, pf.data(), pf.size() * sizeof(PsfFrame), s);
        }
    }
    HIP_TRY(hipGetLastError());
    CatOut co{cat->capacity, cat->n_obj, cat->status, cat->npix, cat->xmin, cat->xmax, cat->ymin, cat->ymax,
              cat->pmin, cat->flux, cat->x, cat->y, cat->x2, cat->y2, cat->xy, cat->peak, cat->flags};
    {
        ProfScope ps(ctx, s, psf ? "peaks_psf" : "peaks");
        launch_peaks(wk, dargs, co, comp_status, f64, pp->sep, pp->cwin, kw, kh, ctx->cus * 4, pargs, pframes,
                     psf ? psf->nmodes : 0, bp->mesh_w, std::max(0, ctx->cus / kXcds), s);
    }
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

extern "C" gp_status gp_peaks(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                              const void* bkg, const gp_det_params* dp, const gp_peak_params* pp, gp_catalog* cat,
                              int32_t* comp_status, void* ws, size_t ws_bytes, void* stream) {
    return peaks_run(ctx, frames, nframes, bp, bkg, dp, pp, nullptr, cat, comp_status, ws, ws_bytes, stream);
}

extern "C" gp_status gp_peaks_psf(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                                  const void* bkg, const gp_det_params* dp, const gp_peak_params* pp,
                                  const gp_psf_model* psf, gp_catalog* cat, int32_t* comp_status, void* ws,
                                  size_t ws_bytes, void* stream) {
    if (!psf) return fail(GP_ERR_INVALID_ARG, "PSF model is NULL");
    return peaks_run(ctx, frames, nframes, bp, bkg, dp, pp, psf, cat, comp_status, ws, ws_bytes, stream);
}

extern "C" gp_status gp_aperture(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                                 const void* bkg, const gp_catalog* cat, const gp_ap_params* ap, gp_phot* out,
                                 void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if ((st = check_ap(ap)) != GP_OK) return st;
    if ((st = check_cat(cat, false)) != GP_OK) return st;
    if (!out || !out->flux || !out->area || !out->bkg) return fail(GP_ERR_INVALID_ARG, "photometry output is NULL");
    if (ap->want_err && !out->fluxerr) return fail(GP_ERR_INVALID_ARG, "fluxerr is NULL with want_err");
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    P.ws_bytes = P.o_recs;
    if ((st = check_ws(P, ws, ws_bytes)) != GP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    // only the descriptors are needed: a one-frame call passes its descriptor
    // with the launch, a batch reads the table at the start of the workspace
    const bool one = nframes == 1;
    DescChunk tail{};
    if ((st = upload_desc(frames, nframes, bp, P, bkg, ws, cat->capacity, nullptr, s, one ? &tail : nullptr)) != GP_OK)
        return st;
    ApArgs a{};
    a.nr = ap->nr;
    a.want_err = ap->want_err ? 1 : 0;
    a.capacity = cat->capacity;
    a.nframes = nframes;
    float rmax = ap->r_out;
    for (int i = 0; i < ap->nr; ++i) {
        a.radii[i] = ap->radii[i];
        rmax = std::max(rmax, ap->radii[i]);
    }
    a.r_in = ap->r_in;
    a.r_out = ap->r_out;
    a.gain = ap->gain;
    a.rmax = rmax;
    {
        // circles in increasing radius (ties keep apertures first)
        std::vector<std::pair<float, int>> c;
        for (int i = 0; i < ap->nr; ++i) c.push_back({ap->radii[i], i});
        c.push_back({ap->r_in, kMaxRadii});
        c.push_back({ap->r_out, kMaxRadii + 1});
        std::stable_sort(c.begin(), c.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        for (size_t j = 0; j < c.size(); ++j) {
            a.crad[j] = c[j].first;
            a.crole[j] = c[j].second;
        }
    }
    ApCat c{cat->n_obj, cat->x, cat->y, cat->flags, out->flux, out->area, out->bkg, out->fluxerr};
    const int total_rows = nframes * cat->capacity;
    {
        ProfScope ps(ctx, s, "aperture");
        int max_nx = 1;
        for (int i = 0; i < nframes; ++i) max_nx = std::max(max_nx, (frames[i].width + bp->mesh_w - 1) / bp->mesh_w);
        const bool f64 = ap->precision == GP_PREC_F64;
        auto run = [&](int per_cu) {
            const int blocks = std::max(1, std::min(ctx->cus * per_cu, (total_rows + 3) / 4));
            launch_aperture((const FrameDesc*)((char*)ws + P.o_desc), one ? &tail.d[0] : nullptr, a, c, total_rows,
                            blocks, bp->mesh_w, max_nx, f64, s);
        };
        // workgroups per CU of the persistent grid
        const std::string key = "aperture:" + std::to_string(ap->nr) + ":" + std::to_string((int)std::ceil(rmax)) +
                                ":" + std::to_string(bp->mesh_w) + (f64 ? ":f64" : ":f32");
        run(choose(ctx, key, {2, 4, 8, 16}, 8, s, run));
    }
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

extern "C" gp_status gp_growth_radii(double fwhm, int32_t cap, int32_t* radii, int32_t* n) {
    if (!n) return fail(GP_ERR_INVALID_ARG, "n is NULL");
    if (!(fwhm > 0.0) || !std::isfinite(fwhm)) return fail(GP_ERR_INVALID_ARG, "fwhm must be positive and finite");
    if (cap < 0 || (cap > 0 && !radii)) return fail(GP_ERR_INVALID_ARG, "radii is NULL with cap > 0");
    const double lo = std::ceil(0.75 * fwhm), hi = std::ceil(5.0 * fwhm);
    if (hi > 1.0e6) return fail(GP_ERR_INVALID_ARG, "fwhm too large");
    int32_t k = 0;
    for (double r = lo; r <= hi; r += 1.0, ++k)
        if (k < cap) radii[k] = (int32_t)r;
    *n = k;
    return GP_OK;
}

namespace {
// The nested top-hat kernels' offset classes (exact: squared distances are
// multiples of 1/4): for each radius, how many offsets join the running sums
// with weight 1 and how many it cuts.  Only the counts are taken here (list
// offsets and the launch's LDS size); k_growth_table classifies the offsets
// itself and computes the areas.
void growth_lists(const gp_growth_params* gp, GrowArgs& a) {
    const int R = gp->radii[gp->nr - 1];
    std::vector<int> nfull(gp->nr, 0), ncut(gp->nr, 0);
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            const double ax = std::fabs((double)dx), ay = std::fabs((double)dy);
            const double nx = std::max(ax - 0.5, 0.0), ny = std::max(ay - 0.5, 0.0);
            const double dmin2 = nx * nx + ny * ny;
            const double dmax2 = (ax + 0.5) * (ax + 0.5) + (ay + 0.5) * (ay + 0.5);
            for (int k = 0; k < gp->nr; ++k) {
                const double r2 = (double)gp->radii[k] * gp->radii[k];
                const double rp2 = (k > 0) ? (double)gp->radii[k - 1] * gp->radii[k - 1] : -1.0;
                if (dmax2 <= r2 && dmax2 > rp2) ++nfull[k];
                if (dmin2 < r2 && r2 < dmax2) ++ncut[k];
            }
        }
    a.full_off[0] = a.cut_off[0] = 0;
    for (int k = 0; k < gp->nr; ++k) {
        a.full_off[k + 1] = a.full_off[k] + nfull[k];
        a.cut_off[k + 1] = a.cut_off[k] + ncut[k];
    }
    a.nfull = a.full_off[gp->nr];
    a.ncut = a.cut_off[gp->nr];
}

size_t growth_table_bytes(const GrowArgs& a) {
    return align256(4 * (size_t)a.nfull) + align256(4 * (size_t)a.ncut) + align256(8 * (size_t)a.ncut);
}
}  // namespace

extern "C" gp_status gp_growth(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                               const void* bkg, const gp_catalog* cat, const gp_growth_params* gp,
                               gp_growth_out* out, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if ((st = check_cat(cat, false)) != GP_OK) return st;
    if (!gp || !gp->radii) return fail(GP_ERR_INVALID_ARG, "growth parameters or radii are NULL");
    if (gp->nr < 1 || gp->nr > kMaxGrowthRadii) return fail(GP_ERR_INVALID_ARG, "nr must be in [1, %d]", kMaxGrowthRadii);
    for (int k = 0; k < gp->nr; ++k) {
        if (gp->radii[k] < 1 || gp->radii[k] > kMaxGrowthRadius)
            return fail(GP_ERR_INVALID_ARG, "radius %d must be in [1, %d]", k, kMaxGrowthRadius);
        if (k > 0 && gp->radii[k] <= gp->radii[k - 1])
            return fail(GP_ERR_INVALID_ARG, "radii must be strictly increasing");
    }
    if (gp->precision != GP_PREC_F32 && gp->precision != GP_PREC_F64)
        return fail(GP_ERR_INVALID_ARG, "unknown precision %d", gp->precision);
    if (!out || !out->sum || !out->area) return fail(GP_ERR_INVALID_ARG, "growth output sum/area is NULL");
    if (!bkg) return fail(GP_ERR_INVALID_ARG, "background buffer is NULL");
    const bool f64 = gp->precision == GP_PREC_F64;
    GrowArgs a{};
    a.nr = gp->nr;
    a.R = gp->radii[gp->nr - 1];
    a.side = 2 * a.R + 1;
    a.capacity = cat->capacity;
    a.nframes = nframes;
    a.want_var = out->var ? 1 : 0;
    for (int k = 0; k < gp->nr; ++k) a.radii[k] = gp->radii[k];
    a.div_magic = (int32_t)(((1u << 20) + a.side - 1) / a.side);
    for (int i = 0; i < a.side * a.side; ++i)
        if ((int)(((uint32_t)i * (uint32_t)a.div_magic) >> 20) != i / a.side)
            return fail(GP_ERR_UNSUPPORTED, "window index split fails for side %d", a.side);
    growth_lists(gp, a);
    int max_nx = 1;
    for (int i = 0; i < nframes; ++i) max_nx = std::max(max_nx, (frames[i].width + bp->mesh_w - 1) / bp->mesh_w);
    // spline pieces a window of `side` columns can touch (knots one mesh apart,
    // the last at least half a mesh from its neighbour)
    a.nixmax = std::max(1, std::min(max_nx + 1, (a.side - 1) / std::max(bp->mesh_w, 1) + 3));
    // wavefronts per workgroup: as many (up to 8) as fit the 160 KB of LDS
    int waves = 8;
    while (waves > 1 && growth_lds_bytes(a.nfull, a.ncut, a.side, a.nixmax, a.want_var, f64, waves) > 160 * 1024)
        --waves;
    if (growth_lds_bytes(a.nfull, a.ncut, a.side, a.nixmax, a.want_var, f64, waves) > 160 * 1024)
        return fail(GP_ERR_UNSUPPORTED, "growth window of radius %d does not fit in LDS", a.R);
    Plan P;
    plan_bkg(frames, nframes, bp, P);
    plan_fixed(nframes, P);
    const size_t o_tab = P.o_recs;
    P.ws_bytes = o_tab + growth_table_bytes(a);
    if ((st = check_ws(P, ws, ws_bytes)) != GP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    const bool one = nframes == 1;
    DescChunk tail{};
    if ((st = upload_desc(frames, nframes, bp, P, bkg, ws, cat->capacity, nullptr, s, one ? &tail : nullptr)) != GP_OK)
        return st;
    char* W = (char*)ws;
    GrowTab t;
    t.full = (int32_t*)(W + o_tab);
    t.cut = (int32_t*)(W + o_tab + align256(4 * (size_t)a.nfull));
    t.cutw = (double*)(W + o_tab + align256(4 * (size_t)a.nfull) + align256(4 * (size_t)a.ncut));
    GrowOut g{cat->n_obj, cat->x, cat->y, out->sum, out->var, out->area, out->flags};
    {
        ProfScope ps(ctx, s, "growth");
        launch_growth_table(a, t, s);
        const int total_rows = nframes * cat->capacity;
        const int blocks = std::max(1, std::min(ctx->cus * 4, (total_rows + waves - 1) / waves));
        hipError_t e = launch_growth((const FrameDesc*)(W + P.o_desc), one ? &tail.d[0] : nullptr, a, t, g, blocks,
                                     waves, f64, s);
        if (e != hipSuccess) return fail(GP_ERR_HIP, "growth launch: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipGetLastError());
    return GP_OK;
}

namespace {
gp_status check_conv(const gp_frame* frames, int32_t nframes, const gp_conv_params* cp) {
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if (!cp) return fail(GP_ERR_INVALID_ARG, "convolution parameters are NULL");
    if (!cp->kx || !cp->ky) return fail(GP_ERR_INVALID_ARG, "convolution taps are NULL");
    if (cp->lx < 1 || cp->ly < 1 || cp->lx > kMaxConvTaps || cp->ly > kMaxConvTaps || !(cp->lx & 1) || !(cp->ly & 1))
        return fail(GP_ERR_INVALID_ARG, "tap counts must be odd and at most %d (got %d, %d)", kMaxConvTaps, cp->lx,
                    cp->ly);
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < cp->lx; ++i) {
        if (!std::isfinite(cp->kx[i])) return fail(GP_ERR_INVALID_ARG, "kx has a non-finite tap");
        sx += cp->kx[i];
    }
    for (int i = 0; i < cp->ly; ++i) {
        if (!std::isfinite(cp->ky[i])) return fail(GP_ERR_INVALID_ARG, "ky has a non-finite tap");
        sy += cp->ky[i];
    }
    if (sx == 0.0 || sy == 0.0) return fail(GP_ERR_INVALID_ARG, "kernel taps sum to zero");
    if (!(cp->gain > 0.f) || !std::isfinite(cp->gain)) return fail(GP_ERR_INVALID_ARG, "gain must be positive");
    if (!(cp->read_noise >= 0.f) || !(cp->dark_current >= 0.f) || !(cp->exptime >= 0.f) ||
        !std::isfinite(cp->read_noise) || !std::isfinite(cp->dark_current) || !std::isfinite(cp->exptime))
        return fail(GP_ERR_INVALID_ARG, "read_noise, dark_current and exptime must be finite and >= 0");
    if (std::isnan(cp->sat_level)) return fail(GP_ERR_INVALID_ARG, "sat_level is NaN");
    if (cp->precision != GP_PREC_F32 && cp->precision != GP_PREC_F64)
        return fail(GP_ERR_INVALID_ARG, "unknown precision %d", cp->precision);
    return GP_OK;
}

// Workspace of a convolution-background call: the frame table, the
// workgroup bases and a flag per frame, then every frame's slice of the two
// working-precision planes (hA / hG and G), of the per-row band flags and of
// the per-tile flags.
struct ConvPlan {
    size_t tab, hb, vb, ff, hA, G, flags, tiles, total;
    std::vector<int64_t> plane, fl, tl;
    std::vector<int32_t> hbase, vbase;
    int64_t htotal = 0, vtotal = 0;
};
ConvPlan conv_plan(const gp_frame* frames, int32_t nframes, const gp_conv_params* cp) {
    ConvPlan p;
    const size_t real = cp->precision == GP_PREC_F64 ? 8 : 4;
    int64_t pe = 0, fb = 0, tb = 0;
    for (int f = 0; f < nframes; ++f) {
        const int64_t W = frames[f].width, H = frames[f].height;
        const int64_t bx = (W + kCvTilePx - 1) / kCvTilePx, by = (H + kCvTilePx - 1) / kCvTilePx;
        p.plane.push_back(pe);
        pe += (W * H + 63) / 64 * 64;
        p.fl.push_back(fb);
        fb += (H * bx + 255) / 256 * 256;
        p.tl.push_back(tb);
        tb += (bx * by + 255) / 256 * 256;
        p.hbase.push_back((int32_t)p.htotal);
        p.htotal += (W + kCvSegPx - 1) / kCvSegPx * H;
        p.vbase.push_back((int32_t)p.vtotal);
        p.vtotal += bx * by;
    }
    p.tab = 256;
    p.hb = p.tab + align256(sizeof(CvFrame) * (size_t)nframes);
    p.vb = p.hb + align256(4 * (size_t)nframes);
    p.ff = p.vb + align256(4 * (size_t)nframes);
    p.hA = p.ff + align256(4 * (size_t)nframes);
    p.G = p.hA + align256(real * (size_t)pe);
    p.flags = p.G + align256(real * (size_t)pe);
    p.tiles = p.flags + align256((size_t)fb);
    p.total = p.tiles + align256((size_t)tb);
    return p;
}
size_t conv_ws_bytes(const gp_frame* frames, int32_t nframes, const gp_conv_params* cp) {
    return conv_plan(frames, nframes, cp).total;
}
}  // namespace

extern "C" gp_status gp_background_conv_ws(const gp_frame* frames, int32_t nframes, const gp_conv_params* cp,
                                           size_t* bytes) {
    gp_status st;
    if ((st = check_conv(frames, nframes, cp)) != GP_OK) return st;
    if (!bytes) return fail(GP_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = conv_ws_bytes(frames, nframes, cp);
    return GP_OK;
}

extern "C" gp_status gp_background_conv(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                                        const uint8_t* const* masks, const gp_conv_params* cp, void* const* back,
                                        void* const* rms, int64_t* unfilled, void* ws, size_t ws_bytes,
                                        void* stream) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st;
    if ((st = check_conv(frames, nframes, cp)) != GP_OK) return st;
    if (!back || !rms) return fail(GP_ERR_INVALID_ARG, "back/rms arrays are NULL");
    for (int f = 0; f < nframes; ++f)
        if (!back[f] || !rms[f]) return fail(GP_ERR_INVALID_ARG, "back/rms of frame %d is NULL", f);
    if (!unfilled) return fail(GP_ERR_INVALID_ARG, "unfilled is NULL");
    if (!ws) return fail(GP_ERR_INVALID_ARG, "workspace is NULL");
    const size_t need = conv_ws_bytes(frames, nframes, cp);
    if (ws_bytes < need)
        return fail(GP_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    const bool f64 = cp->precision == GP_PREC_F64;
    const ConvPlan P = conv_plan(frames, nframes, cp);
    if (P.htotal >= INT32_MAX - 8 || P.vtotal >= INT32_MAX - 8)
        return fail(GP_ERR_UNSUPPORTED, "too many workgroups for one call (%lld, %lld)", (long long)P.htotal,
                    (long long)P.vtotal);
    char* W = (char*)ws;
    CvWork w{};
    w.tab = (CvFrame*)(W + P.tab);
    w.hbase = (int32_t*)(W + P.hb);
    w.vbase = (int32_t*)(W + P.vb);
    w.fflag = (int32_t*)(W + P.ff);
    w.hA = W + P.hA;
    w.G = W + P.G;
    w.flags = (uint8_t*)(W + P.flags);
    w.tiles = (uint8_t*)(W + P.tiles);
    w.unfilled = unfilled;
    std::vector<CvChunk> chunks((nframes + kCvChunk - 1) / kCvChunk);
    for (int f = 0; f < nframes; ++f) {
        CvChunk& c = chunks[f / kCvChunk];
        if (c.count == 0) c.first = f;
        CvFrame& r = c.f[c.count];
        r = CvFrame{};
        r.data = frames[f].data;
        r.mask = masks ? masks[f] : nullptr;
        r.back = back[f];
        r.rms = rms[f];
        r.pitch = frames[f].pitch;
        r.plane = P.plane[f];
        r.flags = P.fl[f];
        r.tiles = P.tl[f];
        r.W = frames[f].width;
        r.H = frames[f].height;
        r.dtype = frames[f].dtype;
        c.hbase[c.count] = P.hbase[f];
        c.vbase[c.count] = P.vbase[f];
        ++c.count;
    }
    CvArgs a{};
    a.lx = cp->lx;
    a.ly = cp->ly;
    a.gain = cp->gain;
    a.read_noise = cp->read_noise;
    a.dark = cp->dark_current;
    a.exptime = cp->exptime;
    a.sat = cp->sat_level;
    a.nm_c1 = 1.0 / (double)cp->gain;
    a.nm_c0 = ((double)cp->read_noise * (double)cp->read_noise + (double)cp->dark_current * (double)cp->exptime) /
              ((double)cp->gain * (double)cp->gain);
    // unit-sum taps: the FP64 sum in tap order, then each tap divided by it
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < cp->lx; ++i) sx += (double)cp->kx[i];
    for (int i = 0; i < cp->ly; ++i) sy += (double)cp->ky[i];
    for (int i = 0; i < cp->lx; ++i) a.kx[i] = (double)cp->kx[i] / sx;
    for (int i = 0; i < cp->ly; ++i) a.ky[i] = (double)cp->ky[i] / sy;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(ctx->device));
    ProfScope ps(ctx, s, "background_conv");
    const hipError_t e = launch_conv(chunks.data(), (int)chunks.size(), nframes, (int)P.htotal, (int)P.vtotal, a, w,
                                     f64, s);
    if (e != hipSuccess) return fail(GP_ERR_HIP, "background convolution: %s", hipGetErrorString(e));
    return GP_OK;
}

// ---------------------------------------------------------------------------
// Captured batches: the three calls over one batch recorded once into a HIP
// graph (on a private stream) and replayed with one launch.  The parameters
// and host arrays are copied, so the caller's may be freed after creation.
struct gp_graph {
    gp_ctx* ctx = nullptr;
    std::vector<gp_frame> frames;
    gp_bkg_params bp{};
    void* bkg = nullptr;
    gp_det_params dp{};
    std::vector<float> kernel;
    gp_catalog cat{};
    std::vector<int32_t*> seg;
    bool has_seg = false;
    int32_t* comp_status = nullptr;
    gp_ap_params ap{};
    std::vector<float> radii;
    gp_phot phot{};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
// record the three calls into a new graph (the context's per-kernel timing is
// off while recording: its events would belong to the capture, not a replay)
gp_status graph_record(gp_graph* g, hipGraph_t* out) {
    gp_ctx* c = g->ctx;
    const bool prof = c->profiling;
    c->profiling = false;
    HIP_TRY(hipSetDevice(c->device));
    hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        c->profiling = prof;
        return fail(GP_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    const int n = (int)g->frames.size();
    gp_status st = gp_background(c, g->frames.data(), n, &g->bp, g->bkg, g->ws, g->ws_bytes, g->cap);
    if (st == GP_OK)
        st = gp_detect(c, g->frames.data(), n, &g->bp, g->bkg, &g->dp, &g->cat, g->has_seg ? g->seg.data() : nullptr,
                       g->comp_status, g->ws, g->ws_bytes, g->cap);
    if (st == GP_OK)
        st = gp_aperture(c, g->frames.data(), n, &g->bp, g->bkg, &g->cat, &g->ap, &g->phot, g->ws, g->ws_bytes,
                         g->cap);
    const std::string msg = g_err;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->cap, &graph);
    c->profiling = prof;
    if (st != GP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        g_err = msg;
        return st;
    }
    if (e != hipSuccess) return fail(GP_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    *out = graph;
    return GP_OK;
}

void graph_free(gp_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
}
}  // namespace

extern "C" gp_status gp_graph_create(gp_ctx* ctx, const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                                     void* bkg, const gp_det_params* dp, gp_catalog* cat, int32_t* const* seg,
                                     int32_t* comp_status, const gp_ap_params* ap, gp_phot* phot, void* ws,
                                     size_t ws_bytes, gp_graph** out) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    if (!out) return fail(GP_ERR_INVALID_ARG, "out is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if ((st = check_bkg(bp, frames, nframes)) != GP_OK) return st;
    if ((st = check_det(dp)) != GP_OK) return st;
    if ((st = check_ap(ap)) != GP_OK) return st;
    if ((st = check_cat(cat, true)) != GP_OK) return st;
    if (!phot) return fail(GP_ERR_INVALID_ARG, "photometry output is NULL");
    gp_graph* g = new gp_graph;
    g->ctx = ctx;
    g->frames.assign(frames, frames + nframes);
    g->bp = *bp;
    g->bkg = bkg;
    g->dp = *dp;
    g->kernel.assign(dp->kernel, dp->kernel + (size_t)dp->kw * dp->kh);
    g->dp.kernel = g->kernel.data();
    g->cat = *cat;
    g->has_seg = seg != nullptr;
    if (seg) g->seg.assign(seg, seg + nframes);
    g->comp_status = comp_status;
    g->ap = *ap;
    g->radii.assign(ap->radii, ap->radii + ap->nr);
    g->ap.radii = g->radii.data();
    g->phot = *phot;
    g->ws = ws;
    g->ws_bytes = ws_bytes;
    hipError_t e;
    if ((e = hipSetDevice(ctx->device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking)) != hipSuccess) {
        graph_free(g);
        return fail(GP_ERR_HIP, "capture stream: %s", hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    if ((st = graph_record(g, &graph)) != GP_OK) {
        graph_free(g);
        return st;
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g->exec = nullptr;
        graph_free(g);
        return fail(GP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = g;
    return GP_OK;
}

extern "C" gp_status gp_graph_launch(gp_graph* g, void* stream) {
    if (!g || !g->exec) return fail(GP_ERR_INVALID_ARG, "graph is NULL");
    HIP_TRY(hipSetDevice(g->ctx->device));
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return GP_OK;
}

extern "C" gp_status gp_graph_rebind(gp_graph* g, const gp_frame* frames, int32_t nframes) {
    if (!g || !g->exec) return fail(GP_ERR_INVALID_ARG, "graph is NULL");
    gp_status st;
    if ((st = check_frames(frames, nframes)) != GP_OK) return st;
    if (nframes != (int32_t)g->frames.size())
        return fail(GP_ERR_INVALID_ARG, "rebind needs %zu frames (got %d)", g->frames.size(), nframes);
    for (int f = 0; f < nframes; ++f) {
        const gp_frame &a = frames[f], &b = g->frames[f];
        if (a.width != b.width || a.height != b.height || a.pitch != b.pitch || a.dtype != b.dtype)
            return fail(GP_ERR_INVALID_ARG, "frame %d: rebind needs the same size, pitch and dtype", f);
    }
    const std::vector<gp_frame> keep = g->frames;
    g->frames.assign(frames, frames + nframes);
    hipGraph_t graph = nullptr;
    if ((st = graph_record(g, &graph)) != GP_OK) {
        g->frames = keep;
        return st;
    }
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res = hipGraphExecUpdateSuccess;
    hipError_t e = hipGraphExecUpdate(g->exec, graph, &bad, &res);
    if (e != hipSuccess || res != hipGraphExecUpdateSuccess) {
        // the topology differs (it should not for equal shapes): instantiate anew
        (void)hipGetLastError();
        hipGraphExec_t fresh = nullptr;
        e = hipGraphInstantiate(&fresh, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            g->frames = keep;
            return fail(GP_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        (void)hipGraphExecDestroy(g->exec);
        g->exec = fresh;
    }
    (void)hipGraphDestroy(graph);
    return GP_OK;
}

extern "C" void gp_graph_destroy(gp_graph* g) {
    if (g) graph_free(g);
}

extern "C" gp_status gp_profile_enable(gp_ctx* ctx, int on) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    ctx->profiling = on != 0;
    return GP_OK;
}

static gp_status drain(gp_ctx* ctx) {
    std::lock_guard<std::mutex> g(ctx->mu);
    for (auto& p : ctx->pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        auto& t = ctx->totals[p.name];
        t.first += ms;
        t.second += 1;
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    return GP_OK;
}

extern "C" gp_status gp_profile_read(gp_ctx* ctx, const char* name, double* total_ms, int64_t* count) {
    if (!ctx || !name) return fail(GP_ERR_INVALID_ARG, "NULL argument");
    gp_status st = drain(ctx);
    if (st != GP_OK) return st;
    auto it = ctx->totals.find(name);
    if (total_ms) *total_ms = it == ctx->totals.end() ? 0.0 : it->second.first;
    if (count) *count = it == ctx->totals.end() ? 0 : it->second.second;
    return GP_OK;
}

extern "C" gp_status gp_profile_reset(gp_ctx* ctx) {
    if (!ctx) return fail(GP_ERR_INVALID_ARG, "context is NULL");
    gp_status st = drain(ctx);
    ctx->totals.clear();
    return st;
}
