// k_args.h -- kernel argument blocks and launcher entry points shared by the
// kernel translation units and the host runtime.
#pragma once
#include "k_common.h"

namespace gpk {

// mesh centres per axis the spline kernels hold in LDS
constexpr int kSplineMaxKnots = 4096;
// frames per call (the aperture kernel keeps their object-count prefix in LDS)
constexpr int kMaxFramesPerCall = 1024;

struct BkgArgs {
    float clip, crowd, mode_a, mode_b;
    int32_t max_iter;
    int32_t fsize;
    int32_t skip_u16;   // the float kernel leaves uint16 meshes to the integer kernel
};

// matched-filter and detection arguments, stored in the workspace
struct DetArgs {
    int32_t kw, kh, separable, conn;
    float thresh, sat;
    int32_t minarea, want_seg;
    float kx[kMaxK], ky[kMaxK];       // normalised 1-D factors (rank-one kernels)
    float kd[kMaxK * kMaxK];          // normalised dense kernel
    double kxd[kMaxK], kyd[kMaxK];    // the same in FP64 (reference variant)
    double kdd[kMaxK * kMaxK];
};

// what the host hands to the argument-writing kernel (the dense kernel is
// normalised on the device)
struct DetArgsIn {
    int32_t kw, kh, separable, conn;
    float thresh, sat;
    int32_t minarea, want_seg;
    float kraw[kMaxK * kMaxK];
    float kx[kMaxK], ky[kMaxK];
    double kxd[kMaxK], kyd[kMaxK];
};

// circles sorted by radius: crole[j] = aperture index (< nr), kMaxRadii for
// r_in, kMaxRadii + 1 for r_out
struct ApArgs {
    int32_t nr, want_err, capacity, nframes;
    float radii[kMaxRadii];
    float r_in, r_out, gain, rmax;
    float crad[kMaxRadii + 2];
    int32_t crole[kMaxRadii + 2];
};

struct ApCat {
    const int32_t* n_obj;
    const double *x, *y;
    uint32_t* flags;
    double *flux, *area, *bkg, *fluxerr;
};

struct CatOut {
    int32_t capacity;
    int32_t *n_obj, *status;
    int32_t *npix, *xmin, *xmax, *ymin, *ymax;
    int64_t* pmin;
    double *flux, *x, *y, *x2, *y2, *xy;
    float* peak;
    uint32_t* flags;
};

// spatially varying matched filter: a reference kernel and up to kMaxModes
// eigenmodes (taps as given, [column][row][mode] with P0 as mode 0, modes
// padded to kMaxModes + 1) and, per frame,
// the coefficient maps (map k of frame f at pf[f].data + k * plane; pixel
// (x, y) reads [(y / bin) * pitch + x / bin])
constexpr int kMaxModes = 8;
constexpr int kPsfTaps = (kMaxModes + 1) * kMaxK * kMaxK;
struct PsfArgs {
    int32_t nmodes, bin, kw, kh;
    float taps[kPsfTaps];
    double tapsd[kPsfTaps];
};
struct PsfFrame {
    const float* data;
    int64_t pitch, plane;
};

// peak detection: separation and centroid half-widths (pixels); psf and pf
// set for the spatially varying filter, else null
struct PeakArgs {
    int32_t sep, cwin;
    const PsfArgs* psf;
    const PsfFrame* pf;
    int32_t mesh_w;   // mesh width of the call (sizes the row cubics of a region row)
};
constexpr int kMaxPeakWin = 7;

// growth curves: integer radii (strictly increasing, <= kMaxGrowthRadius),
// the window half-width R = largest radius, and the offsets of the full and
// cut lists of each radius in the tap table (computed on the host from the
// same exact classification the table kernel uses)
constexpr int kMaxGrowthRadii = 32;
constexpr int kMaxGrowthRadius = 32;
struct GrowArgs {
    int32_t nr, R, side, capacity, nframes, want_var, nixmax, nfull, ncut;
    int32_t div_magic;   // i / side == (i * div_magic) >> 20 for i < side^2
    int32_t radii[kMaxGrowthRadii];
    int32_t full_off[kMaxGrowthRadii + 1], cut_off[kMaxGrowthRadii + 1];
};
struct GrowTab {
    int32_t* full;   // (wy << 16) | wx of each full-list offset
    int32_t* cut;
    double* cutw;    // exact area of the cut pixel for that list's radius
};
struct GrowOut {
    const int32_t* n_obj;
    const double *x, *y;
    double *sum, *var, *area;
    uint32_t* flags;
};

// local background by convolution: separable taps and the noise-model constants
constexpr int kMaxConvTaps = 129;
// taps normalised to unit sum in FP64 on the host and zero-padded to a whole
// number of 8-tap blocks (the kernels' register blocking)
constexpr int kConvTapsPad = (kMaxConvTaps + 7) / 8 * 8;
struct CvArgs {
    int32_t lx, ly;
    float sat, gain, read_noise, dark, exptime;
    double nm_c0, nm_c1;   // R^2 = nm_c1 max(B, 0) + nm_c0 (FP32 maps): 1 / g and (rn^2 + dark t) / g^2
    double kx[kConvTapsPad], ky[kConvTapsPad];
};

// one: the descriptor of a one-frame call, passed with the launch (the kernel
// stores it in the table for the launches that follow), or null
void launch_mesh_stats(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, int max_area, BkgArgs a,
                       int cfg, hipStream_t s);
void launch_mesh_stats_u16(FrameDesc* desc, const FrameDesc* one, int nframes, int total_meshes, int max_area,
                           BkgArgs a, int cfg, hipStream_t s);
void launch_grid_filter(const FrameDesc* desc, int nframes, int total_meshes, int fsize, hipStream_t s);
void launch_spline(const FrameDesc* desc, int nframes, int max_nx, int max_ny, hipStream_t s);
bool filter_spline_fits(int max_nx, int max_ny, int fsize);
void launch_filter_spline(const FrameDesc* desc, int nframes, int max_nx, int max_ny, int fsize, hipStream_t s);
void launch_detect_tiles(const DetWork& wk, const DetArgs* args, bool f64, int rad, int mesh_w, hipStream_t s);
int detect_tiles_per_cu(bool f64, int rad, int mesh_w);
void launch_merge(const DetWork& wk, int conn, int minarea, int persist_blocks, hipStream_t s);
void launch_catalog(const DetWork& wk, const CatOut& cat, int minarea, int persist_blocks, int32_t* comp_status,
                    hipStream_t s);
void launch_seg(const DetWork& wk, int f, int64_t npx, hipStream_t s);
void launch_peaks(const DetWork& wk, const DetArgs* args, const CatOut& cat, int32_t* comp_status, bool f64, int sep,
                  int cwin, int kw, int kh, int persist_blocks, const PsfArgs* psf, const PsfFrame* pf,
                  int nmodes, int mesh_w, int xcd_cus, hipStream_t s);
// copy `bytes` (a multiple of 4) from host memory to device memory through
// kernel arguments (no copy engine, so the call can be captured)
void launch_write_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
size_t peak_lds_bytes(int sep, int cwin, int kw, int kh, bool f64, int mesh_w);
// one: the descriptor of a one-frame call, passed with the launch (the
// workspace table is then not read), or null
void launch_aperture(const FrameDesc* desc, const FrameDesc* one, const ApArgs& a, const ApCat& cat, int total_rows,
                     int blocks, int mesh_w, int max_nx, bool f64, hipStream_t s);
void launch_growth_table(const GrowArgs& a, const GrowTab& t, hipStream_t s);
hipError_t launch_growth(const FrameDesc* desc, const FrameDesc* one, const GrowArgs& a, const GrowTab& t,
                         const GrowOut& g, int blocks, int waves, bool f64, hipStream_t s);
size_t growth_lds_bytes(int nfull, int ncut, int side, int nixmax, int want_var, bool f64, int waves);
// One frame of a convolution-background call.  Every frame has its own
// slices of the working planes (hA / hG and G: element offset plane), of the
// per-row band flags (height x ceil(width / 64) bytes at flags) and of the
// per-tile fill-round flags (one byte per 64 x 64 tile at tiles).
struct CvFrame {
    const void* data;
    const uint8_t* mask;
    void* back;
    void* rms;
    int64_t pitch;
    int64_t plane, flags, tiles;
    int32_t W, H, dtype, pad;
};
constexpr int kCvChunk = 16;   // frame records written per set-up launch
constexpr int kCvSegPx = 2048; // outputs per horizontal workgroup (one row segment)
constexpr int kCvTilePx = 64;  // side of a vertical workgroup's tile and width of a flag band
struct CvChunk {
    int32_t first, count;
    CvFrame f[kCvChunk];
    int32_t hbase[kCvChunk], vbase[kCvChunk];   // first horizontal / vertical workgroup of each frame
};
// device memory of a call: the frame table, the workgroup bases, a flag per
// frame, the two planes, the band and tile flags
struct CvWork {
    CvFrame* tab;
    int32_t *hbase, *vbase, *fflag;
    void *hA, *G;
    uint8_t *flags, *tiles;
    int64_t* unfilled;
};
// chunks: the frame records in kCvChunk groups; htotal / vtotal: workgroups
// of the horizontal / vertical passes over all frames
hipError_t launch_conv(const CvChunk* chunks, int nchunks, int nframes, int htotal, int vtotal, const CvArgs& a,
                       const CvWork& w, bool f64, hipStream_t s);
void launch_bkg_map(const FrameDesc& d, double* bmap, double* rmap, bool f64, hipStream_t s);
void launch_write_desc(const DescChunk& c, FrameDesc* table, hipStream_t s);
void launch_det_setup(const DescChunk& c, FrameDesc* table, const DetArgsIn& in, DetArgs* out, uint32_t* counters,
                      hipStream_t s);

}  // namespace gpk
