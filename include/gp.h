/*
 * gp.h -- C ABI of the MI355X (gfx950) photometry hot path.
 *
 * These calls carry the method, in the order the paper's GPU Implementation
 * section applies its stages to a frame:
 *
 *   gp_background  mesh background: per-mesh kappa-sigma clipped mode and rms
 *                  (the SExtractor method the paper cites), a median filter over
 *                  the mesh grid and a natural bicubic spline that turns the grid
 *                  into the per-pixel background B and noise map R (the paper's
 *                  background subsection: a local background estimate plus a
 *                  per-pixel noise map used as the significance normaliser).
 *   gp_detect      matched-filter detection (source detection subsection): the
 *                  background-subtracted frame M = I - B is correlated with a
 *                  unit-sum kernel using reflected borders, pixels with F > t R
 *                  are grouped into 8- (or 4-) connected components, components
 *                  smaller than minarea are dropped, and the survivors are
 *                  measured (flux, peak, first-moment centroid, second moments).
 *   gp_aperture    circular aperture photometry (adaptive aperture photometry
 *                  subsection): exact pixel/disk overlap sums for each radius,
 *                  an annulus background, and the propagated noise.
 *   gp_peaks       the paper's own detection: local maxima of the significance
 *                  F / R above the threshold with first-moment centroids (in
 *                  place of gp_detect's connected components); gp_peaks_psf
 *                  the same with the spatially varying PSF's filter.
 *   gp_growth      growth curves: top-hat sums of M and of R^2 at every source
 *                  for the integer radii ceil(0.75 FWHM) .. ceil(5 FWHM).
 *   gp_background_conv  the paper's own background: a convolution with
 *                  reflected borders, invalid pixels filled from their valid
 *                  neighbours, and a sky/read/dark noise map (full-frame maps).
 *
 * All of them work on a batch of nframes >= 1 frames of any sizes at once; the
 * plain per-frame use is nframes = 1.
 *
 * Memory.  Every pointer inside gp_frame, gp_catalog, gp_phot and the
 * background and workspace buffers is caller-owned DEVICE memory on the
 * context's device; the library allocates nothing on these paths.  Host
 * pointers appear only in the parameter structs (filter kernel, radii), which
 * are read during the call and may be freed when it returns.
 *
 * Asynchrony.  The calls only enqueue kernels on the given stream (NULL = the
 * default stream) and can be captured into a HIP graph.  Argument errors are
 * returned synchronously.  Data-dependent conditions (more objects than the
 * catalogue holds, more components than the workspace holds) are written to
 * device status words that the caller reads after synchronising.
 *
 * Errors.  A non-GP_OK return leaves a message for gp_last_error() (per host
 * thread).  Nothing is enqueued when a call returns an error.
 *
 * Threads.  A context may be used from several host threads as long as each
 * (workspace, stream) pair is used by one thread at a time.
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gp_status {
    GP_OK = 0,
    GP_ERR_INVALID_ARG = 1,   /* bad argument (returned synchronously)             */
    GP_ERR_UNSUPPORTED = 2,   /* valid but outside what the kernels implement      */
    GP_ERR_WORKSPACE = 3,     /* workspace too small (sync) or component overflow  */
    GP_ERR_CAPACITY = 4,      /* more objects than catalogue rows (device status)  */
    GP_ERR_HIP = 5            /* a HIP runtime call failed                         */
} gp_status;

typedef enum gp_dtype { GP_U16 = 1, GP_F32 = 2 } gp_dtype;

/* Arithmetic of the per-pixel work.  GP_PREC_F32: FP32 per-pixel work with
 * compensated (two-sum) accumulation; FP64 only for the spline solve and the
 * final moment normalisation.  GP_PREC_F64: the same kernels in FP64 end to end
 * (a reference variant of the GPU path, several times slower). */
typedef enum gp_precision { GP_PREC_F32 = 0, GP_PREC_F64 = 1 } gp_precision;

/* One frame: row-major pixels, x = column in [0, width), y = row in
 * [0, height), element (x, y) at data[y * pitch + x] (pitch in elements,
 * >= width, pitch * height < 2^31, else GP_ERR_UNSUPPORTED).  Values must
 * be finite.  Every call takes 1 to 1024 frames (more: GP_ERR_UNSUPPORTED). */
typedef struct gp_frame {
    const void* data;      /* device pointer */
    int32_t width, height;
    int64_t pitch;
    int32_t dtype;         /* gp_dtype */
} gp_frame;

/* Background parameters.  Meshes are mesh_w x mesh_h pixels tiling the frame
 * from (0, 0); the last mesh column/row may be narrower.  Per mesh: sigma0 =
 * std of all pixels; repeat up to max_iter times {med = median, sigma = std,
 * keep pixels with |v - med| <= clip_sigma * sigma} until nothing is removed;
 * back = clipped mean if |sigma - sigma0| < crowd_tol * sigma0, otherwise
 * mode_a * median - mode_b * mean; rms = clipped sigma.  The grids are then
 * median filtered over filter_size x filter_size meshes (odd, 1 = off,
 * truncated at the grid edges) and interpolated by natural cubic splines
 * through the mesh centres, first along y then along x, continued linearly
 * past the outer mesh centres.
 * Limits: 16 <= mesh_w, mesh_h; mesh_w * mesh_h <= 16384; filter_size <= 7;
 * at most 4096 meshes along either axis of a frame (GP_ERR_UNSUPPORTED). */
#define GP_BKG_GRID_GIVEN 1u   /* skip the mesh statistics and the filter: the
                                  caller has written the back/rms grids */
typedef struct gp_bkg_params {
    int32_t mesh_w, mesh_h;
    int32_t filter_size;
    float clip_sigma;      /* 3    */
    float crowd_tol;       /* 0.2  */
    float mode_a, mode_b;  /* 2.5, 1.5 */
    int32_t max_iter;      /* 100  */
    uint32_t flags;        /* GP_BKG_* */
} gp_bkg_params;

/* Layout of one frame's block inside the background buffer (all offsets in
 * bytes from the buffer start, 256-byte aligned).  Grids are double
 * [ny][nx] row-major; coef holds the interpolation as bicubic pieces, double
 * [2][ny+1][nx+1][16] (B then R; piece (jy, ix) covers the rows between mesh
 * centres jy-1 and jy and the columns between centres ix-1 and ix, with the
 * outer pieces extending to the frame edges; coefficient [p*4+q] multiplies
 * (x - X_ix)^p (y - Y_jy)^q where X_ix is the centre max(ix-1, 0) and Y_jy
 * likewise). */
typedef struct gp_bkg_layout {
    int32_t nx, ny;
    int64_t back_raw, rms_raw;   /* per-mesh statistics before the filter */
    int64_t back, rms;           /* filtered grids (what the spline uses)  */
    int64_t coef;
    int64_t iters;               /* int32 [ny][nx]: clipping passes per mesh */
    int64_t bytes;               /* size of this frame's block */
} gp_bkg_layout;

/* Detection parameters.  kernel: HOST pointer to kh x kw floats, row-major,
 * both odd and <= 15; it is normalised to unit sum by the library (used as
 * given when its sum is zero) and applied as a correlation with half-sample
 * reflected borders.  A kernel whose every tap equals the product of its row
 * and column through the peak tap to within 4 float32 rounding units of the
 * tap (a rank-one kernel such as a circular Gaussian) is applied as two 1-D
 * passes; any other kernel is applied densely.  Pixels with F > thresh * R
 * form the mask. */
typedef struct gp_det_params {
    const float* kernel;
    int32_t kw, kh;
    float thresh;
    int32_t minarea;       /* >= 1 */
    int32_t connectivity;  /* 8 or 4 */
    float sat_level;       /* raw value flagged SATURATED (+inf: never) */
    int32_t precision;     /* gp_precision */
} gp_det_params;

/* Aperture parameters.  radii: HOST pointer to nr (1..8) positive radii in
 * pixels; the annulus is [r_in, r_out] with 0 <= r_in < r_out <= 64.
 * gain > 0 adds the Poisson term max(M, 0) / gain to the pixel variance. */
typedef struct gp_ap_params {
    const float* radii;
    int32_t nr;
    float r_in, r_out;
    float gain;
    int32_t want_err;
    int32_t precision;     /* gp_precision */
} gp_ap_params;

/* Object flags */
#define GP_FLAG_SATURATED 1u   /* a raw pixel of the object >= sat_level       */
#define GP_FLAG_EDGE 2u        /* the bounding box touches the frame border    */
#define GP_FLAG_NONPOS 4u      /* sum of M <= 0: moments use unit weights       */
#define GP_FLAG_APER_TRUNC 8u  /* an aperture or the annulus leaves the frame   */

/* Catalogue, structure of arrays.  Frame f's rows are [f*capacity,
 * (f+1)*capacity) of every column; row k holds label k+1.  Labels number the
 * kept components in raster order of their first pixel.  n_obj[f] is the
 * number of components found (it may exceed capacity: then status[f] =
 * GP_ERR_CAPACITY and the first `capacity` labels are stored).  Coordinates
 * are 0-based pixel centres; pmin = y * width + x of the first pixel. */
typedef struct gp_catalog {
    int32_t capacity;
    int32_t* n_obj;        /* [nframes] */
    int32_t* status;       /* [nframes] */
    int32_t *npix, *xmin, *xmax, *ymin, *ymax;
    int64_t* pmin;
    double *flux, *x, *y, *x2, *y2, *xy;
    float* peak;
    uint32_t* flags;
} gp_catalog;

/* Photometry, rows as in the catalogue: flux/area/fluxerr [row][nr],
 * bkg [row].  fluxerr may be NULL when want_err = 0. */
typedef struct gp_phot {
    double* flux;
    double* area;
    double* bkg;
    double* fluxerr;
} gp_phot;

typedef struct gp_ctx gp_ctx;

/* Create a context on HIP device `device`.  tune_cache: path of the JSON file
 * holding autotuned launch shapes (NULL: built-in defaults); read here when it
 * exists, rewritten whenever tuning adds a choice. */
gp_status gp_ctx_create(int device, const char* tune_cache, gp_ctx** out);

/* Autotuning switch (default off).  While on, a gp_background or gp_aperture
 * call whose shape class (mesh area; radii count, r_max, mesh width and
 * precision) has no choice yet times every candidate launch shape of its
 * kernel (mesh statistics: threads x pixels per thread; apertures: workgroups
 * per CU), each twice, synchronously on the call's stream, and keeps the
 * fastest for the context and the cache.  Outputs are those of an ordinary
 * call.  Skipped while the stream is being captured into a graph.  Not a hot
 * path entry: tune once, then switch it off. */
gp_status gp_ctx_set_tuning(gp_ctx* ctx, int32_t on);
void gp_ctx_destroy(gp_ctx* ctx);

/* Message of the last error on this host thread ("" if none). */
const char* gp_last_error(void);

/* Library version string. */
const char* gp_version(void);

/* Size and per-frame layout of the background buffer for a batch.  layouts may
 * be NULL; otherwise it receives nframes entries. */
gp_status gp_background_layout(const gp_frame* frames, int32_t nframes, const gp_bkg_params* bp,
                               gp_bkg_layout* layouts, size_t* bytes);

/* Per-pixel background B and noise map R of frame `index` of the batch, from
 * a background buffer filled by gp_background: device double [height][width]
 * maps (row pitch = width; either may be NULL).  Evaluated exactly as the
 * detection and aperture kernels evaluate them in the given precision
 * (gp_precision).  A diagnostic output (like a background check image); the
 * hot path never materialises these maps. */
gp_status gp_background_map(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                            const gp_bkg_params* bp, const void* bkg, int32_t index,
                            int32_t precision, double* back_map, double* rms_map, void* stream);

/* Local background by convolution (Image Preprocessing and Background
 * Estimation subsection), an alternative to the mesh background:
 *   B = K corr I'  with K = ky kx^T / (sum ky sum kx) and half-sample reflected
 *   borders, where I' is the frame with each invalid pixel (mask != 0, or a
 *   raw value >= sat_level) replaced by the kernel-weighted mean of the valid
 *   pixels around it, (K corr vI) / (K corr v) with v = 1 on valid pixels;
 *   R^2 = (gain max(B, 0) + read_noise^2 + dark_current exptime) / gain^2,
 *   the sky, read-out and dark-current variances of a dark-subtracted frame
 *   in ADU (gain in e-/ADU, read_noise in e-, dark_current in e-/s, exptime
 *   in s).
 * kx, ky: HOST pointers to lx, ly taps (odd, 1..129, non-zero sums).
 * masks: HOST array of nframes DEVICE pointers to uint8 masks with the
 * frame's pitch (NULL array or entries: no mask).  back, rms: HOST arrays of
 * nframes DEVICE pointers to width x height maps (row-major, pitch = width) of
 * float (GP_PREC_F32) or double (GP_PREC_F64).  unfilled: DEVICE int64
 * [nframes], the invalid pixels with no valid pixel under the kernel (filled
 * with 0).  Sums accumulate in FP64; intermediates are stored in the working
 * precision.  Workspace: gp_background_conv_ws bytes, which holds two
 * working-precision planes of every frame (8 bytes per pixel of the batch in
 * FP32, 16 in FP64) plus small per-frame tables: the four passes each run
 * once over all the frames. */
typedef struct gp_conv_params {
    const float* kx;
    int32_t lx;
    const float* ky;
    int32_t ly;
    float sat_level;
    float gain, read_noise, dark_current, exptime;
    int32_t precision;     /* gp_precision */
} gp_conv_params;
gp_status gp_background_conv_ws(const gp_frame* frames, int32_t nframes, const gp_conv_params* cp,
                                size_t* bytes);
gp_status gp_background_conv(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                             const uint8_t* const* masks, const gp_conv_params* cp,
                             void* const* back, void* const* rms, int64_t* unfilled, void* ws,
                             size_t ws_bytes, void* stream);

/* Workspace bytes for running gp_background, gp_detect and gp_aperture on this
 * batch with catalogues of cat_capacity rows per frame and room for
 * comp_capacity connected-component pieces in total (0: a default of
 * max(65536, pixels / 64)).  One workspace serves all three calls. */
gp_status gp_workspace_size(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                            const gp_bkg_params* bp, const gp_det_params* dp,
                            const gp_ap_params* ap, int32_t cat_capacity, int64_t comp_capacity,
                            size_t* bytes);

/* Mesh statistics, grid filter and spline pieces into `bkg` (device buffer of
 * gp_background_layout bytes).  With GP_BKG_GRID_GIVEN only the spline pieces
 * are built from the back/rms grids already in the buffer. */
gp_status gp_background(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                        const gp_bkg_params* bp, void* bkg, void* ws, size_t ws_bytes,
                        void* stream);

/* Detection into the catalogue.  seg: NULL, or a HOST array of nframes
 * pointers, each NULL or a device int32 [height][width] map (row pitch =
 * width) that receives per pixel the label (>= 1), -1 for pixels above
 * threshold in a dropped component, 0 below threshold.  comp_status (device int32[2], may be
 * NULL) receives {GP_OK or GP_ERR_WORKSPACE, pieces needed}.  A batch holds at
 * most 2^31 pixels, each frame counted as ceil(width * height / 1024) * 1024
 * (more: GP_ERR_UNSUPPORTED). */
gp_status gp_detect(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                    const gp_bkg_params* bp, const void* bkg, const gp_det_params* dp,
                    gp_catalog* cat, int32_t* const* seg, int32_t* comp_status, void* ws,
                    size_t ws_bytes, void* stream);

/* gp_detect for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same detection, with the workspace replaced by a static device array of
 * GP_DETECT_NOALLOC_MAX_BYTES that the library holds on every device it runs
 * on until the process ends (its address is looked up when a context is
 * created on the device).  The caller still passes frames, the background
 * buffer (from gp_background) and the catalogue.  The component-piece
 * capacity is whatever the array holds after the batch's fixed sections;
 * overflow is reported through comp_status as with gp_detect.  A batch whose
 * fixed sections alone do not fit returns GP_ERR_UNSUPPORTED (use gp_detect
 * with a workspace).  Every call on a device shares that device's array, and
 * each call writes every part of it that it later reads (nothing needs
 * clearing between calls); two calls that overlap on one device (other
 * streams, other host threads, other contexts) race on the array and their
 * results are undefined.  No allocation, event or stream is created. */
#define GP_DETECT_NOALLOC_MAX_BYTES ((size_t)128 << 20)
gp_status gp_detect_noalloc(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                            const gp_bkg_params* bp, const void* bkg, const gp_det_params* dp,
                            gp_catalog* cat, int32_t* const* seg, int32_t* comp_status, void* stream);

/* Peak detection, the paper's own detection (source detection subsection):
 * the frame minus the background is correlated with the unit-sum kernel and
 * divided by the noise map, nu = F / R (F itself where R = 0); sources are
 * the pixels with F > thresh * R whose nu is a maximum over the
 * (2 sep + 1)^2 window around them inside the frame (ties go to the earlier
 * pixel in raster order, so a plateau gives one peak), refined by a
 * first-moment centroid over the (2 cwin + 1)^2 window inside the frame with
 * weights max(M, 0).  The paper sets both windows from the PSF's FWHM.
 * Uses the kernel, thresh, sat_level and precision of dp (minarea and
 * connectivity are checked but unused).  Catalogue rows, in raster order of
 * the peak pixel: pmin = its index, peak = nu there, x, y, x2, y2, xy = the
 * centroid and second moments, flux = sum of M over the centroid window,
 * npix and the bounding box = that window, flags EDGE (window cut by the
 * border), SATURATED (a raw pixel of the window >= sat_level), NONPOS (no
 * positive M in the window: the peak pixel itself).  n_obj, status and
 * comp_status (peaks recorded) as for gp_detect; gp_aperture runs on the
 * result like on a gp_detect catalogue.  sep and cwin in [0, 7]. */
typedef struct gp_peak_params {
    int32_t sep, cwin;
} gp_peak_params;
gp_status gp_peaks(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                   const gp_bkg_params* bp, const void* bkg, const gp_det_params* dp,
                   const gp_peak_params* pp, gp_catalog* cat, int32_t* comp_status, void* ws,
                   size_t ws_bytes, void* stream);

/* The paper's detection with its spatially varying PSF (Source Detection
 * subsection): the PSF is a reference kernel P0 plus K eigenmodes e_k whose
 * amplitudes c_k vary over the frame, and the matched filter is
 *   S(x, y) = (M corr P0)(x, y) + sum_k c_k(x, y) (M corr e_k)(x, y),
 * K + 1 correlations with half-sample reflected borders, the kernels used as
 * given (no normalisation), the coefficients taken at the output pixel.
 * Peaks, centroids and the catalogue then follow gp_peaks with S in place of
 * F.  kernels: HOST pointer to (nmodes + 1) kernels of kh x kw floats
 * (P0 first, row-major; odd sides <= 15); nmodes in [0, 8]; maps: HOST array
 * of nframes entries, frame f's map k at maps[f].data + k * plane (DEVICE
 * floats), the value for pixel (x, y) at [(y / bin) * pitch + x / bin]
 * (bin = 1: full-frame maps; pitch >= ceil(width / bin)); maps may be NULL
 * when nmodes = 0.  dp: thresh, sat_level and precision are used, its
 * kernel is not.  Each output pixel costs (nmodes + 1) kw kh multiply-adds. */
typedef struct gp_coef_maps {
    const float* data;
    int64_t pitch;         /* elements per map row          */
    int64_t plane;         /* elements between two maps     */
} gp_coef_maps;
typedef struct gp_psf_model {
    const float* kernels;
    int32_t kw, kh;
    int32_t nmodes;
    int32_t bin;
    const gp_coef_maps* maps;
} gp_psf_model;
gp_status gp_peaks_psf(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                       const gp_bkg_params* bp, const void* bkg, const gp_det_params* dp,
                       const gp_peak_params* pp, const gp_psf_model* psf, gp_catalog* cat,
                       int32_t* comp_status, void* ws, size_t ws_bytes, void* stream);

/* Aperture photometry of every catalogued object; also ORs GP_FLAG_APER_TRUNC
 * into cat->flags. */
gp_status gp_aperture(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                      const gp_bkg_params* bp, const void* bkg, const gp_catalog* cat,
                      const gp_ap_params* ap, gp_phot* out, void* ws, size_t ws_bytes,
                      void* stream);

/* Growth curves on top-hat kernels (Adaptive Aperture Photometry subsection:
 * circular apertures of integer radii from ceil(0.75 FWHM) to ceil(5 FWHM),
 * each radius one correlation of the frame with a top-hat kernel, the noise
 * variance propagated through the same kernel, sums in float64).
 *
 * gp_growth_radii: the radii of that rule for a given FWHM (pixels); stores at
 * most cap of them in radii (host memory), *n = how many there are.
 *
 * gp_growth: for every catalogued row (x, y from gp_detect, gp_peaks or the
 * caller) and every radius r_k,
 *   sum[row][k]  = sum over pixels p of T_k(p - c) M(p)
 *   var[row][k]  = sum over pixels p of T_k(p - c) R(p)^2
 *   area[row][k] = sum over pixels p inside the frame of T_k(p - c)
 * where c = (floor(x + 1/2), floor(y + 1/2)) is the pixel holding the
 * centroid, M = I - B and R are the background and noise maps of the
 * background buffer, and T_k(dx, dy) is the exact area of the disk of radius
 * r_k about the centre of pixel (0, 0) inside pixel (dx, dy) (so the interior
 * area is pi r_k^2).  Pixels off the frame contribute nothing.  flags[row] =
 * GP_FLAG_APER_TRUNC when a nonzero tap of the largest kernel falls off the
 * frame (or the position is not a number), else 0; a pixel so far out that
 * no tap reaches the frame gets zero sums.  The catalogue is only read.
 * radii: HOST pointer to nr (1..32) strictly increasing integers in [1, 32].
 * Outputs: device, rows as in the catalogue, [row][nr] doubles; var and flags
 * may be NULL.  Result bits do not depend on the batch or on scheduling.
 * The workspace must hold gp_workspace_size's fixed part plus the tap table
 * (a gp_workspace_size workspace for the same batch always does). */
typedef struct gp_growth_params {
    const int32_t* radii;
    int32_t nr;
    int32_t precision;     /* gp_precision: working precision of M and R */
} gp_growth_params;
typedef struct gp_growth_out {
    double* sum;
    double* var;
    double* area;
    uint32_t* flags;
} gp_growth_out;
gp_status gp_growth_radii(double fwhm, int32_t cap, int32_t* radii, int32_t* n);
gp_status gp_growth(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                    const gp_bkg_params* bp, const void* bkg, const gp_catalog* cat,
                    const gp_growth_params* gp, gp_growth_out* out, void* ws,
                    size_t ws_bytes, void* stream);

/* Captured batch: gp_background -> gp_detect -> gp_aperture over one batch
 * (the arguments of the three calls, one workspace for all of them) recorded
 * once into a HIP graph on a private stream and instantiated; every launch
 * replays the whole sequence with one graph launch on the given stream.  The
 * parameter structs and their host arrays are copied at creation; every
 * device pointer must stay valid while the graph lives.  Creation returns the
 * errors the three calls would (nothing is enqueued then).  Launches of one
 * graph must not overlap (they share its buffers). */
typedef struct gp_graph gp_graph;
gp_status gp_graph_create(gp_ctx* ctx, const gp_frame* frames, int32_t nframes,
                          const gp_bkg_params* bp, void* bkg, const gp_det_params* dp,
                          gp_catalog* cat, int32_t* const* seg, int32_t* comp_status,
                          const gp_ap_params* ap, gp_phot* phot, void* ws, size_t ws_bytes,
                          gp_graph** out);
gp_status gp_graph_launch(gp_graph* g, void* stream);
/* Point the graph at other frames of the same sizes, pitches and dtypes (a
 * new batch of the same shape class, as a server gets it): the sequence is
 * recorded again and the instantiated graph updated in place. */
gp_status gp_graph_rebind(gp_graph* g, const gp_frame* frames, int32_t nframes);
void gp_graph_destroy(gp_graph* g);

/* Per-kernel timing with HIP events recorded on the launch stream.  When
 * enabled, every kernel launch is bracketed by events; gp_profile_read
 * synchronises and returns the summed milliseconds and launch count for the
 * kernel named `name` since the last reset. */
gp_status gp_profile_enable(gp_ctx* ctx, int on);
gp_status gp_profile_read(gp_ctx* ctx, const char* name, double* total_ms, int64_t* count);
gp_status gp_profile_reset(gp_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* GP_H */
