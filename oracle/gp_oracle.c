/*
 * gp_oracle.c -- plain, slow, FP64 CPU oracle of the per-frame photometry hot
 * path: mesh background, matched-filter detection with connected-component
 * labelling and per-object moments, circular exact-overlap aperture photometry.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the HIP
 * library and its Python binding) never links, imports or calls it, and the two
 * share no code, headers, tables or helpers.
 *
 * What the paper fixes (GPU Implementation section, subsections on image
 * preprocessing/background, source detection and adaptive aperture photometry):
 *   - the background is a local estimate and the stage yields a per-pixel noise
 *     map used as the significance normaliser; frames get reflected borders;
 *   - detection is a matched filter: the background-subtracted frame is
 *     correlated with a unit-flux kernel and compared against the noise map
 *     times a threshold in sigma; positions come from first moments;
 *   - photometry sums fluxes in circular apertures, accumulated in float64;
 *     the growth curve of every source over the integer radii from
 *     ceil(0.75 FWHM) to ceil(5 FWHM) is one top-hat correlation per radius
 *     read at the sources, with the variance map through the same kernel;
 *   - the local background can instead be a convolution of the frame with
 *     reflected borders, invalid pixels first filled from their valid
 *     neighbours, with a noise map from the sky, read and dark variances;
 *   - the paper's own detection keeps the local maxima of the matched-filter
 *     significance above the threshold, with first-moment centroids; with a
 *     spatially varying PSF (reference plus eigenmodes with coefficient maps)
 *     the filter is K + 1 correlations weighted by the maps.
 * The paper's own background/detection/photometry use FFTs and peak finding;
 * the mesh statistics follow the published SExtractor method the paper cites
 * (Bertin & Arnouts 1996: kappa-sigma clipping about the median until
 * convergence, clipped mean if sigma changed by less than 20%, otherwise
 * mode = 2.5 median - 1.5 mean), and labelling/moments/exact overlap follow the
 * plain definitions.  Every reading the paper leaves open is a parameter here.
 *
 * Conventions: pixel (x, y) with x the column, y the row, value at the pixel
 * centre, pixel area [x-1/2, x+1/2] x [y-1/2, y+1/2], row-major storage with a
 * pitch (in elements).  All arithmetic is IEEE double; no SIMD, no threads.
 *
 * Parity pins (closed forms, brute force, library routines) live in the test
 * suite; nothing here is checked against itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

/* object flags (bit values are part of the catalogue contract) */
#define OR_FLAG_SATURATED 1u
#define OR_FLAG_EDGE 2u
#define OR_FLAG_NONPOS 4u
#define OR_FLAG_APER_TRUNC 8u

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* median of an ascending array; an even count takes the mean of the two
 * middle order statistics */
static double median_sorted(const double* s, long n) {
    if (n % 2) return s[n / 2];
    return 0.5 * (s[n / 2 - 1] + s[n / 2]);
}

/* mean and population (ddof 0) standard deviation, two passes; exactly zero
 * when every value is the same */
static void mean_std(const double* s, long n, double* mean, double* sd) {
    double acc = 0.0;
    int all_equal = 1;
    for (long i = 0; i < n; ++i) {
        acc += s[i];
        if (s[i] != s[0]) all_equal = 0;
    }
    double m = acc / (double)n;
    if (all_equal) {
        *mean = s[0];
        *sd = 0.0;
        return;
    }
    double v = 0.0;
    for (long i = 0; i < n; ++i) v += (s[i] - m) * (s[i] - m);
    *mean = m;
    *sd = sqrt(v / (double)n);
}

/* ------------------------------------------------------------------------ */
/* Mesh statistics (SExtractor method as cited by the paper)                 */
/* ------------------------------------------------------------------------ */
/*
 * Statistics of one mesh given its pixel values.
 *   sigma0 = std(all values)
 *   if sigma0 == 0: back = value, rms = 0
 *   repeat (at most max_iter times): med = median(S), sigma = std(S),
 *        S <- {v in S : |v - med| <= clip*sigma}; stop when nothing is removed
 *   final med, mean, sigma of S
 *   back = mean if |sigma - sigma0| < crowd*sigma0 else a*med - b*mean
 *   rms = sigma
 * out[0..7] = back, rms, med, mean, sigma0, iterations, clip margin, mode margin.
 * The margins report how close the clip and estimator decisions came to their
 * boundaries (relative to clip*sigma and sigma0): where they are below the
 * rounding of a single-precision evaluation both outcomes are legitimate.
 *
 * Branch policy for those decisions (the reading that a decision within the
 * rounding band may go either way, so the other branch is an equally valid
 * result): a clip decision whose relative margin is below eps_clip is taken
 * as computed (policy field 0), forced to keep the value (1) or forced to
 * drop it (2); the low side (values below the median) is bits 0-1 of
 * `policy`, the high side bits 2-3.  Bit 4 flips the estimator decision when
 * its relative margin is below eps_mode.  policy = 0 is the plain method.
 */
static int mesh_one_policy(const double* vals, long n, double clip, double crowd, double mode_a,
                           double mode_b, int max_iter, double eps_clip, double eps_mode, int policy,
                           double* out) {
    if (n <= 0 || !vals || !out) return OR_EINVAL;
    double* S = (double*)malloc(sizeof(double) * (size_t)n);
    double* T = (double*)malloc(sizeof(double) * (size_t)n);
    if (!S || !T) {
        free(S);
        free(T);
        return OR_ENOMEM;
    }
    memcpy(S, vals, sizeof(double) * (size_t)n);
    /* S is kept in ascending order: dropping elements preserves the order, so
     * one sort serves every median below */
    qsort(S, (size_t)n, sizeof(double), cmp_double);
    double mean0, sig0;
    mean_std(S, n, &mean0, &sig0);
    double margin_clip = INFINITY, margin_mode = INFINITY;
    if (sig0 == 0.0) {
        out[0] = S[0];
        out[1] = 0.0;
        out[2] = S[0];
        out[3] = S[0];
        out[4] = 0.0;
        out[5] = 0.0;
        out[6] = margin_clip;
        out[7] = margin_mode;
        free(S);
        free(T);
        return OR_OK;
    }
    const int pol_lo = policy & 3, pol_hi = (policy >> 2) & 3;
    long ns = n;
    int iters = 0;
    for (int it = 0; it < max_iter; ++it) {
        double med = median_sorted(S, ns);
        double mean, sig;
        mean_std(S, ns, &mean, &sig);
        double lim = clip * sig;
        long nk = 0;
        for (long i = 0; i < ns; ++i) {
            double d = fabs(S[i] - med);
            int keep = d <= lim;
            if (lim > 0.0) {
                double mg = fabs(d - lim) / lim;
                if (mg < margin_clip) margin_clip = mg;
                int pol = (S[i] < med) ? pol_lo : pol_hi;
                if (mg < eps_clip && pol != 0) keep = (pol == 1);
            }
            if (keep) T[nk++] = S[i];
        }
        iters++;
        if (nk == ns || nk == 0) break;
        double* tmp = S;
        S = T;
        T = tmp;
        ns = nk;
    }
    double med = median_sorted(S, ns);
    double mean, sig;
    mean_std(S, ns, &mean, &sig);
    double dsig = fabs(sig - sig0);
    margin_mode = fabs(dsig - crowd * sig0) / sig0;
    int use_mean = dsig < crowd * sig0;
    if ((policy & 16) && margin_mode < eps_mode) use_mean = !use_mean;
    double back = use_mean ? mean : (mode_a * med - mode_b * mean);
    out[0] = back;
    out[1] = sig;
    out[2] = med;
    out[3] = mean;
    out[4] = sig0;
    out[5] = (double)iters;
    out[6] = margin_clip;
    out[7] = margin_mode;
    free(S);
    free(T);
    return OR_OK;
}

int or_mesh_one(const double* vals, long n, double clip, double crowd, double mode_a,
                double mode_b, int max_iter, double* out) {
    return mesh_one_policy(vals, n, clip, crowd, mode_a, mode_b, max_iter, 0.0, 0.0, 0, out);
}

/* The same statistics with the decisions inside the rounding band taken by
 * `policy` (see above). */
int or_mesh_one_policy(const double* vals, long n, double clip, double crowd, double mode_a,
                       double mode_b, int max_iter, double eps_clip, double eps_mode, int policy,
                       double* out) {
    if (policy < 0 || policy > 31 || (policy & 3) == 3 || ((policy >> 2) & 3) == 3) return OR_EINVAL;
    return mesh_one_policy(vals, n, clip, crowd, mode_a, mode_b, max_iter, eps_clip, eps_mode, policy, out);
}

/* number of meshes along one axis */
static long mesh_count(long n, int m) { return (n + m - 1) / m; }

/*
 * Per-mesh statistics over the whole frame.  Mesh (i, j) covers columns
 * [i*mw, min((i+1)*mw, W)) and rows [j*mh, min((j+1)*mh, H)); the last
 * row/column of meshes may be narrower.  stats has 8 doubles per mesh
 * (see or_mesh_one), row-major over (j, i).
 */
int or_mesh_stats(const double* img, long W, long H, long pitch, int mw, int mh, double clip,
                  double crowd, double mode_a, double mode_b, int max_iter, double* stats) {
    if (!img || !stats || W <= 0 || H <= 0 || pitch < W || mw <= 0 || mh <= 0) return OR_EINVAL;
    long nx = mesh_count(W, mw), ny = mesh_count(H, mh);
    double* buf = (double*)malloc(sizeof(double) * (size_t)mw * (size_t)mh);
    if (!buf) return OR_ENOMEM;
    for (long j = 0; j < ny; ++j) {
        for (long i = 0; i < nx; ++i) {
            long x0 = i * mw, x1 = (x0 + mw < W) ? x0 + mw : W;
            long y0 = j * mh, y1 = (y0 + mh < H) ? y0 + mh : H;
            long n = 0;
            for (long y = y0; y < y1; ++y)
                for (long x = x0; x < x1; ++x) buf[n++] = img[y * pitch + x];
            int rc = or_mesh_one(buf, n, clip, crowd, mode_a, mode_b, max_iter,
                                 stats + 8 * (j * nx + i));
            if (rc) {
                free(buf);
                return rc;
            }
        }
    }
    free(buf);
    return OR_OK;
}

/*
 * f x f median filter over an ny x nx grid (f odd; 1 = copy).  The window is
 * truncated at the grid edges; an even number of neighbours takes the mean of
 * the two middle values.
 */
int or_median_filter(const double* in, long nx, long ny, int f, double* out) {
    if (!in || !out || nx <= 0 || ny <= 0 || f <= 0 || (f % 2) == 0) return OR_EINVAL;
    int h = f / 2;
    double* win = (double*)malloc(sizeof(double) * (size_t)f * (size_t)f);
    if (!win) return OR_ENOMEM;
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
            long n = 0;
            for (long b = j - h; b <= j + h; ++b)
                for (long a = i - h; a <= i + h; ++a)
                    if (a >= 0 && a < nx && b >= 0 && b < ny) win[n++] = in[b * nx + a];
            qsort(win, (size_t)n, sizeof(double), cmp_double);
            out[j * nx + i] = median_sorted(win, n);
        }
    free(win);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Natural cubic spline interpolation of the mesh grid                       */
/* ------------------------------------------------------------------------ */
/* knot of mesh k along an axis of n pixels with mesh size m: the geometric
 * centre of the mesh's actual pixel span */
static double knot_pos(long k, long n, int m) {
    long a = k * m, b = (a + m < n) ? a + m : n;
    return 0.5 * (double)(a + b - 1);
}

/* Natural spline second derivatives (zero at both end knots) through
 * (t[k], f[k]), k = 0..n-1, by the tridiagonal (Thomas) elimination. */
static void spline_second(long n, const double* t, const double* f, double* m, double* work) {
    for (long k = 0; k < n; ++k) m[k] = 0.0;
    if (n < 3) return;
    double* c = work;          /* modified super-diagonal */
    double* d = work + n;      /* modified right-hand side */
    /* unknowns m[1..n-2] */
    for (long k = 1; k <= n - 2; ++k) {
        double h0 = t[k] - t[k - 1], h1 = t[k + 1] - t[k];
        double a = h0, b = 2.0 * (h0 + h1), cc = h1;
        double r = 6.0 * ((f[k + 1] - f[k]) / h1 - (f[k] - f[k - 1]) / h0);
        if (k == 1) {
            c[k] = cc / b;
            d[k] = r / b;
        } else {
            double den = b - a * c[k - 1];
            c[k] = cc / den;
            d[k] = (r - a * d[k - 1]) / den;
        }
    }
    m[n - 2] = d[n - 2];
    for (long k = n - 3; k >= 1; --k) m[k] = d[k] - c[k] * m[k + 1];
}

/* Evaluate the spline at x: one knot -> constant, two -> the line through
 * them, otherwise the natural cubic; beyond the end knots the curve continues
 * along the tangent at the end knot. */
static double spline_eval(long n, const double* t, const double* f, const double* m, double x) {
    if (n == 1) return f[0];
    if (x <= t[0]) {
        double h = t[1] - t[0];
        double slope = (f[1] - f[0]) / h - h * (2.0 * m[0] + m[1]) / 6.0;
        return f[0] + slope * (x - t[0]);
    }
    if (x >= t[n - 1]) {
        double h = t[n - 1] - t[n - 2];
        double slope = (f[n - 1] - f[n - 2]) / h + h * (m[n - 2] + 2.0 * m[n - 1]) / 6.0;
        return f[n - 1] + slope * (x - t[n - 1]);
    }
    long k = 0;
    while (k + 1 < n - 1 && x >= t[k + 1]) ++k; /* t[k] <= x < t[k+1] */
    double h = t[k + 1] - t[k];
    double A = (t[k + 1] - x) / h, B = (x - t[k]) / h;
    /* f[k] + B (f[k+1] - f[k]) is the chord (A f[k] + B f[k+1] with A = 1 - B),
     * written so that equal knot values give that value exactly */
    return f[k] + B * (f[k + 1] - f[k]) +
           ((A * A * A - A) * m[k] + (B * B * B - B) * m[k + 1]) * h * h / 6.0;
}

/*
 * Interpolated background at arbitrary points: first along y through the knots
 * of every mesh column (giving V_i(y)), then along x through (cx_i, V_i(y)).
 * grid is ny x nx (row-major), the mesh sizes give the knot positions.
 */
int or_grid_eval(const double* grid, long nx, long ny, long W, long H, int mw, int mh,
                 const double* xs, const double* ys, long npts, double* out) {
    if (!grid || !xs || !ys || !out || nx <= 0 || ny <= 0) return OR_EINVAL;
    double* cx = (double*)malloc(sizeof(double) * (size_t)nx);
    double* cy = (double*)malloc(sizeof(double) * (size_t)ny);
    double* my = (double*)malloc(sizeof(double) * (size_t)(nx * ny));
    double* col = (double*)malloc(sizeof(double) * (size_t)ny);
    double* mcol = (double*)malloc(sizeof(double) * (size_t)ny);
    double* V = (double*)malloc(sizeof(double) * (size_t)nx);
    double* mx = (double*)malloc(sizeof(double) * (size_t)nx);
    long wn = (nx > ny ? nx : ny);
    double* work = (double*)malloc(sizeof(double) * (size_t)(2 * wn));
    if (!cx || !cy || !my || !col || !mcol || !V || !mx || !work) {
        free(cx); free(cy); free(my); free(col); free(mcol); free(V); free(mx); free(work);
        return OR_ENOMEM;
    }
    for (long i = 0; i < nx; ++i) cx[i] = knot_pos(i, W, mw);
    for (long j = 0; j < ny; ++j) cy[j] = knot_pos(j, H, mh);
    /* second derivatives of every column spline, stored [i][j] */
    for (long i = 0; i < nx; ++i) {
        for (long j = 0; j < ny; ++j) col[j] = grid[j * nx + i];
        spline_second(ny, cy, col, mcol, work);
        for (long j = 0; j < ny; ++j) my[i * ny + j] = mcol[j];
    }
    double last_y = NAN;
    for (long p = 0; p < npts; ++p) {
        double y = ys[p];
        if (!(y == last_y)) {
            for (long i = 0; i < nx; ++i) {
                for (long j = 0; j < ny; ++j) col[j] = grid[j * nx + i];
                V[i] = spline_eval(ny, cy, col, my + i * ny, y);
            }
            spline_second(nx, cx, V, mx, work);
            last_y = y;
        }
        out[p] = spline_eval(nx, cx, V, mx, xs[p]);
    }
    free(cx); free(cy); free(my); free(col); free(mcol); free(V); free(mx); free(work);
    return OR_OK;
}

/* Full-resolution interpolated map for rows [y0, y1), every column. */
int or_grid_map(const double* grid, long nx, long ny, long W, long H, int mw, int mh, long y0,
                long y1, double* out) {
    if (y0 < 0 || y1 < y0) return OR_EINVAL;
    long n = (y1 - y0) * W;
    double* xs = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* ys = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!xs || !ys) {
        free(xs);
        free(ys);
        return OR_ENOMEM;
    }
    long p = 0;
    for (long y = y0; y < y1; ++y)
        for (long x = 0; x < W; ++x) {
            xs[p] = (double)x;
            ys[p] = (double)y;
            ++p;
        }
    int rc = or_grid_eval(grid, nx, ny, W, H, mw, mh, xs, ys, n, out);
    free(xs);
    free(ys);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Matched filter                                                            */
/* ------------------------------------------------------------------------ */
/* half-sample symmetric reflection into [0, n): -1 -> 0, -2 -> 1, n -> n-1,
 * repeated for offsets larger than n */
static long reflect(long i, long n) {
    long p = 2 * n;
    long r = i % p;
    if (r < 0) r += p;
    return (r < n) ? r : (p - 1 - r);
}

/*
 * F(x, y) = sum_a sum_b Khat[a][b] M(x + b - hx, y + a - hy)  (a correlation:
 * the kernel is not flipped), Khat = K / sum(K) when the sum is non-zero, with
 * reflected borders.  K is kh x kw, both odd.
 */
int or_filter(const double* M, long W, long H, const double* K, int kw, int kh, double* F) {
    if (!M || !K || !F || W <= 0 || H <= 0 || kw <= 0 || kh <= 0 || !(kw % 2) || !(kh % 2))
        return OR_EINVAL;
    double sum = 0.0;
    for (int a = 0; a < kh * kw; ++a) sum += K[a];
    double norm = (sum != 0.0) ? sum : 1.0;
    int hx = kw / 2, hy = kh / 2;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int a = 0; a < kh; ++a) {
                long yy = reflect(y + a - hy, H);
                for (int b = 0; b < kw; ++b) {
                    long xx = reflect(x + b - hx, W);
                    acc += (K[a * kw + b] / norm) * M[yy * W + xx];
                }
            }
            F[y * W + x] = acc;
        }
    return OR_OK;
}

/*
 * Spatially varying matched filter (Source Detection subsection): with the
 * PSF written as a fixed reference P0 plus K fixed eigenmodes e_k whose
 * amplitudes c_k vary over the frame,
 *   S(x, y) = (M corr P0)(x, y) + sum_k c_k(x, y) (M corr e_k)(x, y),
 * each term a correlation with reflected borders as in or_filter, the
 * kernels used as given (no normalisation).  kernels: (K + 1) kernels of
 * kh x kw, P0 first.  coef: K maps, map k at coef + k * plane, the value for
 * pixel (x, y) at [(y / bin) * pitch + x / bin] (bin = 1: full-frame maps).
 */
int or_filter_varying(const double* M, long W, long H, const double* kernels, int K, int kw, int kh,
                      const double* coef, long pitch, long plane, int bin, double* S) {
    if (!M || !kernels || !S || W <= 0 || H <= 0 || K < 0 || kw <= 0 || kh <= 0 || !(kw % 2) || !(kh % 2) ||
        bin < 1 || (K > 0 && !coef))
        return OR_EINVAL;
    const int hx = kw / 2, hy = kh / 2;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double s = 0.0;
            for (int k = 0; k <= K; ++k) {
                const double* Kk = kernels + (long)k * kh * kw;
                double acc = 0.0;
                for (int a = 0; a < kh; ++a) {
                    const long yy = reflect(y + a - hy, H);
                    for (int b = 0; b < kw; ++b) acc += Kk[a * kw + b] * M[yy * W + reflect(x + b - hx, W)];
                }
                const double c = (k == 0) ? 1.0 : coef[(long)(k - 1) * plane + (y / bin) * pitch + x / bin];
                s += c * acc;
            }
            S[y * W + x] = s;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Threshold and connected components                                       */
/* ------------------------------------------------------------------------ */
/*
 * mask = F > thresh * R (strict).  Components by breadth-first flood fill,
 * 8- or 4-connected, discovered in raster order, so the n-th component found
 * is the one whose first raster pixel is n-th smallest.  Components with
 * fewer than minarea pixels are dropped.  seg receives, per pixel:
 *   k >= 1  label of a kept component (1..nobj in raster order of first pixel)
 *   -1      above threshold but in a dropped component
 *    0      below threshold
 */
int or_threshold_label(const double* F, const double* R, long W, long H, double thresh,
                       int minarea, int conn, int32_t* seg, long* nobj) {
    if (!F || !R || !seg || !nobj || W <= 0 || H <= 0 || (conn != 4 && conn != 8))
        return OR_EINVAL;
    long N = W * H;
    long* queue = (long*)malloc(sizeof(long) * (size_t)N);
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    if (!queue || !tmp) {
        free(queue);
        free(tmp);
        return OR_ENOMEM;
    }
    for (long p = 0; p < N; ++p) tmp[p] = (F[p] > thresh * R[p]) ? -1 : 0; /* -1: unvisited */
    long ncomp = 0;
    /* component sizes, grown as components are found */
    long cap = 1024;
    long* sizes = (long*)malloc(sizeof(long) * (size_t)cap);
    if (!sizes) {
        free(queue);
        free(tmp);
        return OR_ENOMEM;
    }
    for (long p = 0; p < N; ++p) {
        if (tmp[p] != -1) continue;
        ++ncomp;
        if (ncomp >= cap) {
            cap *= 2;
            long* ns = (long*)realloc(sizes, sizeof(long) * (size_t)cap);
            if (!ns) {
                free(queue); free(tmp); free(sizes);
                return OR_ENOMEM;
            }
            sizes = ns;
        }
        long head = 0, tail = 0, cnt = 0;
        queue[tail++] = p;
        tmp[p] = (int32_t)ncomp;
        while (head < tail) {
            long q = queue[head++];
            ++cnt;
            long qx = q % W, qy = q / W;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (!dx && !dy) continue;
                    if (conn == 4 && dx && dy) continue;
                    long nx = qx + dx, ny = qy + dy;
                    if (nx < 0 || nx >= W || ny < 0 || ny >= H) continue;
                    long r = ny * W + nx;
                    if (tmp[r] == -1) {
                        tmp[r] = (int32_t)ncomp;
                        queue[tail++] = r;
                    }
                }
        }
        sizes[ncomp] = cnt;
    }
    /* keep components of at least minarea pixels, renumbered in order */
    int32_t* newlab = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncomp + 1));
    if (!newlab) {
        free(queue); free(tmp); free(sizes);
        return OR_ENOMEM;
    }
    long k = 0;
    newlab[0] = 0;
    for (long c = 1; c <= ncomp; ++c) newlab[c] = (sizes[c] >= minarea) ? (int32_t)(++k) : -1;
    for (long p = 0; p < N; ++p) seg[p] = tmp[p] ? newlab[tmp[p]] : 0;
    *nobj = k;
    free(queue); free(tmp); free(sizes); free(newlab);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-object measurements                                                  */
/* ------------------------------------------------------------------------ */
/*
 * Over the pixels of each labelled object, on the background-subtracted image M:
 *   npix, bbox, first raster pixel pmin, flux = sum M, peak = max M,
 *   SATURATED if any raw I >= sat, EDGE if the bbox touches the frame border,
 *   first moments about pmin: x = xr + Sx/S, y = yr + Sy/S,
 *   second central moments x2 = Sxx/S - (Sx/S)^2, y2, xy likewise,
 *   weights M when S = sum M > 0, otherwise unit weights and NONPOS.
 * Arrays are indexed by label - 1.
 */
int or_measure(const double* I, const double* M, const int32_t* seg, long W, long H, long nobj,
               double sat, int32_t* npix, int32_t* xmin, int32_t* xmax, int32_t* ymin,
               int32_t* ymax, int64_t* pmin, double* flux, double* xc, double* yc, double* x2,
               double* y2, double* xy, double* peak, uint32_t* flags) {
    if (!I || !M || !seg || nobj < 0) return OR_EINVAL;
    for (long k = 0; k < nobj; ++k) {
        npix[k] = 0;
        pmin[k] = -1;
        flux[k] = 0.0;
        peak[k] = -INFINITY;
        flags[k] = 0u;
    }
    /* pass 1: counts, bbox, first pixel, flux, peak, saturation */
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            int32_t l = seg[y * W + x];
            if (l <= 0) continue;
            long k = l - 1;
            double m = M[y * W + x];
            if (npix[k] == 0) {
                pmin[k] = y * W + x;
                xmin[k] = xmax[k] = (int32_t)x;
                ymin[k] = ymax[k] = (int32_t)y;
            }
            npix[k]++;
            if (x < xmin[k]) xmin[k] = (int32_t)x;
            if (x > xmax[k]) xmax[k] = (int32_t)x;
            if (y < ymin[k]) ymin[k] = (int32_t)y;
            if (y > ymax[k]) ymax[k] = (int32_t)y;
            flux[k] += m;
            if (m > peak[k]) peak[k] = m;
            if (I[y * W + x] >= sat) flags[k] |= OR_FLAG_SATURATED;
        }
    /* pass 2: moments about the first pixel */
    double* acc = (double*)calloc((size_t)(nobj > 0 ? nobj : 1) * 12, sizeof(double));
    if (!acc) return OR_ENOMEM;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            int32_t l = seg[y * W + x];
            if (l <= 0) continue;
            long k = l - 1;
            double m = M[y * W + x];
            double dx = (double)(x - pmin[k] % W), dy = (double)(y - pmin[k] / W);
            double* a = acc + 12 * k;
            a[0] += m;
            a[1] += m * dx;
            a[2] += m * dy;
            a[3] += m * dx * dx;
            a[4] += m * dy * dy;
            a[5] += m * dx * dy;
            a[6] += 1.0;
            a[7] += dx;
            a[8] += dy;
            a[9] += dx * dx;
            a[10] += dy * dy;
            a[11] += dx * dy;
        }
    for (long k = 0; k < nobj; ++k) {
        double* a = acc + 12 * k;
        double xr = (double)(pmin[k] % W), yr = (double)(pmin[k] / W);
        const double* w = a;
        if (!(a[0] > 0.0)) {
            flags[k] |= OR_FLAG_NONPOS;
            w = a + 6;
        }
        double S = w[0];
        double mx = w[1] / S, my = w[2] / S;
        xc[k] = xr + mx;
        yc[k] = yr + my;
        x2[k] = w[3] / S - mx * mx;
        y2[k] = w[4] / S - my * my;
        xy[k] = w[5] / S - mx * my;
        if (xmin[k] == 0 || ymin[k] == 0 || xmax[k] == W - 1 || ymax[k] == H - 1)
            flags[k] |= OR_FLAG_EDGE;
    }
    free(acc);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact disk / pixel overlap and aperture sums                             */
/* ------------------------------------------------------------------------ */
/* integral of sqrt(r^2 - t^2) dt from 0 to u, 0 <= u <= r */
static double Phi(double u, double r) {
    double s = r * r - u * u;
    if (s < 0.0) s = 0.0;
    double q = u / r;
    if (q > 1.0) q = 1.0;
    if (q < -1.0) q = -1.0;
    return 0.5 * (u * sqrt(s) + r * r * asin(q));
}

/* signed area of disk(0, r) intersected with the rectangle between (0,0) and
 * (x, y): odd in each argument */
static double Gcorner(double x, double y, double r) {
    double sx = (x < 0.0) ? -1.0 : 1.0, sy = (y < 0.0) ? -1.0 : 1.0;
    double xa = fabs(x), ya = fabs(y);
    if (xa > r) xa = r;
    if (ya > r) ya = r;
    double a;
    if (xa * xa + ya * ya <= r * r) {
        a = xa * ya;
    } else {
        double u0 = sqrt(r * r - ya * ya);
        a = u0 * ya + Phi(xa, r) - Phi(u0, r);
    }
    return sx * sy * a;
}

/* exact area of disk(c, r) intersected with [x0, x1] x [y0, y1].  A rectangle
 * whose nearest point lies on or outside the circle shares no area with the
 * disk, and one whose farthest corner lies on or inside it lies wholly in the
 * disk: those two cases are returned as exactly 0 and the rectangle's area
 * (the corner-integral sum below would leave a rounding residue of a few
 * units of r^2 * 2^-53 instead). */
double or_overlap(double x0, double x1, double y0, double y1, double cx, double cy, double r) {
    if (!(r > 0.0)) return 0.0;
    const double rect = (x1 - x0) * (y1 - y0);
    x0 -= cx; x1 -= cx; y0 -= cy; y1 -= cy;
    double nx = (x0 > 0.0) ? x0 : ((x1 < 0.0) ? -x1 : 0.0);
    double ny = (y0 > 0.0) ? y0 : ((y1 < 0.0) ? -y1 : 0.0);
    if (nx * nx + ny * ny >= r * r) return 0.0;
    double fx = (fabs(x0) > fabs(x1)) ? fabs(x0) : fabs(x1);
    double fy = (fabs(y0) > fabs(y1)) ? fabs(y0) : fabs(y1);
    if (fx * fx + fy * fy <= r * r) return rect;
    return Gcorner(x1, y1, r) - Gcorner(x0, y1, r) - Gcorner(x1, y0, r) + Gcorner(x0, y0, r);
}

/*
 * Circular apertures centred on (xc, yc) for every radius r_k plus an annulus
 * [r_in, r_out]:
 *   w_p(r)  = area(disk(c, r) intersected with pixel p)   (exact)
 *   area_k  = sum_p w_p(r_k),  raw_k = sum_p w_p(r_k) M_p
 *   bkg     = sum_p (w_p(r_out) - w_p(r_in)) M_p / sum_p (w_p(r_out) - w_p(r_in))
 *   flux_k  = raw_k - bkg * area_k
 *   err_k   = sqrt(sum_p w_p(r_k)^2 (R_p^2 + max(M_p, 0) / gain))  (gain <= 0:
 *             no Poisson term)
 * Pixels outside the frame contribute nothing.  An object whose largest circle
 * (aperture or annulus) crosses the frame boundary [-1/2, W-1/2] x [-1/2, H-1/2]
 * gets APER_TRUNC.  Outputs are [n][nr].
 */
int or_aperture(const double* M, const double* R, long W, long H, const double* xc,
                const double* yc, long n, const double* radii, int nr, double r_in,
                double r_out, double gain, int want_err, double* flux, double* area,
                double* bkg, double* fluxerr, uint32_t* flags) {
    if (!M || !xc || !yc || !radii || nr <= 0 || nr > 64) return OR_EINVAL;
    if (want_err && !R) return OR_EINVAL;
    double rmax = r_out;
    for (int k = 0; k < nr; ++k)
        if (radii[k] > rmax) rmax = radii[k];
    double A[64], S[64], V[64];
    for (long o = 0; o < n; ++o) {
        double cx = xc[o], cy = yc[o];
        for (int k = 0; k < nr; ++k) A[k] = S[k] = V[k] = 0.0;
        double Aa = 0.0, Sa = 0.0;
        uint32_t fl = 0u;
        long xa = (long)floor(cx - rmax - 0.5) - 1, xb = (long)ceil(cx + rmax + 0.5) + 1;
        long ya = (long)floor(cy - rmax - 0.5) - 1, yb = (long)ceil(cy + rmax + 0.5) + 1;
        for (long py = ya; py <= yb; ++py)
            for (long px = xa; px <= xb; ++px) {
                double x0 = px - 0.5, x1 = px + 0.5, y0 = py - 0.5, y1 = py + 0.5;
                double wo = or_overlap(x0, x1, y0, y1, cx, cy, r_out);
                double wi = or_overlap(x0, x1, y0, y1, cx, cy, r_in);
                int inside = (px >= 0 && px < W && py >= 0 && py < H);
                double wk[64];
                double wmax = wo;
                for (int k = 0; k < nr; ++k) {
                    wk[k] = or_overlap(x0, x1, y0, y1, cx, cy, radii[k]);
                    if (wk[k] > wmax) wmax = wk[k];
                }
                (void)wmax;
                if (!inside) continue;
                double m = M[py * W + px];
                for (int k = 0; k < nr; ++k) {
                    A[k] += wk[k];
                    S[k] += wk[k] * m;
                    if (want_err) {
                        double var = R[py * W + px] * R[py * W + px];
                        if (gain > 0.0 && m > 0.0) var += m / gain;
                        V[k] += wk[k] * wk[k] * var;
                    }
                }
                Aa += wo - wi;
                Sa += (wo - wi) * m;
            }
        if (cx - rmax < -0.5 || cx + rmax > (double)W - 0.5 || cy - rmax < -0.5 || cy + rmax > (double)H - 0.5)
            fl |= OR_FLAG_APER_TRUNC;
        double b = (Aa > 0.0) ? Sa / Aa : 0.0;
        bkg[o] = b;
        for (int k = 0; k < nr; ++k) {
            area[o * nr + k] = A[k];
            flux[o * nr + k] = S[k] - b * A[k];
            if (want_err && fluxerr) fluxerr[o * nr + k] = sqrt(V[k]);
        }
        if (flags) flags[o] = fl;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Peak detection (the paper's own detection: local maxima of the matched-   */
/* filter significance)                                                      */
/* ------------------------------------------------------------------------ */
/* significance of pixel p: the filtered frame divided by the noise map (a
 * zero noise map leaves F itself) */
static double nu_of(const double* F, const double* R, long p) { return (R[p] > 0.0) ? F[p] / R[p] : F[p]; }

/*
 * Sources are the local maxima of the significance nu = F / R above the
 * threshold (Source Detection subsection: matched filter divided by the noise
 * map, local maxima above a significance threshold found with a maximum
 * filter, sub-pixel positions from a first-moment centroid; the FWHM sets the
 * separation and centroid windows).  Readings:
 *   - candidate: F > thresh * R (the strict threshold of the mask);
 *   - local maximum: nu(p) >= nu(q) for every q of the (2 sep + 1)^2 window
 *     around p inside the frame, strictly > for q earlier in raster order
 *     (one peak per plateau, its first pixel);
 *   - centroid over the (2 cwin + 1)^2 window around the peak inside the
 *     frame with weights max(M, 0): x = px + sum w dx / sum w, and the second
 *     moments about it; with no positive weight the peak pixel itself and
 *     NONPOS;
 *   - flux = sum of M over that window; npix = its pixel count; bbox = the
 *     window; EDGE when the window is cut by the frame border; SATURATED when
 *     a raw pixel of the window reaches sat.
 * Peaks come in raster order of the peak pixel; at most cap are stored, *n
 * receives how many there are.
 */
int or_peaks(const double* I, const double* M, const double* F, const double* R, long W, long H,
             double thresh, int sep, int cwin, double sat, long cap, int32_t* npix, int32_t* xmin,
             int32_t* xmax, int32_t* ymin, int32_t* ymax, int64_t* pidx, double* flux, double* xc,
             double* yc, double* x2, double* y2, double* xy, double* nu, uint32_t* flags, long* n) {
    if (!I || !M || !F || !R || !n || W <= 0 || H <= 0 || sep < 0 || cwin < 0 || cap < 0) return OR_EINVAL;
    long k = 0;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            const long p = y * W + x;
            if (!(F[p] > thresh * R[p])) continue;
            const double v = nu_of(F, R, p);
            int is_max = 1;
            for (long qy = y - sep; qy <= y + sep && is_max; ++qy)
                for (long qx = x - sep; qx <= x + sep; ++qx) {
                    if (qx < 0 || qx >= W || qy < 0 || qy >= H || (qx == x && qy == y)) continue;
                    const long q = qy * W + qx;
                    const double vq = nu_of(F, R, q);
                    if (vq > v || (vq == v && q < p)) {
                        is_max = 0;
                        break;
                    }
                }
            if (!is_max) continue;
            if (k < cap) {
                double sw = 0.0, sx = 0.0, sy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0, fl = 0.0;
                long cnt = 0;
                uint32_t f = 0u;
                const long x0 = x - cwin < 0 ? 0 : x - cwin, x1 = x + cwin >= W ? W - 1 : x + cwin;
                const long y0 = y - cwin < 0 ? 0 : y - cwin, y1 = y + cwin >= H ? H - 1 : y + cwin;
                if (x0 != x - cwin || x1 != x + cwin || y0 != y - cwin || y1 != y + cwin) f |= OR_FLAG_EDGE;
                for (long qy = y0; qy <= y1; ++qy)
                    for (long qx = x0; qx <= x1; ++qx) {
                        const long q = qy * W + qx;
                        const double m = M[q];
                        const double w = m > 0.0 ? m : 0.0;
                        const double dx = (double)(qx - x), dy = (double)(qy - y);
                        sw += w;
                        sx += w * dx;
                        sy += w * dy;
                        sxx += w * dx * dx;
                        syy += w * dy * dy;
                        sxy += w * dx * dy;
                        fl += m;
                        ++cnt;
                        if (I[q] >= sat) f |= OR_FLAG_SATURATED;
                    }
                double mx = 0.0, my = 0.0, vx = 0.0, vy = 0.0, cxy = 0.0;
                if (sw > 0.0) {
                    mx = sx / sw;
                    my = sy / sw;
                    vx = sxx / sw - mx * mx;
                    vy = syy / sw - my * my;
                    cxy = sxy / sw - mx * my;
                } else {
                    f |= OR_FLAG_NONPOS;
                }
                npix[k] = (int32_t)cnt;
                xmin[k] = (int32_t)x0;
                xmax[k] = (int32_t)x1;
                ymin[k] = (int32_t)y0;
                ymax[k] = (int32_t)y1;
                pidx[k] = p;
                flux[k] = fl;
                xc[k] = (double)x + mx;
                yc[k] = (double)y + my;
                x2[k] = vx;
                y2[k] = vy;
                xy[k] = cxy;
                nu[k] = v;
                flags[k] = f;
            }
            ++k;
        }
    *n = k;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Growth curves on top-hat kernels (Adaptive Aperture Photometry subsection) */
/* ------------------------------------------------------------------------ */
/* The integer radii of the growth curve: every integer from ceil(0.75 fwhm)
 * to ceil(5 fwhm).  Stores at most cap of them; *n receives how many there
 * are. */
int or_growth_radii(double fwhm, int cap, int32_t* radii, int* n) {
    if (!(fwhm > 0.0) || !isfinite(fwhm) || !n || cap < 0) return OR_EINVAL;
    const double lo = ceil(0.75 * fwhm), hi = ceil(5.0 * fwhm);
    if (hi > 1.0e6) return OR_EINVAL;
    int k = 0;
    for (double r = lo; r <= hi; r += 1.0, ++k)
        if (k < cap && radii) radii[k] = (int32_t)r;
    *n = k;
    return OR_OK;
}

/* Top-hat kernel of integer radius r, (2r+1) x (2r+1) taps, row-major: the tap
 * at offset (dx, dy) is the exact area of the disk of radius r about the
 * centre of the kernel's middle pixel that falls inside pixel (dx, dy). */
int or_tophat_taps(int r, double* taps) {
    if (r < 0 || !taps) return OR_EINVAL;
    const long side = 2L * r + 1;
    for (long dy = -r; dy <= r; ++dy)
        for (long dx = -r; dx <= r; ++dx)
            taps[(dy + r) * side + (dx + r)] =
                or_overlap(dx - 0.5, dx + 0.5, dy - 0.5, dy + 0.5, 0.0, 0.0, (double)r);
    return OR_OK;
}

/*
 * Growth curves: for each radius r_k, the aperture sum of a source is the
 * correlation of M with the top-hat kernel of radius r_k read at the source,
 * and its variance the correlation of the variance map V with the same
 * kernel; all sums in double.  Readings:
 *   - a source is read at the pixel that holds its centroid,
 *     (floor(x + 1/2), floor(y + 1/2));
 *   - pixels outside the frame contribute nothing (the correlation of a
 *     zero-padded frame); area_k is the sum of the taps that fall inside;
 *   - V goes through the taps themselves (not their squares);
 *   - APER_TRUNC when a nonzero tap of the largest kernel falls outside the
 *     frame.  A source whose pixel lies so far out that no tap reaches the
 *     frame gets zero sums.
 * radii: nr integers >= 1, strictly increasing.  Outputs are [n][nr].
 */
int or_growth(const double* M, const double* V, long W, long H, const double* xs, const double* ys,
              long n, const int32_t* radii, int nr, double* sum, double* var, double* area,
              uint32_t* flags) {
    if (!M || !xs || !ys || !radii || nr <= 0 || W <= 0 || H <= 0) return OR_EINVAL;
    for (int k = 0; k < nr; ++k)
        if (radii[k] < 1 || (k > 0 && radii[k] <= radii[k - 1])) return OR_EINVAL;
    const int R = radii[nr - 1];
    const long side = 2L * R + 1;
    double* taps = (double*)malloc(sizeof(double) * (size_t)side * (size_t)side);
    if (!taps) return OR_EINVAL;
    for (long o = 0; o < n; ++o) {
        for (int k = 0; k < nr; ++k) {
            sum[o * nr + k] = 0.0;
            if (var) var[o * nr + k] = 0.0;
            area[o * nr + k] = 0.0;
        }
        if (flags) flags[o] = 0u;
    }
    for (int k = 0; k < nr; ++k) {
        const int r = radii[k];
        const long sk = 2L * r + 1;
        or_tophat_taps(r, taps);
        for (long o = 0; o < n; ++o) {
            const double fx = floor(xs[o] + 0.5), fy = floor(ys[o] + 0.5);
            if (!(fx >= -(double)R - 1.0 && fx <= (double)W + R && fy >= -(double)R - 1.0 && fy <= (double)H + R)) {
                if (flags) flags[o] = OR_FLAG_APER_TRUNC;
                continue;
            }
            const long cx = (long)fx, cy = (long)fy;
            double s = 0.0, v = 0.0, a = 0.0;
            for (long dy = -r; dy <= r; ++dy)
                for (long dx = -r; dx <= r; ++dx) {
                    const long px = cx + dx, py = cy + dy;
                    if (px < 0 || px >= W || py < 0 || py >= H) continue;
                    const double w = taps[(dy + r) * sk + (dx + r)];
                    s += w * M[py * W + px];
                    if (V) v += w * V[py * W + px];
                    a += w;
                }
            sum[o * nr + k] = s;
            if (var) var[o * nr + k] = v;
            area[o * nr + k] = a;
            if (k == nr - 1 && flags && (cx - r < 0 || cx + r >= W || cy - r < 0 || cy + r >= H))
                flags[o] = OR_FLAG_APER_TRUNC;
        }
    }
    free(taps);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Local background by convolution (Image Preprocessing and Background      */
/* Estimation subsection)                                                   */
/* ------------------------------------------------------------------------ */
/*
 * B = K corr I' with K = ky kx^T / (sum ky sum kx) (a separable smoothing
 * kernel, normalised to unit sum) and reflected borders as in or_filter,
 * where I' is the frame with its invalid pixels filled from their valid
 * neighbours: an invalid pixel p takes
 *   N(p) = sum_q K(q - p) v(q) I(q) / sum_q K(q - p) v(q),
 * the kernel-weighted mean of the valid pixels around it (v = 1 valid, 0
 * invalid; the same reflected borders).  A pixel is invalid when mask[p] != 0
 * (mask may be NULL) or I(p) >= sat.  An invalid pixel with no valid pixel
 * under the kernel is filled with 0 and counted in *unfilled.
 * Noise map, for a dark-subtracted frame in ADU with gain g (e-/ADU), read
 * noise rn (e-), dark current dark (e-/s) and exposure texp (s): the sky,
 * read and dark variances add in electrons,
 *   R^2 = (g max(B, 0) + rn^2 + dark texp) / g^2.
 * kx: lx taps, ky: ly taps, both odd.
 */
int or_background_conv(const double* I, long W, long H, const uint8_t* mask, double sat, const double* kx, int lx,
                       const double* ky, int ly, double gain, double rn, double dark, double texp, double* B,
                       double* R, long* unfilled) {
    if (!I || !kx || !ky || !B || W <= 0 || H <= 0 || lx <= 0 || ly <= 0 || !(lx % 2) || !(ly % 2) ||
        !(gain > 0.0))
        return OR_EINVAL;
    double sx = 0.0, sy = 0.0;
    for (int b = 0; b < lx; ++b) sx += kx[b];
    for (int a = 0; a < ly; ++a) sy += ky[a];
    if (sx == 0.0 || sy == 0.0) return OR_EINVAL;
    const int hx = lx / 2, hy = ly / 2;
    double* F = (double*)malloc(sizeof(double) * (size_t)W * (size_t)H);
    if (!F) return OR_EINVAL;
    long nun = 0;
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            const long p = y * W + x;
            const int valid = !(mask && mask[p]) && I[p] < sat;
            if (valid) {
                F[p] = I[p];
                continue;
            }
            double num = 0.0, den = 0.0;
            for (int a = 0; a < ly; ++a) {
                const long yy = reflect(y + a - hy, H);
                for (int b = 0; b < lx; ++b) {
                    const long q = yy * W + reflect(x + b - hx, W);
                    if ((mask && mask[q]) || !(I[q] < sat)) continue;
                    const double k = (ky[a] / sy) * (kx[b] / sx);
                    num += k * I[q];
                    den += k;
                }
            }
            if (den != 0.0) {
                F[p] = num / den;
            } else {
                F[p] = 0.0;
                ++nun;
            }
        }
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int a = 0; a < ly; ++a) {
                const long yy = reflect(y + a - hy, H);
                for (int b = 0; b < lx; ++b)
                    acc += (ky[a] / sy) * (kx[b] / sx) * F[yy * W + reflect(x + b - hx, W)];
            }
            B[y * W + x] = acc;
            if (R) {
                const double sky = acc > 0.0 ? acc : 0.0;
                R[y * W + x] = sqrt((gain * sky + rn * rn + dark * texp) / (gain * gain));
            }
        }
    free(F);
    if (unfilled) *unfilled = nun;
    return OR_OK;
}
