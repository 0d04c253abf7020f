"""Plain FP64 CPU oracle of the photometry hot path (TEST INFRASTRUCTURE ONLY).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and ``paper_2609_32375_amd``) never imports it and shares no code with
it.  The arithmetic lives in ``gp_oracle.c`` (IEEE double, one thread); this
module only marshals numpy arrays and chains the steps in the order the paper's
GPU Implementation section describes: background -> noise map -> matched filter
-> threshold -> objects -> circular apertures.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "libgporacle.so")

FLAG_SATURATED = 1
FLAG_EDGE = 2
FLAG_NONPOS = 4
FLAG_APER_TRUNC = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no SIMD intrinsics, no OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        up = C.POINTER(C.c_uint32)
        L.or_mesh_one.argtypes = [dp, C.c_long, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.or_mesh_one_policy.argtypes = [dp, C.c_long, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                         C.c_double, C.c_double, C.c_int, dp]
        L.or_mesh_stats.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int, C.c_double,
                                    C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.or_median_filter.argtypes = [dp, C.c_long, C.c_long, C.c_int, dp]
        L.or_grid_eval.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int, dp, dp,
                                   C.c_long, dp]
        L.or_grid_map.argtypes = [dp, C.c_long, C.c_long, C.c_long, C.c_long, C.c_int, C.c_int, C.c_long,
                                  C.c_long, dp]
        L.or_filter.argtypes = [dp, C.c_long, C.c_long, dp, C.c_int, C.c_int, dp]
        L.or_threshold_label.argtypes = [dp, dp, C.c_long, C.c_long, C.c_double, C.c_int, C.c_int, ip,
                                         C.POINTER(C.c_long)]
        L.or_measure.argtypes = [dp, dp, ip, C.c_long, C.c_long, C.c_long, C.c_double, ip, ip, ip, ip, ip,
                                 lp, dp, dp, dp, dp, dp, dp, dp, up]
        L.or_peaks.argtypes = [dp, dp, dp, dp, C.c_long, C.c_long, C.c_double, C.c_int, C.c_int, C.c_double,
                               C.c_long, ip, ip, ip, ip, ip, lp, dp, dp, dp, dp, dp, dp, dp, up, C.POINTER(C.c_long)]
        L.or_overlap.argtypes = [C.c_double] * 7
        L.or_overlap.restype = C.c_double
        L.or_aperture.argtypes = [dp, dp, C.c_long, C.c_long, dp, dp, C.c_long, dp, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_int, dp, dp, dp, dp, up]
        L.or_filter_varying.argtypes = [dp, C.c_long, C.c_long, dp, C.c_int, C.c_int, C.c_int, dp, C.c_long,
                                        C.c_long, C.c_int, dp]
        L.or_background_conv.argtypes = [dp, C.c_long, C.c_long, C.POINTER(C.c_uint8), C.c_double, dp, C.c_int, dp,
                                         C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp,
                                         C.POINTER(C.c_long)]
        L.or_growth_radii.argtypes = [C.c_double, C.c_int, ip, C.POINTER(C.c_int)]
        L.or_tophat_taps.argtypes = [C.c_int, dp]
        L.or_growth.argtypes = [dp, dp, C.c_long, C.c_long, dp, dp, C.c_long, ip, C.c_int, dp, dp, dp, up]
        for f in ("or_background_conv", "or_filter_varying", "or_growth_radii", "or_tophat_taps", "or_growth", "or_mesh_one", "or_mesh_one_policy", "or_mesh_stats", "or_median_filter", "or_grid_eval", "or_grid_map",
                  "or_filter", "or_threshold_label", "or_measure", "or_aperture", "or_peaks"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ----------------------------------------------------------------------------
# Background: mesh statistics, mesh filter, spline map
# ----------------------------------------------------------------------------
MESH_FIELDS = ("back", "rms", "med", "mean", "sigma0", "iters", "margin_clip", "margin_mode")


def mesh_one(values, clip=3.0, crowd=0.2, mode_a=2.5, mode_b=1.5, max_iter=100):
    v = _f64(np.ravel(values))
    out = np.zeros(8)
    _check(lib().or_mesh_one(_p(v), v.size, clip, crowd, mode_a, mode_b, max_iter, _p(out)), "mesh_one")
    return dict(zip(MESH_FIELDS, out))


# Branch policies for decisions inside the rounding band (the reading that such
# a decision may go either way): low-side and high-side clip decisions taken as
# computed (0), kept (1) or dropped (2); bit 4 flips the estimator decision.
MESH_POLICIES = tuple(lo | (hi << 2) | fl for fl in (0, 16) for hi in (0, 1, 2) for lo in (0, 1, 2))


def mesh_one_policy(values, policy, eps_clip, eps_mode, clip=3.0, crowd=0.2, mode_a=2.5, mode_b=1.5,
                    max_iter=100):
    """Mesh statistics with the decisions whose relative margins fall below
    eps_clip / eps_mode taken by `policy` (see MESH_POLICIES)."""
    v = _f64(np.ravel(values))
    out = np.zeros(8)
    _check(lib().or_mesh_one_policy(_p(v), v.size, clip, crowd, mode_a, mode_b, max_iter, eps_clip, eps_mode,
                                    int(policy), _p(out)), "mesh_one_policy")
    return dict(zip(MESH_FIELDS, out))


def mesh_variants(values, eps_clip, eps_mode, clip=3.0, crowd=0.2, mode_a=2.5, mode_b=1.5, max_iter=100):
    """Every distinct result of the mesh statistics over the branch policies:
    the plain result first, then the results with the ambiguous decisions
    taken the other way."""
    out, seen = [], set()
    for pol in MESH_POLICIES:
        st = mesh_one_policy(values, pol, eps_clip, eps_mode, clip, crowd, mode_a, mode_b, max_iter)
        key = (st["back"], st["rms"], st["iters"])
        if key not in seen:
            seen.add(key)
            out.append(st)
    return out


def mesh_stats(img, mesh_w, mesh_h, clip=3.0, crowd=0.2, mode_a=2.5, mode_b=1.5, max_iter=100):
    """Per-mesh statistics; returns a dict of (ny, nx) arrays."""
    a = _f64(img)
    H, W = a.shape
    nx, ny = -(-W // mesh_w), -(-H // mesh_h)
    st = np.zeros((ny, nx, 8))
    _check(lib().or_mesh_stats(_p(a), W, H, W, mesh_w, mesh_h, clip, crowd, mode_a, mode_b, max_iter,
                               _p(st)), "mesh_stats")
    return {k: st[:, :, i].copy() for i, k in enumerate(MESH_FIELDS)}


def median_filter(grid, f):
    g = _f64(grid)
    ny, nx = g.shape
    out = np.zeros_like(g)
    _check(lib().or_median_filter(_p(g), nx, ny, f, _p(out)), "median_filter")
    return out


def grid_map(grid, W, H, mesh_w, mesh_h, y0=0, y1=None):
    g = _f64(grid)
    ny, nx = g.shape
    y1 = H if y1 is None else y1
    out = np.zeros((y1 - y0, W))
    _check(lib().or_grid_map(_p(g), nx, ny, W, H, mesh_w, mesh_h, y0, y1, _p(out)), "grid_map")
    return out


def grid_eval(grid, W, H, mesh_w, mesh_h, xs, ys):
    g = _f64(grid)
    ny, nx = g.shape
    xs = _f64(xs)
    ys = _f64(ys)
    out = np.zeros(xs.size)
    _check(lib().or_grid_eval(_p(g), nx, ny, W, H, mesh_w, mesh_h, _p(xs), _p(ys), xs.size, _p(out)),
           "grid_eval")
    return out


@dataclass
class Background:
    stats: dict          # raw per-mesh statistics (ny, nx)
    back: np.ndarray     # filtered background grid
    rms: np.ndarray      # filtered rms grid
    B: np.ndarray        # interpolated background map (H, W) or None
    R: np.ndarray        # interpolated rms map (H, W) or None


def background(img, p, maps=True):
    st = mesh_stats(img, p.mesh_w, p.mesh_h, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b, p.max_iter)
    back = median_filter(st["back"], p.mesh_filter)
    rms = median_filter(st["rms"], p.mesh_filter)
    H, W = np.shape(img)
    B = grid_map(back, W, H, p.mesh_w, p.mesh_h) if maps else None
    R = grid_map(rms, W, H, p.mesh_w, p.mesh_h) if maps else None
    return Background(st, back, rms, B, R)


# ----------------------------------------------------------------------------
# Detection
# ----------------------------------------------------------------------------
def filter_image(M, K):
    Mm = _f64(M)
    H, W = Mm.shape
    Kk = _f64(K)
    kh, kw = Kk.shape
    F = np.zeros_like(Mm)
    _check(lib().or_filter(_p(Mm), W, H, _p(Kk), kw, kh, _p(F)), "filter")
    return F


def background_conv(I, kx, ky, mask=None, sat=np.inf, gain=1.0, rn=0.0, dark=0.0, texp=0.0):
    """Local background by convolution with reflected borders, invalid pixels
    (mask != 0 or I >= sat) filled from their valid neighbours, and the noise
    map of a dark-subtracted frame.  Returns (B, R, unfilled)."""
    Ii = _f64(I)
    H, W = Ii.shape
    kx, ky = _f64(kx), _f64(ky)
    B = np.zeros_like(Ii)
    R = np.zeros_like(Ii)
    mp = C.POINTER(C.c_uint8)()
    if mask is not None:
        m8 = np.ascontiguousarray(mask, dtype=np.uint8)
        mp = _p(m8, C.c_uint8)
    n = C.c_long(0)
    _check(lib().or_background_conv(_p(Ii), W, H, mp, float(sat), _p(kx), kx.size, _p(ky), ky.size, float(gain),
                                    float(rn), float(dark), float(texp), _p(B), _p(R), C.byref(n)),
           "background_conv")
    return B, R, n.value


def filter_varying(M, kernels, coef=None, bin=1):
    """S = M corr P0 + sum_k c_k (M corr e_k) with reflected borders; kernels
    (K+1, kh, kw) with P0 first, coef (K, ny, nx) maps of bin x bin pixels."""
    Mm = _f64(M)
    H, W = Mm.shape
    ks = _f64(kernels)
    K = ks.shape[0] - 1
    kh, kw = ks.shape[1], ks.shape[2]
    S = np.zeros_like(Mm)
    if K > 0:
        c = _f64(coef)
        assert c.shape[0] == K
        cp, pitch, plane = _p(c), c.shape[2], c.shape[1] * c.shape[2]
    else:
        cp, pitch, plane = C.POINTER(C.c_double)(), 0, 0
    _check(lib().or_filter_varying(_p(Mm), W, H, _p(ks), K, kw, kh, cp, pitch, plane, int(bin), _p(S)),
           "filter_varying")
    return S


def threshold_label(F, R, thresh, minarea, conn):
    Ff, Rr = _f64(F), _f64(R)
    H, W = Ff.shape
    seg = np.zeros((H, W), np.int32)
    n = C.c_long(0)
    _check(lib().or_threshold_label(_p(Ff), _p(Rr), W, H, thresh, minarea, conn, _p(seg, C.c_int32),
                                    C.byref(n)), "threshold_label")
    return seg, int(n.value)


def label_mask(mask, conn=8, minarea=1):
    """Components of a boolean mask (thresholding a 0/1 map against zero)."""
    m = np.asarray(mask, dtype=np.float64)
    return threshold_label(m, np.zeros_like(m), 0.0, minarea, conn)


CAT_FIELDS = ("npix", "xmin", "xmax", "ymin", "ymax", "pmin", "flux", "x", "y", "x2", "y2", "xy",
              "peak", "flags")


def measure(I, M, seg, nobj, sat=np.inf):
    Ii, Mm = _f64(I), _f64(M)
    H, W = Mm.shape
    s = np.ascontiguousarray(seg, dtype=np.int32)
    n = max(nobj, 1)
    ints = {k: np.zeros(n, np.int32) for k in ("npix", "xmin", "xmax", "ymin", "ymax")}
    pmin = np.zeros(n, np.int64)
    dbl = {k: np.zeros(n) for k in ("flux", "x", "y", "x2", "y2", "xy", "peak")}
    flags = np.zeros(n, np.uint32)
    _check(lib().or_measure(_p(Ii), _p(Mm), _p(s, C.c_int32), W, H, nobj, sat,
                            *[_p(ints[k], C.c_int32) for k in ("npix", "xmin", "xmax", "ymin", "ymax")],
                            _p(pmin, C.c_int64), *[_p(dbl[k]) for k in ("flux", "x", "y", "x2", "y2", "xy", "peak")],
                            _p(flags, C.c_uint32)), "measure")
    cat = dict(ints)
    cat["pmin"] = pmin
    cat.update(dbl)
    cat["flags"] = flags
    return {k: v[:nobj] for k, v in cat.items()}


PEAK_FIELDS = ("npix", "xmin", "xmax", "ymin", "ymax", "pmin", "flux", "x", "y", "x2", "y2", "xy", "peak",
               "flags")


def peaks(I, M, F, R, thresh, sep, cwin, sat=np.inf, cap=None):
    """Local maxima of F / R above the threshold with first-moment centroids
    (catalogue columns as measure(); `peak` holds the significance)."""
    Ii, Mm, Ff, Rr = _f64(I), _f64(M), _f64(F), _f64(R)
    H, W = Mm.shape
    cap = W * H if cap is None else cap
    n = C.c_long(0)
    c = max(cap, 1)
    ints = {k: np.zeros(c, np.int32) for k in ("npix", "xmin", "xmax", "ymin", "ymax")}
    pidx = np.zeros(c, np.int64)
    dbl = {k: np.zeros(c) for k in ("flux", "x", "y", "x2", "y2", "xy", "peak")}
    flags = np.zeros(c, np.uint32)
    _check(lib().or_peaks(_p(Ii), _p(Mm), _p(Ff), _p(Rr), W, H, thresh, sep, cwin, sat, cap,
                          *[_p(ints[k], C.c_int32) for k in ("npix", "xmin", "xmax", "ymin", "ymax")],
                          _p(pidx, C.c_int64), *[_p(dbl[k]) for k in ("flux", "x", "y", "x2", "y2", "xy", "peak")],
                          _p(flags, C.c_uint32), C.byref(n)), "peaks")
    k = min(int(n.value), cap)
    out = {q: v[:k] for q, v in ints.items()}
    out["pmin"] = pidx[:k]
    out.update({q: v[:k] for q, v in dbl.items()})
    out["flags"] = flags[:k]
    out["n"] = int(n.value)
    return out


def run_peaks(img, p, sep, cwin, K=None, grids=None):
    """Background -> M = I - B -> F = Khat (x) M -> local maxima of F / R."""
    I = _f64(img)
    H, W = I.shape
    if grids is None:
        bk = background(I, p)
    else:
        back, rms = (_f64(g) for g in grids)
        bk = Background({}, back, rms, grid_map(back, W, H, p.mesh_w, p.mesh_h),
                        grid_map(rms, W, H, p.mesh_w, p.mesh_h))
    M = I - bk.B
    K = p.kernel() if K is None else K
    F = filter_image(M, K)
    return bk, M, F, peaks(I, M, F, bk.R, p.thresh, sep, cwin, p.sat_level)


# ----------------------------------------------------------------------------
# Aperture photometry
# ----------------------------------------------------------------------------
def overlap(x0, x1, y0, y1, cx, cy, r):
    return lib().or_overlap(x0, x1, y0, y1, cx, cy, r)


def aperture(M, R, xs, ys, radii, r_in, r_out, gain=0.0, want_err=True):
    Mm = _f64(M)
    H, W = Mm.shape
    Rr = _f64(R) if R is not None else None
    xs, ys = _f64(xs), _f64(ys)
    n = xs.size
    rad = _f64(radii)
    nr = rad.size
    flux = np.zeros((max(n, 1), nr))
    area = np.zeros((max(n, 1), nr))
    err = np.zeros((max(n, 1), nr))
    bkg = np.zeros(max(n, 1))
    flags = np.zeros(max(n, 1), np.uint32)
    rp = _p(Rr) if Rr is not None else C.POINTER(C.c_double)()
    _check(lib().or_aperture(_p(Mm), rp, W, H, _p(xs), _p(ys), n, _p(rad), nr, r_in, r_out, gain,
                             int(bool(want_err) and Rr is not None), _p(flux), _p(area), _p(bkg),
                             _p(err), _p(flags, C.c_uint32)), "aperture")
    return dict(flux=flux[:n], area=area[:n], bkg=bkg[:n], fluxerr=err[:n], flags=flags[:n])


# ----------------------------------------------------------------------------
# Growth curves on top-hat kernels
# ----------------------------------------------------------------------------
def growth_radii(fwhm):
    """Integer radii ceil(0.75 fwhm) .. ceil(5 fwhm)."""
    n = C.c_int(0)
    _check(lib().or_growth_radii(float(fwhm), 0, C.POINTER(C.c_int32)(), C.byref(n)), "growth_radii")
    out = np.zeros(max(n.value, 1), np.int32)
    _check(lib().or_growth_radii(float(fwhm), n.value, _p(out, C.c_int32), C.byref(n)), "growth_radii")
    return out[: n.value]


def tophat_taps(r):
    """(2r+1)^2 exact-overlap taps of the top-hat kernel of integer radius r."""
    t = np.zeros((2 * r + 1, 2 * r + 1))
    _check(lib().or_tophat_taps(int(r), _p(t)), "tophat_taps")
    return t


def growth(M, V, xs, ys, radii):
    """Growth curves: per source and radius, the top-hat correlation of M and
    of V read at the source's pixel.  Returns dict(sum, var, area, flags)."""
    Mm = _f64(M)
    H, W = Mm.shape
    Vv = _f64(V) if V is not None else None
    xs, ys = _f64(xs), _f64(ys)
    n = xs.size
    rad = np.ascontiguousarray(radii, dtype=np.int32)
    nr = rad.size
    s = np.zeros((max(n, 1), nr))
    v = np.zeros((max(n, 1), nr))
    a = np.zeros((max(n, 1), nr))
    fl = np.zeros(max(n, 1), np.uint32)
    vp = _p(Vv) if Vv is not None else C.POINTER(C.c_double)()
    _check(lib().or_growth(_p(Mm), vp, W, H, _p(xs), _p(ys), n, _p(rad, C.c_int32), nr, _p(s), _p(v), _p(a),
                           _p(fl, C.c_uint32)), "growth")
    return dict(sum=s[:n], var=v[:n], area=a[:n], flags=fl[:n])


# ----------------------------------------------------------------------------
# Whole chain
# ----------------------------------------------------------------------------
@dataclass
class Result:
    bkg: Background
    M: np.ndarray
    F: np.ndarray
    seg: np.ndarray
    cat: dict
    phot: dict


def run(img, p, K=None, grids=None):
    """Background -> M = I - B -> F = Khat (x) M -> mask F > t R -> labelled
    objects with moments -> apertures.  `grids` = (back, rms) skips the mesh
    statistics and filter and interpolates the given grids instead."""
    I = _f64(img)
    H, W = I.shape
    if grids is None:
        bk = background(I, p)
    else:
        back, rms = (_f64(g) for g in grids)
        bk = Background({}, back, rms, grid_map(back, W, H, p.mesh_w, p.mesh_h),
                        grid_map(rms, W, H, p.mesh_w, p.mesh_h))
    M = I - bk.B
    K = p.kernel() if K is None else K
    F = filter_image(M, K)
    seg, n = threshold_label(F, bk.R, p.thresh, p.minarea, p.conn)
    cat = measure(I, M, seg, n, p.sat_level)
    phot = aperture(M, bk.R, cat["x"], cat["y"], list(p.radii), p.r_in, p.r_out, p.gain, p.want_err)
    cat["flags"] = cat["flags"] | phot["flags"]
    return Result(bk, M, F, seg, cat, phot)
