"""ctypes binding of include/gp.h: the same names, argument marshalling only.

Every step of the hot path runs in libgpphot.so (HIP kernels for gfx950).
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpphot.so")

GP_OK, GP_ERR_INVALID_ARG, GP_ERR_UNSUPPORTED, GP_ERR_WORKSPACE, GP_ERR_CAPACITY, GP_ERR_HIP = range(6)
GP_U16, GP_F32 = 1, 2
GP_PREC_F32, GP_PREC_F64 = 0, 1
GP_BKG_GRID_GIVEN = 1
GP_FLAG_SATURATED, GP_FLAG_EDGE, GP_FLAG_NONPOS, GP_FLAG_APER_TRUNC = 1, 2, 4, 8

STATUS_NAMES = {0: "GP_OK", 1: "GP_ERR_INVALID_ARG", 2: "GP_ERR_UNSUPPORTED", 3: "GP_ERR_WORKSPACE",
                4: "GP_ERR_CAPACITY", 5: "GP_ERR_HIP"}


class gp_frame(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch", C.c_int64), ("dtype", C.c_int32)]


class gp_bkg_params(C.Structure):
    _fields_ = [("mesh_w", C.c_int32), ("mesh_h", C.c_int32), ("filter_size", C.c_int32),
                ("clip_sigma", C.c_float), ("crowd_tol", C.c_float), ("mode_a", C.c_float),
                ("mode_b", C.c_float), ("max_iter", C.c_int32), ("flags", C.c_uint32)]


class gp_bkg_layout(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("back_raw", C.c_int64), ("rms_raw", C.c_int64),
                ("back", C.c_int64), ("rms", C.c_int64), ("coef", C.c_int64), ("iters", C.c_int64),
                ("bytes", C.c_int64)]


class gp_det_params(C.Structure):
    _fields_ = [("kernel", C.POINTER(C.c_float)), ("kw", C.c_int32), ("kh", C.c_int32),
                ("thresh", C.c_float), ("minarea", C.c_int32), ("connectivity", C.c_int32),
                ("sat_level", C.c_float), ("precision", C.c_int32)]


class gp_ap_params(C.Structure):
    _fields_ = [("radii", C.POINTER(C.c_float)), ("nr", C.c_int32), ("r_in", C.c_float),
                ("r_out", C.c_float), ("gain", C.c_float), ("want_err", C.c_int32),
                ("precision", C.c_int32)]


class gp_catalog(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("n_obj", C.c_void_p), ("status", C.c_void_p),
                ("npix", C.c_void_p), ("xmin", C.c_void_p), ("xmax", C.c_void_p), ("ymin", C.c_void_p),
                ("ymax", C.c_void_p), ("pmin", C.c_void_p), ("flux", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("x2", C.c_void_p), ("y2", C.c_void_p), ("xy", C.c_void_p),
                ("peak", C.c_void_p), ("flags", C.c_void_p)]


class gp_peak_params(C.Structure):
    _fields_ = [("sep", C.c_int32), ("cwin", C.c_int32)]


class gp_coef_maps(C.Structure):
    _fields_ = [("data", C.c_void_p), ("pitch", C.c_int64), ("plane", C.c_int64)]


class gp_psf_model(C.Structure):
    _fields_ = [("kernels", C.POINTER(C.c_float)), ("kw", C.c_int32), ("kh", C.c_int32), ("nmodes", C.c_int32),
                ("bin", C.c_int32), ("maps", C.POINTER(gp_coef_maps))]


class gp_conv_params(C.Structure):
    _fields_ = [("kx", C.POINTER(C.c_float)), ("lx", C.c_int32), ("ky", C.POINTER(C.c_float)), ("ly", C.c_int32),
                ("sat_level", C.c_float), ("gain", C.c_float), ("read_noise", C.c_float),
                ("dark_current", C.c_float), ("exptime", C.c_float), ("precision", C.c_int32)]


class gp_growth_params(C.Structure):
    _fields_ = [("radii", C.POINTER(C.c_int32)), ("nr", C.c_int32), ("precision", C.c_int32)]


class gp_growth_out(C.Structure):
    _fields_ = [("sum", C.c_void_p), ("var", C.c_void_p), ("area", C.c_void_p), ("flags", C.c_void_p)]


class gp_phot(C.Structure):
    _fields_ = [("flux", C.c_void_p), ("area", C.c_void_p), ("bkg", C.c_void_p), ("fluxerr", C.c_void_p)]


EXPORTS = ("gp_ctx_create", "gp_ctx_destroy", "gp_last_error", "gp_version", "gp_background_layout",
           "gp_workspace_size", "gp_background", "gp_background_map", "gp_detect", "gp_detect_noalloc",
           "gp_peaks", "gp_peaks_psf", "gp_aperture", "gp_growth_radii", "gp_growth", "gp_background_conv_ws",
           "gp_background_conv",
           "gp_profile_enable",
           "gp_profile_read", "gp_profile_reset", "gp_ctx_set_tuning", "gp_graph_create", "gp_graph_launch",
           "gp_graph_rebind", "gp_graph_destroy")

_lib = None


class GpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libgpphot.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2609_32375_amd.build`")
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.gp_ctx_create.argtypes = [C.c_int, C.c_char_p, C.POINTER(vp)]
    L.gp_ctx_destroy.argtypes = [vp]
    L.gp_ctx_destroy.restype = None
    L.gp_last_error.restype = C.c_char_p
    L.gp_version.restype = C.c_char_p
    L.gp_background_layout.argtypes = [C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params),
                                       C.POINTER(gp_bkg_layout), C.POINTER(C.c_size_t)]
    L.gp_workspace_size.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params),
                                    C.POINTER(gp_det_params), C.POINTER(gp_ap_params), i32, i64,
                                    C.POINTER(C.c_size_t)]
    L.gp_background.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp, vp, C.c_size_t, vp]
    L.gp_background_map.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp, i32, i32,
                                    vp, vp, vp]
    L.gp_detect.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp,
                            C.POINTER(gp_det_params), C.POINTER(gp_catalog), C.POINTER(vp), vp, vp,
                            C.c_size_t, vp]
    L.gp_detect_noalloc.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp,
                                    C.POINTER(gp_det_params), C.POINTER(gp_catalog), C.POINTER(vp), vp, vp]
    L.gp_peaks.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp, C.POINTER(gp_det_params),
                           C.POINTER(gp_peak_params), C.POINTER(gp_catalog), vp, vp, C.c_size_t, vp]
    L.gp_aperture.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp,
                              C.POINTER(gp_catalog), C.POINTER(gp_ap_params), C.POINTER(gp_phot), vp,
                              C.c_size_t, vp]
    L.gp_peaks_psf.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp,
                               C.POINTER(gp_det_params), C.POINTER(gp_peak_params), C.POINTER(gp_psf_model),
                               C.POINTER(gp_catalog), vp, vp, C.c_size_t, vp]
    L.gp_background_conv_ws.argtypes = [C.POINTER(gp_frame), i32, C.POINTER(gp_conv_params), C.POINTER(C.c_size_t)]
    L.gp_background_conv.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(vp), C.POINTER(gp_conv_params),
                                     C.POINTER(vp), C.POINTER(vp), vp, vp, C.c_size_t, vp]
    L.gp_growth_radii.argtypes = [C.c_double, i32, C.POINTER(i32), C.POINTER(i32)]
    L.gp_growth.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp, C.POINTER(gp_catalog),
                            C.POINTER(gp_growth_params), C.POINTER(gp_growth_out), vp, C.c_size_t, vp]
    L.gp_graph_create.argtypes = [vp, C.POINTER(gp_frame), i32, C.POINTER(gp_bkg_params), vp,
                                  C.POINTER(gp_det_params), C.POINTER(gp_catalog), C.POINTER(vp), vp,
                                  C.POINTER(gp_ap_params), C.POINTER(gp_phot), vp, C.c_size_t, C.POINTER(vp)]
    L.gp_graph_launch.argtypes = [vp, vp]
    L.gp_graph_rebind.argtypes = [vp, C.POINTER(gp_frame), i32]
    L.gp_graph_destroy.argtypes = [vp]
    L.gp_graph_destroy.restype = None
    L.gp_profile_enable.argtypes = [vp, C.c_int]
    L.gp_ctx_set_tuning.argtypes = [vp, i32]
    L.gp_profile_read.argtypes = [vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(i64)]
    L.gp_profile_reset.argtypes = [vp]
    for f in ("gp_ctx_create", "gp_background_layout", "gp_workspace_size", "gp_background",
              "gp_background_map", "gp_detect", "gp_detect_noalloc", "gp_peaks",
              "gp_aperture", "gp_peaks_psf", "gp_background_conv_ws", "gp_background_conv", "gp_growth_radii", "gp_growth", "gp_profile_enable", "gp_profile_read", "gp_profile_reset", "gp_graph_create",
              "gp_graph_launch", "gp_graph_rebind"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def check(status: int):
    if status != GP_OK:
        raise GpError(status, load().gp_last_error().decode())


# --------------------------------------------------------------------------
# the C-ABI calls under their own names
def gp_ctx_create(device: int = 0, tune_cache: str | None = None):
    h = C.c_void_p()
    check(load().gp_ctx_create(device, tune_cache.encode() if tune_cache else None, C.byref(h)))
    return h


def gp_ctx_destroy(ctx):
    load().gp_ctx_destroy(ctx)


def gp_version() -> str:
    return load().gp_version().decode()


def gp_background_layout(frames, bp):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    lay = (gp_bkg_layout * n)()
    size = C.c_size_t()
    check(load().gp_background_layout(arr, n, C.byref(bp), lay, C.byref(size)))
    return list(lay), size.value


def gp_workspace_size(ctx, frames, bp, dp, ap, cat_capacity, comp_capacity=0):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    size = C.c_size_t()
    check(load().gp_workspace_size(ctx, arr, n, C.byref(bp), C.byref(dp) if dp else None,
                                   C.byref(ap) if ap else None, cat_capacity, comp_capacity, C.byref(size)))
    return size.value


def gp_background(ctx, frames, bp, bkg_ptr, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_background(ctx, arr, n, C.byref(bp), bkg_ptr, ws_ptr, ws_bytes, stream))


def gp_background_map(ctx, frames, bp, bkg_ptr, index, precision, back_ptr, rms_ptr, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_background_map(ctx, arr, n, C.byref(bp), bkg_ptr, index, precision, back_ptr, rms_ptr,
                                   stream))


def gp_detect(ctx, frames, bp, bkg_ptr, dp, cat, seg_ptrs, comp_status_ptr, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    segarr = (C.c_void_p * n)(*seg_ptrs) if seg_ptrs is not None else None
    check(load().gp_detect(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(dp), C.byref(cat), segarr,
                           comp_status_ptr, ws_ptr, ws_bytes, stream))


def gp_detect_noalloc(ctx, frames, bp, bkg_ptr, dp, cat, seg_ptrs, comp_status_ptr, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    segarr = (C.c_void_p * n)(*seg_ptrs) if seg_ptrs is not None else None
    check(load().gp_detect_noalloc(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(dp), C.byref(cat), segarr,
                                   comp_status_ptr, stream))


GP_DETECT_NOALLOC_MAX_BYTES = 128 << 20


def gp_peaks(ctx, frames, bp, bkg_ptr, dp, pp, cat, comp_status_ptr, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_peaks(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(dp), C.byref(pp), C.byref(cat),
                          comp_status_ptr, ws_ptr, ws_bytes, stream))


def gp_aperture(ctx, frames, bp, bkg_ptr, cat, ap, phot, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_aperture(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(cat), C.byref(ap), C.byref(phot),
                             ws_ptr, ws_bytes, stream))


def gp_peaks_psf(ctx, frames, bp, bkg_ptr, dp, pp, psf, cat, comp_status_ptr, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_peaks_psf(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(dp), C.byref(pp), C.byref(psf),
                              C.byref(cat), comp_status_ptr, ws_ptr, ws_bytes, stream))


def gp_background_conv_ws(frames, cp):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    out = C.c_size_t()
    check(load().gp_background_conv_ws(arr, n, C.byref(cp), C.byref(out)))
    return out.value


def gp_background_conv(ctx, frames, mask_ptrs, cp, back_ptrs, rms_ptrs, unfilled_ptr, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    masks = (C.c_void_p * n)(*mask_ptrs) if mask_ptrs is not None else None
    check(load().gp_background_conv(ctx, arr, n, masks, C.byref(cp), (C.c_void_p * n)(*back_ptrs),
                                    (C.c_void_p * n)(*rms_ptrs), unfilled_ptr, ws_ptr, ws_bytes, stream))


def gp_growth_radii(fwhm):
    n = C.c_int32(0)
    check(load().gp_growth_radii(float(fwhm), 0, None, C.byref(n)))
    out = (C.c_int32 * max(n.value, 1))()
    check(load().gp_growth_radii(float(fwhm), n.value, out, C.byref(n)))
    return [int(out[i]) for i in range(n.value)]


def gp_growth(ctx, frames, bp, bkg_ptr, cat, gp, out, ws_ptr, ws_bytes, stream):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_growth(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(cat), C.byref(gp), C.byref(out),
                           ws_ptr, ws_bytes, stream))


def gp_graph_create(ctx, frames, bp, bkg_ptr, dp, cat, seg_ptrs, comp_status_ptr, ap, phot, ws_ptr, ws_bytes):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    segarr = (C.c_void_p * n)(*seg_ptrs) if seg_ptrs is not None else None
    h = C.c_void_p()
    check(load().gp_graph_create(ctx, arr, n, C.byref(bp), bkg_ptr, C.byref(dp), C.byref(cat), segarr,
                                 comp_status_ptr, C.byref(ap), C.byref(phot), ws_ptr, ws_bytes, C.byref(h)))
    return h


def gp_graph_launch(graph, stream):
    check(load().gp_graph_launch(graph, stream))


def gp_graph_rebind(graph, frames):
    n = len(frames)
    arr = (gp_frame * n)(*frames)
    check(load().gp_graph_rebind(graph, arr, n))


def gp_graph_destroy(graph):
    load().gp_graph_destroy(graph)


def gp_ctx_set_tuning(ctx, on: bool):
    check(load().gp_ctx_set_tuning(ctx, 1 if on else 0))


def gp_profile_enable(ctx, on: bool):
    check(load().gp_profile_enable(ctx, 1 if on else 0))


def gp_profile_read(ctx, name: str):
    ms = C.c_double()
    cnt = C.c_int64()
    check(load().gp_profile_read(ctx, name.encode(), C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


def gp_profile_reset(ctx):
    check(load().gp_profile_reset(ctx))
