"""Device buffers and call sequencing around the C ABI (torch for memory/streams).

`Photometry` owns, for a fixed batch geometry, the background buffer, the
workspace, the catalogue and photometry columns (all torch tensors on the
GPU) and enqueues gp_background -> gp_detect -> gp_aperture on a stream.
Nothing here computes any part of the method; it sizes, allocates, fills the
gp_* structs and copies results back.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_NP_DTYPE = {torch.float64: np.float64, torch.float32: np.float32, torch.int32: np.int32,
             torch.int64: np.int64, torch.uint8: np.uint8, torch.int16: np.int16}

from . import _lib as L


@dataclass
class PhotParams:
    mesh_w: int = 64
    mesh_h: int = 64
    mesh_filter: int = 3
    clip_sigma: float = 3.0
    crowd_tol: float = 0.2
    mode_a: float = 2.5
    mode_b: float = 1.5
    max_iter: int = 100
    thresh: float = 1.5
    minarea: int = 5
    conn: int = 8
    radii: Sequence[float] = (3.0, 6.0)
    r_in: float = 10.0
    r_out: float = 15.0
    sat_level: float = math.inf
    gain: float = 0.0
    want_err: bool = True

    @classmethod
    def of(cls, obj) -> "PhotParams":
        """Copy the fields from any object that has them (e.g. a workload spec)."""
        kw = {k: getattr(obj, k) for k in cls.__dataclass_fields__ if hasattr(obj, k)}
        return cls(**kw)


CAT_INT = ("npix", "xmin", "xmax", "ymin", "ymax")
CAT_F64 = ("flux", "x", "y", "x2", "y2", "xy")


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint16:
        return L.GP_U16
    if t.dtype == torch.float32:
        return L.GP_F32
    raise TypeError(f"frames must be uint16 or float32 (got {t.dtype})")


def make_frame(t: torch.Tensor) -> L.gp_frame:
    if not t.is_cuda:
        raise ValueError("frames must be device tensors")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("frames must be 2-D with unit column stride")
    return L.gp_frame(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0), _dtype_code(t))


class Photometry:
    """One batch geometry: shapes, dtypes and parameters fixed at construction.

    autotune: time the candidate launch shapes of this batch's shape classes
    once, here (one synchronous run), and use the fastest from then on;
    tune_cache: JSON file that keeps those choices across contexts."""

    def __init__(self, frames: Sequence[torch.Tensor], params, kernel: np.ndarray, capacity: int,
                 comp_capacity: int = 0, precision: int = L.GP_PREC_F32, device: int = 0,
                 seg: bool = False, ctx=None, autotune: bool = False, tune_cache: Optional[str] = None):
        self.p = PhotParams.of(params)
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else L.gp_ctx_create(device, tune_cache)
        self._own_ctx = ctx is None
        self.frames_t = list(frames)
        self.frames = [make_frame(t) for t in self.frames_t]
        self.n = len(self.frames)
        self.capacity = int(capacity)
        self.kernel = np.ascontiguousarray(kernel, dtype=np.float32)
        self.radii = np.ascontiguousarray(list(self.p.radii), dtype=np.float32)
        p = self.p
        self.bp = L.gp_bkg_params(p.mesh_w, p.mesh_h, p.mesh_filter, p.clip_sigma, p.crowd_tol, p.mode_a,
                                  p.mode_b, p.max_iter, 0)
        kh, kw = self.kernel.shape
        self.dp = L.gp_det_params(self.kernel.ctypes.data_as(C.POINTER(C.c_float)), kw, kh, p.thresh,
                                  p.minarea, p.conn, p.sat_level, precision)
        self.ap = L.gp_ap_params(self.radii.ctypes.data_as(C.POINTER(C.c_float)), len(self.radii), p.r_in,
                                 p.r_out, p.gain, 1 if p.want_err else 0, precision)
        self.layouts, bkg_bytes = L.gp_background_layout(self.frames, self.bp)
        self.ws_bytes = L.gp_workspace_size(self.ctx, self.frames, self.bp, self.dp, self.ap, self.capacity,
                                            comp_capacity)
        dev = self.device
        # the library writes everything it later reads: no clearing needed
        self.bkg = torch.empty(max(bkg_bytes, 256), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        rows = max(self.n * self.capacity, 1)
        nr = len(self.radii)
        self.cat = {k: torch.empty(rows, dtype=torch.int32, device=dev) for k in CAT_INT}
        self.cat.update({k: torch.empty(rows, dtype=torch.float64, device=dev) for k in CAT_F64})
        self.cat["pmin"] = torch.empty(rows, dtype=torch.int64, device=dev)
        self.cat["peak"] = torch.empty(rows, dtype=torch.float32, device=dev)
        self.cat["flags"] = torch.empty(rows, dtype=torch.int32, device=dev)
        self.n_obj = torch.zeros(self.n, dtype=torch.int32, device=dev)
        self.status = torch.zeros(self.n, dtype=torch.int32, device=dev)
        self.comp_status = torch.zeros(2, dtype=torch.int32, device=dev)
        self.phot = {"flux": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                     "area": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                     "fluxerr": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                     "bkg": torch.empty(rows, dtype=torch.float64, device=dev)}
        c = self.cat
        self.gcat = L.gp_catalog(self.capacity, self.n_obj.data_ptr(), self.status.data_ptr(),
                                 *[c[k].data_ptr() for k in CAT_INT], c["pmin"].data_ptr(),
                                 *[c[k].data_ptr() for k in CAT_F64], c["peak"].data_ptr(),
                                 c["flags"].data_ptr())
        ph = self.phot
        self.gphot = L.gp_phot(ph["flux"].data_ptr(), ph["area"].data_ptr(), ph["bkg"].data_ptr(),
                               ph["fluxerr"].data_ptr())
        self.graph = None
        self.grow = None
        self.precision = precision
        self.seg = None
        if seg:
            self.seg = [torch.zeros(t.shape[0], t.shape[1], dtype=torch.int32, device=dev) for t in self.frames_t]
        if autotune:
            L.gp_ctx_set_tuning(self.ctx, True)
            try:
                self.run()
                torch.cuda.synchronize(self.device)
            finally:
                L.gp_ctx_set_tuning(self.ctx, False)

    def close(self):
        if self.graph is not None and self.ctx:
            L.gp_graph_destroy(self.graph)
            self.graph = None
        if self._own_ctx and self.ctx:
            L.gp_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def rebind(self, frames: Sequence[torch.Tensor]):
        """Point the batch at other frames of the same shapes and dtypes."""
        if len(frames) != self.n:
            raise ValueError("rebind needs the same number of frames")
        new = [make_frame(t) for t in frames]
        for a, b in zip(new, self.frames):
            if (a.width, a.height, a.pitch, a.dtype) != (b.width, b.height, b.pitch, b.dtype):
                raise L.GpError(L.GP_ERR_INVALID_ARG, "rebind needs the same shapes, pitches and dtypes")
        self.frames_t = list(frames)
        self.frames = new
        if self.graph is not None:
            L.gp_graph_rebind(self.graph, self.frames)

    def stream_ptr(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def background(self, stream=None, grid_given: bool = False):
        bp = L.gp_bkg_params.from_buffer_copy(self.bp)
        if grid_given:
            bp.flags |= L.GP_BKG_GRID_GIVEN
        L.gp_background(self.ctx, self.frames, bp, C.c_void_p(self.bkg.data_ptr()),
                        C.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.stream_ptr(stream))

    def detect(self, stream=None):
        seg = [s.data_ptr() for s in self.seg] if self.seg is not None else None
        L.gp_detect(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.dp, self.gcat, seg,
                    C.c_void_p(self.comp_status.data_ptr()), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                    self.stream_ptr(stream))

    def peaks(self, sep: int, cwin: int, stream=None):
        """The paper's detection (local maxima of F / R, first-moment
        centroids) into the catalogue, in place of detect()."""
        L.gp_peaks(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.dp,
                   L.gp_peak_params(int(sep), int(cwin)), self.gcat, C.c_void_p(self.comp_status.data_ptr()),
                   C.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.stream_ptr(stream))

    def peaks_psf(self, sep: int, cwin: int, kernels: np.ndarray, coef: Optional[Sequence[torch.Tensor]] = None,
                  bin: int = 1, stream=None):
        """The paper's detection with a spatially varying PSF: kernels
        (K+1, kh, kw) float32 with the reference first, coef one device
        tensor (K, ceil(H / bin), ceil(W / bin)) float32 per frame."""
        ks = np.ascontiguousarray(kernels, dtype=np.float32)
        K, kh, kw = ks.shape[0] - 1, ks.shape[1], ks.shape[2]
        maps = None
        if K > 0:
            if coef is None or len(coef) != self.n:
                raise ValueError("one coefficient-map tensor per frame is needed")
            arr = []
            for c in coef:
                if c.dtype != torch.float32 or c.dim() != 3 or c.shape[0] != K or c.stride(2) != 1:
                    raise ValueError("coefficient maps must be float32 (K, rows, cols) with unit column stride")
                arr.append(L.gp_coef_maps(c.data_ptr(), c.stride(1), c.stride(0)))
            maps = (L.gp_coef_maps * self.n)(*arr)
        psf = L.gp_psf_model(ks.ctypes.data_as(C.POINTER(C.c_float)), kw, kh, K, int(bin), maps)
        L.gp_peaks_psf(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.dp,
                       L.gp_peak_params(int(sep), int(cwin)), psf, self.gcat,
                       C.c_void_p(self.comp_status.data_ptr()), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                       self.stream_ptr(stream))

    def aperture(self, stream=None):
        L.gp_aperture(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.gcat, self.ap,
                      self.gphot, C.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.stream_ptr(stream))

    def growth(self, radii, stream=None, want_var: bool = True):
        """Growth curves of every catalogued source: top-hat sums of M (and of
        R^2) at the source's pixel for each integer radius (see
        growth_radii()).  Results come back under "growth" in results()."""
        rad = np.ascontiguousarray(radii, dtype=np.int32)
        nr = rad.size
        rows = max(self.n * self.capacity, 1)
        if self.grow is None or self.grow["sum"].shape[1] != nr:
            dev = self.device
            self.grow = {"sum": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                         "var": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                         "area": torch.empty(rows, nr, dtype=torch.float64, device=dev),
                         "flags": torch.empty(rows, dtype=torch.int32, device=dev)}
        g = self.grow
        self._grow_radii = rad
        gp = L.gp_growth_params(rad.ctypes.data_as(C.POINTER(C.c_int32)), nr, self.precision)
        out = L.gp_growth_out(g["sum"].data_ptr(), g["var"].data_ptr() if want_var else None, g["area"].data_ptr(),
                              g["flags"].data_ptr())
        L.gp_growth(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.gcat, gp, out,
                    C.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.stream_ptr(stream))

    def run(self, stream=None):
        self.background(stream)
        self.detect(stream)
        self.aperture(stream)

    def capture(self):
        """Record the three calls over this batch into a library graph (once);
        replay() then runs them with one graph launch, and rebind() updates
        the graph for other frames of the same shapes."""
        if self.graph is None:
            seg = [s.data_ptr() for s in self.seg] if self.seg is not None else None
            self.graph = L.gp_graph_create(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), self.dp,
                                           self.gcat, seg, C.c_void_p(self.comp_status.data_ptr()), self.ap,
                                           self.gphot, C.c_void_p(self.ws.data_ptr()), self.ws_bytes)
        return self

    def replay(self, stream=None):
        if self.graph is None:
            self.capture()
        L.gp_graph_launch(self.graph, self.stream_ptr(stream))

    # ------------------------------------------------------------------
    # host-side inspection (tests, bench)
    def grids(self, f: int):
        lay = self.layouts[f]
        ny, nx = lay.ny, lay.nx
        raw = self.bkg

        def view(off, n, dt):
            return raw[off: off + n * np.dtype(dt).itemsize].view(
                {np.float64: torch.float64, np.int32: torch.int32}[dt]).cpu().numpy()
        out = {k: view(getattr(lay, k), nx * ny, np.float64).reshape(ny, nx)
               for k in ("back_raw", "rms_raw", "back", "rms")}
        out["iters"] = view(lay.iters, nx * ny, np.int32).reshape(ny, nx)
        out["coef"] = view(lay.coef, 2 * (ny + 1) * (nx + 1) * 16, np.float64).reshape(2, ny + 1, nx + 1, 16)
        return out

    def maps(self, f: int, precision: int = L.GP_PREC_F32):
        """Per-pixel background and noise maps of frame f (float64, synchronises)."""
        t = self.frames_t[f]
        H, W = t.shape
        B = torch.empty(H, W, dtype=torch.float64, device=self.device)
        R = torch.empty(H, W, dtype=torch.float64, device=self.device)
        L.gp_background_map(self.ctx, self.frames, self.bp, C.c_void_p(self.bkg.data_ptr()), f, precision,
                            C.c_void_p(B.data_ptr()), C.c_void_p(R.data_ptr()), self.stream_ptr())
        torch.cuda.synchronize(self.device)
        return B.cpu().numpy(), R.cpu().numpy()

    def set_grids(self, f: int, back: np.ndarray, rms: np.ndarray):
        """Write the background/rms grids of frame f (used with grid_given)."""
        lay = self.layouts[f]
        for off, g in ((lay.back, back), (lay.rms, rms)):
            a = torch.from_numpy(np.ascontiguousarray(g, dtype=np.float64).ravel())
            self.bkg[off: off + a.numel() * 8].copy_(a.view(torch.uint8))

    def set_catalog(self, f: int, x: np.ndarray, y: np.ndarray, flags: Optional[np.ndarray] = None):
        """Write object centres of frame f (used to run the aperture stage alone)."""
        n = len(x)
        if n > self.capacity:
            raise ValueError("more objects than capacity")
        base = f * self.capacity
        self.cat["x"][base: base + n] = torch.as_tensor(np.asarray(x, np.float64), device=self.device)
        self.cat["y"][base: base + n] = torch.as_tensor(np.asarray(y, np.float64), device=self.device)
        fl = np.zeros(n, np.int32) if flags is None else np.asarray(flags, np.int32)
        self.cat["flags"][base: base + n] = torch.as_tensor(fl, device=self.device)
        self.n_obj[f] = n
        self.status[f] = 0

    def results(self, f: int = 0, sync: bool = True):
        """Catalogue and photometry of frame f as numpy arrays.  sync=False when
        the caller already knows the work is done (e.g. an event completed).
        The frame's rows of every column are packed on the device and brought
        over in one copy."""
        if sync:
            torch.cuda.synchronize(self.device)
        hdr = torch.stack([self.n_obj[f], self.status[f]]).cpu().numpy()
        n, st = int(hdr[0]), int(hdr[1])
        k = min(n, self.capacity)
        base = f * self.capacity
        cols = [("cat", name, t) for name, t in self.cat.items()] + \
               [("phot", name, t) for name, t in self.phot.items()]
        if self.grow is not None:
            cols += [("growth", name, t) for name, t in self.grow.items()]
        parts = [t[base: base + k].reshape(-1).view(torch.uint8) for _, _, t in cols]
        parts.append(self.comp_status.reshape(-1).view(torch.uint8))
        flat = torch.cat(parts).cpu().numpy()
        out = {"cat": {}, "phot": {}, "growth": {}}
        off = 0
        for (grp, name, t), pt in zip(cols, parts):
            nb = pt.numel()
            shape = (k,) + tuple(t.shape[1:])
            out[grp][name] = flat[off: off + nb].view(_NP_DTYPE[t.dtype]).reshape(shape).copy()
            off += nb
        comp = flat[off:].view(_NP_DTYPE[self.comp_status.dtype]).tolist()
        out["cat"]["flags"] = out["cat"]["flags"].astype(np.uint32)
        if self.grow is not None:
            out["growth"]["flags"] = out["growth"]["flags"].astype(np.uint32)
        return dict(n_obj=n, status=st, cat=out["cat"], phot=out["phot"], growth=out["growth"], comp_status=comp,
                    seg=self.seg[f].cpu().numpy() if self.seg is not None else None)


def run_plain(frame: torch.Tensor, params, kernel: np.ndarray, capacity: int, **kw):
    """One frame through background -> detect -> aperture; returns the results."""
    ph = Photometry([frame], params, kernel, capacity, **kw)
    ph.run()
    out = ph.results(0)
    out["grids"] = ph.grids(0)
    ph.close()
    return out


def growth_radii(fwhm: float) -> List[int]:
    """Integer radii ceil(0.75 fwhm) .. ceil(5 fwhm) of the growth curves (the
    library's rule)."""
    return L.gp_growth_radii(fwhm)


class ConvBackground:
    """The paper's own background for a batch of frames: a convolution with
    reflected borders (separable taps kx, ky), invalid pixels (mask or
    >= sat_level) filled from their valid neighbours, and the noise map of a
    dark-subtracted frame from gain, read noise and dark current.  run()
    fills self.back / self.rms (one (H, W) tensor per frame, float32 or
    float64 by precision) and self.unfilled (int64 per frame)."""

    def __init__(self, frames: Sequence[torch.Tensor], kx, ky, gain: float, read_noise: float = 0.0,
                 dark_current: float = 0.0, exptime: float = 0.0, sat_level: float = math.inf,
                 precision: int = L.GP_PREC_F32, device: int = 0, ctx=None):
        self.device = torch.device("cuda", device)
        self.ctx = ctx if ctx is not None else L.gp_ctx_create(device, None)
        self._own_ctx = ctx is None
        self.frames_t = list(frames)
        self.frames = [make_frame(t) for t in self.frames_t]
        self.kx = np.ascontiguousarray(kx, dtype=np.float32)
        self.ky = np.ascontiguousarray(ky, dtype=np.float32)
        self.cp = L.gp_conv_params(self.kx.ctypes.data_as(C.POINTER(C.c_float)), self.kx.size,
                                   self.ky.ctypes.data_as(C.POINTER(C.c_float)), self.ky.size, sat_level, gain,
                                   read_noise, dark_current, exptime, precision)
        self.ws_bytes = L.gp_background_conv_ws(self.frames, self.cp)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        dt = torch.float64 if precision == L.GP_PREC_F64 else torch.float32
        self.back = [torch.empty(t.shape[0], t.shape[1], dtype=dt, device=self.device) for t in self.frames_t]
        self.rms = [torch.empty(t.shape[0], t.shape[1], dtype=dt, device=self.device) for t in self.frames_t]
        self.unfilled = torch.zeros(len(self.frames), dtype=torch.int64, device=self.device)

    def run(self, masks: Optional[Sequence[Optional[torch.Tensor]]] = None, stream=None):
        mp = None
        if masks is not None:
            mp = []
            for m, t in zip(masks, self.frames_t):
                if m is None:
                    mp.append(None)
                    continue
                if m.dtype != torch.uint8 or m.shape != t.shape or m.stride() != t.stride():
                    raise ValueError("masks must be uint8 with the frame's shape and strides")
                mp.append(m.data_ptr())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.gp_background_conv(self.ctx, self.frames, mp, self.cp, [b.data_ptr() for b in self.back],
                             [r.data_ptr() for r in self.rms], C.c_void_p(self.unfilled.data_ptr()),
                             C.c_void_p(self.ws.data_ptr()), self.ws_bytes, C.c_void_p(s.cuda_stream))

    def close(self):
        if self._own_ctx and self.ctx:
            L.gp_ctx_destroy(self.ctx)
            self.ctx = None
