"""Seeded synthetic star fields and run parameters for the photometry hot path.

This module is shared by the GPU path's tests/bench and by the oracle's tests.
It holds none of the method's arithmetic: it only draws scenes (sky, stars,
noise, cosmic rays), builds the un-normalised filter kernel that is handed to
both sides as an input, and names the workloads.

Workloads follow the paper's frame sizes (4.2 to 151.2 MP, Table of datasets)
and source counts (hundreds to ~134k per frame, Introduction); the paper's own
frames are not available, so these synthetic fields stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "Params", "Frame", "gaussian_kernel", "make_frame", "config_params",
    "CONFIGS", "batch_frames", "arrival_stream", "crop",
]


# ----------------------------------------------------------------------------
# Run parameters (the method's knobs; the same object configures both sides)
# ----------------------------------------------------------------------------
@dataclass
class Params:
    mesh_w: int = 64
    mesh_h: int = 64
    mesh_filter: int = 3          # f x f median over the mesh grid (1 = off)
    clip_sigma: float = 3.0       # kappa of the kappa-sigma clip about the median
    crowd_tol: float = 0.2        # sigma change below which the clipped mean is used
    mode_a: float = 2.5           # mode = a*median - b*mean otherwise
    mode_b: float = 1.5
    max_iter: int = 100
    kernel_size: int = 5          # odd, square Gaussian matched filter
    kernel_fwhm: float = 3.0
    thresh: float = 1.5           # detection threshold in units of the rms map
    minarea: int = 5
    conn: int = 8
    radii: Sequence[float] = (3.0, 6.0)
    r_in: float = 10.0
    r_out: float = 15.0
    sat_level: float = math.inf
    gain: float = 0.0             # <= 0: no Poisson term in the aperture error
    want_err: bool = True

    def kernel(self) -> np.ndarray:
        return gaussian_kernel(self.kernel_size, self.kernel_fwhm)

    def to_dict(self):
        d = asdict(self)
        d["radii"] = list(self.radii)
        return d


def gaussian_kernel(size: int, fwhm: float) -> np.ndarray:
    """Un-normalised circular Gaussian exp(-(a^2+b^2)/2s^2), s = FWHM/(2 sqrt(2 ln 2)).

    The filter step normalises it to unit sum itself (the paper normalises PSF
    stamps to unit flux), so it is handed over as-is.
    """
    assert size % 2 == 1 and size >= 1
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    h = size // 2
    a = np.arange(-h, h + 1, dtype=np.float64)
    g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * s * s))
    return g.astype(np.float32)


# ----------------------------------------------------------------------------
# Scene rendering helpers
# ----------------------------------------------------------------------------
def _powerlaw_fluxes(rng, n, fmin=1e3, fmax=1e6):
    """dN/dF ~ F^-1.5 on [fmin, fmax] by inverse CDF."""
    u = rng.random(n)
    a, b = fmin ** -0.5, fmax ** -0.5
    return (a - u * (a - b)) ** -2.0


def _erf(x):
    # vectorised erf via math.erf is slow; use numpy-friendly scipy if present
    try:
        from scipy.special import erf
        return erf(x)
    except Exception:  # pragma: no cover
        return np.vectorize(math.erf)(x)


def _add_gaussian_stars(img, xs, ys, fl, fwhm):
    """Pixel-integrated Gaussian PSFs (products of erf differences)."""
    H, W = img.shape
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    hw = int(math.ceil(6.0 * fwhm))
    k = np.arange(-hw, hw + 1)
    inv = 1.0 / (s * math.sqrt(2.0))
    for x0, y0, f in zip(xs, ys, fl):
        ix, iy = int(round(x0)), int(round(y0))
        px = ix + k
        py = iy + k
        gx = 0.5 * (_erf((px + 0.5 - x0) * inv) - _erf((px - 0.5 - x0) * inv))
        gy = 0.5 * (_erf((py + 0.5 - y0) * inv) - _erf((py - 0.5 - y0) * inv))
        mx = (px >= 0) & (px < W)
        my = (py >= 0) & (py < H)
        if not mx.any() or not my.any():
            continue
        img[np.ix_(py[my], px[mx])] += f * np.outer(gy[my], gx[mx])


class _MoffatBank:
    """Unit-sum Moffat stamps (beta given), 5x5 sub-sampled per pixel, on a grid
    of FWHM values and 1/8-pixel phases; stars pick the nearest entry."""

    def __init__(self, beta=3.0, fwhm_lo=2.0, fwhm_hi=5.0, dfwhm=0.1, nphase=8):
        self.beta = beta
        self.fwhms = np.arange(fwhm_lo, fwhm_hi + 1e-9, dfwhm)
        self.nphase = nphase
        self.cache = {}

    def stamp(self, fwhm_idx, phx, phy):
        key = (fwhm_idx, phx, phy)
        st = self.cache.get(key)
        if st is not None:
            return st
        fwhm = self.fwhms[fwhm_idx]
        beta = self.beta
        alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
        hw = int(math.ceil(6.0 * fwhm))
        ox = phx / self.nphase
        oy = phy / self.nphase
        sub = (np.arange(5) + 0.5) / 5.0 - 0.5
        k = np.arange(-hw, hw + 1, dtype=np.float64)
        xx = (k[None, :, None, None] + sub[None, None, None, :]) - ox
        yy = (k[:, None, None, None] + sub[None, None, :, None]) - oy
        r2 = xx * xx + yy * yy
        prof = (1.0 + r2 / (alpha * alpha)) ** (-beta)
        st = prof.mean(axis=(2, 3))
        st /= st.sum()
        self.cache[key] = st
        return st

    def render(self, img, xs, ys, fl, fw):
        H, W = img.shape
        fidx = np.clip(np.rint((fw - self.fwhms[0]) / (self.fwhms[1] - self.fwhms[0])), 0,
                       len(self.fwhms) - 1).astype(int)
        for x0, y0, f, fi in zip(xs, ys, fl, fidx):
            ix, iy = int(math.floor(x0)), int(math.floor(y0))
            phx = int((x0 - ix) * self.nphase) % self.nphase
            phy = int((y0 - iy) * self.nphase) % self.nphase
            st = self.stamp(int(fi), phx, phy)
            hw = st.shape[0] // 2
            xa, xb = ix - hw, ix + hw + 1
            ya, yb = iy - hw, iy + hw + 1
            cxa, cxb = max(xa, 0), min(xb, W)
            cya, cyb = max(ya, 0), min(yb, H)
            if cxa >= cxb or cya >= cyb:
                continue
            img[cya:cyb, cxa:cxb] += f * st[cya - ya:cyb - ya, cxa - xa:cxb - xa]


def _noise(rng, expected, read_noise=10.0):
    """Poisson(expected) counts (gain 1 e-/ADU) plus Gaussian read noise."""
    lam = np.clip(expected, 0.0, None)
    out = rng.poisson(lam).astype(np.float64)
    out += rng.normal(0.0, read_noise, size=expected.shape)
    return out


# ----------------------------------------------------------------------------
# Workload definitions
# ----------------------------------------------------------------------------
@dataclass
class Frame:
    image: np.ndarray                 # float32 or uint16, shape (H, W)
    params: Params
    name: str = ""
    truth: Optional[dict] = None      # injected positions / fluxes


CONFIGS = {
    "c1": dict(W=2048, H=2048, dtype="f32", seed=0),
    "c2": dict(W=6144, H=6144, dtype="f32", seed=1),
    "c3": dict(W=12300, H=12300, dtype="f32", seed=2),
}


def config_params(name: str) -> Params:
    """Run parameters of each named workload."""
    if name == "c1":
        return Params(mesh_w=64, mesh_h=64, kernel_size=5, kernel_fwhm=3.0, thresh=1.5,
                      minarea=5, conn=8, radii=(3.0, 6.0), r_in=10.0, r_out=15.0)
    if name in ("c2", "c3"):
        return Params(mesh_w=128, mesh_h=128, kernel_size=9, kernel_fwhm=3.5, thresh=1.5,
                      minarea=5, conn=8, radii=(3.0, 6.0, 9.0), r_in=13.0, r_out=18.0,
                      sat_level=(65535.0 if name == "c3" else math.inf))
    raise KeyError(name)


def _sky_c1(W, H):
    x = np.arange(W, dtype=np.float64)
    return np.broadcast_to(1000.0 + 0.05 * x[None, :], (H, W)).copy()


def _sky_vignette(W, H, level=800.0, amp=0.05):
    x = np.arange(W, dtype=np.float64)
    y = np.arange(H, dtype=np.float64)
    return level * (1.0 + amp * np.sin(2 * np.pi * y / H)[:, None] * np.sin(2 * np.pi * x / W)[None, :])


def make_frame(name: str = "c1", seed: Optional[int] = None, W: Optional[int] = None,
               H: Optional[int] = None, nstars: Optional[int] = None,
               dtype: Optional[str] = None) -> Frame:
    """Render one synthetic frame of a named workload.

    c1: 2048^2 f32, sky 1000 + 0.05 x, 300 Gaussian stars (FWHM 3).
    c2: 6144^2 f32, sky 800 (1 + 0.05 sin sin), 20,000 Moffat stars (beta 3,
        FWHM 2..5 growing with the distance from the frame centre).
    c3: 12300^2 f32 crowded field, 134,000 Moffat stars, a bright population
        tuned so that about 2% of pixels saturate at 65535, 5,000 single-pixel
        cosmic-ray hits, clipped at 65535.
    Sizes, seeds, star counts and dtype can be overridden for small cases.
    """
    base = CONFIGS.get(name, CONFIGS["c1"])
    W = W or base["W"]
    H = H or base["H"]
    seed = base["seed"] if seed is None else seed
    dtype = dtype or base["dtype"]
    rng = np.random.Generator(np.random.PCG64(seed))
    params = config_params(name if name in ("c1", "c2", "c3") else "c1")
    area_scale = (W * H) / (base["W"] * base["H"])
    truth = {}
    if name == "c1":
        n = nstars if nstars is not None else max(1, int(round(300 * area_scale)))
        sky = _sky_c1(W, H)
        xs = rng.uniform(0, W, n)
        ys = rng.uniform(0, H, n)
        fl = _powerlaw_fluxes(rng, n)
        stars = np.zeros((H, W))
        _add_gaussian_stars(stars, xs, ys, fl, 3.0)
        img = _noise(rng, sky + stars)
        truth = dict(x=xs, y=ys, flux=fl)
    else:
        default_n = 20000 if name == "c2" else 134000
        n = nstars if nstars is not None else max(1, int(round(default_n * area_scale)))
        sky = _sky_vignette(W, H)
        xs = rng.uniform(0, W, n)
        ys = rng.uniform(0, H, n)
        fl = _powerlaw_fluxes(rng, n)
        rho = np.hypot(xs - W / 2.0, ys - H / 2.0)
        fw = 2.0 + 3.0 * rho / max(rho.max(), 1e-9)
        bank = _MoffatBank()
        if name == "c3":
            # bright population: log-uniform flux in [1e7, 1e9], chosen with
            # probability p_b; p_b bisected so that ~2% of pixels saturate
            ub = rng.random(n)
            fb = 10.0 ** rng.uniform(7.0, 9.0, n)
            sat_px = _saturated_footprints(bank, fb, fw, sky_level=800.0, sat=65535.0)
            target = 0.02 * W * H
            lo, hi = 0.0, 1.0
            for _ in range(40):
                mid = 0.5 * (lo + hi)
                if sat_px[ub < mid].sum() < target:
                    lo = mid
                else:
                    hi = mid
            bright = ub < 0.5 * (lo + hi)
            fl = np.where(bright, fb, fl)
            truth["bright"] = bright
        stars = np.zeros((H, W))
        bank.render(stars, xs, ys, fl, fw)
        img = _noise(rng, sky + stars)
        if name == "c3":
            ncr = max(1, int(round(5000 * area_scale)))
            cx = rng.integers(0, W, ncr)
            cy = rng.integers(0, H, ncr)
            img[cy, cx] += rng.uniform(2000.0, 50000.0, ncr)
            truth["cr_x"] = cx
            truth["cr_y"] = cy
        if name == "c3":
            img = np.minimum(img, 65535.0)
        truth.update(x=xs, y=ys, flux=fl, fwhm=fw)
    if dtype == "u16":
        out = np.clip(np.rint(img), 0, 65535).astype(np.uint16)
    else:
        out = img.astype(np.float32)
    return Frame(image=out, params=params, name=name, truth=truth)


def _saturated_footprints(bank, fb, fw, sky_level, sat):
    """Pixels of each star's stamp that would reach `sat` if the star were bright."""
    fidx = np.clip(np.rint((fw - bank.fwhms[0]) / (bank.fwhms[1] - bank.fwhms[0])), 0,
                   len(bank.fwhms) - 1).astype(int)
    out = np.zeros(len(fb))
    peak = {}
    for i, (f, fi) in enumerate(zip(fb, fidx)):
        st = peak.get(fi)
        if st is None:
            st = np.sort(bank.stamp(int(fi), 0, 0).ravel())[::-1]
            peak[fi] = st
        out[i] = np.count_nonzero(f * st >= sat - sky_level)
    return out


def crop(frame: Frame, x0: int, y0: int, w: int, h: int) -> Frame:
    """A sub-frame of a larger frame (same parameters)."""
    img = np.ascontiguousarray(frame.image[y0:y0 + h, x0:x0 + w])
    return Frame(image=img, params=frame.params, name=f"{frame.name}[{x0}:{x0+w},{y0}:{y0+h}]")


# ----------------------------------------------------------------------------
# Batch and arrival-stream workloads
# ----------------------------------------------------------------------------
def batch_frames(scale: float = 1.0, count_scale: float = 1.0, seed0: int = 1000):
    """64 uint16 frames of uneven sizes: 24 x 2048^2, 24 x 4096^2, 16 x 9600x6400
    (W x H), each with log-uniform 300..40,000 Gaussian stars as in c1.
    `scale` shrinks every side (for tests); `count_scale` the number of frames."""
    shapes = [(2048, 2048)] * 24 + [(4096, 4096)] * 24 + [(9600, 6400)] * 16
    if count_scale != 1.0:
        keep = max(1, int(round(len(shapes) * count_scale)))
        idx = np.linspace(0, len(shapes) - 1, keep).round().astype(int)
        shapes = [shapes[i] for i in idx]
    out = []
    for i, (w, h) in enumerate(shapes):
        r = np.random.Generator(np.random.PCG64(seed0 + i))
        u = r.random()
        n = int(round(300.0 * (40000.0 / 300.0) ** u * scale * scale))
        W = max(16, int(round(w * scale)))
        H = max(16, int(round(h * scale)))
        f = make_frame("c1", seed=seed0 + i, W=W, H=H, nstars=max(1, n), dtype="u16")
        f.name = f"batch{i}_{W}x{H}"
        out.append(f)
    return out


def arrival_stream(rate: float = 4.0, duration: float = 60.0, seed: int = 5):
    """Poisson arrival times (s) and shape classes ('c1','c2','c3') drawn uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, times, kinds = 0.0, [], []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        times.append(t)
        kinds.append(["c1", "c2", "c3"][int(rng.integers(0, 3))])
    return np.array(times), kinds


# ----------------------------------------------------------------------------
# Device-side rendering for the large batch / stream workloads (seconds in
# numpy become milliseconds on the GPU).  Same scene recipe as the c1 frames:
# sky 1000 + 0.05 x, erf-integrated Gaussian stars (FWHM 3), power-law fluxes,
# Poisson counts (gain 1) plus N(0, 10^2) read noise; uint16 by rounding and
# clipping.  Positions and fluxes come from numpy PCG64 (seeded); the noise
# from a seeded torch generator on the device.
# ----------------------------------------------------------------------------
def render_gpu(W: int, H: int, nstars: int, seed: int, fwhm: float = 3.0, dtype: str = "u16",
               device: str = "cuda"):
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = rng.uniform(0, W, nstars)
    ys = rng.uniform(0, H, nstars)
    fl = _powerlaw_fluxes(rng, nstars)
    dev = torch.device(device)
    x = torch.arange(W, device=dev, dtype=torch.float32)
    img = (1000.0 + 0.05 * x)[None, :].repeat(H, 1)
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    hw = int(math.ceil(6.0 * fwhm))
    k = torch.arange(-hw, hw + 1, device=dev, dtype=torch.float64)
    inv = 1.0 / (s * math.sqrt(2.0))
    flat = img.view(-1)
    for c0 in range(0, nstars, 4096):
        x0 = torch.as_tensor(xs[c0:c0 + 4096], device=dev)
        y0 = torch.as_tensor(ys[c0:c0 + 4096], device=dev)
        f0 = torch.as_tensor(fl[c0:c0 + 4096], device=dev)
        px = torch.round(x0)[:, None] + k[None, :]
        py = torch.round(y0)[:, None] + k[None, :]
        gx = 0.5 * (torch.erf((px + 0.5 - x0[:, None]) * inv) - torch.erf((px - 0.5 - x0[:, None]) * inv))
        gy = 0.5 * (torch.erf((py + 0.5 - y0[:, None]) * inv) - torch.erf((py - 0.5 - y0[:, None]) * inv))
        st = f0[:, None, None] * gy[:, :, None] * gx[:, None, :]
        X = px[:, None, :].expand_as(st)
        Y = py[:, :, None].expand_as(st)
        ok = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
        idx = (Y[ok] * W + X[ok]).long()
        flat.index_add_(0, idx, st[ok].float())
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    out = torch.poisson(img.clamp_min(0), generator=g)
    out += 10.0 * torch.randn(img.shape, device=dev, generator=g)
    if dtype == "u16":
        return torch.round(out).clamp(0, 65535).to(torch.int32).to(torch.uint16)
    return out.float()


def batch_shapes(count_scale: float = 1.0, seed0: int = 1000):
    """(W, H, nstars, seed) of the 64-frame uneven batch: 24 x 2048^2,
    24 x 4096^2, 16 x 9600x6400, log-uniform 300..40,000 stars each."""
    shapes = [(2048, 2048)] * 24 + [(4096, 4096)] * 24 + [(9600, 6400)] * 16
    if count_scale != 1.0:
        keep = max(1, int(round(len(shapes) * count_scale)))
        idx = np.linspace(0, len(shapes) - 1, keep).round().astype(int)
        shapes = [shapes[i] for i in idx]
    out = []
    for i, (w, h) in enumerate(shapes):
        r = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(round(300.0 * (40000.0 / 300.0) ** r.random()))
        out.append((w, h, n, seed0 + i))
    return out


def psf_model(nmodes: int = 5, size: int = 9, fwhm: float = 3.0, seed: int = 0) -> np.ndarray:
    """A reference kernel plus nmodes eigenmodes, float32 (nmodes + 1, size,
    size): the reference is a unit-sum circular Gaussian, the modes are
    zero-sum deviation patterns (the Gaussian times dx, dy, dx^2 - dy^2,
    dx dy, r^2 - <r^2>, then random smooth patterns), each scaled to a peak of
    a few percent of the reference's, as a PCA of star stamps about their
    mean gives.  Synthetic stand-in for a fitted eigen-PSF model."""
    rng = np.random.default_rng(seed)
    g = gaussian_kernel(size, fwhm).astype(np.float64)
    g /= g.sum()
    h = size // 2
    yy, xx = np.mgrid[-h:h + 1, -h:h + 1].astype(np.float64)
    shapes = [xx, yy, xx * xx - yy * yy, xx * yy, xx * xx + yy * yy]
    out = [g]
    for k in range(nmodes):
        base = shapes[k] if k < len(shapes) else rng.normal(0, 1, (size, size))
        e = base * g
        e -= e.mean()
        e *= rng.uniform(0.02, 0.05) * g.max() / max(np.abs(e).max(), 1e-30)
        out.append(e)
    return np.ascontiguousarray(np.stack(out), dtype=np.float32)


def coef_maps(nmodes: int, W: int, H: int, bin: int = 1, seed: int = 0) -> np.ndarray:
    """Smooth coefficient maps, float32 (nmodes, ceil(H / bin), ceil(W /
    bin)): low-order polynomials of the normalised position with O(1)
    amplitude, evaluated at each bin's first pixel (the amplitudes of the PSF
    modes vary slowly over a wide field)."""
    rng = np.random.default_rng(seed)
    ny, nx = -(-H // bin), -(-W // bin)
    v = (np.arange(ny) * bin / max(H, 1))[:, None] - 0.5
    u = (np.arange(nx) * bin / max(W, 1))[None, :] - 0.5
    out = np.empty((nmodes, ny, nx))
    for k in range(nmodes):
        c = rng.normal(0, 1, 6)
        out[k] = c[0] + c[1] * u + c[2] * v + c[3] * u * u + c[4] * u * v + c[5] * v * v
    return np.ascontiguousarray(out, dtype=np.float32)


def coef_maps_gpu(torch, nmodes: int, W: int, H: int, seed: int = 0, device: str = "cuda"):
    """coef_maps at full resolution (bin 1), rendered on the device as one
    float32 tensor (nmodes, H, W) (large frames: no host round trip)."""
    rng = np.random.default_rng(seed)
    v = (torch.arange(H, device=device, dtype=torch.float32) / max(H, 1) - 0.5)[:, None]
    u = (torch.arange(W, device=device, dtype=torch.float32) / max(W, 1) - 0.5)[None, :]
    out = torch.empty(nmodes, H, W, device=device, dtype=torch.float32)
    for k in range(nmodes):
        c = [float(x) for x in rng.normal(0, 1, 6)]
        out[k] = c[0] + c[1] * u + c[2] * v + c[3] * u * u + c[4] * u * v + c[5] * v * v
    return out
