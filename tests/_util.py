"""Helpers shared by the parity tests (comparison, ambiguity, GPU runs)."""
from __future__ import annotations

import dataclasses
import math
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# tolerances of the contract
TOL_BKG_REL = 1e-5      # background and rms maps / grids, relative
TOL_FLUX_REL = 1e-6     # fluxes, relative to the sum's condition sum(w |M|)
TOL_CEN = 1e-4          # centroid, px
TOL_MOM_ABS = 1e-4      # second moments, px^2 (+ 1e-6 relative)
# a threshold decision within this relative margin may go either way in FP32
AMBIG_T = 1e-5
# mesh decisions: relative margins of the clip and estimator tests
AMBIG_MESH = 1e-5


def f32(x):
    return float(np.float32(x))


def f32_params(p):
    """Parameters as the GPU sees them (its ABI carries them as float32)."""
    q = dataclasses.replace(p)
    for k in ("clip_sigma", "crowd_tol", "mode_a", "mode_b", "thresh", "r_in", "r_out", "gain"):
        setattr(q, k, f32(getattr(p, k)))
    q.radii = tuple(f32(r) for r in p.radii)
    if math.isfinite(p.sat_level):
        q.sat_level = f32(p.sat_level)
    return q


def header_functions():
    """Function names declared in include/gp.h."""
    txt = open(os.path.join(ROOT, "include", "gp.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gp_status|void|const char\*)\s+(gp_\w+)\s*\(", txt, re.M)))


def mesh_ambiguous(st):
    return (st["margin_clip"] < AMBIG_MESH) | (st["margin_mode"] < AMBIG_MESH)


def thresh_ambiguous(F, R, t):
    return np.abs(F - t * R) <= AMBIG_T * (np.abs(F) + t * np.abs(R))


def gpu_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def cmp_catalog(gcat, ocat, M, seg, tag=""):
    """GPU catalogue vs oracle measurements of the same labels."""
    n = len(ocat["npix"])
    assert len(gcat["npix"]) == n, (tag, len(gcat["npix"]), n)
    if n == 0:
        return {}
    for k in ("npix", "xmin", "xmax", "ymin", "ymax", "pmin"):
        np.testing.assert_array_equal(gcat[k].astype(np.int64), ocat[k].astype(np.int64), err_msg=f"{tag} {k}")
    np.testing.assert_array_equal(gcat["flags"] & 7, ocat["flags"] & 7, err_msg=f"{tag} flags")
    # condition of the sums: sum |M| over each object
    absM = np.bincount(seg[seg > 0].ravel() - 1, weights=np.abs(M[seg > 0]).ravel(), minlength=n)
    err = {}
    dflux = np.abs(gcat["flux"] - ocat["flux"])
    err["flux"] = float(np.max(dflux / np.maximum(absM, 1e-300)))
    assert np.all(dflux <= TOL_FLUX_REL * np.maximum(np.abs(ocat["flux"]), absM)), (tag, err["flux"])
    for k in ("x", "y"):
        d = np.abs(gcat[k] - ocat[k])
        err[k] = float(d.max())
        assert np.all(d <= TOL_CEN), (tag, k, d.max())
    for k in ("x2", "y2", "xy"):
        d = np.abs(gcat[k] - ocat[k])
        err[k] = float(d.max())
        assert np.all(d <= TOL_MOM_ABS + 1e-6 * np.abs(ocat[k])), (tag, k, d.max())
    dp = np.abs(gcat["peak"].astype(np.float64) - ocat["peak"])
    assert np.all(dp <= 1e-6 * np.abs(ocat["peak"]) + 1e-3), (tag, "peak", dp.max())
    return err


def cmp_phot(gphot, ophot, cond, cond_ann, tag="", mmax=None):
    """GPU photometry vs oracle; cond[k, j] = sum w |M| of aperture j, cond_ann
    = the annulus' weighted mean |M|; mmax[k] = max |M| near object k (a pixel
    the circle barely touches may get a weight of ~1e-7 on one side and 0 on
    the other: that difference, at most the area error times max |M|, is
    allowed on top of the relative tolerance)."""
    err = {}
    if len(ophot["flux"]) == 0:
        return err
    da = np.abs(gphot["area"] - ophot["area"])
    err["area"] = float(da.max())
    assert np.all(da <= 1e-6 * np.maximum(ophot["area"], 1.0)), (tag, "area", da.max())
    db = np.abs(gphot["bkg"] - ophot["bkg"])
    err["bkg"] = float(np.max(db / np.maximum(cond_ann, 1e-300)))
    assert np.all(db <= TOL_FLUX_REL * np.maximum(np.abs(ophot["bkg"]), cond_ann) + 1e-12), (tag, "bkg", err["bkg"])
    df = np.abs(gphot["flux"] - ophot["flux"])
    scale = cond + np.abs(ophot["bkg"])[:, None] * ophot["area"]
    floor = 0.0 if mmax is None else da * np.asarray(mmax)[:, None]
    err["flux"] = float(np.max(np.maximum(df - floor, 0) / np.maximum(scale, 1e-300)))
    assert np.all(df <= TOL_FLUX_REL * np.maximum(np.abs(ophot["flux"]), scale) + floor), (tag, "flux", err["flux"])
    if "fluxerr" in ophot and np.any(ophot["fluxerr"]):
        de = np.abs(gphot["fluxerr"] - ophot["fluxerr"])
        err["fluxerr"] = float(np.max(de / np.maximum(ophot["fluxerr"], 1e-300)))
        assert np.all(de <= 1e-5 * ophot["fluxerr"] + 1e-9), (tag, "fluxerr", err["fluxerr"])
    return err


def phot_condition(M, xs, ys, p):
    """sum w |M| per aperture and the annulus mean |M| (oracle on |M|)."""
    import oracle
    o = oracle.aperture(np.abs(M), None, xs, ys, list(p.radii), p.r_in, p.r_out, want_err=False)
    raw = o["flux"] + o["bkg"][:, None] * o["area"]
    return raw, np.abs(o["bkg"])


def box_max_abs(M, xs, ys, r):
    """max |M| over the pixels within r + 1 of each centre (inside the frame)."""
    H, W = M.shape
    out = np.zeros(len(xs))
    for i, (x, y) in enumerate(zip(xs, ys)):
        x0, x1 = max(int(np.floor(x - r - 1)), 0), min(int(np.ceil(x + r + 1)) + 1, W)
        y0, y1 = max(int(np.floor(y - r - 1)), 0), min(int(np.ceil(y + r + 1)) + 1, H)
        if x0 < x1 and y0 < y1:
            out[i] = np.abs(M[y0:y1, x0:x1]).max()
    return out
