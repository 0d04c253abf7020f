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
TOL_B64_ABS = 1e-9      # FP64 background map against the oracle's spline, ADU
TOL_R64_REL = 1e-12     # FP64 noise map against the oracle's spline, relative
TOL_CEN = 1e-4          # centroid, px
TOL_MOM_ABS = 1e-4      # second moments, px^2 (+ 1e-6 relative)
# a threshold decision within this relative margin may go either way in FP32
AMBIG_T = 1e-5
# mesh decisions: relative margins of the clip test (|v - med| against k sigma,
# evaluated in FP32 from a correctly rounded threshold and difference: at most
# about 2^-23 relative) and of the estimator test (FP64 on the GPU); a decision
# inside this band may go either way, and the oracle is re-run with it flipped
AMBIG_MESH = 1e-6
# FP32 rounding unit; the exact-overlap weight of a pixel cut by a circle of
# radius r is computed from coordinates of magnitude <= r + 1 and is trusted to
# EPS_W_ULPS units of u (r + 1) absolute (a float32 emulation of the formula
# against the exact oracle area peaks at 1.3 u (r + 1))
U32 = 2.0 ** -24
U64 = 2.0 ** -53
EPS_W_ULPS = 8.0


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


def _mesh_close(gb, gr, gi, st):
    ok_b = abs(gb - st["back"]) <= TOL_BKG_REL * abs(st["back"])
    ok_r = abs(gr - st["rms"]) <= TOL_BKG_REL * abs(st["rms"])
    return bool(ok_b and ok_r and int(gi) == int(st["iters"]))


def mesh_match(vals, gb, gr, gi, p, plain=None):
    """Check one mesh's GPU statistics (back, rms, clipping passes) against the
    oracle.  A mesh with a decision inside the rounding band may take either
    branch: the oracle is re-run with each such decision flipped and the GPU
    must match one of the results.  Returns the oracle result matched and
    whether it was a flipped one; raises AssertionError when none matches."""
    st = plain if plain is not None else oracle_mesh_one(vals, p)
    if _mesh_close(gb, gr, gi, st):
        return st, False
    if st["margin_clip"] < AMBIG_MESH or st["margin_mode"] < AMBIG_MESH:
        import oracle
        for v in oracle.mesh_variants(vals, AMBIG_MESH, AMBIG_MESH, p.clip_sigma, p.crowd_tol, p.mode_a,
                                      p.mode_b, p.max_iter)[1:]:
            if _mesh_close(gb, gr, gi, v):
                return v, True
    raise AssertionError(f"mesh: GPU back {gb!r} rms {gr!r} passes {gi} vs oracle back {st['back']!r} "
                         f"rms {st['rms']!r} passes {st['iters']} (margins {st['margin_clip']:.3g}, "
                         f"{st['margin_mode']:.3g}), no branch variant matches")


def oracle_mesh_one(vals, p):
    import oracle
    return oracle.mesh_one(vals, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b, p.max_iter)


def check_meshes(img, g, p, picks=None):
    """Every mesh of the frame (or the (j, i) in picks) against the oracle with
    mesh_match.  Returns the raw grids the oracle accepts (each mesh's matched
    branch, for an oracle chain downstream) and the number of meshes matched by
    a flipped branch."""
    H, W = img.shape
    ny, nx = g["back_raw"].shape
    back = np.full((ny, nx), np.nan)
    rms = np.full((ny, nx), np.nan)
    flipped = 0
    cells = picks if picks is not None else [(j, i) for j in range(ny) for i in range(nx)]
    for (j, i) in cells:
        x0, y0 = i * p.mesh_w, j * p.mesh_h
        vals = img[y0:min(y0 + p.mesh_h, H), x0:min(x0 + p.mesh_w, W)].astype(np.float64)
        st, fl = mesh_match(vals, g["back_raw"][j, i], g["rms_raw"][j, i], g["iters"][j, i], p)
        back[j, i], rms[j, i] = st["back"], st["rms"]
        flipped += fl
    return back, rms, flipped


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


def cmp_phot(gphot, ophot, cond, cond_ann, allow, tag=""):
    """GPU photometry vs oracle.  cond[k, j] = sum w |M| of aperture j and
    cond_ann = the annulus' weighted mean |M| (the conditions of the sums);
    allow = weight_allowance(...): what the FP32 weights of cut pixels may add,
    from the oracle's geometry and M alone."""
    err = {}
    if len(ophot["flux"]) == 0:
        return err
    da = np.abs(gphot["area"] - ophot["area"])
    err["area"] = float(da.max())
    assert np.all(da <= 1e-6 * np.maximum(ophot["area"], 1.0)), (tag, "area", da.max())
    db = np.abs(gphot["bkg"] - ophot["bkg"])
    err["bkg"] = float(np.max(db / np.maximum(cond_ann, 1e-300)))
    tol_b = TOL_FLUX_REL * np.maximum(np.abs(ophot["bkg"]), cond_ann) + allow["bkg"] + 1e-12
    assert np.all(db <= tol_b), (tag, "bkg", err["bkg"])
    df = np.abs(gphot["flux"] - ophot["flux"])
    scale = cond + np.abs(ophot["bkg"])[:, None] * ophot["area"]
    err["flux"] = float(np.max(df / np.maximum(scale, 1e-300)))
    err["flux_allow_share"] = float(np.max(allow["flux"] / np.maximum(scale, 1e-300)))
    tol = TOL_FLUX_REL * np.maximum(np.abs(ophot["flux"]), scale) + allow["flux"]
    assert np.all(df <= tol), (tag, "flux", err["flux"], float(np.max(df - tol)))
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


def _near_circle(M, xc, yc, r):
    """sum |M| and count over the frame pixels a circle of radius r may cut:
    nearest corner within r (1 + 1e-6) and farthest beyond r (1 - 1e-6)."""
    H, W = M.shape
    x0, x1 = max(int(np.floor(xc - r - 1)), 0), min(int(np.ceil(xc + r + 1)) + 1, W)
    y0, y1 = max(int(np.floor(yc - r - 1)), 0), min(int(np.ceil(yc + r + 1)) + 1, H)
    if x0 >= x1 or y0 >= y1:
        return 0.0, 0
    yy, xx = np.mgrid[y0:y1, x0:x1]
    ax, ay = np.abs(xx - xc), np.abs(yy - yc)
    dmin = np.hypot(np.maximum(ax - 0.5, 0.0), np.maximum(ay - 0.5, 0.0))
    dmax = np.hypot(ax + 0.5, ay + 0.5)
    near = (dmin <= r * (1 + 1e-6)) & (dmax >= r * (1 - 1e-6))
    return float(np.abs(M[y0:y1, x0:x1][near]).sum()), int(near.sum())


def weight_allowance(M, xs, ys, p, ophot, precision=0):
    """What the exact-overlap weights, computed in FP32 (precision 0) or FP64,
    may add to the flux and annulus errors: every pixel a circle of radius r
    cuts carries a weight error of at most EPS_W_ULPS u (r + 1), so
      raw_k        <- eps_k sum_cut(k) |M|,     A_k <- eps_k n_cut(k)
      annulus mean <- (eps_in S_in + eps_out S_out + |bkg| (eps_in n_in + eps_out n_out)) / A_ann
      flux_k       <- raw_k + |bkg| A_k-term + A_k (annulus term).
    Only the oracle's M, centres and photometry enter."""
    u = U32 if precision == 0 else U64
    eps = lambda r: EPS_W_ULPS * u * (r + 1.0)
    n = len(xs)
    nr = len(p.radii)
    af = np.zeros((n, nr))
    ab = np.zeros(n)
    for k in range(n):
        xc, yc = float(xs[k]), float(ys[k])
        bk = abs(float(ophot["bkg"][k]))
        s_in, n_in = _near_circle(M, xc, yc, p.r_in)
        s_out, n_out = _near_circle(M, xc, yc, p.r_out)
        a_ann = np.pi * (p.r_out ** 2 - p.r_in ** 2)
        ab[k] = (eps(p.r_in) * (s_in + bk * n_in) + eps(p.r_out) * (s_out + bk * n_out)) / a_ann
        for j, r in enumerate(p.radii):
            s_j, n_j = _near_circle(M, xc, yc, r)
            af[k, j] = eps(r) * (s_j + bk * n_j) + float(ophot["area"][k, j]) * ab[k]
    return {"flux": af, "bkg": ab}


def peak_ambiguous(F, R, t, sep):
    """Pixels whose peak decision FP32 may take either way: the threshold test
    within the rounding band, or nu = F / R within 1e-5 (relative) of the
    largest other nu of its window."""
    from scipy import ndimage
    nu = np.where(R > 0, F / np.where(R > 0, R, 1.0), F)
    H, W = nu.shape
    best = np.full_like(nu, -np.inf)
    pad = np.pad(nu, sep, mode="constant", constant_values=-np.inf)
    for dy in range(-sep, sep + 1):
        for dx in range(-sep, sep + 1):
            if dx == 0 and dy == 0:
                continue
            best = np.maximum(best, pad[sep + dy:sep + dy + H, sep + dx:sep + dx + W])
    close = np.abs(nu - best) <= AMBIG_T * (np.abs(nu) + np.abs(best))
    return thresh_ambiguous(F, R, t) | (close & (F > t * R))


def growth_allowance(A, xs, ys, radii):
    """What the FP64 top-hat taps of cut pixels may differ by between the two
    sides, as (sum over cut pixels of |A| times it, cut-pixel count times it)
    per source and radius.  The oracle's tap is a signed sum of four corner
    integrals, each a sum of up to three terms of magnitude <= r^2, each
    rounded within a few units of 2^-53 (32 u r^2 in all; the same formula in
    long double puts the largest actual difference at 15.6 u r^2, radius
    32); the device's cancellation-free area is within 8 u (r + 1).  Only the oracle-side frame and positions enter: the
    circle is centred on the pixel holding the position."""
    n, nr = len(xs), len(radii)
    sa = np.zeros((n, nr))
    na = np.zeros((n, nr))
    H, W = A.shape
    R = max(radii)
    for i in range(n):
        fx, fy = np.floor(xs[i] + 0.5), np.floor(ys[i] + 0.5)
        if not (np.isfinite(fx) and np.isfinite(fy)) or not (-R - 1 <= fx <= W + R and -R - 1 <= fy <= H + R):
            continue
        for j, r in enumerate(radii):
            e = 32 * U64 * r * r + EPS_W_ULPS * U64 * (r + 1.0)
            s, c = _near_circle(A, float(fx), float(fy), float(r))
            sa[i, j] = e * s
            na[i, j] = e * c
    return sa, na
