"""GPU path vs the FP64 oracle, through the C ABI (needs an MI355X).

Stage-isolated checks feed each GPU stage the oracle's upstream output, so a
difference is attributable to that stage; decisions whose margins fall below
FP32 rounding (mesh clip / estimator tests, threshold tests) are excluded and
counted, everything else must match to the stated tolerances, labels bit for
bit.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from synth import Params, gaussian_kernel, make_frame
from tests._util import (AMBIG_T, TOL_B64_ABS, TOL_BKG_REL, TOL_R64_REL, TOL_CEN, TOL_MOM_ABS, check_meshes, cmp_catalog, cmp_phot, f32_params,
                         growth_allowance, mesh_ambiguous, peak_ambiguous, phot_condition, thresh_ambiguous, weight_allowance)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    from paper_2609_32375_amd import pipeline
    return pipeline


def _dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def _params(name="c1", **kw):
    from synth import config_params
    p = config_params(name)
    for k, v in kw.items():
        setattr(p, k, v)
    return f32_params(p)


# ----------------------------------------------------------------------------
# mesh statistics and the background interpolation
# ----------------------------------------------------------------------------
MESH_CASES = [
    ("c1", 300, 200, "f32", 64, 64, 0),
    ("c1", 257, 131, "u16", 64, 64, 1),
    ("c2", 390, 270, "f32", 128, 128, 2),
    ("c1", 200, 150, "f32", 17, 23, 3),
    ("c1", 40, 30, "f32", 64, 64, 4),        # frame smaller than one mesh
    ("c1", 300, 250, "u16", 96, 80, 5),      # 7680-pixel meshes: the 512 x 16 launch shape
]


def _structured_meshes(m, seed):
    """A frame of 4 x 2 meshes of m x m float32 pixels, each with a value
    distribution that stresses one part of the clipping loop: heavy ties
    (2 integer levels), a bright source over a third of the mesh (the median
    moves far between passes), tiny values of both signs, a two-level mesh,
    a bimodal mixture, a Gaussian sky with a few saturated pixels, a bright
    compact star and a steep gradient."""
    rng = np.random.default_rng(seed)
    n = m * m
    ties = 1000.0 + rng.integers(0, 2, n)
    ties[rng.choice(n, n // 50, replace=False)] = 60000.0
    src = 500.0 + 5.0 * rng.standard_normal(n)
    src[: n // 3] += 800.0 + 200.0 * rng.standard_normal(n // 3)
    tiny = 1e-3 * rng.standard_normal(n)
    two = np.where(rng.random(n) < 0.7, 3.0, 7.0)
    bim = np.concatenate([100.0 + rng.standard_normal(n - n // 4), 140.0 + rng.standard_normal(n // 4)])
    rng.shuffle(bim)
    sat = 2000.0 + 30.0 * rng.standard_normal(n)
    sat[rng.choice(n, 40, replace=False)] = 65535.0
    # a bright compact star with a bleed trail: many clipping passes, whole
    # per-thread runs (columns) above the clip window, the median drifting down
    yy, xx = np.mgrid[0:m, 0:m]
    rr2 = (xx - 0.4 * m) ** 2 + (yy - 0.55 * m) ** 2
    star = 800.0 + 40.0 * rng.standard_normal((m, m)) + 60000.0 / (1.0 + rr2 / 9.0) ** 1.5
    star[:, int(0.4 * m) - 2: int(0.4 * m) + 3] += 30000.0       # its bleed trail, full height
    star = np.minimum(star, 65535.0).ravel()
    ramp = (300.0 + 4000.0 * xx / m + 20.0 * rng.standard_normal((m, m))).ravel()
    blocks = [x.reshape(m, m) for x in (ties, src, tiny, two, bim, sat, star, ramp)]
    img = np.block([[blocks[0], blocks[1], blocks[2], blocks[3]], [blocks[4], blocks[5], blocks[6], blocks[7]]])
    return np.ascontiguousarray(img.astype(np.float32))


@pytest.mark.parametrize("m", [64, 128])
def test_mesh_statistics_structured(P, m):
    """Tie-heavy, drifting, tiny, two-level and bimodal meshes (4096 and 16384
    pixels: both launch shapes of the statistics kernel)."""
    _say("structured meshes", m)
    img = _structured_meshes(m, 7 + m)
    p = _params("c1", mesh_w=m, mesh_h=m, mesh_filter=1)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=64)
    ph.background()
    g = ph.grids(0)
    # every mesh: those with a decision inside the rounding band must match
    # the oracle re-run with that decision taken either way
    _, _, flipped = check_meshes(img, g, p)
    st = oracle.mesh_stats(img.astype(np.float64), m, m, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b, p.max_iter)
    _say("ambiguous", int(mesh_ambiguous(st).sum()), "matched a flipped branch", flipped,
         "iters", st["iters"].ravel().tolist())
    ph.close()


def _structured_meshes_u16(m, seed):
    """uint16 meshes (4 x 3 of m x m) for the integer statistics kernel: the
    float structured set rounded and clipped (ties, a bright source over a
    third, two levels, bimodal, saturated pixels, a saturated star with a
    bleed trail, a steep ramp), plus a Gaussian sky, values spread over the
    whole 16-bit range, a tight cluster with a far saturated block, and a
    mesh of one value plus a single different pixel."""
    base = _structured_meshes(m, seed).astype(np.float64)
    blocks = [base[:m, i * m:(i + 1) * m] for i in range(4)] + [base[m:, i * m:(i + 1) * m] for i in range(4)]
    blocks[2] = 20.0 + blocks[2] * 1e4                   # the tiny mesh, lifted into integers
    rng = np.random.default_rng(seed + 1)
    n = m * m
    sky = (1000.0 + 33.0 * rng.standard_normal(n)).reshape(m, m)
    spread = rng.uniform(0, 65535, n).reshape(m, m)
    far = (500.0 + 3.0 * rng.standard_normal(n))
    far[: n // 10] = 65535.0
    rng.shuffle(far)
    one = np.full(n, 4321.0)
    one[n // 2] = 4400.0
    blocks += [sky, spread, far.reshape(m, m), one.reshape(m, m)]
    img = np.block([blocks[0:4], blocks[4:8], blocks[8:12]])
    return np.ascontiguousarray(np.clip(np.rint(img), 0, 65535).astype(np.uint16))


@pytest.mark.parametrize("m", [64, 96, 128])
def test_mesh_statistics_structured_u16(P, m):
    """The integer statistics kernel of uint16 frames on meshes that stress
    its window, bisection and interval paths (4096, 9216 and 16384 pixels)."""
    _say("structured uint16 meshes", m)
    img = _structured_meshes_u16(m, 17 + m)
    p = _params("c1", mesh_w=m, mesh_h=m, mesh_filter=1)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=64)
    ph.background()
    g = ph.grids(0)
    _, _, flipped = check_meshes(img, g, p)
    st = oracle.mesh_stats(img.astype(np.float64), m, m, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b, p.max_iter)
    _say("ambiguous", int(mesh_ambiguous(st).sum()), "flipped", flipped, "iters", st["iters"].ravel().tolist())
    ph.close()


@pytest.mark.parametrize("case", MESH_CASES, ids=lambda c: f"{c[0]}-{c[1]}x{c[2]}-{c[3]}-m{c[4]}x{c[5]}")
def test_mesh_statistics_match_oracle(P, case):
    name, W, H, dt, mw, mh, seed = case
    _say("mesh case", case)
    fr = make_frame(name, seed=100 + seed, W=W, H=H, dtype=dt)
    p = _params(name, mesh_w=mw, mesh_h=mh)
    img = fr.image
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=64)
    ph.background()
    g = ph.grids(0)
    _, _, flipped = check_meshes(img, g, p)
    st = oracle.mesh_stats(img.astype(np.float64), mw, mh, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b, p.max_iter)
    _say("meshes", st["back"].size, "ambiguous", int(mesh_ambiguous(st).sum()), "matched a flipped branch", flipped)
    # the grid filter is exact given the same raw grid
    np.testing.assert_array_equal(g["back"], oracle.median_filter(g["back_raw"], p.mesh_filter))
    np.testing.assert_array_equal(g["rms"], oracle.median_filter(g["rms_raw"], p.mesh_filter))
    ph.close()


@pytest.mark.parametrize("f", [1, 3, 5, 7])
@pytest.mark.parametrize("W", [700, 4200])
def test_grid_filter_every_size(P, f, W):
    # sizes 1-5 keep the window in registers, 7 in LDS; ragged grid edges.
    # 22 x 14 meshes: sizes 1-5 run inside the y-spline launch; 132 x 14 (more
    # than 127 knots along x) and size 7: the separate filter kernel
    fr = make_frame("c1", seed=5, W=W, H=430, dtype="f32")
    p = _params("c1", mesh_w=32, mesh_h=32, mesh_filter=f)
    ph = P.Photometry([_dev(fr.image)], p, p.kernel(), capacity=64)
    ph.background()
    g = ph.grids(0)
    np.testing.assert_array_equal(g["back"], oracle.median_filter(g["back_raw"], f))
    np.testing.assert_array_equal(g["rms"], oracle.median_filter(g["rms_raw"], f))
    ph.close()


# the splines by knots on the solved axis: up to 63 one wavefront per spline
# (5x4, 5x5, 1x1, 8x3, 2x63, 63x3, 63x63 with ragged last meshes), 64 to 127
# one workgroup (64x3, 100x2, 107x3, 3x107, 127x127), above 127 the Thomas
# kernels, with up to 100 knots in LDS and longer axes on global scratch
# (132x3: x on global scratch, y in LDS; 3x132: the converse)
@pytest.mark.parametrize("shape", [(300, 200, 64, 64), (130, 77, 32, 16), (50, 20, 64, 64), (1000, 40, 128, 16),
                                   (100, 2000, 64, 32), (1008, 40, 16, 16), (1003, 999, 16, 16),
                                   (1024, 40, 16, 16), (1600, 24, 16, 16), (1700, 40, 16, 16), (40, 1700, 16, 16),
                                   (2025, 2030, 16, 16), (2100, 40, 16, 16), (40, 2100, 16, 16)])
def test_background_maps_match_oracle_spline(P, shape):
    W, H, mw, mh = shape
    _say("map case", shape)
    rng = np.random.default_rng(W + H)
    nx, ny = -(-W // mw), -(-H // mh)
    back = 1000 + 30 * rng.standard_normal((ny, nx))
    rms = 20 + 3 * rng.random((ny, nx))
    img = np.zeros((H, W), np.float32)
    p = _params("c1", mesh_w=mw, mesh_h=mh)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=16)
    ph.set_grids(0, back, rms)
    ph.background(grid_given=True)
    B, R = ph.maps(0)
    Bo = oracle.grid_map(back, W, H, mw, mh)
    Ro = oracle.grid_map(rms, W, H, mw, mh)
    eb = np.abs(B - Bo).max()
    er = (np.abs(R - Ro) / np.abs(Ro)).max()
    _say("max |dB|", eb, "max rel dR", er)
    assert eb <= 5e-5                      # ADU: ~5e-8 relative, far inside 1e-5
    assert er <= TOL_BKG_REL
    B64, R64 = ph.maps(0, precision=1)
    assert np.abs(B64 - Bo).max() <= TOL_B64_ABS and (np.abs(R64 - Ro) / Ro).max() <= TOL_R64_REL
    ph.close()


def test_constant_sky_gives_constant_background(P):
    img = np.full((150, 220), 812.5, np.float32)
    p = _params("c1", mesh_w=32, mesh_h=32)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=16)
    ph.background()
    ph.detect()
    B, R = ph.maps(0)
    assert np.all(B == 812.5) and np.all(R == 0.0)
    r = ph.results(0)
    assert r["n_obj"] == 0 and r["status"] == 0
    ph.close()


# ----------------------------------------------------------------------------
# labelling: a given mask through constant sky, zero rms and a delta kernel
# ----------------------------------------------------------------------------
def _mask_cases():
    rng = np.random.default_rng(0)
    cases = []
    for d in (0.02, 0.3, 0.55, 0.9):
        cases.append((f"rand{d}", rng.random((150, 200)) < d))
    full = np.ones((130, 129), bool)
    cases.append(("full", full))
    cases.append(("empty", np.zeros((70, 70), bool)))
    checker = (np.add.outer(np.arange(100), np.arange(140)) % 2).astype(bool)
    cases.append(("checker", checker))
    snake = np.zeros((140, 200), bool)
    for r in range(0, 140, 2):
        snake[r, :] = True
        if r + 1 < 140:
            snake[r + 1, 199 if (r // 2) % 2 == 0 else 0] = True
    cases.append(("snake", snake))
    # diagonal chains across tile corners
    diag = np.zeros((200, 200), bool)
    for i in range(200):
        diag[i, i] = True
        diag[i, 199 - i] = True
    cases.append(("diag", diag))
    # anti-diagonal stripes: long 8-connected chains through every tile (deep
    # union-find trees, concurrent finds)
    yy, xx = np.mgrid[0:256, 0:256]
    cases.append(("stripes", (xx + yy) % 7 == 0))
    tiny = rng.random((3, 5)) < 0.5
    cases.append(("tiny", tiny))
    one = np.ones((1, 1), bool)
    cases.append(("one", one))
    return cases


@pytest.mark.parametrize("mesh", [16, 64])   # 64: row cubics of at most 4 pieces, union pairs in less LDS
@pytest.mark.parametrize("conn", [8, 4])
@pytest.mark.parametrize("case", _mask_cases(), ids=lambda c: c[0])
def test_labels_bit_exact_for_given_mask(P, case, conn, mesh):
    name, mask = case
    _say("mask case", name, conn, mesh)
    H, W = mask.shape
    c, A = 500.0, 100.0
    rng = np.random.default_rng(H * W)
    amp = A + 50.0 * rng.random(mask.shape)
    img = (c + np.where(mask, amp, 0.0)).astype(np.float32)
    minarea = 3
    p = _params("c1", mesh_w=mesh, mesh_h=mesh, conn=conn, minarea=minarea, thresh=1.5)
    K = np.zeros((3, 3), np.float32)
    K[1, 1] = 1.0
    nx, ny = -(-W // mesh), -(-H // mesh)
    ph = P.Photometry([_dev(img)], p, K, capacity=max(8, W * H), seg=True)
    ph.set_grids(0, np.full((ny, nx), c), np.zeros((ny, nx)))
    ph.background(grid_given=True)
    seg_o, n_o = oracle.label_mask(mask, conn, minarea)
    M = img.astype(np.float64) - c
    ocat = oracle.measure(img, M, seg_o, n_o)
    for rep in range(3):      # the labelling runs concurrently: repeat it
        ph.detect()
        r = ph.results(0)
        assert r["status"] == 0 and r["comp_status"][0] == 0
        assert r["n_obj"] == n_o
        np.testing.assert_array_equal(r["seg"], seg_o)
        cmp_catalog(r["cat"], ocat, M, seg_o, tag=f"{name} run {rep}")
    ph.close()


# ----------------------------------------------------------------------------
# detection and photometry on star fields, stage-isolated
# ----------------------------------------------------------------------------
FIELD_CASES = [
    ("c1", 320, 256, "f32", 11),
    ("c1", 333, 211, "u16", 12),
    ("c2", 400, 300, "f32", 13),
]


def _field(case):
    name, W, H, dt, seed = case
    nst = max(10, int(W * H / 4e3))
    fr = make_frame(name, seed=seed, W=W, H=H, dtype=dt, nstars=nst)
    p = f32_params(fr.params)
    p.mesh_w = p.mesh_h = 64
    return fr, p


def _kernel_cases():
    """Filter kernels beyond the workloads' own: square Gaussians of every
    separable radius (0..7), a non-square rank-one kernel and two kernels that
    are not rank one (asymmetric random, and a Gaussian with one tap changed by
    1e-5 of its peak), all through the detection kernel's other code paths."""
    rng = np.random.default_rng(77)
    out = [(f"gauss{k}", gaussian_kernel(k, 3.0)) for k in (1, 3, 7, 11, 13, 15)]
    g = np.exp(-0.5 * (np.arange(-1, 2) / 1.2) ** 2)
    h = np.exp(-0.5 * (np.arange(-3, 4) / 1.7) ** 2)
    out.append(("rank1_3x7", np.outer(g, h).astype(np.float32)))
    out.append(("dense_7x5", (0.2 + rng.random((7, 5))).astype(np.float32)))
    near = gaussian_kernel(9, 3.5).copy()
    near[3, 5] += 1e-5 * near.max()
    out.append(("near_rank1_9x9", near))
    return out


def _detect_stage(P, case, prec, K=None):
    fr, p = _field(case)
    img = fr.image
    I = img.astype(np.float64)
    ob = oracle.background(I, p, maps=True)
    M = I - ob.B
    K = p.kernel() if K is None else K
    F = oracle.filter_image(M, K)
    ph = P.Photometry([_dev(img)], p, K, capacity=4096, seg=True, precision=prec)
    ph.set_grids(0, ob.back, ob.rms)
    ph.background(grid_given=True)
    ph.detect()
    r = ph.results(0)
    assert r["status"] == 0 and r["comp_status"][0] == 0
    seg_g = r["seg"]
    mask_g = seg_g != 0
    # the oracle's mask, with every decision inside the rounding band taken the
    # way the GPU took it (both branches are correct there)
    mask_o = F > p.thresh * ob.R
    amb = thresh_ambiguous(F, ob.R, p.thresh)
    diff = mask_g != mask_o
    _say("mask pixels", int(mask_o.sum()), "differ", int(diff.sum()), "ambiguous", int(amb.sum()))
    assert np.all(amb[diff])
    mask_ref = np.where(amb, mask_g, mask_o)
    seg_o, n_o = oracle.label_mask(mask_ref, p.conn, p.minarea)
    np.testing.assert_array_equal(seg_g, seg_o)
    assert r["n_obj"] == n_o
    ocat = oracle.measure(I, M, seg_o, n_o, p.sat_level)
    err = cmp_catalog(r["cat"], ocat, M, seg_o, tag=str(case))
    _say("catalogue errors", err)
    return fr, p, ph, ob, M, ocat


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", FIELD_CASES, ids=lambda c: f"{c[0]}-{c[1]}x{c[2]}-{c[3]}")
def test_detection_stage_isolated(P, case, prec):
    _say("detect case", case, prec)
    fr, p, ph, ob, M, ocat = _detect_stage(P, case, prec)
    # apertures at the oracle's centroids, on the same background
    xs, ys = ocat["x"], ocat["y"]
    ph.set_catalog(0, xs, ys, ocat["flags"])
    ph.aperture()
    r = ph.results(0)
    oph = oracle.aperture(M, ob.R, xs, ys, list(p.radii), p.r_in, p.r_out, p.gain, p.want_err)
    cond, cond_ann = phot_condition(M, xs, ys, p)
    allow = weight_allowance(M, xs, ys, p, oph, precision=prec)
    err = cmp_phot(r["phot"], oph, cond, cond_ann, allow, tag=str(case))
    _say("photometry errors", err)
    trunc = (r["cat"]["flags"] & 8) != 0
    np.testing.assert_array_equal(trunc, (oph["flags"] & 8) != 0)
    ph.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("kcase", _kernel_cases(), ids=lambda c: c[0])
def test_detection_every_filter_path(P, kcase, prec):
    name, K = kcase
    _say("kernel case", name, K.shape, prec)
    case = ("c1", 300, 230, "f32", 17)
    _, _, ph, _, _, _ = _detect_stage(P, case, prec, K=K)
    ph.close()


@pytest.mark.parametrize("case", FIELD_CASES[:2], ids=lambda c: f"{c[0]}-{c[1]}x{c[2]}-{c[3]}")
def test_aperture_stage_isolated_exact_centres(P, case):
    _say("aperture case", case)
    fr, p = _field(case)
    img = fr.image
    I = img.astype(np.float64)
    H, W = img.shape
    ob = oracle.background(I, p, maps=True)
    M = I - ob.B
    rng = np.random.default_rng(5)
    n = 300
    xs = rng.uniform(-3, W + 3, n)
    ys = rng.uniform(-3, H + 3, n)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=n)
    ph.set_grids(0, ob.back, ob.rms)
    ph.background(grid_given=True)
    ph.set_catalog(0, xs, ys)
    ph.aperture()
    r = ph.results(0)
    oph = oracle.aperture(M, ob.R, xs, ys, list(p.radii), p.r_in, p.r_out, p.gain, p.want_err)
    cond, cond_ann = phot_condition(M, xs, ys, p)
    allow = weight_allowance(M, xs, ys, p, oph)
    err = cmp_phot(r["phot"], oph, cond, cond_ann, allow, tag=str(case))
    _say("photometry errors", err)
    np.testing.assert_array_equal((r["cat"]["flags"] & 8) != 0, (oph["flags"] & 8) != 0)
    ph.close()


def test_aperture_constant_image_closed_form(P):
    c = 7.25
    W = H = 120
    img = np.full((H, W), c, np.float32)
    p = _params("c2")
    nx, ny = -(-W // p.mesh_w), -(-H // p.mesh_h)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=64)
    ph.set_grids(0, np.zeros((ny, nx)), np.ones((ny, nx)))
    ph.background(grid_given=True)
    rng = np.random.default_rng(1)
    xs = 60 + rng.uniform(-2, 2, 40)
    ys = 60 + rng.uniform(-2, 2, 40)
    ph.set_catalog(0, xs, ys)
    ph.aperture()
    r = ph.results(0)
    for k, rad in enumerate(p.radii):
        np.testing.assert_allclose(r["phot"]["area"][:, k], math.pi * rad * rad, rtol=2e-7)
        np.testing.assert_allclose(r["phot"]["flux"][:, k], 0.0, atol=1e-6 * c * math.pi * rad * rad)
    np.testing.assert_allclose(r["phot"]["bkg"], c, rtol=1e-7)
    ph.close()


# ----------------------------------------------------------------------------
# whole chain, batches and failure paths
# ----------------------------------------------------------------------------
# ----------------------------------------------------------------------------
# peak detection (the paper's own), stage-isolated
# ----------------------------------------------------------------------------
PEAK_CASES = [
    # name, W, H, dtype, seed, thresh, sep, cwin, kernel
    ("c1", 333, 257, "f32", 51, 1.5, 3, 3, None),
    ("c1", 300, 211, "u16", 52, 5.0, 3, 4, None),
    ("c1", 420, 180, "f32", 53, 3.0, 1, 2, "dense"),
    ("c1", 257, 300, "f32", 54, 2.0, 6, 7, None),
    ("c1", 129, 70, "f32", 55, 1.5, 0, 0, None),
]


def _cmp_peak_catalogues(r, o, M, F, R, thresh, sep):
    """GPU peaks against the oracle's: the two sets differ only at pixels
    whose decisions are ambiguous in FP32 (threshold or window maximum), and
    every common peak agrees field by field."""
    assert r["status"] == 0 and r["comp_status"][0] == 0
    amb = peak_ambiguous(F, R, thresh, sep).ravel()
    g_set, o_set = set(r["cat"]["pmin"].tolist()), set(o["pmin"].tolist())
    diff = sorted(g_set ^ o_set)
    _say("peaks gpu", len(g_set), "oracle", len(o_set), "differ", len(diff), "ambiguous px", int(amb.sum()))
    assert len(o_set) > 3
    assert all(amb[q] for q in diff), [q for q in diff if not amb[q]]
    assert np.all(np.diff(r["cat"]["pmin"]) > 0)
    common = sorted(g_set & o_set)
    gi = {q: i for i, q in enumerate(r["cat"]["pmin"].tolist())}
    oi = {q: i for i, q in enumerate(o["pmin"].tolist())}
    ig = np.array([gi[q] for q in common])
    io = np.array([oi[q] for q in common])
    g, c = r["cat"], {k: v[io] for k, v in o.items() if k != "n"}
    for k in ("npix", "xmin", "xmax", "ymin", "ymax"):
        np.testing.assert_array_equal(g[k][ig], c[k], err_msg=k)
    np.testing.assert_array_equal(g["flags"][ig], c["flags"])
    # flux of the window: tolerance on the sum of |M| over it
    absM = np.array([np.abs(M[c["ymin"][k]:c["ymax"][k] + 1, c["xmin"][k]:c["xmax"][k] + 1]).sum()
                     for k in range(len(io))])
    assert np.all(np.abs(g["flux"][ig] - c["flux"]) <= 1e-6 * np.maximum(np.abs(c["flux"]), absM))
    for k in ("x", "y"):
        assert np.all(np.abs(g[k][ig] - c[k]) <= TOL_CEN), (k, np.abs(g[k][ig] - c[k]).max())
    for k in ("x2", "y2", "xy"):
        assert np.all(np.abs(g[k][ig] - c[k]) <= TOL_MOM_ABS + 1e-6 * np.abs(c[k])), k
    assert np.all(np.abs(g["peak"][ig] - c["peak"]) <= 2e-6 * np.abs(c["peak"]) + 1e-6)
    return len(common)


PSF_CASES = [
    # W, H, dtype, seed, thresh, sep, cwin, nmodes, kernel side, coefficient-map bin
    # [, mesh size (64 if absent)]
    (333, 257, "f32", 91, 3.0, 3, 3, 5, 9, 1),
    (300, 211, "u16", 92, 5.0, 3, 3, 5, 9, 16),
    (257, 190, "f32", 93, 2.0, 2, 4, 8, 15, 7),
    (200, 150, "f32", 94, 2.0, 4, 2, 0, 7, 1),
    (190, 130, "f32", 95, 2.5, 3, 3, 3, (7, 5), 1),   # a non-square kernel
    (400, 300, "f32", 96, 1.0, 2, 2, 5, 13, 1),       # low threshold: hundreds of noise peaks
    # 16-px meshes: the tile's row-cubic table (8 pieces a row) is larger
    # than nu, which it shares in the varying filter's LDS layout
    (300, 220, "f32", 98, 3.0, 3, 3, 5, 13, 1, 16),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", PSF_CASES,
                         ids=lambda c: f"{c[0]}x{c[1]}-{c[2]}-K{c[7]}-k{c[8]}-bin{c[9]}" + (f"-mesh{c[10]}" if len(c) > 10 else ""))
def test_peaks_psf_stage_isolated(P, case, prec):
    """gp_peaks_psf against the oracle's varying filter and peaks on the
    oracle's background grids, with synthetic eigen-PSF models and smooth
    coefficient maps (full-frame and binned)."""
    from synth import coef_maps, psf_model
    W, H, dt, seed, t, sep, cw, K, side, b = case[:10]
    mesh = case[10] if len(case) > 10 else 64
    _say("psf peak case", case, prec)
    fr = make_frame("c1", seed=seed, W=W, H=H, dtype=dt, nstars=max(8, W * H // 2500))
    p = f32_params(fr.params)
    p.mesh_w = p.mesh_h = mesh
    p.thresh = t
    p.sat_level = 60000.0
    if isinstance(side, tuple):
        kw, kh = side
        ks = psf_model(K, max(kw, kh), 3.0, seed)[:, (max(kw, kh) - kh) // 2:(max(kw, kh) + kh) // 2,
                                                   (max(kw, kh) - kw) // 2:(max(kw, kh) + kw) // 2].copy()
    else:
        ks = psf_model(K, side, 3.0, seed)
    cm = coef_maps(K, W, H, b, seed + 1)
    I = fr.image.astype(np.float64)
    ob = oracle.background(I, p, maps=True)
    M = I - ob.B
    S = oracle.filter_varying(M, ks.astype(np.float64), cm.astype(np.float64) if K else None, bin=b)
    o = oracle.peaks(I, M, S, ob.R, p.thresh, sep, cw, p.sat_level)
    ph = P.Photometry([_dev(fr.image)], p, p.kernel(), capacity=8192, precision=prec)
    ph.set_grids(0, ob.back, ob.rms)
    ph.background(grid_given=True)
    ph.peaks_psf(sep, cw, ks, [torch.from_numpy(cm).cuda()] if K else None, bin=b)
    n = _cmp_peak_catalogues(ph.results(0), o, M, S, ob.R, p.thresh, sep)
    _say("common peaks", n)
    ph.close()


def test_peaks_psf_without_modes_equals_gp_peaks(P):
    """With no eigenmodes and P0 of unit sum, gp_peaks_psf finds what gp_peaks
    finds with P0 as its kernel (up to FP32 ties at the threshold)."""
    from synth import psf_model
    fr = make_frame("c1", seed=97, W=300, H=220, nstars=30)
    p = f32_params(fr.params)
    ks = psf_model(0, 9, 3.0, 1)
    a = P.Photometry([_dev(fr.image)], p, ks[0], capacity=4096)
    a.background()
    a.peaks(3, 3)
    ra = a.results(0)
    a.peaks_psf(3, 3, ks)
    rb = a.results(0)
    _say("plain", ra["n_obj"], ra["status"], ra["cat"]["pmin"][:6], ra["cat"]["peak"][:6])
    _say("psf", rb["n_obj"], rb["status"], rb["cat"]["pmin"][:6], rb["cat"]["peak"][:6])
    assert ra["n_obj"] > 5
    common = np.intersect1d(ra["cat"]["pmin"], rb["cat"]["pmin"])
    assert len(common) >= ra["n_obj"] - 2 and len(common) >= rb["n_obj"] - 2
    a.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", PEAK_CASES, ids=lambda c: f"{c[1]}x{c[2]}-{c[3]}-t{c[5]}-s{c[6]}-c{c[7]}-{c[8] or 'gauss'}")
def test_peaks_stage_isolated(P, case, prec):
    name, W, H, dt, seed, t, sep, cw, kk = case
    _say("peak case", case, prec)
    fr = make_frame(name, seed=seed, W=W, H=H, dtype=dt, nstars=max(8, W * H // 2500))
    p = f32_params(fr.params)
    p.mesh_w = p.mesh_h = 64
    p.thresh = t
    p.sat_level = 60000.0
    K = p.kernel() if kk is None else (0.3 + np.random.default_rng(seed).random((7, 5))).astype(np.float32)
    I = fr.image.astype(np.float64)
    ob = oracle.background(I, p, maps=True)
    M = I - ob.B
    F = oracle.filter_image(M, K)
    o = oracle.peaks(I, M, F, ob.R, p.thresh, sep, cw, p.sat_level)
    ph = P.Photometry([_dev(fr.image)], p, K, capacity=8192, precision=prec)
    ph.set_grids(0, ob.back, ob.rms)
    ph.background(grid_given=True)
    ph.peaks(sep, cw)
    r = ph.results(0)
    _cmp_peak_catalogues(r, o, M, F, ob.R, p.thresh, sep)
    # the apertures run on the peak catalogue
    ph.aperture()
    ra = ph.results(0)
    rad = np.asarray(p.radii)
    rm = max(max(p.radii), p.r_out)
    x, y = ra["cat"]["x"], ra["cat"]["y"]
    inner = (x - rm >= -0.5) & (x + rm <= W - 0.5) & (y - rm >= -0.5) & (y + rm <= H - 0.5)
    np.testing.assert_allclose(ra["phot"]["area"][inner], np.broadcast_to(np.pi * rad ** 2, (inner.sum(), rad.size)),
                               rtol=1e-6)
    ph.close()


# ----------------------------------------------------------------------------
# growth curves on top-hat kernels, stage-isolated
# ----------------------------------------------------------------------------
GROWTH_CASES = [
    # name, W, H, dtype, seed, radii
    ("c1", 333, 257, "f32", 61, list(range(3, 16))),    # FWHM 3: radii 3..15
    ("c2", 300, 211, "u16", 62, list(range(3, 19))),    # FWHM 3.5: radii 3..18
    ("c1", 129, 70, "f32", 63, [1, 2, 5, 9]),
    ("c1", 200, 150, "f32", 64, list(range(1, 33))),    # the largest window (radius 32)
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", GROWTH_CASES, ids=lambda c: f"{c[1]}x{c[2]}-{c[3]}-r{c[5][0]}..{c[5][-1]}")
def test_growth_stage_isolated(P, case, prec):
    """Top-hat sums of M and R^2 at given positions against the oracle on the
    oracle's own background grids.  The FP64 path pins the tap table (areas
    to FP64 rounding); the FP32 path adds the FP32 evaluation of M and R."""
    name, W, H, dt, seed, radii = case
    _say("growth case", case, prec)
    fr = make_frame(name, seed=seed, W=W, H=H, dtype=dt, nstars=max(8, W * H // 2500))
    p = f32_params(fr.params)
    p.mesh_w = p.mesh_h = 64
    I = fr.image.astype(np.float64)
    ob = oracle.background(I, p, maps=True)
    M = I - ob.B
    V = ob.R ** 2
    rng = np.random.default_rng(seed)
    n = 400
    xs = rng.uniform(-40, W + 40, n)
    ys = rng.uniform(-40, H + 40, n)
    # half-integers round up; far off the frame; not a number
    xs[:8] = [10.5, -0.5, W - 0.5, W - 0.5 - 1e-9, -1e6, 1e30, np.nan, W / 2]
    ys[:8] = [20.5, H / 2, H / 2, 7.0, 5.0, 5.0, 5.0, np.inf]
    ph = P.Photometry([_dev(fr.image)], p, p.kernel(), capacity=n, precision=prec)
    ph.set_grids(0, ob.back, ob.rms)
    ph.background(grid_given=True)
    ph.set_catalog(0, xs, ys)
    ph.growth(radii)
    r = ph.results(0)["growth"]
    o = oracle.growth(M, V, xs, ys, radii)
    np.testing.assert_array_equal(r["flags"], o["flags"])
    # taps: both sides FP64 exact-overlap areas, which may differ at cut pixels
    # by the allowance below; summation adds a few units of 2^-53 of the area
    sa_m, na = growth_allowance(np.abs(M), xs, ys, radii)
    sa_v, _ = growth_allowance(V, xs, ys, radii)
    da = np.abs(r["area"] - o["area"])
    assert np.all(da <= na + 8 * 2.0 ** -53 * o["area"]), float(np.max(da - na))
    # sums: per pixel M within a few units of the working precision of |M| + |B|
    # (FP64: within the FP64 background map's agreement with the spline)
    u = 2.0 ** -24 if prec == 0 else 2.0 ** -53
    cond = oracle.growth(np.abs(M) + np.abs(ob.B), None, xs, ys, radii)["sum"]
    tol = 8 * u * cond + sa_m + (TOL_B64_ABS * o["area"] if prec == 1 else 0.0)
    ds = np.abs(r["sum"] - o["sum"])
    q = ds / np.maximum(cond, 1e-300)
    i, k = np.unravel_index(int(np.argmax(q)), q.shape)
    _say("growth sum err / cond", float(q[i, k]), "at", (xs[i], ys[i]), "r", radii[k], "tap allowance share",
         float(np.max(sa_m / np.maximum(tol, 1e-300))))
    assert np.all(ds <= tol), float(np.max(ds - tol))
    dv = np.abs(r["var"] - o["var"])
    tv = (16 * u + (2.5 * TOL_R64_REL if prec == 1 else 0.0)) * o["var"] + sa_v
    assert np.all(dv <= tv), float(np.max(dv / np.maximum(o["var"], 1e-300)))
    # sources that no tap reaches: zero sums
    far = ~np.isfinite(xs) | ~np.isfinite(ys) | (np.abs(xs) > 1e5)
    assert not np.any(r["sum"][far]) and not np.any(r["area"][far])
    ph.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
def test_growth_taps_on_a_zero_background(P, prec):
    """With B = 0 both sides sum the same float32 pixels: only the taps and
    the summation order differ, so the sums agree to FP64 rounding in both
    working precisions (this pins the tap table and its lists)."""
    W, H = 170, 140
    rng = np.random.default_rng(81)
    img = (rng.normal(0, 30, (H, W)) + 5 * np.arange(W)[None, :]).astype(np.float32)
    p = _params("c1")
    nx, ny = -(-W // p.mesh_w), -(-H // p.mesh_h)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=300, precision=prec)
    ph.set_grids(0, np.zeros((ny, nx)), np.full((ny, nx), 3.0))
    ph.background(grid_given=True)
    xs = rng.uniform(-5, W + 5, 300)
    ys = rng.uniform(-5, H + 5, 300)
    ph.set_catalog(0, xs, ys)
    radii = list(range(1, 33))
    ph.growth(radii)
    r = ph.results(0)["growth"]
    M = img.astype(np.float64)
    o = oracle.growth(M, np.full((H, W), 9.0), xs, ys, radii)
    cond = oracle.growth(np.abs(M), None, xs, ys, radii)["sum"]
    sa_m, na = growth_allowance(np.abs(M), xs, ys, radii)
    ds = np.abs(r["sum"] - o["sum"])
    _say("zero-background growth err / cond", float(np.max(ds / np.maximum(cond, 1e-300))))
    assert np.all(ds <= 8 * 2.0 ** -53 * cond + sa_m), float(np.max(ds - 8 * 2.0 ** -53 * cond - sa_m))
    assert np.all(np.abs(r["area"] - o["area"]) <= na + 8 * 2.0 ** -53 * o["area"])
    assert np.all(np.abs(r["var"] - o["var"]) <= 9.0 * (na + 8 * 2.0 ** -53 * o["area"]))
    np.testing.assert_array_equal(r["flags"], o["flags"])
    ph.close()


def test_growth_constant_image_closed_form(P):
    c = 7.25
    W, H = 150, 120
    img = np.full((H, W), c, np.float32)
    p = _params("c2")
    nx, ny = -(-W // p.mesh_w), -(-H // p.mesh_h)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=64)
    ph.set_grids(0, np.zeros((ny, nx)), np.full((ny, nx), 2.0))
    ph.background(grid_given=True)
    rng = np.random.default_rng(2)
    xs = 75 + rng.uniform(-3, 3, 40)
    ys = 60 + rng.uniform(-3, 3, 40)
    ph.set_catalog(0, xs, ys)
    radii = P.growth_radii(3.5)
    ph.growth(radii)
    r = ph.results(0)["growth"]
    a = np.pi * np.asarray(radii, np.float64) ** 2
    np.testing.assert_allclose(r["area"], np.broadcast_to(a, r["area"].shape), rtol=1e-13)
    np.testing.assert_allclose(r["sum"], c * r["area"], rtol=1e-15)
    np.testing.assert_allclose(r["var"], 4.0 * r["area"], rtol=1e-7)
    assert not np.any(r["flags"])
    ph.close()


def test_growth_batch_matches_single_frames(P):
    frs = [make_frame("c1", seed=71, W=300, H=260, nstars=30),
           make_frame("c1", seed=72, W=130, H=90, nstars=8, dtype="u16"),
           make_frame("c2", seed=73, W=450, H=128, nstars=25)]
    p = f32_params(frs[0].params)
    K = p.kernel()
    devs = [_dev(f.image) for f in frs]
    radii = P.growth_radii(3.0)
    batch = P.Photometry(devs, p, K, capacity=1024)
    batch.background()
    batch.peaks(3, 3)
    batch.growth(radii)
    for i, d in enumerate(devs):
        one = P.Photometry([d], p, K, capacity=1024)
        one.background()
        one.peaks(3, 3)
        one.growth(radii)
        a, b = batch.results(i), one.results(0)
        assert a["n_obj"] == b["n_obj"] > 0
        for k in a["growth"]:
            np.testing.assert_array_equal(a["growth"][k], b["growth"][k], err_msg=k)
        # interior sources: area pi r^2
        W, H = frs[i].image.shape[1], frs[i].image.shape[0]
        cx = np.floor(a["cat"]["x"] + 0.5)
        cy = np.floor(a["cat"]["y"] + 0.5)
        R = max(radii)
        inner = (cx - R >= 0) & (cx + R < W) & (cy - R >= 0) & (cy + R < H)
        np.testing.assert_array_equal(a["growth"]["flags"] != 0, ~inner)
        np.testing.assert_allclose(a["growth"]["area"][inner],
                                   np.broadcast_to(np.pi * np.asarray(radii, float) ** 2,
                                                   (int(inner.sum()), len(radii))), rtol=1e-13)
        one.close()
    batch.close()


# ----------------------------------------------------------------------------
# local background by convolution
# ----------------------------------------------------------------------------
CONV_CASES = [
    # W, H, dtype, seed, lx, ly, mask kind, sat
    (600, 400, "f32", 111, 33, 33, "blobs", np.inf),
    (333, 211, "u16", 112, 31, 9, "blobs", 60000.0),
    (300, 200, "f32", 113, 129, 129, "none", np.inf),   # the largest kernel
    (257, 131, "f32", 114, 1, 1, "blobs", np.inf),      # delta kernel: holes stay unfilled
    (200, 150, "f32", 115, 65, 17, "hole", np.inf),     # a hole wider than the kernel
    # two horizontal segments; invalid pixels on the four borders, at the
    # segment seam and at band edges (the reach of the fill passes)
    (2300, 150, "f32", 116, 65, 65, "edges", np.inf),
    (40, 30, "u16", 117, 65, 33, "blobs", 60000.0),   # narrower than the kernel: repeated reflections
    (700, 300, "u16", 118, 65, 65, "none", 30000.0),  # saturated star cores only
    (260, 190, "f32", 119, 129, 129, "blobs", np.inf),  # the largest kernel with fills (largest LDS stage)
]


def _conv_inputs(case):
    W, H, dt, seed, lx, ly, mk, sat = case
    fr = make_frame("c1", seed=seed, W=W, H=H, dtype=dt, nstars=max(8, W * H // 3000))
    rng = np.random.default_rng(seed)
    kx = (0.2 + rng.random(lx)).astype(np.float32)     # asymmetric taps
    ky = (0.2 + rng.random(ly)).astype(np.float32)
    mask = None
    if mk == "blobs":
        mask = np.zeros((H, W), np.uint8)
        for _ in range(12):
            cx, cy, r = rng.integers(0, W), rng.integers(0, H), rng.integers(1, 6)
            mask[max(cy - r, 0):cy + r + 1, max(cx - r, 0):cx + r + 1] = 1
    elif mk == "hole":
        mask = np.zeros((H, W), np.uint8)
        mask[20:130, 30:160] = 1
    elif mk == "edges":
        mask = np.zeros((H, W), np.uint8)
        for x, y in ((0, 17), (W - 1, 40), (90, 0), (1500, H - 1), (0, 0), (W - 1, H - 1), (2047, 70), (2048, 71),
                     (2040, 110), (63, 120), (64, 121), (W - 2, 5)):
            mask[y, x] = 1
    return fr.image, kx, ky, mask, sat


def _conv_tolerances(I, kx, ky, mask, sat, B, prec, gain):
    """Bounds from oracle-side quantities: the condition K corr |I'| of the
    sums, the FP32 storage of the intermediates (FP32 path) or the oracle's own
    2-D summation (FP64 path), and the fill's division by K corr v."""
    from scipy import ndimage
    K = np.outer(ky.astype(float) / ky.astype(float).sum(), kx.astype(float) / kx.astype(float).sum())
    I = I.astype(np.float64)
    v = np.ones_like(I) if mask is None else (mask == 0).astype(float)
    v *= (I < sat)
    Aabs = ndimage.correlate(v * np.abs(I), K, mode="reflect")
    Cv = ndimage.correlate(v, K, mode="reflect")
    with np.errstate(divide="ignore", invalid="ignore"):
        Nabs = np.where(Cv > 0, Aabs / Cv, 0.0)
    lx, ly = kx.size, ky.size
    if prec == 0:
        g = 8 * 2.0 ** -24
    else:
        g = (lx * ly + 2 * (lx + ly) + 8) * 2.0 ** -53
    with np.errstate(divide="ignore", invalid="ignore"):
        eN = np.where((v == 0) & (Cv > 0), g * (Aabs + Nabs * Cv) / Cv, 0.0)
    cond = Aabs + ndimage.correlate((1 - v) * Nabs, K, mode="reflect")
    return g * cond + ndimage.correlate(eN, K, mode="reflect") + g * np.abs(B)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "fp64"])
@pytest.mark.parametrize("case", CONV_CASES, ids=lambda c: f"{c[0]}x{c[1]}-{c[2]}-k{c[4]}x{c[5]}-{c[6]}")
def test_background_conv_against_oracle(P, case, prec):
    _say("conv case", case, prec)
    I, kx, ky, mask, sat = _conv_inputs(case)
    # the parameters as the float32 values the library receives
    gain, rn, dark, texp = (float(np.float32(q)) for q in (1.6, 7.0, 0.05, 120.0))
    Bo, Ro, no = oracle.background_conv(I, kx.astype(np.float64), ky.astype(np.float64), mask=mask, sat=sat,
                                        gain=gain, rn=rn, dark=dark, texp=texp)
    cb = P.ConvBackground([_dev(I)], kx, ky, gain, rn, dark, texp, sat, precision=prec)
    cb.run([_dev(mask)] if mask is not None else None)
    torch.cuda.synchronize()
    B = cb.back[0].cpu().numpy().astype(np.float64)
    R = cb.rms[0].cpu().numpy().astype(np.float64)
    ng = int(cb.unfilled[0].item())
    assert ng == no, (ng, no)
    tol = _conv_tolerances(I, kx, ky, mask, sat, Bo, prec, gain)
    dB = np.abs(B - Bo)
    _say("conv |dB| max", float(dB.max()), "share of tolerance", float(np.max(dB / np.maximum(tol, 1e-300))),
         "unfilled", no)
    assert np.all(dB <= tol), float(np.max(dB - tol))
    u = 2.0 ** -24 if prec == 0 else 2.0 ** -53
    tR = 0.5 * tol / (gain * np.maximum(Ro, 1e-300)) + 4 * u * Ro
    assert np.all(np.abs(R - Ro) <= tR), float(np.max(np.abs(R - Ro) - tR))
    cb.close()


def test_background_conv_constant_frame_and_batch(P):
    """A constant frame comes back unchanged; a batch of frames (uint16 and
    float32, several sizes) equals per-frame calls bit for bit."""
    c = np.full((150, 260), 812.0, np.float32)
    kx = np.hanning(67)[1:-1].astype(np.float32)
    ky = np.hanning(35)[1:-1].astype(np.float32)
    cb = P.ConvBackground([_dev(c)], kx, ky, 2.0)
    cb.run()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cb.back[0].cpu().numpy(), c)
    np.testing.assert_allclose(cb.rms[0].cpu().numpy(), np.sqrt(812.0 / 2.0), rtol=1e-6)
    cb.close()
    frs = [make_frame("c1", seed=121, W=300, H=260, nstars=30).image,
           make_frame("c1", seed=122, W=130, H=90, nstars=8, dtype="u16").image,
           make_frame("c1", seed=123, W=450, H=128, nstars=25).image]
    masks = [None, (np.random.default_rng(1).random((90, 130)) < 0.02).astype(np.uint8), None]
    devs = [_dev(f) for f in frs]
    mdev = [None if m is None else _dev(m) for m in masks]
    batch = P.ConvBackground(devs, kx, ky, 1.5, 5.0, sat_level=60000.0)
    batch.run(mdev)
    for i, d in enumerate(devs):
        one = P.ConvBackground([d], kx, ky, 1.5, 5.0, sat_level=60000.0)
        one.run([mdev[i]])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(batch.back[i].cpu().numpy(), one.back[0].cpu().numpy())
        np.testing.assert_array_equal(batch.rms[i].cpu().numpy(), one.rms[0].cpu().numpy())
        assert int(batch.unfilled[i].item()) == int(one.unfilled[0].item())
        one.close()
    batch.close()


def _grown(mask):
    """mask grown by one pixel in the 8-neighbourhood"""
    g = mask.copy()
    g[1:, :] |= mask[:-1, :]
    g[:-1, :] |= mask[1:, :]
    g2 = g.copy()
    g2[:, 1:] |= g[:, :-1]
    g2[:, :-1] |= g[:, 1:]
    return g2


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_end_to_end_against_oracle(P, seed):
    """GPU chain vs oracle chain.  Meshes are checked one by one (a mesh with a
    decision inside the rounding band may match the oracle with that decision
    flipped); the oracle chain then runs downstream of the grids it accepts.
    Objects whose pixels (grown by one) hold no ambiguous threshold decision
    must appear identically in both catalogues; every other GPU object must
    touch an ambiguous pixel."""
    fr = make_frame("c1", seed=seed, W=384, H=320, nstars=40)
    p = f32_params(fr.params)
    img = fr.image
    I = img.astype(np.float64)
    ph = P.Photometry([_dev(img)], p, p.kernel(), capacity=2048, seg=True)
    ph.run()
    r = ph.results(0)
    g = ph.grids(0)
    back_raw, rms_raw, flipped = check_meshes(img, g, p)
    back = oracle.median_filter(back_raw, p.mesh_filter)
    rms = oracle.median_filter(rms_raw, p.mesh_filter)
    res = oracle.run(I, p, grids=(back, rms))
    amb_px = thresh_ambiguous(res.F, res.bkg.R, p.thresh)
    ocat, gcat = res.cat, r["cat"]
    n_o = len(ocat["npix"])
    clean = np.array([not np.any(amb_px & _grown(res.seg == k + 1)) for k in range(n_o)], bool)
    _say("meshes matched a flipped branch", flipped, "objects gpu", r["n_obj"], "oracle", n_o,
         "ambiguous objects", int((~clean).sum()), "ambiguous px", int(amb_px.sum()))
    assert clean.sum() >= max(1, 0.8 * n_o)
    gi = {int(pm): i for i, pm in enumerate(gcat["pmin"])}
    idx_o = np.nonzero(clean)[0]
    assert all(int(ocat["pmin"][k]) in gi for k in idx_o), "a clean oracle object is missing on the GPU"
    idx_g = np.array([gi[int(ocat["pmin"][k])] for k in idx_o])
    # the same pixels: each clean object's GPU label covers exactly its pixels
    for k, kg in zip(idx_o, idx_g):
        np.testing.assert_array_equal(r["seg"] == kg + 1, res.seg == k + 1)
    sub_g = {q: v[idx_g] for q, v in gcat.items()}
    sub_o = {q: v[idx_o] for q, v in ocat.items()}
    seg_sub = np.zeros_like(res.seg)
    for t, k in enumerate(idx_o):
        seg_sub[res.seg == k + 1] = t + 1
    err = cmp_catalog(sub_g, sub_o, res.M, seg_sub, tag="e2e")
    # GPU objects not among the clean ones lie on ambiguous pixels
    others = np.setdiff1d(np.arange(r["n_obj"]), idx_g)
    for kg in others:
        assert np.any(amb_px & _grown(r["seg"] == kg + 1)), ("unexplained GPU object", int(kg))
    # apertures of the clean objects at the oracle's centres
    xs, ys = sub_o["x"], sub_o["y"]
    oph = {q: v[idx_o] for q, v in res.phot.items()}
    cond, cond_ann = phot_condition(res.M, xs, ys, p)
    gph = {q: v[idx_g] for q, v in r["phot"].items()}
    perr = cmp_phot(gph, oph, cond, cond_ann, weight_allowance(res.M, xs, ys, p, oph), tag="e2e")
    _say("e2e errors", err, perr)
    ph.close()


def test_batch_matches_single_frames(P):
    frs = [make_frame("c1", seed=31, W=300, H=260, nstars=30),
           make_frame("c1", seed=32, W=130, H=90, nstars=8, dtype="u16"),
           make_frame("c1", seed=33, W=450, H=128, nstars=25)]
    p = f32_params(frs[0].params)
    K = p.kernel()
    devs = [_dev(f.image) for f in frs]
    batch = P.Photometry(devs, p, K, capacity=1024, seg=True)
    batch.run()
    for i, d in enumerate(devs):
        one = P.Photometry([d], p, K, capacity=1024, seg=True)
        one.run()
        a, b = batch.results(i), one.results(0)
        assert a["n_obj"] == b["n_obj"] > 0
        np.testing.assert_array_equal(a["seg"], b["seg"])
        # bit for bit: every sum is formed in a fixed order or from exact terms
        for k in a["cat"]:
            np.testing.assert_array_equal(a["cat"][k], b["cat"][k], err_msg=k)
        for k in a["phot"]:
            np.testing.assert_array_equal(a["phot"][k], b["phot"][k], err_msg=k)
        ga, gb = batch.grids(i), one.grids(0)
        for k in ("back_raw", "rms_raw", "back", "rms", "coef"):
            np.testing.assert_array_equal(ga[k], gb[k])
        one.close()
    batch.close()


def _same_results(a, b, tag):
    assert a["n_obj"] == b["n_obj"] and a["status"] == b["status"], tag
    for grp in ("cat", "phot"):
        for k in a[grp]:
            np.testing.assert_array_equal(a[grp][k], b[grp][k], err_msg=f"{tag} {grp}.{k}")


def test_graph_replay_matches_direct_calls(P):
    """The three calls over an uneven uint16/float32 batch captured once into a
    HIP graph: every replay (with other work and synchronisations between the
    replays) gives, bit for bit, the results of direct calls and of per-frame
    calls."""
    frs = [make_frame("c1", seed=91, W=700, H=520, nstars=60, dtype="u16"),
           make_frame("c1", seed=92, W=257, H=190, nstars=15),
           make_frame("c1", seed=93, W=1030, H=300, nstars=70, dtype="u16"),
           make_frame("c1", seed=94, W=64, H=900, nstars=12)]
    p = f32_params(frs[0].params)
    K = p.kernel()
    devs = [_dev(f.image) for f in frs]
    direct = P.Photometry(devs, p, K, capacity=2048)
    direct.run()
    ref = [direct.results(i) for i in range(len(devs))]
    singles = []
    for i, d in enumerate(devs):
        one = P.Photometry([d], p, K, capacity=2048)
        one.run()
        singles.append(one.results(0))
        one.close()
        _same_results(ref[i], singles[i], f"frame {i} batch vs alone")
    gb = P.Photometry(devs, p, K, capacity=2048)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gb.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gb.run()
    for rep in range(4):
        # eager work between replays: another batch through direct calls
        direct.run()
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(devs)):
            _same_results(gb.results(i), ref[i], f"replay {rep} frame {i}")
        del junk
    del g
    gb.close()
    direct.close()


def test_library_graph_replay_and_rebind(P):
    """gp_graph_create records the three calls over an uneven batch once;
    every gp_graph_launch (with other work and synchronisations between
    launches) reproduces direct calls bit for bit, and gp_graph_rebind to other
    frames of the same shapes gives what direct calls give on those frames."""
    def frames(seed0):
        return [make_frame("c1", seed=seed0, W=610, H=480, nstars=50, dtype="u16"),
                make_frame("c1", seed=seed0 + 1, W=300, H=199, nstars=20),
                make_frame("c1", seed=seed0 + 2, W=900, H=257, nstars=40, dtype="u16")]
    a = [_dev(f.image) for f in frames(110)]
    b = [_dev(f.image) for f in frames(120)]
    p = f32_params(frames(110)[0].params)
    K = p.kernel()

    def direct(devs):
        ph = P.Photometry(devs, p, K, capacity=2048)
        ph.run()
        out = [ph.results(i) for i in range(len(devs))]
        ph.close()
        return out
    ra, rb = direct(a), direct(b)
    g = P.Photometry(a, p, K, capacity=2048).capture()
    other = P.Photometry(b, p, K, capacity=2048)
    for rep in range(3):
        other.run()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(a)):
            _same_results(g.results(i), ra[i], f"launch {rep} frame {i}")
    g.rebind(b)
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(b)):
            _same_results(g.results(i), rb[i], f"rebound launch {rep} frame {i}")
    g.rebind(a)
    g.replay()
    for i in range(len(a)):
        _same_results(g.results(i), ra[i], f"rebound back, frame {i}")
    from paper_2609_32375_amd import _lib as L
    with pytest.raises(L.GpError):
        g.rebind([a[1], a[0], a[2]])        # other shapes: refused, graph unchanged
    g.replay()
    _same_results(g.results(0), ra[0], "after a refused rebind")
    g.close()
    other.close()


def test_capacity_overflow_keeps_first_labels(P):
    fr = make_frame("c1", seed=41, W=320, H=320, nstars=60)
    p = f32_params(fr.params)
    dev = _dev(fr.image)
    full = P.Photometry([dev], p, p.kernel(), capacity=4096)
    full.run()
    a = full.results(0)
    n = a["n_obj"]
    assert n > 6
    small = P.Photometry([dev], p, p.kernel(), capacity=5)
    small.run()
    b = small.results(0)
    assert b["status"] == 4 and b["n_obj"] == n
    for k in ("pmin", "npix", "x", "y"):
        np.testing.assert_array_equal(b["cat"][k], a["cat"][k][:5])
    full.close()
    small.close()


def test_component_overflow_reports_required_size(P):
    mask = (np.add.outer(np.arange(128), np.arange(128)) % 2).astype(bool)
    img = np.where(mask, 600.0, 500.0).astype(np.float32)
    p = _params("c1", mesh_w=16, mesh_h=16, conn=4, minarea=1)
    K = np.ones((1, 1), np.float32)
    ph = P.Photometry([_dev(img)], p, K, capacity=16, comp_capacity=100)
    ph.set_grids(0, np.full((8, 8), 500.0), np.zeros((8, 8)))
    ph.background(grid_given=True)
    ph.detect()
    r = ph.results(0)
    assert r["comp_status"][0] == 3 and r["comp_status"][1] == 128 * 128 // 2
    assert r["status"] == 3
    ph.close()


def test_invalid_arguments_fail_synchronously(P):
    from paper_2609_32375_amd import _lib as L
    img = _dev(np.zeros((64, 64), np.float32))
    p = _params("c1")
    ph = P.Photometry([img], p, p.kernel(), capacity=8)
    bad_k = np.ones((4, 4), np.float32)
    with pytest.raises(L.GpError) as e:
        P.Photometry([img], p, bad_k, capacity=8)
    assert e.value.status == L.GP_ERR_INVALID_ARG
    q = _params("c1", minarea=0)
    with pytest.raises(L.GpError):
        P.Photometry([img], q, p.kernel(), capacity=8)
    q = _params("c1", conn=6)
    with pytest.raises(L.GpError):
        P.Photometry([img], q, p.kernel(), capacity=8)
    # undersized workspace
    with pytest.raises(L.GpError) as e:
        L.gp_detect(ph.ctx, ph.frames, ph.bp, ph.bkg.data_ptr(), ph.dp, ph.gcat, None, None,
                    ph.ws.data_ptr(), 1024, ph.stream_ptr())
    assert e.value.status == L.GP_ERR_WORKSPACE
    # a detection batch holds at most 2^31 pixels (rejected while planning,
    # before any device access: the frame pointers are dummies)
    big = [L.gp_frame(1, 32768, 40000, 32768, 1)] * 2
    with pytest.raises(L.GpError) as e:
        L.gp_detect(ph.ctx, big, ph.bp, ph.bkg.data_ptr(), ph.dp, ph.gcat, None, None,
                    ph.ws.data_ptr(), 1 << 40, ph.stream_ptr())
    assert e.value.status == L.GP_ERR_UNSUPPORTED and "2^31" in L.load().gp_last_error().decode()
    ph.close()


def test_autotuning_keeps_results_and_writes_the_cache(P, tmp_path):
    import json
    fr = make_frame("c1", seed=41, W=512, H=384, nstars=40)
    p = f32_params(fr.params)
    d = _dev(fr.image)
    ref = P.Photometry([d], p, p.kernel(), capacity=1024)
    ref.run()
    a = ref.results(0)
    path = str(tmp_path / "tune.json")
    tuned = P.Photometry([d], p, p.kernel(), capacity=1024, autotune=True, tune_cache=path)
    tuned.run()
    b = tuned.results(0)
    cache = json.load(open(path))
    _say("tuned", cache)
    assert any(k.startswith("mesh_stats:") for k in cache) and any(k.startswith("aperture:") for k in cache)
    assert a["n_obj"] == b["n_obj"] > 0
    for k in ("npix", "xmin", "xmax", "ymin", "ymax", "pmin"):
        np.testing.assert_array_equal(a["cat"][k], b["cat"][k])
    for k in ("flux", "area", "bkg", "fluxerr"):
        np.testing.assert_allclose(a["phot"][k], b["phot"][k], rtol=1e-12, atol=1e-9)
    # a new context reads the choices back
    again = P.Photometry([d], p, p.kernel(), capacity=1024, tune_cache=path)
    again.run()
    c = again.results(0)
    np.testing.assert_array_equal(b["cat"]["pmin"], c["cat"]["pmin"])
    for o in (ref, tuned, again):
        o.close()
