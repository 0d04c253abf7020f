"""The full-size workloads in the launch configuration bench.py times, checked
against the FP64 oracle on sampled outputs (needs an MI355X).

c2 is the 6144 x 6144 float32 field (20,000 stars, mesh 128, 9x9 filter,
apertures 3/6/9 px, annulus 13-18 px), c3 the 12300 x 12300 float32 field
(134,000 stars).  The GPU runs the whole path once per workload; the oracle
then recomputes, one by one, what it can afford at that size:

  * mesh statistics of sampled meshes (each mesh's own pixels);
  * the grid median filter on the whole grid (exact);
  * the background and noise maps at sampled pixels, from the GPU's grids;
  * sampled objects: their component and moments from a window around the
    GPU's bounding box (M from the GPU's grids, filter halo reflected at the
    frame border as on the GPU), skipped when a threshold decision nearby is
    within FP32 rounding;
  * apertures of sampled objects on a window around each centre;

and checks properties that hold for every object at any size (raster order of
labels, minarea, bounding boxes, aperture areas, the truncation flag).
"""
import math
import sys

import numpy as np
import pytest

import oracle
from synth import make_frame
from tests._util import (TOL_BKG_REL, box_max_abs, cmp_phot, f32_params, mesh_ambiguous, phot_condition,
                         thresh_ambiguous)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CAPACITY = {"c2": 65536, "c3": 262144}     # as bench.py
FLAG_SAT, FLAG_EDGE, FLAG_NONPOS, FLAG_TRUNC = 1, 2, 4, 8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _reflect(i, n):
    p = 2 * n
    r = np.mod(i, p)
    return np.where(r < n, r, p - 1 - r)


@pytest.fixture(scope="module", params=["c2", "c3"])
def full(request):
    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry
    name = request.param
    _say("full-size workload", name)
    fr = make_frame(name)
    img = fr.image
    H, W = img.shape
    dev = torch.from_numpy(img).cuda()
    ph = Photometry([dev], fr.params, fr.params.kernel(), capacity=CAPACITY[name])
    ph.run()
    r = ph.results(0)
    g = ph.grids(0)
    # maps on the device, sampled there
    B = torch.empty(H, W, dtype=torch.float64, device=dev.device)
    R = torch.empty(H, W, dtype=torch.float64, device=dev.device)
    import ctypes as C
    L.gp_background_map(ph.ctx, ph.frames, ph.bp, C.c_void_p(ph.bkg.data_ptr()), 0, L.GP_PREC_F32,
                        C.c_void_p(B.data_ptr()), C.c_void_p(R.data_ptr()), ph.stream_ptr())
    torch.cuda.synchronize()
    _say(name, "objects", r["n_obj"], "status", r["status"])
    yield dict(name=name, fr=fr, p=f32_params(fr.params), img=img, r=r, g=g, B=B, R=R)
    del B, R
    ph.close()
    torch.cuda.empty_cache()


def test_fullsize_status_and_catalogue_properties(full):
    r, p, img = full["r"], full["p"], full["img"]
    H, W = img.shape
    n = r["n_obj"]
    assert r["status"] == 0 and 0 < n <= CAPACITY[full["name"]]
    c, ph = r["cat"], r["phot"]
    assert len(c["npix"]) == n
    # canonical labels: raster order of the first pixel
    assert np.all(np.diff(c["pmin"]) > 0)
    assert np.all(c["npix"] >= p.minarea)
    assert np.all((c["xmin"] <= c["xmax"]) & (c["ymin"] <= c["ymax"]))
    assert np.all((c["xmin"] >= 0) & (c["ymin"] >= 0) & (c["xmax"] < W) & (c["ymax"] < H))
    assert np.all(c["npix"] <= (c["xmax"] - c["xmin"] + 1) * (c["ymax"] - c["ymin"] + 1))
    py, px = np.divmod(c["pmin"], W)
    assert np.all((py == c["ymin"]) & (px >= c["xmin"]) & (px <= c["xmax"]))
    edge = (c["xmin"] == 0) | (c["ymin"] == 0) | (c["xmax"] == W - 1) | (c["ymax"] == H - 1)
    np.testing.assert_array_equal((c["flags"] & FLAG_EDGE) != 0, edge)
    # apertures: areas within the disks, the truncation flag geometric
    rad = np.asarray(p.radii, np.float64)
    # (the areas are summed with FP32 weights: relative 1e-6, as against the oracle)
    assert np.all(ph["area"] >= 0) and np.all(ph["area"] <= np.pi * rad[None, :] ** 2 * (1 + 1e-6))
    rm = max(max(p.radii), p.r_out)
    x, y = c["x"], c["y"]
    trunc = (x - rm < -0.5) | (x + rm > W - 0.5) | (y - rm < -0.5) | (y + rm > H - 0.5)
    np.testing.assert_array_equal((c["flags"] & FLAG_TRUNC) != 0, trunc)
    inner = ~trunc
    np.testing.assert_allclose(ph["area"][inner], np.broadcast_to(np.pi * rad ** 2, ph["area"][inner].shape),
                               rtol=1e-6)
    assert np.all(ph["fluxerr"] > 0)


def test_fullsize_meshes_sampled(full):
    img, p, g = full["img"], full["p"], full["g"]
    H, W = img.shape
    ny, nx = g["back_raw"].shape
    rng = np.random.default_rng(11)
    picks = {(ny - 1, nx - 1), (0, 0), (ny - 1, 0), (0, nx - 1)}
    while len(picks) < 40:
        picks.add((int(rng.integers(ny)), int(rng.integers(nx))))
    checked = 0
    for (j, i) in sorted(picks):
        x0, y0 = i * p.mesh_w, j * p.mesh_h
        w, h = min(p.mesh_w, W - x0), min(p.mesh_h, H - y0)
        st = oracle.mesh_stats(img[y0:y0 + h, x0:x0 + w].astype(np.float64), w, h, p.clip_sigma, p.crowd_tol,
                               p.mode_a, p.mode_b, p.max_iter)
        if mesh_ambiguous(st)[0, 0]:
            continue
        checked += 1
        assert abs(g["back_raw"][j, i] - st["back"][0, 0]) <= TOL_BKG_REL * abs(st["back"][0, 0]), (j, i)
        assert abs(g["rms_raw"][j, i] - st["rms"][0, 0]) <= TOL_BKG_REL * abs(st["rms"][0, 0]), (j, i)
        assert g["iters"][j, i] == int(st["iters"][0, 0]), (j, i)
    _say("meshes checked", checked, "of", len(picks))
    assert checked >= 24
    # the grid median filter, whole grid, exactly
    np.testing.assert_array_equal(g["back"], oracle.median_filter(g["back_raw"], p.mesh_filter))
    np.testing.assert_array_equal(g["rms"], oracle.median_filter(g["rms_raw"], p.mesh_filter))


def test_fullsize_maps_sampled(full):
    img, p, g = full["img"], full["p"], full["g"]
    H, W = img.shape
    rng = np.random.default_rng(12)
    n = 4000
    xs = np.concatenate([rng.integers(0, W, n), [0, W - 1, 0, W - 1]])
    ys = np.concatenate([rng.integers(0, H, n), [0, 0, H - 1, H - 1]])
    Bo = oracle.grid_eval(g["back"], W, H, p.mesh_w, p.mesh_h, xs.astype(np.float64), ys.astype(np.float64))
    Ro = oracle.grid_eval(g["rms"], W, H, p.mesh_w, p.mesh_h, xs.astype(np.float64), ys.astype(np.float64))
    ix = torch.as_tensor(ys * W + xs, device=full["B"].device)
    Bg = full["B"].reshape(-1)[ix].cpu().numpy()
    Rg = full["R"].reshape(-1)[ix].cpu().numpy()
    eb, er = np.abs(Bg - Bo).max(), (np.abs(Rg - Ro) / Ro).max()
    _say("maps: max |dB|", eb, "max rel dR", er)
    assert eb <= 5e-5 and er <= TOL_BKG_REL


def _window(img, gb, gr, p, x0, x1, y0, y1, halo):
    """I, M, R over [x0, x1) x [y0, y1) and F over it (M taken on the window
    grown by `halo`, reflected at the frame border as the filter does)."""
    H, W = img.shape
    rows = _reflect(np.arange(y0 - halo, y1 + halo), H)
    cols = _reflect(np.arange(x0 - halo, x1 + halo), W)
    yy, xx = np.meshgrid(rows, cols, indexing="ij")
    Bx = oracle.grid_eval(gb, W, H, p.mesh_w, p.mesh_h, xx.ravel().astype(np.float64),
                          yy.ravel().astype(np.float64)).reshape(xx.shape)
    Ix = img[yy, xx].astype(np.float64)
    Mx = Ix - Bx
    Fx = oracle.filter_image(Mx, p.kernel())
    sl = (slice(halo, halo + (y1 - y0)), slice(halo, halo + (x1 - x0)))
    yy0, xx0 = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    R = oracle.grid_eval(gr, W, H, p.mesh_w, p.mesh_h, xx0.ravel().astype(np.float64),
                         yy0.ravel().astype(np.float64)).reshape(xx0.shape)
    return Ix[sl], Mx[sl], R, Fx[sl]


def test_fullsize_objects_sampled(full):
    img, p, g, r = full["img"], full["p"], full["g"], full["r"]
    H, W = img.shape
    c = r["cat"]
    n = r["n_obj"]
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([rng.choice(n, min(n, 48), replace=False), [0, n - 1]]))
    kr = p.kernel_size // 2
    checked = skipped = 0
    for k in idx:
        m = 3
        x0, x1 = max(int(c["xmin"][k]) - m, 0), min(int(c["xmax"][k]) + m + 1, W)
        y0, y1 = max(int(c["ymin"][k]) - m, 0), min(int(c["ymax"][k]) + m + 1, H)
        I, M, R, F = _window(img, g["back"], g["rms"], p, x0, x1, y0, y1, kr)
        seg, _ = oracle.threshold_label(F, R, p.thresh, 1, p.conn)
        py, px = divmod(int(c["pmin"][k]), W)
        lab = seg[py - y0, px - x0]
        amb = thresh_ambiguous(F, R, p.thresh)
        if lab <= 0:
            assert amb[py - y0, px - x0], ("first pixel below threshold", k)
            skipped += 1
            continue
        comp = seg == lab
        grown = comp.copy()
        grown[1:, :] |= comp[:-1, :]
        grown[:-1, :] |= comp[1:, :]
        grown[:, 1:] |= grown[:, :-1].copy()
        grown[:, :-1] |= grown[:, 1:].copy()
        if np.any(amb & grown):
            skipped += 1
            continue
        # the component must lie inside the window away from its cut edges
        inner = np.ones_like(comp)
        if y0 > 0:
            inner[0, :] = False
        if y1 < H:
            inner[-1, :] = False
        if x0 > 0:
            inner[:, 0] = False
        if x1 < W:
            inner[:, -1] = False
        assert not np.any(comp & ~inner), ("component reaches the window edge", k)
        o = oracle.measure(I, M, comp.astype(np.int32), 1, p.sat_level)
        assert int(o["npix"][0]) == int(c["npix"][k]), k
        assert (int(o["xmin"][0]) + x0, int(o["xmax"][0]) + x0, int(o["ymin"][0]) + y0, int(o["ymax"][0]) + y0) == \
            (int(c["xmin"][k]), int(c["xmax"][k]), int(c["ymin"][k]), int(c["ymax"][k])), k
        oy, ox = divmod(int(o["pmin"][0]), x1 - x0)
        assert (oy + y0) * W + ox + x0 == int(c["pmin"][k]), k
        absM = np.abs(M[comp]).sum()
        assert abs(c["flux"][k] - o["flux"][0]) <= 1e-6 * max(abs(o["flux"][0]), absM), k
        assert abs(c["x"][k] - (o["x"][0] + x0)) <= 1e-4 and abs(c["y"][k] - (o["y"][0] + y0)) <= 1e-4, k
        for q in ("x2", "y2", "xy"):
            assert abs(c[q][k] - o[q][0]) <= 1e-4 + 1e-6 * abs(o[q][0]), (k, q)
        assert abs(float(c["peak"][k]) - o["peak"][0]) <= 1e-6 * abs(o["peak"][0]) + 1e-3, k
        assert (int(c["flags"][k]) & (FLAG_SAT | FLAG_NONPOS)) == (int(o["flags"][0]) & (FLAG_SAT | FLAG_NONPOS)), k
        checked += 1
    _say("objects checked", checked, "skipped (threshold within rounding)", skipped)
    assert checked >= 0.8 * len(idx)


def test_fullsize_apertures_sampled(full):
    img, p, g, r = full["img"], full["p"], full["g"], full["r"]
    H, W = img.shape
    c, phot = r["cat"], r["phot"]
    n = r["n_obj"]
    rng = np.random.default_rng(14)
    idx = np.unique(np.concatenate([rng.choice(n, min(n, 64), replace=False), [0, n - 1]]))
    # include objects whose apertures leave the frame
    tr = np.nonzero(c["flags"] & FLAG_TRUNC)[0]
    if tr.size:
        idx = np.unique(np.concatenate([idx, rng.choice(tr, min(tr.size, 8), replace=False)]))
    rm = max(max(p.radii), p.r_out)
    for k in idx:
        xc, yc = float(c["x"][k]), float(c["y"][k])
        x0, x1 = max(int(math.floor(xc - rm)) - 2, 0), min(int(math.ceil(xc + rm)) + 3, W)
        y0, y1 = max(int(math.floor(yc - rm)) - 2, 0), min(int(math.ceil(yc + rm)) + 3, H)
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        fx, fy = xx.ravel().astype(np.float64), yy.ravel().astype(np.float64)
        B = oracle.grid_eval(g["back"], W, H, p.mesh_w, p.mesh_h, fx, fy).reshape(xx.shape)
        R = oracle.grid_eval(g["rms"], W, H, p.mesh_w, p.mesh_h, fx, fy).reshape(xx.shape)
        M = img[y0:y1, x0:x1].astype(np.float64) - B
        xs, ys = np.array([xc - x0]), np.array([yc - y0])
        o = oracle.aperture(M, R, xs, ys, list(p.radii), p.r_in, p.r_out, p.gain, p.want_err)
        cond, cond_ann = phot_condition(M, xs, ys, p)
        gph = {q: phot[q][k:k + 1] for q in ("flux", "area", "bkg", "fluxerr")}
        cmp_phot(gph, o, cond, cond_ann, tag=f"{full['name']} object {k}",
                 mmax=box_max_abs(M, xs, ys, rm))
    _say("apertures checked", len(idx))
