"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Every check here compares the oracle with something other than itself: closed
forms, library routines (scipy.ndimage, scipy.interpolate, scipy.integrate,
numpy statistics), brute force, or invariants.  Each is chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign or index, a
transposed operand) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, interpolate, ndimage

import oracle
from synth import Params, gaussian_kernel, make_frame


# ----------------------------------------------------------------------------
# exact disk / pixel overlap
# ----------------------------------------------------------------------------
def _quad_overlap(x0, x1, y0, y1, cx, cy, r):
    """Area by 1-D quadrature of the clipped chord length (scipy.integrate)."""
    def h(x):
        u = x - cx
        if abs(u) >= r:
            return 0.0
        s = math.sqrt(r * r - u * u)
        lo, hi = max(y0, cy - s), min(y1, cy + s)
        return max(0.0, hi - lo)
    a, b = max(x0, cx - r), min(x1, cx + r)
    if a >= b:
        return 0.0
    pts = [p for p in (cx - math.sqrt(max(r * r - (y - cy) ** 2, 0.0)) for y in (y0, y1))] + \
          [p for p in (cx + math.sqrt(max(r * r - (y - cy) ** 2, 0.0)) for y in (y0, y1))]
    pts = sorted(p for p in pts if a < p < b)
    val, _ = integrate.quad(h, a, b, points=pts or None, epsabs=1e-13, epsrel=1e-12, limit=200)
    return val


@pytest.mark.parametrize("r", [0.3, 0.5, 1.0, 2.7, 3.0, 6.0, 9.0, 15.0, 18.0])
@pytest.mark.parametrize("c", [(0.0, 0.0), (0.5, 0.5), (0.37, -0.21), (10.123, 5.777)])
def test_overlap_sums_to_pi_r2(r, c):
    cx, cy = c
    tot = 0.0
    R = int(math.ceil(r)) + 2
    for py in range(int(math.floor(cy)) - R, int(math.floor(cy)) + R + 1):
        for px in range(int(math.floor(cx)) - R, int(math.floor(cx)) + R + 1):
            tot += oracle.overlap(px - .5, px + .5, py - .5, py + .5, cx, cy, r)
    assert abs(tot - math.pi * r * r) <= 1e-12 * max(1.0, math.pi * r * r)


def test_overlap_special_cases():
    # small disk centred in a pixel
    for r in (0.1, 0.25, 0.5):
        assert abs(oracle.overlap(-.5, .5, -.5, .5, 0.0, 0.0, r) - math.pi * r * r) < 1e-15
    # pixel entirely inside the disk
    assert oracle.overlap(2.5, 3.5, 0.5, 1.5, 0.0, 0.0, 5.0) == pytest.approx(1.0, abs=1e-14)
    # entirely outside
    assert oracle.overlap(5.5, 6.5, 5.5, 6.5, 0.0, 0.0, 5.0) == 0.0
    # a pixel quadrant of a centred disk with r >= sqrt(2)/2 covers the pixel
    assert oracle.overlap(-.5, .5, -.5, .5, 0, 0, 0.75) == pytest.approx(1.0, abs=1e-14)
    # r = 0 -> nothing
    assert oracle.overlap(-.5, .5, -.5, .5, 0, 0, 0.0) == 0.0


def test_overlap_exact_outside_and_inside():
    # a pixel whose nearest point is just outside the circle shares no area,
    # and one whose farthest corner is just inside lies wholly in the disk,
    # exactly (no rounding residue of the corner integrals)
    rng = np.random.default_rng(8)
    for _ in range(400):
        cx, cy = rng.uniform(-0.5, 0.5, 2)
        px, py = (int(v) for v in rng.integers(-15, 16, 2))
        x0, x1, y0, y1 = px - .5, px + .5, py - .5, py + .5
        nx = max(x0 - cx, cx - x1, 0.0)
        ny = max(y0 - cy, cy - y1, 0.0)
        fx = max(abs(x0 - cx), abs(x1 - cx))
        fy = max(abs(y0 - cy), abs(y1 - cy))
        gap = 10.0 ** rng.uniform(-9, -2)
        near, far = math.hypot(nx, ny), math.hypot(fx, fy)
        if near > 2 * gap:
            assert oracle.overlap(x0, x1, y0, y1, cx, cy, near * (1 - gap)) == 0.0
        assert oracle.overlap(x0, x1, y0, y1, cx, cy, far * (1 + gap)) == 1.0
    # a circle ending just beyond the last row contributes nothing to the frame
    M = np.ones((50, 40))
    o = oracle.aperture(M, None, [20.3], [52.5 + 1e-6], [3.0], 5.0, 8.0, want_err=False)
    assert o["area"][0, 0] == 0.0 and o["flux"][0, 0] == 0.0


def test_overlap_symmetries_and_quadrature():
    rng = np.random.default_rng(7)
    for _ in range(300):
        r = rng.uniform(0.2, 20.0)
        cx, cy = rng.uniform(-1, 1, 2)
        px, py = rng.integers(-int(r) - 2, int(r) + 3, 2)
        w = oracle.overlap(px - .5, px + .5, py - .5, py + .5, cx, cy, r)
        # x <-> y swap
        w2 = oracle.overlap(py - .5, py + .5, px - .5, px + .5, cy, cx, r)
        # reflection x -> -x
        w3 = oracle.overlap(-px - .5, -px + .5, py - .5, py + .5, -cx, cy, r)
        assert abs(w - w2) < 1e-12 and abs(w - w3) < 1e-12
        assert -1e-12 <= w <= 1.0 + 1e-12   # f64 cancellation ~ eps * r^2
        q = _quad_overlap(px - .5, px + .5, py - .5, py + .5, cx, cy, r)
        assert abs(w - q) < 1e-9, (r, cx, cy, px, py, w, q)


# ----------------------------------------------------------------------------
# aperture sums
# ----------------------------------------------------------------------------
def test_aperture_constant_image():
    H = W = 80
    c = 7.25
    M = np.full((H, W), c)
    R = np.full((H, W), 2.0)
    xs = np.array([40.0, 33.3, 41.71])
    ys = np.array([40.0, 45.6, 38.02])
    radii = [3.0, 6.0, 9.0]
    out = oracle.aperture(M, R, xs, ys, radii, 13.0, 18.0)
    for k, r in enumerate(radii):
        np.testing.assert_allclose(out["area"][:, k], math.pi * r * r, rtol=1e-12)
        np.testing.assert_allclose(out["flux"][:, k], 0.0, atol=1e-9)
    np.testing.assert_allclose(out["bkg"], c, rtol=1e-13)
    assert not np.any(out["flags"])


def test_aperture_recovers_injected_flux():
    H = W = 96
    s = 3.0 / (2 * math.sqrt(2 * math.log(2)))
    F0 = 12345.0
    x0, y0 = 47.3, 49.8
    from scipy.special import erf
    px = np.arange(W)
    py = np.arange(H)
    gx = 0.5 * (erf((px + .5 - x0) / (s * math.sqrt(2))) - erf((px - .5 - x0) / (s * math.sqrt(2))))
    gy = 0.5 * (erf((py + .5 - y0) / (s * math.sqrt(2))) - erf((py - .5 - y0) / (s * math.sqrt(2))))
    M = F0 * np.outer(gy, gx)
    out = oracle.aperture(M, None, [x0], [y0], [20.0], 30.0, 40.0, want_err=False)
    assert out["bkg"][0] == pytest.approx(0.0, abs=1e-12)
    assert out["flux"][0, 0] == pytest.approx(F0, rel=1e-9)


def test_aperture_truncation_flag_and_error():
    M = np.ones((40, 40))
    R = np.full((40, 40), 3.0)
    out = oracle.aperture(M, R, [2.0, 20.0], [20.0, 20.0], [0.4], 5.0, 10.0)
    assert out["flags"][0] & oracle.FLAG_APER_TRUNC
    assert not out["flags"][1] & oracle.FLAG_APER_TRUNC
    # a disk inside one pixel: error = R * w with w = pi r^2
    w = math.pi * 0.16
    assert out["fluxerr"][1, 0] == pytest.approx(3.0 * w, rel=1e-12)
    # Poisson term: sqrt(w^2 (R^2 + M/gain))
    out2 = oracle.aperture(M * 4.0, R, [20.0], [20.0], [0.4], 5.0, 10.0, gain=2.0)
    assert out2["fluxerr"][0, 0] == pytest.approx(w * math.sqrt(9.0 + 2.0), rel=1e-12)


# ----------------------------------------------------------------------------
# matched filter
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 3, 5, 9, 15])
def test_filter_delta_kernel_is_identity(k):
    rng = np.random.default_rng(k)
    M = rng.normal(size=(23, 31)).astype(np.float32).astype(np.float64)
    K = np.zeros((k, k))
    K[k // 2, k // 2] = 2.5   # any scale: the kernel is normalised to unit sum
    F = oracle.filter_image(M, K)
    assert np.array_equal(F, M)


def test_filter_constant_and_scipy_reflect():
    rng = np.random.default_rng(3)
    M = np.full((17, 29), 3.5)
    K = gaussian_kernel(9, 3.5).astype(np.float64)
    np.testing.assert_allclose(oracle.filter_image(M, K), 3.5, rtol=1e-14)
    # random image and an asymmetric kernel against scipy.ndimage.correlate
    # (mode 'reflect' is the half-sample mirror)
    M = rng.normal(size=(37, 23))
    K = rng.uniform(0.1, 1.0, size=(5, 7))
    ref = ndimage.correlate(M, K / K.sum(), mode="reflect")
    np.testing.assert_allclose(oracle.filter_image(M, K), ref, rtol=1e-12, atol=1e-12)
    # kernel larger than the frame: repeated reflection
    M = rng.normal(size=(3, 4))
    K = rng.uniform(0.1, 1.0, size=(9, 9))
    ref = ndimage.correlate(M, K / K.sum(), mode="reflect")
    np.testing.assert_allclose(oracle.filter_image(M, K), ref, rtol=1e-12, atol=1e-12)
    # zero-sum kernel is applied as given
    K = np.array([[0, 0, 0], [-1, 0, 1], [0, 0, 0]], float)
    ref = ndimage.correlate(M, K, mode="reflect")
    np.testing.assert_allclose(oracle.filter_image(M, K), ref, atol=1e-14)


# ----------------------------------------------------------------------------
# spline interpolation of the mesh grid
# ----------------------------------------------------------------------------
def _knots(n, m):
    return np.array([0.5 * (k * m + min(k * m + m, n) - 1) for k in range(-(-n // m))])


@pytest.mark.parametrize("nx,ny", [(5, 4), (1, 6), (2, 3), (7, 1), (2, 2), (3, 3)])
def test_spline_matches_scipy_natural(nx, ny):
    rng = np.random.default_rng(nx * 10 + ny)
    mw, mh = 16, 12
    W, H = nx * mw - 5, ny * mh - 3          # ragged last meshes
    nx_, ny_ = -(-W // mw), -(-H // mh)
    assert (nx_, ny_) == (nx, ny)
    G = rng.normal(size=(ny, nx)) * 10 + 100
    cx, cy = _knots(W, mw), _knots(H, mh)

    def natural(t, f):
        if len(t) == 1:
            return lambda x: np.full_like(np.asarray(x, float), f[0])
        if len(t) == 2:
            return lambda x: f[0] + (f[1] - f[0]) / (t[1] - t[0]) * (np.asarray(x) - t[0])
        cs = interpolate.CubicSpline(t, f, bc_type="natural")
        d0, d1 = cs(t[0], 1), cs(t[-1], 1)

        def ev(x):
            x = np.asarray(x, float)
            out = cs(np.clip(x, t[0], t[-1]))
            out = np.where(x < t[0], f[0] + d0 * (x - t[0]), out)
            out = np.where(x > t[-1], f[-1] + d1 * (x - t[-1]), out)
            return out
        return ev

    ys = np.arange(H)
    xs = np.arange(W)
    V = np.stack([natural(cy, G[:, i])(ys) for i in range(nx)], axis=1)   # (H, nx)
    ref = np.stack([natural(cx, V[y])(xs) for y in range(H)])
    got = oracle.grid_map(G, W, H, mw, mh)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-10)


def test_spline_reproduces_planes():
    mw = mh = 10
    W, H = 57, 43
    cx, cy = _knots(W, mw), _knots(H, mh)
    G = 3.0 + 0.25 * cx[None, :] - 0.5 * cy[:, None]
    got = oracle.grid_map(G, W, H, mw, mh)
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    np.testing.assert_allclose(got, 3.0 + 0.25 * x - 0.5 * y, atol=1e-11)


# ----------------------------------------------------------------------------
# mesh statistics
# ----------------------------------------------------------------------------
def test_mesh_constant_sky():
    img = np.full((100, 130), 812.5)
    st = oracle.mesh_stats(img, 32, 32)
    assert np.all(st["back"] == 812.5) and np.all(st["rms"] == 0.0)
    p = Params(mesh_w=32, mesh_h=32, mesh_filter=3)
    bk = oracle.background(img, p)
    assert np.all(bk.B == 812.5) and np.all(bk.R == 0.0)


def test_mesh_no_clip_case_equals_numpy():
    # a uniform spread never reaches 3 sigma from its median: no pixel is
    # clipped, sigma is unchanged, so back = mean and rms = std (numpy)
    rng = np.random.default_rng(11)
    v = rng.uniform(0, 1, 4096)
    st = oracle.mesh_one(v)
    assert st["iters"] == 1
    assert st["back"] == pytest.approx(np.mean(v), rel=1e-14)
    assert st["rms"] == pytest.approx(np.std(v), rel=1e-13)
    assert st["med"] == pytest.approx(np.median(v), rel=0, abs=0)


def test_mesh_outlier_removed_and_mode_rule():
    rng = np.random.default_rng(12)
    core = rng.uniform(-1, 1, 999)
    v = np.concatenate([core, [1e4]])
    st = oracle.mesh_one(v)
    # the outlier inflates sigma0 far beyond 20%: mode = 2.5 med - 1.5 mean of the rest
    assert st["sigma0"] == pytest.approx(np.std(v), rel=1e-13)
    assert st["rms"] == pytest.approx(np.std(core), rel=1e-12)
    assert st["back"] == pytest.approx(2.5 * np.median(core) - 1.5 * np.mean(core), rel=1e-12, abs=1e-12)
    # a small symmetric contamination keeps sigma within 20%: clipped mean
    v2 = np.concatenate([rng.normal(0, 1, 20000), [4.5, -4.6]])
    st2 = oracle.mesh_one(v2)
    assert abs(st2["rms"] - st2["sigma0"]) < 0.2 * st2["sigma0"]
    assert st2["back"] == pytest.approx(st2["mean"], rel=0, abs=0)


def _brute_mesh(v, clip=3.0, crowd=0.2, a=2.5, b=1.5, max_iter=100):
    """Independent re-statement with numpy primitives (median, std, masks)."""
    S = np.asarray(v, float)
    s0 = np.std(S) if S.min() != S.max() else 0.0
    if s0 == 0:
        return S[0], 0.0
    for _ in range(max_iter):
        med = np.median(S)
        sd = np.std(S) if S.min() != S.max() else 0.0
        keep = S[np.abs(S - med) <= clip * sd]
        if keep.size == S.size or keep.size == 0:
            break
        S = keep
    med, mean = np.median(S), np.mean(S)
    sd = np.std(S) if S.min() != S.max() else 0.0
    back = mean if abs(sd - s0) < crowd * s0 else a * med - b * mean
    return back, sd


def test_mesh_against_numpy_restatement():
    rng = np.random.default_rng(5)
    for trial in range(40):
        n = int(rng.integers(1, 3000))
        v = rng.normal(1000, 30, n)
        if trial % 3 == 0:
            v[: n // 10] += rng.uniform(100, 5e4, n // 10)   # a star in the mesh
        if trial % 5 == 0:
            v = np.round(v)                                  # integer data with ties
        b, s = _brute_mesh(v)
        st = oracle.mesh_one(v)
        assert st["back"] == pytest.approx(b, rel=1e-12, abs=1e-9)
        assert st["rms"] == pytest.approx(s, rel=1e-12, abs=1e-12)


def _brute_mesh_policy(v, eps, lo, hi, flip, clip=3.0, crowd=0.2, a=2.5, b=1.5, max_iter=100):
    """numpy re-statement of the clip loop in which every decision whose
    relative margin |(|v - med| - k sigma)| / (k sigma) is below eps is forced:
    0 = as computed, 1 = keep, 2 = drop (lo: values below the median, hi: the
    rest); flip: the estimator decision is flipped when its margin is below eps."""
    S = np.sort(np.asarray(v, float))
    s0 = np.std(S)
    for _ in range(max_iter):
        med = np.median(S)
        lim = clip * np.std(S)
        d = np.abs(S - med)
        keep = d <= lim
        amb = np.abs(d - lim) / lim < eps
        pol = np.where(S < med, lo, hi)
        keep = np.where(amb & (pol == 1), True, np.where(amb & (pol == 2), False, keep))
        if keep.all() or not keep.any():
            break
        S = S[keep]
    med, mean, sd = np.median(S), np.mean(S), np.std(S)
    use_mean = abs(sd - s0) < crowd * s0
    if flip and abs(abs(sd - s0) - crowd * s0) / s0 < eps:
        use_mean = not use_mean
    return (mean if use_mean else a * med - b * mean), sd


def test_mesh_branch_policy_against_numpy_restatement():
    # a wide band (5% of the clip limit) makes many decisions ambiguous, so
    # every forced branch changes the result; each policy must equal the
    # numpy re-statement of the same forcing, and policy 0 the plain method
    rng = np.random.default_rng(9)
    eps = 0.05
    changed = 0
    for trial in range(12):
        n = int(rng.integers(200, 3000))
        v = rng.normal(500, 20, n)
        v[: n // 8] += rng.uniform(50, 3000, n // 8)
        if trial % 3 == 0:
            v = np.round(v)
        plain = oracle.mesh_one(v)
        st0 = oracle.mesh_one_policy(v, 0, eps, eps)
        assert (st0["back"], st0["rms"], st0["iters"]) == (plain["back"], plain["rms"], plain["iters"])
        distinct = set()
        for pol in oracle.MESH_POLICIES:
            lo, hi, flip = pol & 3, (pol >> 2) & 3, bool(pol & 16)
            st = oracle.mesh_one_policy(v, pol, eps, eps)
            bb, ss = _brute_mesh_policy(v, eps, lo, hi, flip)
            assert st["back"] == pytest.approx(bb, rel=1e-12, abs=1e-9), (trial, pol)
            assert st["rms"] == pytest.approx(ss, rel=1e-12, abs=1e-12), (trial, pol)
            distinct.add(round(st["back"], 9))
        changed += len(distinct) > 1
    assert changed >= 8, changed
    # with a band of zero width no policy changes anything
    v = rng.normal(0, 1, 1000)
    ref = oracle.mesh_one(v)
    for pol in oracle.MESH_POLICIES:
        st = oracle.mesh_one_policy(v, pol, 0.0, 0.0)
        assert (st["back"], st["rms"]) == (ref["back"], ref["rms"])
    with pytest.raises(RuntimeError):
        oracle.mesh_one_policy(v, 3, 0.1, 0.1)


def test_mesh_decision_margins_against_numpy_restatement():
    """The clip margin is the smallest | |v - med| - k sigma | / (k sigma) over
    every value of every pass, the mode margin | |sigma - sigma0| - crowd
    sigma0 | / sigma0 at the end: both recomputed here with numpy."""
    rng = np.random.default_rng(13)
    for trial in range(25):
        n = int(rng.integers(50, 2500))
        v = rng.normal(800, 25, n)
        if trial % 2 == 0:
            v[: n // 6] += rng.uniform(30, 2000, n // 6)
        if trial % 4 == 0:
            v = np.round(v)
        S = np.sort(v)
        s0 = np.std(S)
        mclip = np.inf
        for _ in range(100):
            med, lim = np.median(S), 3.0 * np.std(S)
            d = np.abs(S - med)
            mclip = min(mclip, float(np.min(np.abs(d - lim) / lim)))
            keep = d <= lim
            if keep.all() or not keep.any():
                break
            S = S[keep]
        mmode = abs(abs(np.std(S) - s0) - 0.2 * s0) / s0
        st = oracle.mesh_one(v)
        assert st["margin_clip"] == pytest.approx(mclip, rel=1e-9, abs=1e-15), trial
        assert st["margin_mode"] == pytest.approx(mmode, rel=1e-9, abs=1e-15), trial
    # a constant mesh decides nothing: both margins infinite
    st = oracle.mesh_one(np.full(100, 7.0))
    assert st["margin_clip"] == np.inf and st["margin_mode"] == np.inf


def test_mesh_gaussian_sky_statistics():
    rng = np.random.default_rng(2)
    c, sn = 1000.0, 10.0
    img = c + rng.normal(0, sn, size=(256, 256))
    st = oracle.mesh_stats(img, 64, 64)
    n = 64 * 64
    assert np.all(np.abs(st["back"] - c) < 5 * sn / math.sqrt(n) * 3)
    assert np.all(np.abs(st["rms"] / sn - 1) < 0.05)


def test_background_linear_ramp_is_exact():
    # symmetric distribution in every mesh (actual-centre knots) and a spline
    # that reproduces lines: B equals the plane (filter off)
    W, H = 200, 150
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    img = 500.0 + 0.3 * x + 0.1 * y + 0.0 * x * y
    p = Params(mesh_w=32, mesh_h=32, mesh_filter=1)
    bk = oracle.background(img, p)
    np.testing.assert_allclose(bk.B, img, rtol=0, atol=1e-9)


def test_median_filter_against_scipy():
    rng = np.random.default_rng(4)
    G = rng.normal(size=(9, 12))
    got = oracle.median_filter(G, 3)
    # interior: plain 3x3 median (scipy.ndimage.median_filter)
    ref = ndimage.median_filter(G, size=3, mode="nearest")
    np.testing.assert_allclose(got[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=0, atol=0)
    # corner: mean of the two middle values of the 2x2 window
    w = np.sort(G[:2, :2].ravel())
    assert got[0, 0] == pytest.approx(0.5 * (w[1] + w[2]), abs=0)
    assert np.array_equal(oracle.median_filter(G, 1), G)


# ----------------------------------------------------------------------------
# connected components
# ----------------------------------------------------------------------------
def _canon_scipy(mask, conn):
    st = ndimage.generate_binary_structure(2, 1 if conn == 4 else 2)
    lab, n = ndimage.label(mask, structure=st)
    # renumber by first raster pixel
    order = {}
    flat = lab.ravel()
    out = np.zeros_like(flat)
    nxt = 0
    for i, l in enumerate(flat):
        if l and l not in order:
            nxt += 1
            order[l] = nxt
    for l, k in order.items():
        out[flat == l] = k
    return out.reshape(mask.shape), n


@pytest.mark.parametrize("conn", [4, 8])
def test_ccl_all_4x4_masks(conn):
    st = ndimage.generate_binary_structure(2, 1 if conn == 4 else 2)
    for bits in range(1 << 16):
        m = np.array([(bits >> i) & 1 for i in range(16)], bool).reshape(4, 4)
        seg, n = oracle.label_mask(m, conn)
        lab, n2 = ndimage.label(m, structure=st)
        assert n == n2
        # same partition, numbered by first raster pixel
        if n:
            firsts = [np.flatnonzero(lab.ravel() == k)[0] for k in range(1, n2 + 1)]
            order = np.argsort(firsts)
            for newk, oldk in enumerate(order, start=1):
                assert np.array_equal(seg == newk, lab == oldk + 1)


@pytest.mark.parametrize("conn", [4, 8])
def test_ccl_random_and_adversarial(conn):
    rng = np.random.default_rng(conn)
    shapes = []
    for d in (0.05, 0.3, 0.5, 0.6, 0.95):
        shapes.append(rng.random((64, 64)) < d)
    # spiral
    sp = np.zeros((41, 41), bool)
    x = y = 20
    dx, dy, step = 1, 0, 1
    while 0 <= x < 41 and 0 <= y < 41:
        for _ in range(2):
            for _ in range(step):
                if 0 <= x < 41 and 0 <= y < 41:
                    sp[y, x] = True
                x += dx * 1
                y += dy * 1
            dx, dy = -dy, dx
        step += 2
    shapes.append(sp)
    comb = np.zeros((30, 70), bool)
    comb[0, :] = True
    comb[:, ::2] = True
    shapes.append(comb)
    snake = np.zeros((70, 130), bool)
    for r in range(0, 70, 2):
        snake[r, :] = True
        snake[r + 1 if r + 1 < 70 else r, (129 if (r // 2) % 2 == 0 else 0)] = True
    shapes.append(snake)
    shapes.append(np.ones((33, 65), bool))
    checker = (np.add.outer(np.arange(20), np.arange(21)) % 2).astype(bool)
    shapes.append(checker)
    for m in shapes:
        seg, n = oracle.label_mask(m, conn)
        ref, n2 = _canon_scipy(m, conn)
        assert n == n2
        assert np.array_equal(seg, ref)


def test_minarea_and_seg_convention():
    m = np.zeros((10, 10), bool)
    m[1, 1] = True                      # single pixel: dropped
    m[5:7, 5:8] = True                  # 6 pixels: kept
    F = m.astype(float)
    seg, n = oracle.threshold_label(F, np.zeros_like(F), 0.0, 5, 8)
    assert n == 1
    assert seg[1, 1] == -1 and np.all(seg[5:7, 5:8] == 1) and seg[0, 0] == 0
    # strict threshold: F == t R is not detected
    F = np.full((4, 4), 3.0)
    R = np.full((4, 4), 2.0)
    _, n = oracle.threshold_label(F, R, 1.5, 1, 8)
    assert n == 0
    _, n = oracle.threshold_label(F + 1e-12, R, 1.5, 1, 8)
    assert n == 1


# ----------------------------------------------------------------------------
# moments
# ----------------------------------------------------------------------------
def _measure(M, conn=8, I=None, sat=np.inf):
    seg, n = oracle.threshold_label(np.where(M != 0, 1.0, 0.0), np.zeros_like(M), 0.0, 1, conn)
    return oracle.measure(M if I is None else I, M, seg, n, sat), seg


def test_moments_closed_forms():
    M = np.zeros((12, 14))
    M[3, 9] = 5.0
    cat, _ = _measure(M)
    assert cat["x"][0] == 9.0 and cat["y"][0] == 3.0
    assert cat["x2"][0] == 0 and cat["y2"][0] == 0 and cat["xy"][0] == 0
    assert cat["flux"][0] == 5.0 and cat["npix"][0] == 1 and cat["pmin"][0] == 3 * 14 + 9
    M = np.zeros((12, 14))
    M[4:7, 2:5] = 2.0
    cat, _ = _measure(M)
    assert cat["x"][0] == pytest.approx(3.0) and cat["y"][0] == pytest.approx(5.0)
    assert cat["x2"][0] == pytest.approx(2.0 / 3.0) and cat["y2"][0] == pytest.approx(2.0 / 3.0)
    assert cat["xy"][0] == pytest.approx(0.0, abs=1e-15)
    assert (cat["xmin"][0], cat["xmax"][0], cat["ymin"][0], cat["ymax"][0]) == (2, 4, 4, 6)
    M = np.zeros((5, 5))
    M[2, 1:3] = 1.0
    cat, _ = _measure(M)
    assert cat["x2"][0] == pytest.approx(0.25) and cat["y2"][0] == 0.0


def test_moments_symmetry_translation_and_nonpos():
    rng = np.random.default_rng(9)
    blob = rng.uniform(1, 5, (7, 7))
    blob = blob + blob[::-1, :]                  # mirror symmetric in y
    blob = blob + blob[:, ::-1]                  # and in x
    M = np.zeros((30, 30))
    M[10:17, 12:19] = blob
    cat, _ = _measure(M)
    assert cat["xy"][0] == pytest.approx(0.0, abs=1e-12)
    assert cat["x"][0] == pytest.approx(15.0) and cat["y"][0] == pytest.approx(13.0)
    M2 = np.zeros((30, 30))
    M2[13:20, 5:12] = blob
    cat2, _ = _measure(M2)
    assert cat2["x"][0] - cat["x"][0] == pytest.approx(-7.0)
    assert cat2["y"][0] - cat["y"][0] == pytest.approx(3.0)
    for k in ("x2", "y2", "xy"):
        assert cat2[k][0] == pytest.approx(cat[k][0], rel=1e-12, abs=1e-12)
    # sum M <= 0: unit weights and NONPOS
    M = np.zeros((9, 9))
    M[2:5, 2:5] = -1.0
    M[3, 3] = 0.5
    seg, n = oracle.threshold_label(np.where(M != 0, 1.0, 0.0), np.zeros_like(M), 0.0, 1, 8)
    cat = oracle.measure(M, M, seg, n)
    assert cat["flags"][0] & oracle.FLAG_NONPOS
    assert cat["x"][0] == pytest.approx(3.0) and cat["x2"][0] == pytest.approx(2.0 / 3.0)


def test_flags_edge_and_saturation():
    M = np.zeros((10, 10))
    M[0:2, 4:6] = 1.0
    M[6:8, 6:8] = 2.0
    I = M.copy()
    I[7, 7] = 70000.0
    cat, _ = _measure(M, I=I, sat=65535.0)
    assert cat["flags"][0] & oracle.FLAG_EDGE and not cat["flags"][0] & oracle.FLAG_SATURATED
    assert cat["flags"][1] & oracle.FLAG_SATURATED and not cat["flags"][1] & oracle.FLAG_EDGE
    assert cat["peak"][1] == 2.0


# ----------------------------------------------------------------------------
# whole chain: statistical sanity on injected stars
# ----------------------------------------------------------------------------
def test_chain_finds_injected_stars():
    fr = make_frame("c1", seed=3, W=256, H=256, nstars=12)
    p = fr.params
    res = oracle.run(fr.image, p)
    t = fr.truth
    bright = t["flux"] > 2e4
    found = 0
    for x0, y0 in zip(t["x"][bright], t["y"][bright]):
        d = np.hypot(res.cat["x"] - x0, res.cat["y"] - y0)
        if d.size and d.min() < 1.0:
            found += 1
    assert found == bright.sum()
    # large-aperture fluxes of bright isolated stars approach the injected flux
    assert np.all(np.isfinite(res.phot["flux"]))


# ----------------------------------------------------------------------------
# peak detection (local maxima of the significance, first-moment centroids)
# ----------------------------------------------------------------------------
def test_peaks_equal_scipy_maximum_filter():
    # continuous random significance (no ties): peaks = above threshold and
    # equal to the maximum filter over the window truncated at the edges
    from scipy import ndimage
    rng = np.random.default_rng(21)
    for trial in range(8):
        H, W = rng.integers(20, 70, 2)
        F = rng.normal(0, 3, (H, W))
        R = rng.uniform(0.5, 2.0, (H, W))
        M = rng.normal(0, 1, (H, W))
        sep = int(rng.integers(0, 5))
        t = 1.0
        nu = F / R
        mx = ndimage.maximum_filter(nu, size=2 * sep + 1, mode="constant", cval=-np.inf)
        want = np.flatnonzero(((F > t * R) & (nu == mx)).ravel())
        got = oracle.peaks(M, M, F, R, t, sep, 1)
        np.testing.assert_array_equal(got["pmin"], want)
        assert got["n"] == want.size
        np.testing.assert_array_equal(got["peak"], nu.ravel()[want])


def test_peaks_plateau_and_separation():
    F = np.zeros((20, 30))
    R = np.ones_like(F)
    F[5:8, 10:13] = 7.0                 # a 3 x 3 plateau: one peak, its first pixel
    F[12, 4] = 5.0                      # two maxima 3 px apart
    F[12, 7] = 6.0
    M = F.copy()
    got = oracle.peaks(M, M, F, R, 1.0, 3, 1)
    assert list(got["pmin"]) == [5 * 30 + 10, 12 * 30 + 7]
    got = oracle.peaks(M, M, F, R, 1.0, 2, 1)
    assert list(got["pmin"]) == [5 * 30 + 10, 12 * 30 + 4, 12 * 30 + 7]
    # threshold strict: F == t R is not a candidate
    got = oracle.peaks(M, M, F, R, 7.0, 1, 1)
    assert list(got["pmin"]) == []


def test_peak_centroid_closed_forms():
    # a blob symmetric about a pixel centre: centroid at that pixel, xy = 0
    H, W = 41, 37
    yy, xx = np.mgrid[0:H, 0:W]
    M = np.exp(-((xx - 17) ** 2 + (yy - 21) ** 2) / (2 * 1.7 ** 2)) * 100
    F, R = M.copy(), np.ones_like(M)
    got = oracle.peaks(M, M, F, R, 1.0, 3, 4)
    assert got["n"] == 1 and got["pmin"][0] == 21 * W + 17
    assert got["x"][0] == 17.0 and got["y"][0] == 21.0 and abs(got["xy"][0]) < 1e-14
    assert got["x2"][0] == pytest.approx(got["y2"][0], rel=1e-14)
    # a uniform 3 x 3 block with a 1-pixel window: x2 = y2 = 2/3
    M = np.zeros((9, 9))
    M[3:6, 3:6] = 2.0
    F = M.copy()
    F[4, 4] = 3.0
    got = oracle.peaks(M, M, F, np.ones_like(F), 1.0, 1, 1)
    assert got["n"] == 1 and got["x"][0] == 4.0 and got["y"][0] == 4.0
    assert got["x2"][0] == pytest.approx(2 / 3, rel=1e-14) and got["y2"][0] == pytest.approx(2 / 3, rel=1e-14)
    assert got["flux"][0] == pytest.approx(18.0) and got["npix"][0] == 9
    # translation invariance of the centroid offset
    rng = np.random.default_rng(5)
    M = rng.uniform(-1, 5, (30, 30))
    F = np.zeros_like(M)
    F[12, 14] = 10.0
    a = oracle.peaks(M, M, F, np.ones_like(F), 1.0, 2, 3)
    M2 = np.roll(np.roll(M, 4, axis=0), 3, axis=1)
    F2 = np.roll(np.roll(F, 4, axis=0), 3, axis=1)
    b = oracle.peaks(M2, M2, F2, np.ones_like(F2), 1.0, 2, 3)
    assert b["x"][0] == pytest.approx(a["x"][0] + 3, abs=1e-12)
    assert b["y"][0] == pytest.approx(a["y"][0] + 4, abs=1e-12)


def test_peak_centroid_against_numpy_and_flags():
    rng = np.random.default_rng(8)
    H, W = 60, 50
    I = rng.uniform(0, 100, (H, W))
    I[2, 30] = 65535.0
    M = rng.normal(2, 3, (H, W))
    F = rng.normal(0, 2, (H, W))
    R = rng.uniform(0.8, 1.2, (H, W))
    c = 3
    got = oracle.peaks(I, M, F, R, 1.5, 2, c, sat=65535.0)
    assert got["n"] > 10
    for k in range(got["n"]):
        y, x = divmod(int(got["pmin"][k]), W)
        y0, y1, x0, x1 = max(y - c, 0), min(y + c, H - 1), max(x - c, 0), min(x + c, W - 1)
        win = M[y0:y1 + 1, x0:x1 + 1]
        w = np.maximum(win, 0)
        gy, gx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        mx, my = (w * (gx - x)).sum() / w.sum(), (w * (gy - y)).sum() / w.sum()
        assert got["x"][k] == pytest.approx(x + mx, abs=1e-12) and got["y"][k] == pytest.approx(y + my, abs=1e-12)
        assert got["x2"][k] == pytest.approx((w * (gx - x) ** 2).sum() / w.sum() - mx * mx, abs=1e-10)
        assert got["flux"][k] == pytest.approx(win.sum(), abs=1e-10)
        edge = (x - c < 0) or (y - c < 0) or (x + c >= W) or (y + c >= H)
        assert bool(got["flags"][k] & oracle.FLAG_EDGE) == edge
        sat = bool((I[y0:y1 + 1, x0:x1 + 1] >= 65535.0).any())
        assert bool(got["flags"][k] & oracle.FLAG_SATURATED) == sat
    # capacity: the first peaks in raster order are kept, the count is whole
    few = oracle.peaks(I, M, F, R, 1.5, 2, c, sat=65535.0, cap=3)
    assert few["n"] == got["n"] and list(few["pmin"]) == list(got["pmin"][:3])


# ----------------------------------------------------------------------------
# growth curves on top-hat kernels
# ----------------------------------------------------------------------------
def test_growth_radii_rule():
    # ceil(0.75 F) .. ceil(5 F): FWHM 3 gives 3..15
    assert list(oracle.growth_radii(3.0)) == list(range(3, 16))
    assert list(oracle.growth_radii(3.5)) == list(range(3, 19))
    assert list(oracle.growth_radii(4.0)) == list(range(3, 21))   # 0.75 * 4 = 3 exactly
    assert list(oracle.growth_radii(1.0)) == [1, 2, 3, 4, 5]
    assert list(oracle.growth_radii(0.5)) == [1, 2, 3]
    assert list(oracle.growth_radii(2.2)) == list(range(2, 12))
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(RuntimeError):
            oracle.growth_radii(bad)


@pytest.mark.parametrize("r", [1, 2, 3, 6, 15])
def test_tophat_taps_against_quadrature(r):
    t = oracle.tophat_taps(r)
    assert t.shape == (2 * r + 1, 2 * r + 1)
    # sum of the taps = pi r^2; eight-fold symmetry (up to the corner sums' rounding)
    assert abs(t.sum() - math.pi * r * r) <= 1e-13 * math.pi * r * r
    for tt in (t[::-1, :], t[:, ::-1], t.T):
        np.testing.assert_allclose(t, tt, rtol=0, atol=1e-14 * r * r)
    # interior taps exactly 1, taps wholly outside exactly 0, the rest by quadrature
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = t[dy + r, dx + r]
            far = math.hypot(abs(dx) + .5, abs(dy) + .5)
            near = math.hypot(max(abs(dx) - .5, 0), max(abs(dy) - .5, 0))
            if far <= r:
                assert w == 1.0
            elif near >= r:
                assert w == 0.0
            elif (dx + dy) % 3 == 0 or r <= 3:
                q = _quad_overlap(dx - .5, dx + .5, dy - .5, dy + .5, 0.0, 0.0, float(r))
                assert abs(w - q) < 1e-10, (r, dx, dy, w, q)


def _segment(d, r):
    """Area of the part of a disk of radius r beyond a line at distance d from its centre."""
    if d >= r:
        return 0.0
    return r * r * math.acos(d / r) - d * math.sqrt(r * r - d * d)


def test_growth_constant_image_and_one_edge():
    H, W = 70, 90
    c, v = 3.5, 0.75
    M = np.full((H, W), c)
    V = np.full((H, W), v)
    radii = [2, 3, 5, 8, 11]
    # interior sources: c pi r^2, v pi r^2 (a variance through the squared taps would differ)
    xs = np.array([45.2, 44.5, 50.49])
    ys = np.array([35.0, 30.7, 29.51])
    o = oracle.growth(M, V, xs, ys, radii)
    for k, r in enumerate(radii):
        np.testing.assert_allclose(o["area"][:, k], math.pi * r * r, rtol=1e-13)
        np.testing.assert_allclose(o["sum"][:, k], c * math.pi * r * r, rtol=1e-13)
        np.testing.assert_allclose(o["var"][:, k], v * math.pi * r * r, rtol=1e-13)
    assert not np.any(o["flags"])
    # a source at column cx near the left edge only: the frame edge x = -1/2 is a
    # straight line at distance cx + 1/2 from the centre, cutting off a segment
    for cx in (0, 1, 3, 6, 10):
        o = oracle.growth(M, V, [cx + 0.2], [35.0], radii)
        for k, r in enumerate(radii):
            want = math.pi * r * r - _segment(cx + 0.5, r)
            assert abs(o["area"][0, k] - want) < 1e-11 * r * r, (cx, r, o["area"][0, k], want)
            assert abs(o["sum"][0, k] - c * want) < 1e-11 * c * r * r
        assert bool(o["flags"][0] & oracle.FLAG_APER_TRUNC) == (cx < max(radii))


def _fft_correlate_zero_padded(M, t):
    """Correlation of the zero-padded frame with taps t by the FFT (the
    paper's evaluation), full output indexed like M."""
    H, W = M.shape
    r = t.shape[0] // 2
    sh = (H + 2 * r, W + 2 * r)
    FM = np.fft.rfft2(M, sh)
    FK = np.fft.rfft2(t[::-1, ::-1], sh)   # correlation = convolution with the flipped kernel
    full = np.fft.irfft2(FM * FK, sh)
    return full[r:r + H, r:r + W]


def test_growth_equals_scipy_correlate_and_fft():
    rng = np.random.default_rng(11)
    H, W = 61, 83
    M = rng.normal(0, 10, (H, W)) + 20 * np.sin(np.arange(W) / 7.0)[None, :] + np.arange(H)[:, None]
    V = rng.uniform(0.5, 4.0, (H, W))
    radii = [1, 3, 4, 7, 12]
    xs = rng.uniform(-0.49, W - 0.51, 60)
    ys = rng.uniform(-0.49, H - 0.51, 60)
    xs[:4] = [0.0, W - 1.0, 10.5, 20.5 - 1e-12]
    ys[:4] = [0.0, H - 1.0, 7.5, 30.5]
    o = oracle.growth(M, V, xs, ys, radii)
    cx = np.floor(xs + 0.5).astype(int)
    cy = np.floor(ys + 0.5).astype(int)
    assert cx[2] == 11 and cx[3] == 20
    for k, r in enumerate(radii):
        t = oracle.tophat_taps(r)
        cm = ndimage.correlate(M, t, mode="constant", cval=0.0)
        cv = ndimage.correlate(V, t, mode="constant", cval=0.0)
        ca = ndimage.correlate(np.ones_like(M), t, mode="constant", cval=0.0)
        scale = ndimage.correlate(np.abs(M), t, mode="constant", cval=0.0)
        np.testing.assert_allclose(o["sum"][:, k], cm[cy, cx], rtol=0, atol=1e-12 * scale[cy, cx].max())
        np.testing.assert_allclose(o["var"][:, k], cv[cy, cx], rtol=1e-13)
        np.testing.assert_allclose(o["area"][:, k], ca[cy, cx], rtol=1e-13)
        ff = _fft_correlate_zero_padded(M, t)
        np.testing.assert_allclose(o["sum"][:, k], ff[cy, cx], rtol=0, atol=1e-10 * scale[cy, cx].max())
    trunc = (cx - max(radii) < 0) | (cx + max(radii) >= W) | (cy - max(radii) < 0) | (cy + max(radii) >= H)
    np.testing.assert_array_equal((o["flags"] & oracle.FLAG_APER_TRUNC) != 0, trunc)


def test_growth_delta_reads_the_centroid_pixel_and_is_monotone():
    H, W = 40, 50
    M = np.zeros((H, W))
    M[20, 11] = 1.0
    radii = [1, 2]
    t1 = oracle.tophat_taps(1)
    # x = 10.5 rounds to pixel 11 (the delta at the kernel centre); 10.49 to pixel 10
    o = oracle.growth(M, None, [10.5, 10.49, 11.0], [20.0, 20.0, 19.4], radii)
    assert o["sum"][0, 0] == t1[1, 1] == 1.0
    assert o["sum"][1, 0] == t1[1, 2]
    assert o["sum"][2, 0] == t1[2, 1]   # reads (11, 19): the delta is one row below
    # sources far off the frame: nothing reaches it
    o = oracle.growth(M, None, [-40.0, 1e30, 10.0], [5.0, 5.0, float("nan")], radii)
    assert not np.any(o["sum"]) and not np.any(o["area"])
    assert np.all(o["flags"] == oracle.FLAG_APER_TRUNC)
    # non-negative frames: growth curves are non-decreasing in r
    rng = np.random.default_rng(3)
    P = rng.uniform(0, 5, (H, W))
    o = oracle.growth(P, P, rng.uniform(0, W, 30), rng.uniform(0, H, 30), list(range(1, 13)))
    assert np.all(np.diff(o["sum"], axis=1) >= 0) and np.all(np.diff(o["area"], axis=1) > 0)


# ----------------------------------------------------------------------------
# spatially varying matched filter
# ----------------------------------------------------------------------------
def _eigen_model(K, kw, kh, seed):
    """A reference kernel of unit sum and K zero-sum deviation patterns."""
    rng = np.random.default_rng(seed)
    P0 = gaussian_kernel(kw, 2.5).astype(np.float64) if kw == kh else rng.random((kh, kw))
    P0 = P0 / P0.sum()
    modes = rng.normal(0, 0.02, (K, kh, kw))
    modes -= modes.mean(axis=(1, 2), keepdims=True)
    return np.concatenate([P0[None], modes])


def test_varying_filter_without_modes_is_the_plain_filter():
    rng = np.random.default_rng(4)
    M = rng.normal(0, 10, (37, 53))
    ks = _eigen_model(0, 7, 7, 1)
    S = oracle.filter_varying(M, ks)
    np.testing.assert_allclose(S, oracle.filter_image(M, ks[0]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(S, ndimage.correlate(M, ks[0], mode="reflect"), rtol=0, atol=1e-12)


def test_varying_filter_with_constant_maps_is_one_correlation():
    rng = np.random.default_rng(5)
    H, W = 41, 29
    M = rng.normal(0, 10, (H, W)) + np.arange(W)[None, :]
    ks = _eigen_model(5, 9, 5, 2)
    a = rng.normal(0, 2, 5)
    coef = np.broadcast_to(a[:, None, None], (5, H, W)).copy()
    S = oracle.filter_varying(M, ks, coef)
    Keff = ks[0] + np.tensordot(a, ks[1:], axes=1)
    np.testing.assert_allclose(S, ndimage.correlate(M, Keff, mode="reflect"), rtol=0, atol=1e-11)


def test_varying_filter_is_the_local_psf_at_each_pixel():
    """Brute force: at each output pixel assemble that pixel's kernel
    P0 + sum c_k(x, y) e_k and correlate the mirrored window with it."""
    rng = np.random.default_rng(6)
    H, W = 23, 31
    K, kh, kw = 3, 5, 7
    M = rng.normal(0, 10, (H, W))
    ks = _eigen_model(K, kw, kh, 3)
    yy, xx = np.mgrid[0:H, 0:W]
    coef = np.stack([np.sin(xx / 5.0) + yy / 10.0, np.cos(yy / 3.0) * xx / 20.0, (xx - yy) / 15.0])
    S = oracle.filter_varying(M, ks, coef)
    Mp = np.pad(M, ((kh // 2, kh // 2), (kw // 2, kw // 2)), mode="symmetric")   # half-sample mirror
    for y in range(H):
        for x in range(W):
            Kp = ks[0] + np.tensordot(coef[:, y, x], ks[1:], axes=1)
            want = float(np.sum(Kp * Mp[y:y + kh, x:x + kw]))
            assert abs(S[y, x] - want) <= 1e-11 * (1 + abs(want)), (x, y)


def test_varying_filter_binned_maps_equal_expanded_maps():
    rng = np.random.default_rng(7)
    H, W, b = 45, 38, 8
    M = rng.normal(0, 10, (H, W))
    ks = _eigen_model(2, 5, 5, 4)
    small = rng.normal(0, 1, (2, -(-H // b), -(-W // b)))
    full = np.repeat(np.repeat(small, b, axis=1), b, axis=2)[:, :H, :W]
    np.testing.assert_array_equal(oracle.filter_varying(M, ks, small, bin=b), oracle.filter_varying(M, ks, full))


# ----------------------------------------------------------------------------
# local background by convolution
# ----------------------------------------------------------------------------
def _k2(kx, ky):
    kx = np.asarray(kx, float) / np.sum(kx)
    ky = np.asarray(ky, float) / np.sum(ky)
    return np.outer(ky, kx)


@pytest.mark.parametrize("lx,ly", [(1, 1), (9, 5), (31, 31), (65, 129)])
def test_background_conv_constant_image(lx, ly):
    I = np.full((37, 53), 812.25)
    B, R, n = oracle.background_conv(I, np.hanning(lx + 2)[1:-1], np.ones(ly), gain=1.5)
    np.testing.assert_allclose(B, 812.25, rtol=1e-14)
    assert n == 0


def test_background_conv_delta_kernel_is_identity():
    rng = np.random.default_rng(21)
    I = rng.normal(100, 10, (20, 30))
    mask = np.zeros(I.shape, np.uint8)
    mask[5, 7] = mask[11, 2] = 1
    B, _, n = oracle.background_conv(I, [2.0], [3.0], mask=mask)
    ok = mask == 0
    np.testing.assert_array_equal(B[ok], I[ok])
    # an invalid pixel with only itself under the kernel cannot be filled
    assert n == 2 and B[5, 7] == 0.0 and B[11, 2] == 0.0


def test_background_conv_equals_scipy_separable_reflect():
    rng = np.random.default_rng(22)
    H, W = 41, 67
    I = rng.normal(500, 20, (H, W)) + 3 * np.arange(W)[None, :]
    kx = rng.uniform(0.2, 1.0, 11)      # asymmetric: a flipped kernel would differ
    ky = rng.uniform(0.2, 1.0, 7)
    B, _, n = oracle.background_conv(I, kx, ky)
    t = ndimage.correlate1d(I, kx / kx.sum(), axis=1, mode="reflect")
    t = ndimage.correlate1d(t, ky / ky.sum(), axis=0, mode="reflect")
    np.testing.assert_allclose(B, t, rtol=1e-13)
    assert n == 0


def test_background_conv_fill_equals_normalised_convolution():
    rng = np.random.default_rng(23)
    H, W = 45, 60
    I = rng.normal(300, 15, (H, W))
    I[10:14, 20:26] = 70000.0              # a saturated blob (invalid through sat)
    mask = np.zeros((H, W), np.uint8)
    mask[30:37, 40:45] = 1                 # a masked compact source
    mask[0, 0] = 1
    kx = rng.uniform(0.1, 1.0, 9)
    ky = rng.uniform(0.1, 1.0, 13)
    B, _, n = oracle.background_conv(I, kx, ky, mask=mask, sat=65535.0)
    K = _k2(kx, ky)
    v = ((mask == 0) & (I < 65535.0)).astype(float)
    num = ndimage.correlate(v * I, K, mode="reflect")
    den = ndimage.correlate(v, K, mode="reflect")
    Ip = np.where(v > 0, I, num / den)
    np.testing.assert_allclose(B, ndimage.correlate(Ip, K, mode="reflect"), rtol=1e-12)
    assert n == 0


def test_background_conv_counts_unfillable_pixels():
    H, W = 40, 40
    I = np.full((H, W), 10.0)
    mask = np.zeros((H, W), np.uint8)
    mask[5:30, 5:30] = 1                    # a hole far wider than the kernel
    B, _, n = oracle.background_conv(I, np.ones(5), np.ones(3), mask=mask)
    v = (mask == 0).astype(float)
    reach = ndimage.correlate(v, np.ones((3, 5)), mode="reflect")
    want = int(np.sum((mask != 0) & (reach == 0)))
    assert n == want > 0


def test_noise_map_adds_sky_dark_and_read_variances():
    """Monte Carlo: a dark-subtracted pixel of sky s (ADU) with gain g, read
    noise rn and dark current d over texp has variance (g s + rn^2 + d texp) / g^2."""
    rng = np.random.default_rng(24)
    g, rn, d, texp, s = 1.7, 6.5, 0.8, 30.0, 240.0
    n = 400_000
    e = rng.poisson(g * s, n) + rng.poisson(d * texp, n) - d * texp + rng.normal(0, rn, n)
    adu = e / g
    _, R, _ = oracle.background_conv(np.full((8, 8), s), [1.0], [1.0], gain=g, rn=rn, dark=d, texp=texp)
    assert abs(np.var(adu) / R[0, 0] ** 2 - 1.0) < 0.01
    assert abs(np.mean(adu) - s) < 0.1


def test_background_conv_keeps_planes_inside():
    """A symmetric unit-sum kernel reproduces a plane away from the borders."""
    H, W = 50, 70
    yy, xx = np.mgrid[0:H, 0:W]
    I = 100.0 + 0.5 * xx - 0.25 * yy
    B, _, _ = oracle.background_conv(I, np.hanning(13)[1:-1], np.hanning(9)[1:-1])
    np.testing.assert_allclose(B[6:-6, 8:-8], I[6:-6, 8:-8], rtol=1e-13)
