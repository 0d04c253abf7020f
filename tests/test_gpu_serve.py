"""Serving: continuous batching returns, for every request, the result it gets
alone; admission respects the HBM budget and the slot count (needs a GPU)."""
import numpy as np
import pytest

from synth import make_frame
from tests._util import f32_params

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solo(P, img, p, K, cap):
    ph = P.Photometry([torch.from_numpy(img).cuda()], p, K, cap)
    ph.run()
    r = ph.results(0)
    ph.close()
    return r


def test_results_alone_equal_results_in_the_mix():
    from paper_2609_32375_amd import pipeline as P
    from paper_2609_32375_amd.serve import Request, Server, latency_stats
    frs = [make_frame("c1", seed=60 + i, W=w, H=h, nstars=n, dtype=dt)
           for i, (w, h, n, dt) in enumerate([(300, 260, 30, "f32"), (512, 128, 20, "u16"), (200, 200, 12, "f32"),
                                               (640, 300, 40, "u16"), (256, 256, 25, "f32"), (96, 400, 10, "f32")])]
    p = f32_params(frs[0].params)
    K = p.kernel()
    cap = 2048
    solo = [_solo(P, f.image, p, K, cap) for f in frs]
    # a tight budget forces deferral; half the frames come from the host
    srv = Server(p, K, capacity=cap, slots=3, streams=2)
    fps = [srv.footprint(f.image) for f in frs]
    srv.budget = int(max(fps) * 2.5)
    reqs = []
    for i, f in enumerate(frs):
        frame = f.image if i % 2 else torch.from_numpy(f.image).cuda()
        reqs.append(Request(i, frame, arrival=0.002 * i))
    peak = [0]
    orig = srv._admit

    def admit():
        ok = orig()
        peak[0] = max(peak[0], srv.resident)
        assert sum(len(e.reqs) for e in srv.inflight) <= srv.slots
        return ok
    srv._admit = admit
    srv.run(reqs)
    assert peak[0] <= srv.budget
    for r, s in zip(reqs, solo):
        a = r.result
        assert a["n_obj"] == s["n_obj"] and a["status"] == s["status"] == 0
        for k in ("pmin", "npix", "xmin", "xmax", "ymin", "ymax", "flags"):
            np.testing.assert_array_equal(a["cat"][k], s["cat"][k], err_msg=k)
        for k in ("flux", "x", "y", "x2", "y2", "xy", "peak"):
            np.testing.assert_array_equal(a["cat"][k], s["cat"][k], err_msg=k)
        for k in a["phot"]:
            np.testing.assert_array_equal(a["phot"][k], s["phot"][k], err_msg=k)
        assert r.latency is not None and r.latency >= 0
    st = latency_stats(reqs)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    with pytest.raises(ValueError):
        srv.submit(Request(99, np.zeros((4096, 4096), np.float32)))
    srv.close()


def test_batches_stay_within_the_detection_pixel_limit():
    # sixteen 151 MP requests queued at once with room for all of them: one
    # batch would hold 2.4 G pixels, above gp_detect's 2^31, so the server
    # splits them; every request gets the result it gets alone
    from paper_2609_32375_amd import pipeline as P
    from paper_2609_32375_amd.serve import MAX_BATCH_BLOCKS, Request, Server, pixel_blocks
    from synth import config_params, render_gpu
    img = render_gpu(12300, 12300, 2000, 71)
    p = config_params("c3")
    K = p.kernel()
    cap = 65536
    ph = P.Photometry([img], p, K, cap)
    ph.run()
    solo = ph.results(0)
    ph.close()
    assert 16 * pixel_blocks(img) > MAX_BATCH_BLOCKS and MAX_BATCH_BLOCKS * 1024 == 1 << 31
    srv = Server(p, K, capacity=cap, slots=32, streams=2)
    sizes = []
    orig = srv._admit

    def admit():
        n0 = len(srv.inflight)
        ok = orig()
        if ok and len(srv.inflight) > n0:
            sizes.append(len(srv.inflight[-1].reqs))
        return ok
    srv._admit = admit
    reqs = [Request(i, img, arrival=0.0) for i in range(16)]
    srv.run(reqs)
    srv.close()
    assert sizes and max(sizes) * pixel_blocks(img) <= MAX_BATCH_BLOCKS
    for r in reqs:
        a = r.result
        assert a["status"] == 0 and a["n_obj"] == solo["n_obj"] > 0
        np.testing.assert_array_equal(a["cat"]["pmin"], solo["cat"]["pmin"])
        np.testing.assert_array_equal(a["phot"]["flux"], solo["phot"]["flux"])


def test_idle_batches_stay_within_the_budget():
    """A stream of many distinct frame shapes: finished batch objects kept for
    reuse count against the HBM budget and are released (oldest first) when a
    request would not fit, so the server's allocations never exceed it."""
    from paper_2609_32375_amd.serve import Request, Server
    rng = np.random.default_rng(3)
    shapes = [(int(w), int(h)) for w, h in zip(rng.integers(200, 700, 10), rng.integers(150, 600, 10))]
    frames = [torch.from_numpy(make_frame("c1", seed=80 + i, W=w, H=h, nstars=10).image).cuda()
              for i, (w, h) in enumerate(shapes)]
    p = f32_params(make_frame("c1", seed=80, W=64, H=64, nstars=1).params)
    K = p.kernel()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    srv = Server(p, K, capacity=1024, slots=4, streams=2)
    fps = [srv.footprint(f) for f in frames]
    srv.budget = int(3.2 * max(fps))
    peak = 0
    for wave in range(4):
        order = rng.permutation(len(frames))
        reqs = [Request(i, frames[j], arrival=0.0) for i, j in enumerate(order)]
        srv.run(reqs)
        torch.cuda.synchronize()
        used = torch.cuda.memory_allocated() - base
        peak = max(peak, used)
        assert srv.resident == 0
        assert srv.idle_bytes <= srv.budget
        assert used <= srv.budget, (wave, used, srv.budget)
        for r in reqs:
            assert r.result["status"] == 0
    srv.close()
    assert torch.cuda.memory_allocated() - base <= 4096
