"""gp_detect_noalloc (static device scratch) against gp_detect with a
workspace, through the C ABI: bit-identical catalogues and label maps on two
calls in a row, the second on a smaller frame (needs an MI355X)."""
import ctypes as C

import numpy as np
import pytest

from synth import make_frame
from tests._util import f32_params

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run_both(fr, cap):
    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry
    p = f32_params(fr.params)
    dev = torch.from_numpy(fr.image).cuda()
    ph = Photometry([dev], p, p.kernel(), capacity=cap, seg=True)
    ph.background()
    ph.detect()                        # gp_detect with the caller's workspace
    a = ph.results(0)
    # clear the outputs so that nothing of the first call can pass for the second
    for t in list(ph.cat.values()) + [ph.n_obj, ph.status, ph.comp_status] + ph.seg:
        t.fill_(-7 if t.dtype != torch.float64 else float("nan"))
    torch.cuda.synchronize()
    segp = [s.data_ptr() for s in ph.seg]
    L.gp_detect_noalloc(ph.ctx, ph.frames, ph.bp, C.c_void_p(ph.bkg.data_ptr()), ph.dp, ph.gcat, segp,
                        C.c_void_p(ph.comp_status.data_ptr()), ph.stream_ptr())
    b = ph.results(0)
    ph.close()
    return a, b


def _same(a, b):
    assert a["status"] == b["status"] == 0 and a["n_obj"] == b["n_obj"] > 0
    assert a["comp_status"] == b["comp_status"]
    np.testing.assert_array_equal(a["seg"], b["seg"])
    for k in a["cat"]:
        np.testing.assert_array_equal(a["cat"][k], b["cat"][k], err_msg=k)


def test_noalloc_detection_equals_workspace_detection_twice():
    big = make_frame("c1", seed=301, W=1400, H=1100, nstars=160)
    small = make_frame("c1", seed=302, W=530, H=410, nstars=40, dtype="u16")
    a, b = _run_both(big, 4096)
    _same(a, b)
    a2, b2 = _run_both(small, 1024)
    _same(a2, b2)
    assert b2["n_obj"] < b["n_obj"]


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry
    fr = make_frame("c1", seed=303, W=200, H=150, nstars=5)
    p = f32_params(fr.params)
    ph = Photometry([torch.from_numpy(fr.image).cuda()], p, p.kernel(), capacity=64)
    # four 16384 x 16000 frames (dummy pointers: rejected while planning,
    # before any device access): their fixed detection sections exceed 128 MiB
    big = [L.gp_frame(1, 16384, 16000, 16384, L.GP_F32)] * 4
    with pytest.raises(L.GpError) as e:
        L.gp_detect_noalloc(ph.ctx, big, ph.bp, C.c_void_p(ph.bkg.data_ptr()), ph.dp, ph.gcat, None, None,
                            ph.stream_ptr())
    assert e.value.status == L.GP_ERR_UNSUPPORTED
    assert "static scratch" in L.load().gp_last_error().decode()
    ph.close()
