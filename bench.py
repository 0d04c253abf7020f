#!/usr/bin/env python3
"""Benchmark of the photometry hot path on one MI355X.

Headline workload: the uneven batch of 64 uint16 frames (24 x 2048^2,
24 x 4096^2, 16 x 9600x6400; 300-40,000 Gaussian stars each; mesh 64, 5x5
Gaussian filter, threshold 1.5 sigma, minarea 5, 8-connected, apertures 3/6 px,
annulus 10-15 px), already resident in HBM.  A step is one pass of the whole
path -- gp_background, gp_detect, gp_aperture -- over all 64 frames, run as
one launch of the library's captured graph.  The same frames through plain
per-frame calls are timed beside it (queued back to back on one stream, and
as a client that waits for each frame's catalogue).  Further forms: the
6144^2 and 12300^2 float32 fields per frame (FP32 and FP64 variants of the
path); the paper's own path over the batch (peaks with the fixed kernel, then
with the spatially varying PSF, then top-hat growth curves); the background
by convolution over the batch; and a served Poisson stream of mixed uint16
frames.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-forms]
                  [--stream-seconds S]

Helper modes for the roofline's `traffic` figure (rocprofv3 counters):
  python bench.py --profile-only [--workload batch|c2|c3]   the workload's
                                            direct calls only, a few steps
  python bench.py --copy-calibration MIB    one elementwise copy (torch.neg) of
                                            MIB MiB, whose known bytes scale
                                            FETCH_SIZE / WRITE_SIZE
  python bench.py --traffic KERNEL FETCH.csv WRITE.csv CAL_FETCH.csv CAL_WRITE.csv
                                            writes profiles/traffic_<KERNEL>_<workload>.json
  python bench.py --form paper|background_conv   one form of the batch alone
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "extracted MP/s + p50/p99 frame latency, batched/served vs plain, 1 MI355X"
KERNEL_NAMES = ("mesh_stats", "filter_spline", "grid_filter", "spline", "setup", "detect_tiles", "merge", "catalog",
                "aperture")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch", choices=["batch", "c1", "c2", "c3"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the per-frame and served forms")
    ap.add_argument("--stream-seconds", type=float, default=60.0, help="length of the Poisson arrival stream")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the workload's direct calls (autotuned), for counter collection")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--form", choices=["paper", "background_conv"], default=None,
                    help="run only this form of the batch (for a kernel trace of its kernels)")
    ap.add_argument("--traffic", nargs=5, metavar=("KERNEL", "FETCH", "WRITE", "CAL_FETCH", "CAL_WRITE"))
    ap.add_argument("--traffic-last", type=int, default=5,
                    help="dispatches counted: the last N of the kernel (the profiled run's steps)")
    return ap.parse_args()


CAL_KERNEL = "neg"   # name fragment of the calibration copy kernel
# the source file of each timed kernel: a traffic figure is only reported while
# the file is unchanged since its counters were taken
KERNEL_SOURCE = {"mesh_stats": "k_background.hip", "detect_tiles": "k_detect.hip", "aperture": "k_aperture.hip"}
KERNEL_FRAGMENT = {"mesh_stats": "k_mesh_stats", "detect_tiles": "k_detect_tiles", "aperture": "k_aperture"}


def source_sha1(kern):
    import hashlib
    path = os.path.join(ROOT, "paper_2609_32375_amd", "csrc", KERNEL_SOURCE[kern])
    return hashlib.sha1(open(path, "rb").read()).hexdigest()


def copy_calibration(mib):
    """Run one float32 elementwise copy of `mib` MiB (after a warm-up launch)."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_bytes_each_way": n * 4}), flush=True)


def counter_mean(path, fragment, counter, last=None):
    """Mean of a counter (summed over its instances) per dispatch of the kernels
    whose name contains `fragment`, from a rocprofv3 counter_collection.csv;
    `last`: only the last that many such dispatches (the timed steps, after the
    launch-shape autotuning that runs the kernel's other shapes first)."""
    import csv
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if fragment in r["Kernel_Name"] and r["Counter_Name"] == counter:
                per[int(r["Dispatch_Id"])] = per.get(int(r["Dispatch_Id"]), 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernels named *{fragment}* in {path}")
    ids = sorted(per)[-last:] if last else sorted(per)
    return sum(per[i] for i in ids) / len(ids), len(ids)


def write_traffic(a):
    kern, fetch, write, cfetch, cwrite = a.traffic
    frag = KERNEL_FRAGMENT[kern]
    fk, nf = counter_mean(fetch, frag, "FETCH_SIZE", a.traffic_last)
    wk, nw = counter_mean(write, frag, "WRITE_SIZE", a.traffic_last)
    cfk, _ = counter_mean(cfetch, CAL_KERNEL, "FETCH_SIZE")
    cwk, _ = counter_mean(cwrite, CAL_KERNEL, "WRITE_SIZE")
    cal_bytes = a.copy_calibration * (1 << 20) if a.copy_calibration else 1 << 30
    sf, sw = cal_bytes / (cfk * 1024), cal_bytes / (cwk * 1024)
    out = {"kernel": kern, "workload": a.workload, "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
           "dispatches": [nf, nw], "calibration_bytes": cal_bytes, "calibration_fetch_kib": cfk,
           "calibration_write_kib": cwk, "fetch_scale": sf, "write_scale": sw,
           "bytes_per_launch": int(fk * 1024 * sf + wk * 1024 * sw), "source_sha1": source_sha1(kern)}
    path = os.path.join(ROOT, "profiles", f"traffic_{kern}_{a.workload}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def kernel_bytes(name, frames_px_bytes, n_obj, rmax, bpp):
    """Algorithmic bytes one launch of a kernel must move: one read of every
    frame for the mesh statistics and the detection, the pixels of every
    object's outer circle for the apertures."""
    if name in ("mesh_stats", "detect_tiles"):
        return frames_px_bytes
    if name == "aperture":
        return n_obj * math.pi * rmax * rmax * bpp
    return None


def traffic_of(kern, workload):
    tfile = os.path.join(ROOT, "profiles", f"traffic_{kern}_{workload}.json")
    if not os.path.exists(tfile):
        return None
    try:
        tj = json.load(open(tfile))
        return tj.get("bytes_per_launch") if tj.get("source_sha1") == source_sha1(kern) else None
    except Exception:
        return None


def event_time(torch, fn, reps, stream=None):
    """Milliseconds per call of fn(), GPU events around `reps` calls queued
    back to back (one synchronisation at the end)."""
    s = stream or torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def kernel_profile(torch, L, ph, steps):
    """Mean milliseconds per launch of each kernel (events on the launch stream)."""
    L.gp_profile_reset(ph.ctx)
    L.gp_profile_enable(ph.ctx, True)
    for _ in range(steps):
        ph.run()
    torch.cuda.synchronize()
    L.gp_profile_enable(ph.ctx, False)
    out = {}
    for name in KERNEL_NAMES:
        tot, cnt = L.gp_profile_read(ph.ctx, name)
        if cnt:
            out[name] = tot / cnt
    return out


def roofline(kern_ms, frames_px_bytes, n_obj, rmax, bpp, workload):
    dom = max((k for k in kern_ms if kernel_bytes(k, frames_px_bytes, n_obj, rmax, bpp)), key=lambda k: kern_ms[k])
    alg = kernel_bytes(dom, frames_px_bytes, n_obj, rmax, bpp)
    achieved = alg / (kern_ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_of(dom, workload),
            "kernel_ms": round(kern_ms[dom], 4), "algorithmic_bytes": int(alg)}


# ----------------------------------------------------------------------------
def batch_frames(torch):
    from synth import batch_shapes, render_gpu
    t0 = time.time()
    shapes = batch_shapes()
    frames = [render_gpu(w, h, n, seed) for (w, h, n, seed) in shapes]
    torch.cuda.synchronize()
    log(f"batch: {len(frames)} uint16 frames rendered in {time.time() - t0:.1f}s")
    return frames


def profile_only(a):
    """Direct calls of the workload for a few steps (counter collection)."""
    import torch
    from paper_2609_32375_amd.pipeline import Photometry
    from synth import config_params, make_frame
    if a.workload == "batch":
        frames = batch_frames(torch)
        p = config_params("c1")
        cap = 65536
    else:
        fr = make_frame(a.workload)
        frames = [torch.from_numpy(fr.image).cuda()]
        p = fr.params
        cap = 262144 if a.workload == "c3" else 65536
    tune = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"gpphot_tune_prof_{os.getpid()}.json")
    ph = Photometry(frames, p, p.kernel(), capacity=cap, autotune=True, tune_cache=tune)
    for _ in range(a.profile_steps):
        ph.run()
    torch.cuda.synchronize()
    print(json.dumps({"workload": a.workload, "steps": a.profile_steps, "objects": int(ph.n_obj.sum().item())}),
          flush=True)
    ph.close()


def main():
    a = parse()
    if a.traffic:
        write_traffic(a)
        return
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}): this build measures one MI355X; "
              "sharding across GPUs is a design note", file=sys.stderr)
        sys.exit(2)
    if a.profile_only:
        profile_only(a)
        return
    if a.form:
        import torch
        fn = {"paper": form_peaks, "background_conv": form_background_conv}[a.form]
        print(json.dumps(fn(torch, a)), flush=True)
        return
    if a.workload != "batch":
        out = single_frame_line(a)
        print(json.dumps(out), flush=True)
        return
    import torch

    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry
    from synth import config_params

    frames = batch_frames(torch)
    p = config_params("c1")
    K = p.kernel()
    npx = [f.shape[0] * f.shape[1] for f in frames]
    mp = sum(npx) / 1e6
    cap = 65536
    # launch shapes tuned once here, before anything is timed
    tune = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"gpphot_tune_batch_{os.getpid()}.json")
    batch = Photometry(frames, p, K, capacity=cap, autotune=True, tune_cache=tune)
    tuned = json.load(open(tune)) if os.path.exists(tune) else {}
    log(f"autotuned launch shapes: {tuned}")
    batch.capture()
    for _ in range(a.warmup):
        batch.replay()
    torch.cuda.synchronize()
    n_obj = [int(v) for v in batch.n_obj.cpu().tolist()]
    status = [int(v) for v in batch.status.cpu().tolist()]
    log(f"objects {sum(n_obj)} status {set(status)}")
    # timed region: K graph launches, each the whole path over all 64 frames
    stream = torch.cuda.current_stream()
    lat = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(a.steps):
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        batch.replay()
        s1.record(stream)
        lat.append((s0, s1))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.steps
    lat_ms = np.array([x.elapsed_time(y) for x, y in lat])
    value = mp / (ms / 1e3)
    log(f"batched (one graph launch over 64 frames): {ms:.3f} ms/step, {value:.1f} MP/s")
    # per-kernel durations of the same batch (direct calls, events on the launch stream)
    kern = kernel_profile(torch, L, batch, a.profile_steps)
    log("kernel ms:", {k: round(v, 4) for k, v in kern.items()})
    rmax = max(p.r_out, max(p.radii))
    roof = roofline(kern, 2 * sum(npx), sum(n_obj), rmax, 2, "batch")
    step_bytes = 2 * 2 * sum(npx) + sum(n_obj) * math.pi * rmax * rmax * 2
    # results of the graph launches are those of direct calls (checked in the tests)
    batch.close()
    del batch
    torch.cuda.empty_cache()
    plain = plain_forms(torch, frames, p, K, cap, a)
    log(f"plain per-frame: queued {plain['queued_ms']:.3f} ms ({mp / plain['queued_ms'] * 1e3:.0f} MP/s), "
        f"waiting for each catalogue {plain['client_ms']:.3f} ms ({mp / plain['client_ms'] * 1e3:.0f} MP/s)")
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "MP/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch: 64 uint16 frames of uneven sizes (24 x 2048^2, 24 x 4096^2, 16 x 9600x6400; "
                               "1486.4 MP), 300-40,000 Gaussian stars each; mesh 64, 5x5 filter, apertures 3/6 px, "
                               "annulus 10-15 px; one launch of the captured graph per step",
                   "frames": len(frames), "mp": round(mp, 2), "objects": sum(n_obj), "autotuned": tuned},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "note": "a batch's frames all complete at the end of its launch"},
        "vs_plain": {"plain_queued_mp_s": round(mp / plain["queued_ms"] * 1e3, 1),
                     "plain_queued_ms": round(plain["queued_ms"], 3),
                     "speedup_vs_plain_queued": round(plain["queued_ms"] / ms, 3),
                     "plain_client_mp_s": round(mp / plain["client_ms"] * 1e3, 1),
                     "plain_client_ms": round(plain["client_ms"], 3),
                     "speedup_vs_plain_client": round(plain["client_ms"] / ms, 3),
                     "plain_frame_latency_ms": plain["frame_latency"]},
        "step_hbm_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels_ms": {k: round(v, 4) for k, v in kern.items()},
        "roofline": roof,
    }
    out["copy_ceiling_gbs"] = round(copy_ceiling(torch), 1)
    cpu_frames = [f.cpu().numpy() for f in frames[:24]] + [f.cpu().numpy() for f in frames[24:32]]
    del frames
    torch.cuda.empty_cache()
    if not a.no_forms:
        out["forms"] = {}
        for w in ("c2", "c3"):
            out["forms"][w] = frame_form(torch, w, a)
            torch.cuda.empty_cache()
        out["forms"]["peaks"] = form_peaks(torch, a)
        torch.cuda.empty_cache()
        out["forms"]["background_conv"] = form_background_conv(torch, a)
        torch.cuda.empty_cache()
        out["forms"]["served"] = form_served(torch, a)
        torch.cuda.empty_cache()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cpu_frames, p)
    print(json.dumps(out), flush=True)


def plain_forms(torch, frames, p, K, cap, a):
    """The batch's frames through plain per-frame calls: (i) queued back to
    back on one stream, timed with GPU events; (ii) a client that waits for
    each frame's catalogue (synchronise and copy the results) before the next."""
    from paper_2609_32375_amd.pipeline import Photometry
    singles = [Photometry([f], p, K, capacity=cap) for f in frames]
    for s in singles:
        s.run()
    torch.cuda.synchronize()

    def all_frames():
        for s in singles:
            s.run()
    reps = max(2, a.steps // 5)
    queued = event_time(torch, all_frames, reps)
    t = time.perf_counter()
    lat = []
    for _ in range(reps):
        for s in singles:
            t1 = time.perf_counter()
            s.run()
            s.results(0)
            lat.append(time.perf_counter() - t1)
    client = (time.perf_counter() - t) * 1e3 / reps
    for s in singles:
        s.close()
    lat = np.array(lat) * 1e3
    return {"queued_ms": queued, "client_ms": client,
            "frame_latency": {"p50": round(float(np.percentile(lat, 50)), 3),
                              "p99": round(float(np.percentile(lat, 99)), 3)}}


def copy_ceiling(torch, mib=1024, reps=10):
    """Read + write GB/s of a plain elementwise copy (torch.neg) of `mib` MiB:
    the practical HBM ceiling next to the 8 TB/s peak."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    ms = event_time(torch, lambda: torch.neg(x, out=y), reps)
    del x, y
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def frame_form(torch, w, a):
    """One float32 field per step through direct calls, FP32 path and the FP64
    variant: ms per frame, MP/s, the dominant kernel's roofline."""
    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry
    from synth import make_frame
    t0 = time.time()
    fr = make_frame(w)
    img = fr.image
    H, W = img.shape
    log(f"frame {w} {W}x{H} generated in {time.time() - t0:.1f}s")
    dev = torch.from_numpy(img).cuda()
    p = fr.params
    cap = 262144 if w == "c3" else 65536
    tune = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"gpphot_tune_{w}_{os.getpid()}.json")
    res = {"workload": f"{w}: {W}x{H} float32 star field, plain per-frame calls"}
    for prec in (0, 1):
        ph = Photometry([dev], p, p.kernel(), capacity=cap, precision=prec, autotune=True, tune_cache=tune)
        for _ in range(3):
            ph.run()
        torch.cuda.synchronize()
        ms = event_time(torch, ph.run, max(5, a.steps // 2))
        n_obj = int(ph.n_obj[0].item())
        key = "fp64" if prec else "fp32"
        res[key] = {"ms": round(ms, 4), "mp_s": round(W * H / 1e6 / (ms / 1e3), 1), "objects": n_obj}
        if prec == 0:
            kern = kernel_profile(torch, L, ph, a.profile_steps)
            rmax = max(p.r_out, max(p.radii))
            res[key]["kernels_ms"] = {k: round(v, 4) for k, v in kern.items()}
            res[key]["roofline"] = roofline(kern, 4 * W * H, n_obj, rmax, 4, w)
            res[key]["step_hbm_frac"] = round((8 * W * H + n_obj * math.pi * rmax * rmax * 4) /
                                              (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        ph.close()
        log(f"{w} {key}: {ms:.3f} ms/frame")
    del dev
    return res


def single_frame_line(a):
    """--workload c1|c2|c3: the per-frame FP32 step as the JSON line."""
    import torch
    r = frame_form(torch, a.workload, a)
    f = r["fp32"]
    mp = f["mp_s"] * f["ms"] / 1e3
    return {"metric": METRIC, "value": f["mp_s"], "unit": "MP/s", "n_gpus": 1, "steps": max(5, a.steps // 2),
            "warmup": 3, "ms_per_step": f["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": {"workload": r["workload"], "mp": round(mp, 2),
                                                           "objects": f["objects"]},
            "kernels_ms": f["kernels_ms"], "roofline": f["roofline"], "fp64_variant": r["fp64"]}


def form_peaks(torch, a):
    """The paper's own path on the batch, direct calls: gp_background ->
    gp_peaks (first pass: the fixed Gaussian kernel, local maxima of F / R
    above 5 sigma, separation and centroid half-widths 3 px = ceil(FWHM)) ->
    gp_peaks_psf (second pass: reference PSF plus 5 eigenmodes of 13 x 13
    taps with full-frame coefficient maps, the paper's K) -> gp_growth
    (top-hat growth curves over the radii ceil(0.75 FWHM) .. ceil(5 FWHM) =
    3..15 px for FWHM 3).  The PSF fit between the passes is not timed."""
    from paper_2609_32375_amd import _lib as L
    from paper_2609_32375_amd.pipeline import Photometry, growth_radii
    from synth import coef_maps_gpu, config_params, psf_model
    frames = batch_frames(torch)
    p = config_params("c1")
    p.thresh = 5.0
    radii = growth_radii(3.0)
    K = 5
    ks = psf_model(K, 13, 3.0, 11)
    maps = [coef_maps_gpu(torch, K, f.shape[1], f.shape[0], 100 + i) for i, f in enumerate(frames)]
    npx = [f.shape[0] * f.shape[1] for f in frames]
    mp = sum(npx) / 1e6
    ph = Photometry(frames, p, p.kernel(), capacity=65536)

    def step():
        ph.background()
        ph.peaks(3, 3)
        ph.peaks_psf(3, 3, ks, maps)
        ph.growth(radii)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    ms = event_time(torch, step, max(3, a.steps // 4))
    n = int(ph.n_obj.sum().item())
    L.gp_profile_reset(ph.ctx)
    L.gp_profile_enable(ph.ctx, True)
    for _ in range(a.profile_steps):
        step()
    torch.cuda.synchronize()
    L.gp_profile_enable(ph.ctx, False)
    kern = {}
    for name in ("mesh_stats", "peaks", "peaks_psf", "growth"):
        tot, cnt = L.gp_profile_read(ph.ctx, name)
        if cnt:
            kern[name] = round(tot / cnt, 4)
    ph.close()
    del frames, maps
    log(f"paper path: {ms:.3f} ms per batch, {n} peaks")
    return {"workload": "the 64-frame uint16 batch; background, peaks (5 sigma, sep 3, cwin 3), peaks with the "
                        "varying PSF (reference + 5 modes, 13 x 13, full-frame maps), growth curves (radii 3..15)",
            "ms": round(ms, 3), "mp_s": round(mp / ms * 1e3, 1), "peaks": n, "kernels_ms": kern,
            "peaks_hbm_frac": round(2 * sum(npx) / (kern.get("peaks", 1e9) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "peaks_psf_tflops": round(2 * (K + 1) * 13 * 13 * sum(npx) / (kern.get("peaks_psf", 1e9) * 1e-3) / 1e12,
                                      1),
            "growth_sources_per_s": round(n / (kern.get("growth", 1e9) * 1e-3), 1)}


def form_background_conv(torch, a):
    """The paper's own background on the batch: gp_background_conv with a
    separable Gaussian of FWHM 32 px (65 taps per axis), saturated pixels
    (>= 65535) filled from their valid neighbours, and the noise map of a
    gain 1.5 e-/ADU, 5 e- read-noise frame; one call over the 64 frames."""
    import numpy as np
    from paper_2609_32375_amd.pipeline import ConvBackground
    frames = batch_frames(torch)
    npx = sum(f.shape[0] * f.shape[1] for f in frames)
    t = np.arange(-32, 33, dtype=np.float64)
    k = np.exp(-0.5 * (t / (32.0 / 2.3548)) ** 2).astype(np.float32)
    cb = ConvBackground(frames, k, k, 1.5, 5.0, 0.0, 0.0, sat_level=65535.0)
    for _ in range(2):
        cb.run()
    torch.cuda.synchronize()
    ms = event_time(torch, cb.run, max(3, a.steps // 4))
    unf = int(cb.unfilled.sum().item())
    cb.close()
    del frames, cb
    log(f"background by convolution: {ms:.3f} ms per batch")
    return {"workload": "the 64-frame uint16 batch; background by convolution (65 x 65 separable Gaussian, "
                        "saturated pixels filled), noise map", "ms": round(ms, 3),
            "mp_s": round(npx / 1e6 / ms * 1e3, 1), "unfilled": unf,
            # the two passes every pixel takes (A = K corr vI): 2 x 65 FMAs per pixel
            "fp64_tflops_a_passes": round(2 * 2 * 65 * npx / (ms * 1e-3) / 1e12, 2)}


def form_served(torch, a):
    """Mixed 4.2 / 37.7 / 151.3 MP uint16 requests (shapes uniform over the
    three), device-resident, each with its shape's parameters: (i) Poisson
    arrivals at 4 /s over the stream length: p50/p99 latency; (ii) all queued
    at once (saturating) against the same requests through plain per-frame
    calls that wait for each catalogue; (iii) with a 4 GB HBM budget, which
    binds; (iv) frames coming from host memory.  Servers are timed after a
    throwaway server in the same process (the first one's rate is reported
    beside)."""
    from paper_2609_32375_amd.pipeline import Photometry
    from paper_2609_32375_amd.serve import Request, Server, latency_stats
    from synth import arrival_stream, config_params, render_gpu
    shp = {"c1": (2048, 2048, 300), "c2": (6144, 6144, 20000), "c3": (12300, 12300, 134000)}
    pools, params, kernels = {}, {}, {}
    for kname, (w, h, n) in shp.items():
        pools[kname] = [render_gpu(w, h, n, 3000 + 10 * list(shp).index(kname) + j) for j in range(3)]
        params[kname] = config_params(kname)
        kernels[kname] = params[kname].kernel()
    torch.cuda.synchronize()
    cap = 262144
    times, kinds = arrival_stream(rate=4.0, duration=a.stream_seconds)
    reqs_of = lambda arr, src=pools: [Request(i, src[k][i % 3], arrival=t, params=params[k], kernel=kernels[k])
                                      for i, (t, k) in enumerate(zip(arr, kinds))]
    mp = sum(pools[k][0].shape[0] * pools[k][0].shape[1] for k in kinds) / 1e6
    zero = np.zeros(len(kinds))

    def saturating(srv, src=pools):
        for _ in range(2):                          # warm-up (allocator, graphs)
            srv.run(reqs_of(zero, src))
        t = time.perf_counter()
        done = srv.run(reqs_of(zero, src))
        return time.perf_counter() - t, latency_stats(done)

    # the first server of a process runs about a fifth slower than every later
    # one (its device busy time is the same; the gap is idle time): one
    # throwaway server first, so the figures are a long-running server's
    warm = Server(params["c1"], kernels["c1"], capacity=cap, slots=16, streams=2)
    first_s, _ = saturating(warm)
    warm.close()
    srv = Server(params["c1"], kernels["c1"], capacity=cap, slots=16, streams=2)
    sat_s, sat_lat = saturating(srv)
    # plain: the same requests one at a time, each catalogue waited for
    plain = {k: Photometry([pools[k][0]], params[k], kernels[k], capacity=cap) for k in shp}
    for k in shp:
        plain[k].run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i, k in enumerate(kinds):
        plain[k].rebind([pools[k][i % 3]])
        plain[k].run()
        plain[k].results(0)
    plain_s = time.perf_counter() - t
    for k in shp:
        plain[k].close()
    log(f"served saturating {mp / sat_s:.0f} MP/s vs plain {mp / plain_s:.0f} MP/s; open loop over "
        f"{a.stream_seconds:.0f} s next")
    done = srv.run(reqs_of(times))
    open_lat = latency_stats(done)
    srv.close()
    srv_ng = Server(params["c1"], kernels["c1"], capacity=cap, slots=16, streams=2, graphs=False)
    ng_s, _ = saturating(srv_ng)
    srv_ng.close()
    srv4 = Server(params["c1"], kernels["c1"], capacity=cap, slots=16, streams=2, hbm_budget=4 << 30)
    b4_s, b4_lat = saturating(srv4)
    srv4.close()
    host = {k: [pools[k][j].cpu().numpy() for j in range(3)] for k in shp}
    srvh = Server(params["c1"], kernels["c1"], capacity=cap, slots=16, streams=2)
    host_s, host_lat = saturating(srvh, host)
    srvh.close()
    log(f"served: open loop {open_lat}; without graphs {mp / ng_s:.0f} MP/s; 4 GB budget {mp / b4_s:.0f} MP/s; "
        f"host-sourced {mp / host_s:.0f} MP/s")
    r = lambda x: round(x, 2)
    return {"workload": f"{len(kinds)} requests, shapes uniform over 2048^2 / 6144^2 / 12300^2 uint16, "
                        f"device-resident, Poisson 4/s over {a.stream_seconds:.0f} s",
            "mp": round(mp, 1), "p50_ms": r(open_lat.get("p50_ms", 0)), "p99_ms": r(open_lat.get("p99_ms", 0)),
            "saturating_mp_s": round(mp / sat_s, 1), "plain_mp_s": round(mp / plain_s, 1),
            "first_server_saturating_mp_s": round(mp / first_s, 1),
            "speedup_vs_plain": round(plain_s / sat_s, 3),
            "saturating_p50_ms": r(sat_lat.get("p50_ms", 0)), "saturating_p99_ms": r(sat_lat.get("p99_ms", 0)),
            "saturating_without_graphs_mp_s": round(mp / ng_s, 1),
            "budget_4gb": {"saturating_mp_s": round(mp / b4_s, 1), "p50_ms": r(b4_lat.get("p50_ms", 0)),
                           "p99_ms": r(b4_lat.get("p99_ms", 0))},
            "host_sourced": {"saturating_mp_s": round(mp / host_s, 1), "p50_ms": r(host_lat.get("p50_ms", 0)),
                             "p99_ms": r(host_lat.get("p99_ms", 0))},
            "slots": 16, "streams": 2}


def _oracle_frame(args):
    """One frame through the FP64 oracle chain (a worker process)."""
    img, pd = args
    import oracle
    from synth import Params
    p = Params(**pd)
    t = time.perf_counter()
    oracle.run(img.astype(np.float64), p)
    return img.shape[0] * img.shape[1], time.perf_counter() - t


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames, p):
    """The FP64 oracle on the host cores, frame-parallel (one frame per worker
    process), over a bounded sample of the batch: its 24 2048^2 frames and
    eight of its 4096^2 frames; plus one 2048^2 frame on one core."""
    import multiprocessing as mp
    workers = max(1, min(int(os.environ.get("OMP_NUM_THREADS", "16")), os.cpu_count() or 1, 16))
    pd = p.to_dict()
    jobs = [(f, pd) for f in frames]
    ctx = mp.get_context("spawn")
    t = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_frame, jobs, chunksize=1)
    wall = time.perf_counter() - t
    px = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    one = _oracle_frame(jobs[0])
    log(f"oracle: {px / 1e6:.0f} MP in {wall:.1f} s on {workers} processes ({cpu_s:.0f} s of CPU work)")
    return {"value": round(px / 1e6 / wall, 3), "unit": "MP/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(frames)} frames of the batch (24 x 2048^2, {len(frames) - 24} x 4096^2 uint16, "
                      f"{px / 1e6:.0f} MP), full FP64 chain, one frame per worker process, {wall:.1f} s wall",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "single_core": {"value": round(one[0] / 1e6 / one[1], 3), "unit": "MP/s",
                            "sample": f"one 2048^2 uint16 frame, {one[1]:.2f} s"}}


if __name__ == "__main__":
    main()
