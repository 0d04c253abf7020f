"""Serving: continuous batching of frames over the C ABI.

Requests (frames of any size, u16 or f32, on the host or already in HBM)
arrive over time.  The loop admits waiting requests in arrival order while a
slot is free and their HBM footprint fits the budget, launches every request
admitted at one poll as one batch (one gp_background / gp_detect /
gp_aperture sequence over all of them) on the next stream of a small pool, and
keeps going: batches from consecutive polls run concurrently on the device
while earlier ones finish.  A finished batch's results are downloaded by a
worker thread, so admission never waits on a copy; once they are on the host
the batch releases its slots and footprint and hands each request its
catalogue and photometry.

Everything per pixel runs in the HIP library; this module schedules.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, List, Optional

import numpy as np
import torch

from . import _lib as L
from .pipeline import Photometry

# a detection batch holds at most 2^31 pixels, each frame counted in whole
# 1024-pixel blocks (larger batches are refused by gp_detect)
MAX_BATCH_BLOCKS = 1 << 21


def pixel_blocks(frame) -> int:
    h, w = frame.shape[-2], frame.shape[-1]
    return -(-(int(h) * int(w)) // 1024)


@dataclass
class Request:
    rid: int
    frame: Any                      # numpy array (host) or torch tensor (device)
    arrival: float = 0.0            # seconds on the server clock
    params: Any = None              # per-request parameters (None: the server's)
    kernel: Any = None              # per-request filter kernel (None: the server's)
    footprint: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[dict] = None

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.arrival


@dataclass
class _Epoch:
    reqs: List[Request]
    ph: Photometry
    stream: torch.cuda.Stream
    done: torch.cuda.Event
    dev_frames: list = field(default_factory=list)
    key: Any = None


class Server:
    """Continuous-batching server for one GPU.

    hbm_budget: bytes of HBM the server may hold: the in-flight requests
    (frames, background buffers, workspace, catalogue) plus the finished batch
    objects kept for reuse; None = 90% of the free memory at start.  Idle batch
    objects are released, least recently used first, whenever a request would
    not fit otherwise.
    slots: most requests queued or running on the device (a finished batch
    whose results are still being downloaded no longer holds slots, only its
    HBM).  streams: concurrent batches.  max_batch: most requests per batch
    (default: slots / streams).
    """

    def __init__(self, params, kernel, capacity: int = 65536, hbm_budget: Optional[int] = None,
                 slots: int = 16, streams: int = 2, device: int = 0, max_batch: Optional[int] = None,
                 graphs: bool = True):
        self.params = params
        self.kernel = np.ascontiguousarray(kernel, dtype=np.float32)
        self.capacity = capacity
        self.device = torch.device("cuda", device)
        self.ctx = L.gp_ctx_create(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.slots = slots
        # run each batch as a captured library graph, kept with its batch
        # object per shape class and rebound to the next batch's frames
        self.graphs = graphs
        # a batch takes at most its stream's share of the slots, so the next
        # batch can start on the other stream while one is being retired
        self.max_batch = max_batch or max(1, slots // max(1, streams))
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self._next_stream = 0
        self.waiting: deque = deque()
        self.inflight: List[_Epoch] = []
        self.downloading: list = []          # (epoch, future of its results)
        self._pool = ThreadPoolExecutor(max_workers=1)
        self.resident = 0
        self.t0 = time.perf_counter()
        self.finished: List[Request] = []
        self._ws_cache = {}
        # batch objects (buffers sized for a set of shapes) kept for reuse, in
        # least-recently-used order: (key, serial) -> Photometry; their HBM is
        # counted in idle_bytes against the budget
        self._idle: "OrderedDict" = OrderedDict()
        self._idle_serial = 0
        self.idle_bytes = 0

    # ------------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def footprint(self, frame, params=None) -> int:
        """HBM bytes a request holds while in flight (its frame, its share of
        the background buffer and workspace, its catalogue rows)."""
        H, W = frame.shape
        bpp = 2 if frame.dtype in (np.uint16, torch.uint16) else 4
        fr = L.gp_frame(1, W, H, W, L.GP_U16 if bpp == 2 else L.GP_F32)
        p = params if params is not None else self.params
        bp = L.gp_bkg_params(p.mesh_w, p.mesh_h, p.mesh_filter, p.clip_sigma, p.crowd_tol, p.mode_a, p.mode_b,
                             p.max_iter, 0)
        key = (W, H, bpp, p.mesh_w, p.mesh_h)
        if key not in self._ws_cache:
            _, bkg = L.gp_background_layout([fr], bp)
            ws = L.gp_workspace_size(self.ctx, [fr], bp, None, None, self.capacity, 0)
            self._ws_cache[key] = bkg + ws
        nr = len(p.radii)
        cat = self.capacity * (5 * 4 + 8 + 6 * 8 + 4 + 4 + 3 * nr * 8 + 8)
        own = W * H * bpp if not (isinstance(frame, torch.Tensor) and frame.is_cuda) else 0
        return own + self._ws_cache[key] + cat

    def submit(self, req: Request):
        req.footprint = self.footprint(req.frame, req.params)
        if req.footprint > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint} bytes, above the budget {self.budget}")
        self.waiting.append(req)

    # ------------------------------------------------------------------
    def _download(self, ep):
        res = [ep.ph.results(i, sync=False) for i in range(len(ep.reqs))]
        return res, self.now()

    def _retire(self):
        keep = []
        for ep in self.inflight:
            if ep.done.query():
                self.downloading.append((ep, self._pool.submit(self._download, ep)))
            else:
                keep.append(ep)
        self.inflight = keep
        still = []
        for ep, fut in self.downloading:
            if fut.done():
                res, t = fut.result()
                for r, out in zip(ep.reqs, res):
                    r.result = out
                    r.t_done = t
                    self.resident -= r.footprint
                    self.finished.append(r)
                self._park(ep.key, ep.ph)
            else:
                still.append((ep, fut))
        self.downloading = still

    # ------------------------------------------------------------------
    @staticmethod
    def _bytes(ph) -> int:
        """HBM held by a batch object's buffers."""
        n = ph.bkg.numel() + ph.ws.numel()
        for t in list(ph.cat.values()) + list(ph.phot.values()) + [ph.n_obj, ph.status, ph.comp_status]:
            n += t.numel() * t.element_size()
        if ph.seg is not None:
            n += sum(t.numel() * t.element_size() for t in ph.seg)
        return int(n)

    def _park(self, key, ph):
        self._idle_serial += 1
        self._idle[(key, self._idle_serial)] = ph
        self.idle_bytes += self._bytes(ph)

    def _take_idle(self, key):
        for k in reversed(self._idle):
            if k[0] == key:
                ph = self._idle.pop(k)
                self.idle_bytes -= self._bytes(ph)
                return ph
        return None

    def _evict(self, need: int) -> bool:
        """Release idle batch objects, oldest first, until `need` more bytes fit
        the budget; True when they do."""
        while self._idle and self.resident + self.idle_bytes + need > self.budget:
            _, ph = self._idle.popitem(last=False)
            self.idle_bytes -= self._bytes(ph)
            ph.close()
            del ph
        return self.resident + self.idle_bytes + need <= self.budget

    def _key(self, r):
        return (id(r.params) if r.params is not None else None, id(r.kernel) if r.kernel is not None else None)

    def _admit(self):
        """Start one batch: the oldest arrived request plus every other arrived
        request with the same parameters, while slots and footprint allow."""
        batch = []
        # requests on the device: a batch being downloaded holds only its HBM
        n_inflight = sum(len(e.reqs) for e in self.inflight)
        now = self.now()
        key = None
        keep = deque()
        blocks = 0
        while self.waiting:
            r = self.waiting.popleft()
            fits = (len(batch) < self.max_batch and r.arrival <= now and n_inflight + len(batch) < self.slots
                    and blocks + pixel_blocks(r.frame) <= MAX_BATCH_BLOCKS
                    and self._evict(r.footprint))
            if fits and (key is None or self._key(r) == key):
                key = self._key(r)
                r.t_admit = now
                self.resident += r.footprint
                blocks += pixel_blocks(r.frame)
                batch.append(r)
            else:
                keep.append(r)
                if r.arrival > now or not batch and not fits:
                    break      # FIFO: nothing behind an unadmittable head starts first
        keep.extend(self.waiting)
        self.waiting = keep
        if not batch:
            return False
        stream = self.streams[self._next_stream % len(self.streams)]
        self._next_stream += 1
        with torch.cuda.stream(stream):
            devs = []
            for r in batch:
                f = r.frame
                if isinstance(f, torch.Tensor) and f.is_cuda:
                    devs.append(f)
                else:
                    t = torch.as_tensor(f)
                    devs.append(t.to(self.device, non_blocking=True))
            params = batch[0].params if batch[0].params is not None else self.params
            kernel = batch[0].kernel if batch[0].kernel is not None else self.kernel
            bkey = (key, tuple((tuple(t.shape), t.dtype) for t in devs))
            ph = self._take_idle(bkey)
            if ph is not None:
                ph.rebind(devs)
            else:
                ph = Photometry(devs, params, kernel, self.capacity, ctx=self.ctx)
                if self.graphs:
                    ph.capture()
            if self.graphs:
                ph.replay(stream)
            else:
                ph.run(stream)
            done = torch.cuda.Event()
            done.record(stream)
        self.inflight.append(_Epoch(batch, ph, stream, done, devs, bkey))
        return True

    def poll(self):
        self._retire()
        while self._admit():
            pass

    def drain(self, poll_sleep: float = 2e-4):
        while self.waiting or self.inflight or self.downloading:
            self.poll()
            if self.inflight or self.waiting or self.downloading:
                time.sleep(poll_sleep)

    def run(self, requests: List[Request], poll_sleep: float = 2e-4):
        """Serve requests whose `arrival` times are relative to now; returns
        them finished, with latencies."""
        self.t0 = time.perf_counter()
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r)
        self.drain(poll_sleep)
        return requests

    def close(self):
        for ep in self.inflight:
            ep.done.synchronize()
            ep.ph.close()
        self.inflight = []
        for ep, fut in self.downloading:
            fut.result()
            ep.ph.close()
        self.downloading = []
        self._pool.shutdown(wait=True)
        for ph in self._idle.values():
            ph.close()
        self._idle = OrderedDict()
        self.idle_bytes = 0
        if self.ctx:
            L.gp_ctx_destroy(self.ctx)
            self.ctx = None


def latency_stats(reqs: List[Request]):
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}
