"""Served form: simulated camera streams driving the library's request loop.

Cameras produce binary foreground masks (moving ellipses plus salt noise,
``workloads.CameraStream``).  Frames are pre-rendered into device-resident
rings so rendering stays off the measured path.  Arrivals are independent
Poisson processes per camera at ``rate / n_cameras``; each arrival submits the
camera's next ring frame to a ``binding.Server``.  The server (C++, in
libccl) admits frames by its HBM budget, batches whatever is admitted onto
idle worker streams and stamps completions; this module only schedules
arrivals, collects the stamps and releases label slots.

Latency of a frame = completion seen by the server - submission.
Throughput = completed frames / (last completion - first submission),
both stamped by the server.
"""
from __future__ import annotations

import ctypes
import statistics
import time
from dataclasses import dataclass

import numpy as np

from . import binding
from . import workloads as wl


@dataclass
class ServeResult:
    mode: str
    offered_fps: float
    frames: int
    fps: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    duration_s: float

    def as_dict(self):
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in self.__dict__.items()}


def make_rings(shapes=wl.CAMERA_SHAPES, ring: int = 8, seed_base: int = 50000):
    """Render `ring` frames per camera on the host, upload them; returns the
    per-camera lists of (host uint8 array, device tensor)."""
    import torch

    rings = []
    for cam in wl.camera_streams(seed_base, shapes):
        frames = []
        for _ in range(ring):
            h = cam.step()
            frames.append((h, torch.from_numpy(h).cuda()))
        rings.append(frames)
    torch.cuda.synchronize()
    return rings


def arrival_schedule(rate: float, duration_s: float, n_cams: int, seed: int):
    """Merged Poisson arrivals: sorted (t_seconds, camera) pairs."""
    rng = wl.rng_for(seed)
    ev = []
    for c in range(n_cams):
        t = 0.0
        lam = rate / n_cams
        while True:
            t += float(rng.exponential(1.0 / lam))
            if t >= duration_s:
                break
            ev.append((t, c))
    ev.sort()
    return ev


def copy_labels(ptr: int, H: int, W: int) -> np.ndarray:
    """Copy one frame's labels out of a server slot (device pointer)."""
    import torch

    out = torch.empty((H, W), dtype=torch.int32, device="cuda")
    rt = binding._load_hip_runtime()
    rt.hipMemcpy.restype = ctypes.c_int
    rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    rc = rt.hipMemcpy(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr), H * W * 4, 3)
    if rc != 0:
        raise binding.CclError("hipMemcpy of a label slot failed (%d)" % rc)
    return out.cpu().numpy().view(np.uint32)


def run(rings, rate: float, duration_s: float, plain: bool, conn: int = 8, n_workers: int = 2,
        max_batch: int = 8, hbm_budget: int = None, seed: int = 7, check=None, config=None,
        check_all: bool = False):
    """Drive one server at an offered load of `rate` frames/s for `duration_s`.

    check: optional callable(tag, frame_host, labels_numpy) run after the run
    on the frames whose labels are copied out when they complete: about six
    spread over the run, or every frame with check_all."""
    shapes = [r[0][0].shape for r in rings]
    max_px = max(h * w for h, w in shapes)
    if hbm_budget is None:
        hbm_budget = 64 * max_px * 4  # 64 frame slots of labels
    srv = binding.Server(max_px, hbm_budget, n_workers=n_workers, max_batch=max_batch,
                         conn=conn, plain=plain, config=config)
    sched = arrival_schedule(rate, duration_s, len(rings), seed)
    idx = [0] * len(rings)
    meta = {}
    lat = []
    done_ts = []
    keep = {}
    step = 1 if check_all else max(1, len(sched) // 6)
    want_check = set(range(0, len(sched), step)) if check else set()
    sub_ts = []
    t0 = time.perf_counter_ns()
    i = 0

    def drain_once():
        for tag, ptr, slot, ts, ta, tl, td in srv.poll():
            if td < 0:
                raise binding.CclError("frame %d failed in the server" % tag)
            lat.append((td - ts) * 1e-6)
            done_ts.append(td)
            sub_ts.append(ts)
            if tag in want_check:
                # copy the labels out now: a held slot would block admission
                keep[tag] = copy_labels(ptr, *meta[tag][1].shape)
            srv.release(slot)

    while i < len(sched):
        t_arr, cam = sched[i]
        target = t0 + int(t_arr * 1e9)
        while time.perf_counter_ns() < target:
            drain_once()
        frame_h, frame_d = rings[cam][idx[cam] % len(rings[cam])]
        idx[cam] += 1
        meta[i] = (cam, frame_h)
        rc = srv.submit(frame_d, i)
        if rc != 0:
            raise binding.CclError("ccl_server_submit failed: %d" % rc)
        i += 1
    while srv.pending() > 0:
        drain_once()
        time.sleep(0.0001)
    drain_once()
    srv.close()
    if check:
        for tag, labels in sorted(keep.items()):
            check(tag, meta[tag][1], labels)
    n = len(lat)
    span = (max(done_ts) - min(done_ts)) * 1e-9 if n > 1 else 0.0
    lat_sorted = sorted(lat)
    p = lambda q: lat_sorted[min(n - 1, int(q * n))] if n else float("nan")
    # throughput over the whole run: first submission to last completion
    total_s = (max(done_ts) - min(sub_ts)) * 1e-9 if n else float("nan")
    return ServeResult("plain" if plain else "batched", rate, n, n / total_s if n else 0.0,
                       p(0.50), p(0.99), statistics.mean(lat) if n else float("nan"),
                       max(lat) if n else float("nan"), span)


def saturation_fps(rings, plain: bool, conn: int = 8, n_frames: int = 400, **kw):
    """Throughput with every frame submitted at once (closed loop on the GPU)."""
    res = run(rings, rate=1e9, duration_s=n_frames / 1e9, plain=plain, conn=conn, **kw)
    return res.fps
