"""Continuous-batching render server (Python side).

`Server` wraps the library's server: scenes registered once stay resident in
HBM; `submit` queues a render request and returns a ticket; the library's
scheduler thread admits queued requests into batched launches as in-flight
slots and the HBM budget allow, on two streams so that one batch's
preprocessing overlaps the previous batch's sort and blend.

`bench_serving` replays seeded Poisson request traces over sixteen resident
outdoor-like scenes (0.2M-3M Gaussians, log-uniform sizes, SH degree 3) at
random orbit poses and resolutions, through a batched server and through a
one-request-at-a-time server, and reports arrival-to-completion p50/p99 latency
and frames/s for each.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import native
from .native import P, check
from .render import GaussianScene

__all__ = ["Server", "bench_serving"]


class Server:
    """A render server on its own library context (device memory from hipMalloc,
    so the scheduler thread never calls back into Python)."""

    def __init__(self, device: int = 0, max_slots: int = 16, max_batch: int = 8, hbm_budget_bytes: int = 0,
                 sort_variant: int = 0):
        self.L = native.load()
        self.device = torch.device("cuda", device)
        ctx = P()
        check(self.L.cds_create(ctypes.byref(ctx), device, None))
        self._ctx = ctx
        opts = native.CdsServerOpts(int(max_slots), int(max_batch), int(hbm_budget_bytes), int(sort_variant), 0)
        h = P()
        try:
            check(self.L.cds_server_create(ctx, ctypes.byref(opts), ctypes.byref(h)))
        except Exception:
            self.L.cds_destroy(ctx)
            self._ctx = None
            raise
        self.handle = h
        self._scenes = []   # keeps the registered tensors alive
        self._outs = {}     # ticket -> output tensor, kept alive until collected

    def add_scene(self, scene: GaussianScene) -> int:
        torch.cuda.synchronize(self.device)  # uploads complete before the server's streams read them
        sid = ctypes.c_int32()
        st = scene.struct()
        check(self.L.cds_server_add_scene(self.handle, ctypes.byref(st), ctypes.byref(sid)))
        self._scenes.append(scene)
        return sid.value

    def submit(self, scene_id: int, cam, out: torch.Tensor | None = None):
        """Queue a render; returns (ticket, out).  `out` ([3,H,W] float32 on the
        server's device) is written by the server and valid once `poll` says so."""
        cs = native.camera_struct(cam)
        if out is None:
            out = torch.empty((3, cs.height, cs.width), dtype=torch.float32, device=self.device)
            torch.cuda.synchronize(self.device)
        elif tuple(out.shape) != (3, cs.height, cs.width) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor of shape [3,H,W]")
        t = ctypes.c_uint64()
        check(self.L.cds_server_submit(self.handle, int(scene_id), ctypes.byref(cs), out.data_ptr(),
                                       ctypes.byref(t)))
        self._outs[t.value] = out
        return t.value, out

    def poll(self, ticket: int):
        """(done, latency_ms): latency from submit to completion, once done.  A
        done ticket is collected and cannot be polled again."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        try:
            check(self.L.cds_server_poll(self.handle, int(ticket), ctypes.byref(done), ctypes.byref(lat)))
        except native.CdsError:
            self._outs.pop(ticket, None)
            raise
        if done.value:
            self._outs.pop(ticket, None)
            return True, lat.value
        return False, None

    def drain(self):
        check(self.L.cds_server_drain(self.handle))

    def stats(self) -> dict:
        s = native.CdsServerStats()
        check(self.L.cds_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in native.CdsServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self.L.cds_server_destroy(self.handle)
            self.handle = None
        if getattr(self, "_ctx", None):
            self.L.cds_destroy(self._ctx)
            self._ctx = None
        self._outs.clear()
        self._scenes = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _OutputRing:
    """Reusable output images per resolution; a slot is reused only after the
    request that last wrote it has completed."""

    def __init__(self, device, per_res: int):
        self.device = device
        self.per_res = per_res
        self.bufs = {}
        self.next = {}

    def get(self, w, h):
        key = (w, h)
        if key not in self.bufs:
            self.bufs[key] = [torch.empty((3, h, w), dtype=torch.float32, device=self.device)
                              for _ in range(self.per_res)]
            self.next[key] = 0
        i = self.next[key]
        self.next[key] = (i + 1) % self.per_res
        return key, i, self.bufs[key][i]


def _replay(server: Server, scene_ids, reqs, ring: _OutputRing):
    """Submit `reqs` at their arrival times (seconds from the start) and collect
    every completion.  Returns per-request latency (ms, scheduled arrival to
    completion) and the span from the first arrival to the last completion."""
    from .scenes import orbit_camera
    torch.cuda.synchronize(server.device)
    n = len(reqs)
    lateness = np.zeros(n)
    lat = np.full(n, np.nan)
    done_at = np.zeros(n)
    owner = {}          # (res, slot) -> request index still using that buffer
    open_t = {}         # ticket -> request index

    def collect(block_on=None):
        for t in list(open_t):
            d, l = server.poll(t)
            if d:
                i = open_t.pop(t)
                lat[i] = lateness[i] + l
                done_at[i] = reqs[i][0] + lat[i] * 1e-3
        if block_on is not None:
            while block_on in open_t.values():
                time.sleep(5e-5)
                collect()

    cams = [orbit_camera(w, h, radius=4.0, azimuth_deg=az, elevation_deg=el) for (_, _, w, h, az, el) in reqs]
    t0 = time.perf_counter()
    for i, (arr, sid, w, h, _, _) in enumerate(reqs):
        while True:
            now = time.perf_counter() - t0
            if now >= arr:
                break
            collect()
            if arr - now > 1e-3:
                time.sleep(min(arr - now - 5e-4, 2e-3))
        key, slot, out = ring.get(w, h)
        if (key, slot) in owner:
            collect(block_on=owner[(key, slot)])
        lateness[i] = (time.perf_counter() - t0 - arr) * 1e3
        t, _ = server.submit(scene_ids[sid], cams[i], out)
        owner[(key, slot)] = i
        open_t[t] = i
    server.drain()
    collect()
    assert not open_t, "requests left open after drain"
    span = float(done_at.max() - reqs[0][0]) if n else 0.0
    return lat, span


def _summary(lat, span, stats):
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "frames_per_s": round(len(lat) / span, 2) if span > 0 else None,
            "requests": int(len(lat)), "batches": stats["batches"],
            "peak_workspace_gb": round(stats["peak_workspace_bytes"] / 1e9, 3),
            "peak_held_gb": round(stats["peak_held_bytes"] / 1e9, 3)}


def bench_serving(quick: bool = True, device: int = 0, loads=(0.5, 0.8, 0.95), requests_per_load=None,
                  max_slots: int = 16, max_batch: int = 8, hbm_budget_bytes: int = 16 << 30, seed: int = 5,
                  scene_sizes=None):
    """Serving benchmark over sixteen resident scenes; see the module docstring.

    The one-at-a-time capacity (requests/s) is measured first with a closed
    loop; each offered load is a fraction of it.  Both servers replay the same
    trace.  Latency runs from the scheduled arrival to the completion event."""
    from . import scenes as S
    dev = torch.device("cuda", device)
    sizes = scene_sizes or S.serving_scene_sizes(seed)
    count = requests_per_load or (300 if quick else 2000)
    t_gen = time.perf_counter()
    resident = [GaussianScene.from_numpy(S.scene_outdoor(seed * 1000 + k, n), device=dev)
                for k, n in enumerate(sizes)]
    t_gen = time.perf_counter() - t_gen
    out = {"scenes": len(sizes), "gaussians": int(sum(sizes)),
           "resident_gb": round(sum(s.nbytes() for s in resident) / 1e9, 3),
           "resolutions": [f"{w}x{h}" for w, h in S.SERVING_RESOLUTIONS],
           "hbm_budget_gb": round(hbm_budget_bytes / 1e9, 2), "max_slots": max_slots, "max_batch": max_batch,
           "requests_per_load": count, "scene_generation_s": round(t_gen, 1)}
    fifo = Server(device, max_slots=1, max_batch=1, hbm_budget_bytes=hbm_budget_bytes)
    batched = Server(device, max_slots=max_slots, max_batch=max_batch, hbm_budget_bytes=hbm_budget_bytes)
    ring = _OutputRing(dev, per_res=max(2 * max_slots, 32))
    try:
        ids = {}
        for name, srv in (("fifo", fifo), ("batched", batched)):
            ids[name] = [srv.add_scene(s) for s in resident]
        # warm-up: grow both servers' workspaces on the largest requests
        big = int(np.argmax(sizes))
        warm = [(0.0, big, 1920, 1080, 30.0 * k, 0.0) for k in range(2 * max_batch)]
        warm += S.serving_requests(seed + 100, 4 * max_batch, len(sizes), 1e9)
        for name, srv in (("fifo", fifo), ("batched", batched)):
            _replay(srv, ids[name], warm, ring)
        # one-at-a-time capacity: everything arrives at once
        cap_reqs = [(0.0,) + r[1:] for r in S.serving_requests(seed + 200, min(count, 200), len(sizes), 1.0)]
        lat, span = _replay(fifo, ids["fifo"], cap_reqs, ring)
        capacity = len(cap_reqs) / span
        out["fifo_capacity_rps"] = round(capacity, 2)
        out["loads"] = {}
        for k, load in enumerate(loads):
            reqs = S.serving_requests(seed + 300 + k, count, len(sizes), load * capacity)
            res = {"offered_rps": round(load * capacity, 2)}
            for name, srv in (("fifo", fifo), ("batched", batched)):
                s0 = srv.stats()
                lat, span = _replay(srv, ids[name], reqs, ring)
                s1 = srv.stats()
                st = {"batches": s1["batches"] - s0["batches"], "peak_workspace_bytes": s1["peak_workspace_bytes"],
                      "peak_held_bytes": s1["peak_held_bytes"]}
                res[name] = _summary(lat, span, st)
            out["loads"][str(load)] = res
        # saturation: the whole trace at once through the batched server
        sat = [(0.0,) + r[1:] for r in S.serving_requests(seed + 400, count, len(sizes), 1.0)]
        s0 = batched.stats()
        lat, span = _replay(batched, ids["batched"], sat, ring)
        s1 = batched.stats()
        out["batched_capacity_rps"] = round(len(sat) / span, 2)
        out["batched_saturation"] = _summary(lat, span, {"batches": s1["batches"] - s0["batches"],
                                                         "peak_workspace_bytes": s1["peak_workspace_bytes"],
                                                         "peak_held_bytes": s1["peak_held_bytes"]})
    finally:
        fifo.close()
        batched.close()
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--full", action="store_true")
    a = ap.parse_args()
    print(json.dumps(bench_serving(quick=not a.full)), flush=True)
