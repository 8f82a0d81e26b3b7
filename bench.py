"""Benchmark: frames/s of the MI355X Gaussian-splatting rasterizer.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]

A step is one forward render (preprocess, scan, duplicate, sort, ranges,
blend) of the configuration's synthetic scene, inputs resident in HBM, one
frame at a time (`value`); the same frames are also timed with two in flight
on two streams (`fwd_fps_2_in_flight`).  The run also times forward+backward steps (forward, L1 loss gradient,
backward) and reports per-stage times from HIP events recorded on the render
stream, the roofline position of the dominant kernel, and the CPU oracle timed
on the host cores.  Prints one JSON line.
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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed), TFLOP/s

# Algorithmic HBM bytes of each forward stage's kernels (each byte the
# computation must move once): see roofline().


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "room"])
    ap.add_argument("--blend-variant", type=int, default=0)
    ap.add_argument("--sort-variant", type=int, default=0, choices=[0, 1, 2, 3, 4])
    ap.add_argument("--sort-algo", default="auto", choices=["auto", "onesweep", "reduce_scan"])
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true")
    ap.add_argument("--no-in-flight", action="store_true",
                    help="skip the two-frames-in-flight timing (kernel traces of one frame at a time)")
    ap.add_argument("--quick-serving", action="store_true",
                    help="300 requests per load instead of 2000")
    ap.add_argument("--cpu-budget-s", type=float, default=40.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB three times (the known-size reference "
                         "for scaling the HBM traffic counters) and exit")
    return ap.parse_args()


def calibrate_copy(gib, reps=3):
    """A plain device-to-device copy of exactly `gib` GiB in and out per
    repetition: under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, what the
    counters read for it is the scale for every other kernel's reading."""
    import torch
    n = (gib << 30) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_gib": gib, "repetitions": reps}), flush=True)


def roofline(stages, scene, K, passes, info, first_pass_ms, variant, algo):
    """Roofline position of the dominant forward stage: algorithmic bytes per
    launch of its main kernel over that kernel's average launch duration, from
    the HIP events the library records on the render stream."""
    n = scene.n
    sh_bytes = 4 * 3 * (scene.sh_degree + 1) ** 2
    tiles = int(info.tiles_x) * int(info.tiles_y)
    nvis = int(info.num_visible)
    tile_passes = max(int(passes) - 4, 1)
    tile_bits = max(1, (tiles - 1).bit_length())
    tile_digit_bits = -(-tile_bits // tile_passes)  # widest digit of the balanced split
    # between tile passes a key travels as one packed word (remaining tile bits
    # and Gaussian index) when they fit 32 bits
    value_bits = max(1, (n - 1).bit_length())
    packed = tile_passes > 1 and (tile_bits - tile_digit_bits) + value_bits <= 32
    word = 4 if packed else 8
    table = {
        # kernel, launches per frame, algorithmic bytes per launch
        # preprocess: 40 B of geometry + SH in, 61 B of splat state out per Gaussian,
        # 24 B of visible counts per workgroup of 256, and the depth sort's
        # look-back words it clears (4 passes x 256 digits per 4096 Gaussians)
        "preprocess_ms": ("k_preprocess_counted<false>", 1,
                          (40 + sh_bytes + 61) * n + 24 * (-(-n // 256)) + 4 * 4 * 256 * (-(-n // 4096))),
        # compaction of the visible splats: 16 B read per Gaussian, 20 B written per visible one
        "scan_ms": ("k_scan_sums + k_vis_scatter", 1, 16 * n + 20 * nvis),
        # depth order: 4 onesweep passes over (u32 depth, u32 position) of the visible splats
        "depth_order_ms": ("k_sort_pass_onesweep<u32,8> (depth digits)", 4, 16 * nvis),
        # duplicate: 8 B per key (tile id, value) + 24 B per Gaussian read
        "duplicate_ms": ("k_duplicate", 1, 8 * K + 24 * n),
        # tile sort, its first pass: keys generated from the splat records in
        # depth order (4 B offset + 16 B record per visible splat, 4 B owner per
        # 1024 keys read) and written once as packed words (else tile id + value)
        # (512-thread workgroups from 2^23 keys on, as the library chooses)
        "sort_ms": (f"k_sort_pass_gen<{tile_digit_bits}, {512 if K >= (1 << 23) else 256}>", 1,
                    20 * nvis + 4 * (K // 1024 + 1) + word * K),
    }
    if variant in (0, 4) and int(info.num_row_entries) > 0:
        # row-wise placement: the last kernel reads each row-list entry (8 B)
        # and writes each key's value (4 B); its time is the tile stage's
        # minus the column counts and starts before it (its own event)
        table["sort_ms"] = ("k_rp_place_cols", 1, 8 * int(info.num_row_entries) + 4 * K)
    elif variant == 1:  # first pass over (u64 key, u32 value) pairs written by k_duplicate
        table["sort_ms"] = (f"k_sort_pass_onesweep<u64,{tile_digit_bits}> (first pass)", 1, 24 * K)
    elif algo == "reduce_scan":  # first pass over (u32 tile, u32 value) pairs written by k_duplicate
        table["sort_ms"] = (f"k_sort_pass_rts<u32,{tile_digit_bits}> (first pass)", 1, (8 + word) * K)
    table.update({
        # ranges from sorted keys (sort variant 1): read 4 B per key, write 8 B per tile
        "ranges_ms": ("k_ranges4", 1, 4 * K + 8 * tiles),
    })
    dom = max(stages, key=stages.get)
    if dom not in table:
        return {"kernel": dom.replace("_ms", ""), "bound": "alu", "achieved": None, "peak": None,
                "unit": None, "frac": None, "traffic": None, "stage_ms": round(stages[dom], 4)}
    kernel, launches, nbytes = table[dom]
    per_launch_ms = stages[dom] / launches
    if dom == "sort_ms":  # the kernel alone, from its own events
        per_launch_ms = stages[dom] - first_pass_ms if kernel == "k_rp_place_cols" else first_pass_ms
    achieved = nbytes / (per_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(kernel)
    return {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": int(nbytes), "launches_per_frame": launches,
            "avg_launch_ms": round(per_launch_ms, 4),
            # what bounds it instead: the VALU-busy fraction of the same profile
            # (reported with the traffic, i.e. while the kernel source is unchanged)
            "valu_busy": measured_valu_busy(kernel) if traffic is not None else None}


def measured_valu_busy(kernel):
    """VALU-busy fraction of `kernel` from the committed rocprofv3 activity
    table (SQ_ACTIVE_INST_VALU over SIMD cycles), or None."""
    path = os.path.join(ROOT, "profiles", "c2_utilisation.txt")
    try:
        with open(path) as f:
            for line in f:
                if line.startswith(kernel + " ") or line.startswith(kernel[:34] + " "):
                    return float(line[34:].split()[1])
    except (OSError, ValueError, IndexError):
        return None
    return None


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none for this kernel or its source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(kernel)
    if not ent:
        return None
    src = os.path.join(ROOT, ent["source"])
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    return ent["bytes_per_launch"] if sha == ent["source_sha256"] else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _subsample(scene, frac, seed=0):
    n = scene["n"]
    m = max(1, int(n * frac))
    idx = np.random.default_rng(seed).choice(n, m, replace=False)
    idx.sort()
    s = {k: (np.ascontiguousarray(v[..., idx]) if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    s["n"] = m
    return s


def cpu_baseline(scene, cam, budget_s):
    """The FP64 oracle, as it is, on the host cores: full forward frames of the
    same scene and camera (the oracle's projection, keys, sort, ranges and
    blend): one warm-up frame, then the median of three timed frames on every
    core the process may use, plus one frame on a single thread over a random
    1/16 subsample of the Gaussians (same image).  Falls back to a 1/8
    subsample for the all-core frames when three full frames would exceed
    the budget; the sample is stated in the output.  Also returns the last
    all-core oracle result (its per-pixel counts give the blend's algorithmic
    work)."""
    from oracle import oracle as O
    cores = O.get_threads()
    t0 = time.perf_counter()
    O.render(scene, cam)  # warm-up (loads the library), and the frame-time estimate
    t_full = time.perf_counter() - t0
    frac, label = 1.0, "full frames"
    if t_full * 3 > budget_s:
        frac, label = 1 / 8, "frames of a 1/8 random subsample of the Gaussians"
    s = scene if frac == 1.0 else _subsample(scene, frac)
    if frac != 1.0:
        O.render(s, cam)  # warm-up of the sample
    times, res = [], None
    for _ in range(3):
        t0 = time.perf_counter()
        res = O.render(s, cam)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    # one thread, on a 1/16 subsample, and the same subsample on every core for the ratio
    s16 = _subsample(scene, 1 / 16, seed=1)
    t0 = time.perf_counter()
    O.render(s16, cam)
    t_all16 = time.perf_counter() - t0
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        O.render(s16, cam)
        t_one16 = time.perf_counter() - t0
    finally:
        O.set_threads(cores)
    out = {"value": round(1.0 / dt, 5), "unit": "frames/s", "cores": cores, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{label} ({s['n']} Gaussians, {cam.width}x{cam.height}), FP64 C oracle, OpenMP over "
                     f"Gaussians and pixels, single-threaded stable sort; 1 warm-up + median of 3 "
                     f"({', '.join(f'{t:.2f}' for t in times)} s)",
           "single_thread": {"value": round(1.0 / t_one16, 5), "unit": "frames/s",
                             "sample": f"one frame of a 1/16 random subsample ({s16['n']} Gaussians, "
                                       f"{cam.width}x{cam.height}) on one thread: {t_one16:.2f} s "
                                       f"against {t_all16:.2f} s on {cores} threads"}}
    return out, res


# Algorithmic VALU issue slots of the blend per (pixel, splat) pair, counted
# from the arithmetic Alg. 1 needs in float32: an examined pair needs the
# offset (2 sub), the quadratic form (7 mul/fma/add), the power > 0 test, the
# exponential (one transcendental, a quarter-rate instruction: 4 slots),
# alpha = min(0.99, o G) (2), the 1/255 test, T (1 - alpha) (2) and its test:
# 21 slots.  A blended pair adds the weight alpha T and three colour FMAs (4)
# and the contributor index (1): 5 slots.  The backward pass examines each
# position up to the pixel's last contributor (the same 21 slots to recover
# alpha) and, per blended pair, recovers T by a reciprocal (2), updates the
# three composited-behind colours (6), forms dL/dalpha (6) and the nine 2D
# gradient terms (16): 30 slots.  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.3e12 non-packed lane slots per second.
VALU_SLOTS_PEAK = 256 * 4 * 16 * 2.4e9
SLOTS_EXAMINED, SLOTS_BLENDED, SLOTS_BWD_BLENDED = 21, 5, 30


def blend_work(o):
    """Algorithmic pair counts of one frame from the oracle's per-pixel
    counts: examined pairs, blended pairs, and the backward pass's examined
    positions (up to the last contributor)."""
    ne = int(o["n_eval"].astype(np.int64).sum())
    nb = int(o["n_used"].astype(np.int64).sum())
    nc = int(o["n_contrib"].astype(np.int64).sum())
    return {"examined_pairs": ne, "blended_pairs": nb, "backward_examined_pairs": nc}


def blend_roofline(work, blend_ms, blend_bwd_ms=None):
    fwd_slots = SLOTS_EXAMINED * work["examined_pairs"] + SLOTS_BLENDED * work["blended_pairs"]
    out = {"bound": "alu", "unit": "lane-slots/s", "peak": VALU_SLOTS_PEAK,
           "algorithmic_slots": fwd_slots, "avg_launch_ms": round(blend_ms, 4),
           "achieved": round(fwd_slots / (blend_ms * 1e-3), 1),
           "frac": round(fwd_slots / (blend_ms * 1e-3) / VALU_SLOTS_PEAK, 4), **work}
    if blend_bwd_ms:
        bwd_slots = SLOTS_EXAMINED * work["backward_examined_pairs"] + SLOTS_BWD_BLENDED * work["blended_pairs"]
        out["backward"] = {"algorithmic_slots": bwd_slots, "avg_launch_ms": round(blend_bwd_ms, 4),
                           "frac": round(bwd_slots / (blend_bwd_ms * 1e-3) / VALU_SLOTS_PEAK, 4)}
    return out


def tile_statistics(o, W, H):
    """Table 3's workload shape from one frame: splats per tile (mean and
    variance over the tiles) and the fraction of its tile's splats a pixel
    examines (mean over pixels with a non-empty list)."""
    lens = (o["ranges"][:, 1].astype(np.int64) - o["ranges"][:, 0])
    tiles_x = (W + 15) // 16
    ys, xs = np.mgrid[0:H, 0:W]
    L = lens[(ys // 16) * tiles_x + xs // 16]
    nz = L > 0
    frac = float((o["n_eval"][nz] / L[nz]).mean()) if nz.any() else 0.0
    return {"splats_per_tile_mean": round(float(lens.mean()), 1), "splats_per_tile_var": round(float(lens.var()), 1),
            "splats_per_tile_max": int(lens.max()), "processed_fraction": round(frac, 4)}


class Bench:
    """Times forward and forward+backward frames of one scene on the render
    stream, with stage times from the library's HIP events."""

    def __init__(self, R, scene_np, cam, args):
        import torch
        from paper_2509_25626_amd.render import GaussianScene
        self.R, self.cam, self.args = R, cam, args
        self.dev = torch.device("cuda", 0)
        self.scene = GaussianScene.from_numpy(scene_np, device=self.dev)
        # two frame objects used in turn: a frame's stage events are read after
        # the next frame has been enqueued, so reading them never stalls the stream
        self.frames = [R.acquire_frame(), R.acquire_frame()]
        H, W = cam.height, cam.width
        self.out = (torch.empty((3, H, W), device=self.dev), torch.empty((H, W), device=self.dev),
                    torch.empty((H, W), dtype=torch.int32, device=self.dev))

    def fwd(self, fr, timing=False, for_backward=False):
        a = self.args
        return self.R.forward(self.scene, self.cam, frame=fr, blend_variant=a.blend_variant, out=self.out,
                              timing=timing, sort_variant=a.sort_variant, sort_algo=a.sort_algo,
                              for_backward=for_backward)

    @staticmethod
    def _accumulate(acc, fr):
        for k, v in fr.stage_times().items():
            acc[k] = acc.get(k, 0.0) + v

    def _run(self, step, steps, warmup):
        """Seconds per step over `steps` timed steps (no stage events: the
        events of stage timing cost the stream a few microseconds each), then
        the stage times from a separate run of up to 10 steps with them."""
        import torch
        for i in range(max(2, warmup)):
            step(self.frames[i % 2])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(self.frames[i % 2])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        acc = {}
        nst = max(2, min(steps, 10))
        for i in range(nst):
            step(self.frames[i % 2], timing=True)
            if i > 0:
                self._accumulate(acc, self.frames[(i - 1) % 2])
        torch.cuda.synchronize()
        self._accumulate(acc, self.frames[(nst - 1) % 2])
        return dt, {k: v / nst for k, v in acc.items()}

    def forward(self, steps, warmup):
        dt, st = self._run(self.fwd, steps, warmup)
        stages = {k: v for k, v in st.items() if not k.endswith("backward_ms") and k != "sort_first_pass_ms"}
        return dt, stages, st.get("sort_first_pass_ms", 0.0)

    def forward_in_flight(self, steps, warmup):
        """Seconds per forward frame with two frames in flight: frames go in
        turn to two streams, each with its own frame object and output
        buffers, so one frame's preprocess runs beside the other's depth sort
        and tile lists.  Every frame is rendered in full."""
        import torch
        H, W = self.cam.height, self.cam.width
        outs = [self.out] + [(torch.empty((3, H, W), device=self.dev), torch.empty((H, W), device=self.dev),
                              torch.empty((H, W), dtype=torch.int32, device=self.dev))]
        streams = [torch.cuda.current_stream(self.dev), torch.cuda.Stream(self.dev)]
        a = self.args

        def render(i):
            with torch.cuda.stream(streams[i % 2]):
                self.R.forward(self.scene, self.cam, frame=self.frames[i % 2], blend_variant=a.blend_variant,
                               out=outs[i % 2], sort_variant=a.sort_variant, sort_algo=a.sort_algo)

        for i in range(max(2, warmup)):
            render(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            render(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def forward_backward(self, steps, warmup):
        import torch
        from paper_2509_25626_amd import scenes as S
        H, W = self.cam.height, self.cam.width
        target = torch.from_numpy(S.target_image(40, W, H)).to(self.dev)
        grads = {k: torch.empty_like(getattr(self.scene, k)) for k in
                 ("means", "log_scales", "quats", "opacity_logits", "sh")}
        dl = torch.empty((3, H, W), device=self.dev)
        loss = torch.empty(1, device=self.dev)

        def step(fr, timing=False):
            rgb, T, nc, _ = self.fwd(fr, timing, for_backward=True)
            self.R.l1_loss_grad(rgb, target, dl, loss)
            self.R.backward(fr, self.scene, self.cam, T, nc, dl, grads)

        dt, st = self._run(step, steps, warmup)
        return dt, {k: v for k, v in st.items() if k.endswith("backward_ms")}

    def close(self):
        for f in self.frames:
            self.R.release_frame(f)
        self.scene = None


def other_config(R, name, args, backward):
    """Forward (and forward+backward) frames/s of another configuration with
    the same kernels, plus its stage times."""
    import torch
    from paper_2509_25626_amd import scenes as S
    scene_np, cam = S.config_scene(name)
    b = Bench(R, scene_np, cam, args)
    steps = max(5, args.steps // 2)
    dt, stages, _ = b.forward(steps, max(2, args.warmup // 2))
    info = b.frames[0].info()
    res = {"workload": f"{name}: {scene_np['n']} Gaussians SH{scene_np['sh_degree']}, {cam.width}x{cam.height}",
           "fwd_fps": round(1.0 / dt, 2), "fwd_ms": round(dt * 1e3, 4), "keys": int(info.num_keys),
           "visible": int(info.num_visible), "stage_ms": {k: round(v, 4) for k, v in stages.items()}}
    if name == "c1":
        res["fwd_us"] = round(dt * 1e6, 1)
    if backward:
        dtb, bst = b.forward_backward(steps, max(2, args.warmup // 2))
        res["fwd_bwd_fps"] = round(1.0 / dtb, 2)
        res["fwd_bwd_ms"] = round(dtb * 1e3, 4)
        res["backward_stage_ms"] = {k: round(v, 4) for k, v in bst.items()}
    b.close()
    del b
    torch.cuda.synchronize()
    return res, scene_np, cam, stages


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the renderer has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2509_25626_amd import scenes as S
    from paper_2509_25626_amd.render import Renderer

    scene_np, cam = S.config_scene(args.config)
    R = Renderer(0)
    b = Bench(R, scene_np, cam, args)
    H, W = cam.height, cam.width
    t_fwd, stages, first_pass_ms = b.forward(args.steps, args.warmup)
    info = b.frames[0].info()
    t_fly = None if args.no_in_flight else b.forward_in_flight(args.steps, args.warmup)
    K, passes = int(info.num_keys), int(info.sort_passes)
    roof = roofline(stages, b.scene, K, passes, info, first_pass_ms, args.sort_variant, args.sort_algo)

    # forward frames/s with two frames in flight on two streams (a sequence of
    # frames rendered back to back); `value` is one frame at a time
    result_extra = ({"fwd_fps_2_in_flight": round(1.0 / t_fly, 3), "fwd_ms_2_in_flight": round(t_fly * 1e3, 4)}
                    if t_fly else {})
    bwd_stages = {}
    if not args.no_backward:
        t_fb, bwd_stages = b.forward_backward(args.steps, max(2, args.warmup // 2))
        result_extra["fwd_bwd_fps"] = round(1.0 / t_fb, 3)
        result_extra["fwd_bwd_ms"] = round(t_fb * 1e3, 4)
        result_extra["backward_stage_ms"] = {k: round(v, 4) for k, v in bwd_stages.items()}
    b.close()
    del b
    torch.cuda.synchronize()

    others = {}
    if not args.no_other_configs and args.config == "c2":
        for name in ("c1", "c4", "c3", "room"):
            res, sc_o, cam_o, st_o = other_config(R, name, args, backward=(name == "c4"))
            if name == "room":
                # the paper's blend-bound regime: Table 3's statistics and the blend's work
                from oracle import oracle as O
                o = O.render(sc_o, cam_o, round_f32=True)
                res["table3"] = tile_statistics(o, cam_o.width, cam_o.height)
                res["blend_roofline"] = blend_roofline(blend_work(o), st_o["blend_ms"])
                for v in (1, 3, 5):
                    args_v = argparse.Namespace(**{**vars(args), "blend_variant": v})
                    rv, _, _, stv = other_config(R, name, args_v, backward=False)
                    res[f"blend_variant_{v}_ms"] = round(stv["blend_ms"], 4)
            if name == "c1":
                for v in (1, 3, 5):
                    args_v = argparse.Namespace(**{**vars(args), "blend_variant": v})
                    rv, _, _, stv = other_config(R, name, args_v, backward=False)
                    res[f"blend_variant_{v}_ms"] = round(stv["blend_ms"], 4)
            others[name] = res

    serving = None
    if not args.no_serving:
        try:
            from paper_2509_25626_amd import serve
            serving = serve.bench_serving(quick=args.quick_serving)
        except Exception as e:  # serving is reported when available
            serving = {"error": str(e)[:200]}

    cpu = None
    blend_roof = None
    if not args.no_cpu_baseline:
        cpu, o = cpu_baseline(scene_np, cam, args.cpu_budget_s)
        if o is not None and o["image"].shape[1:] == (H, W) and "full" in cpu["sample"]:
            work = blend_work(o)
            blend_roof = blend_roofline(work, stages["blend_ms"], bwd_stages.get("blend_backward_ms"))
            blend_roof["table3"] = tile_statistics(o, W, H)

    fps = 1.0 / t_fwd
    line = {
        "metric": "frames/s at 3M Gaussians 1.3MP (fwd, fwd+bwd); p50/p99 batched-serve ms",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_fwd * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "float32 storage and blending; the projection's decisions (cull, radius, tile "
                      "rectangle, depth bits) and the blend's quadratic form are evaluated in float64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {scene_np['n']} Gaussians SH{scene_np['sh_degree']}, {W}x{H}, "
                               "16x16 tiles, forward render", "gaussians": scene_np["n"], "width": W,
                   "height": H, "keys": K, "sort_passes": passes, "parallelism": "single GPU"},
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        **result_extra,
        "other_configs": others or None,
        "serving": serving,
        "roofline": roof,
        "blend_roofline": blend_roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    R.close()


if __name__ == "__main__":
    main()
