"""Benchmark: frames/s of the MI355X Gaussian-splatting rasterizer.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]

A step is one forward render (preprocess, scan, duplicate, sort, ranges,
blend) of the configuration's synthetic scene, inputs resident in HBM.  The
same run also times forward+backward steps (forward, L1 loss gradient,
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
    ap.add_argument("--sort-variant", type=int, default=0, choices=[0, 1, 2, 3])
    ap.add_argument("--sort-algo", default="auto", choices=["auto", "onesweep", "reduce_scan"])
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=40.0)
    return ap.parse_args()


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
        # preprocess: 40 B of geometry + SH in, 61 B of splat state out per Gaussian
        "preprocess_ms": ("k_preprocess", 1, (40 + sh_bytes + 61) * n),
        # compaction of the visible splats: 16 B read per Gaussian, 20 B written per visible one
        "scan_ms": ("k_vis_count + k_vis_scatter", 1, 16 * n + 20 * nvis),
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
    if variant == 1:  # first pass over (u64 key, u32 value) pairs written by k_duplicate
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
    if dom == "sort_ms":  # the first pass alone, from its own event
        per_launch_ms = first_pass_ms
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


def cpu_baseline(scene, cam, budget_s):
    """The FP64 oracle, as it is, on the host cores: one full forward frame of
    the same scene and camera (the oracle's projection, keys, sort, ranges and
    blend).  Falls back to a 1/8 Gaussian subsample when a full frame would
    exceed the budget; the sample is stated in the output."""
    from oracle import oracle as O
    import multiprocessing
    cores = int(os.environ.get("OMP_NUM_THREADS", multiprocessing.cpu_count()))
    n = scene["n"]
    # estimate from a 1/64 subsample first
    def sub(frac):
        m = max(1, int(n * frac))
        idx = np.random.default_rng(0).choice(n, m, replace=False)
        idx.sort()
        s = {k: (np.ascontiguousarray(v[..., idx]) if isinstance(v, np.ndarray) else v)
             for k, v in scene.items()}
        s["n"] = m
        return s
    t0 = time.perf_counter()
    O.render(sub(1 / 64), cam)
    t_small = time.perf_counter() - t0
    frac, label = 1.0, "one full frame"
    if t_small * 64 > budget_s:
        frac, label = 1 / 8, "one frame of a 1/8 random subsample of the Gaussians"
    s = scene if frac == 1.0 else sub(frac)
    t0 = time.perf_counter()
    O.render(s, cam)
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{label} ({s['n']} Gaussians, {cam.width}x{cam.height}), FP64 C oracle, "
                      f"OpenMP over Gaussians and pixels, single-threaded stable sort; {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2509_25626_amd import scenes as S
    from paper_2509_25626_amd.render import GaussianScene, Renderer

    scene_np, cam = S.config_scene(args.config)
    dev = torch.device("cuda", 0)
    scene = GaussianScene.from_numpy(scene_np, device=dev)
    R = Renderer(0)
    # two frame objects used in turn: a frame's stage events are read after the
    # next frame has been enqueued, so reading them never stalls the stream
    frames = [R.acquire_frame(), R.acquire_frame()]
    frame = frames[0]
    H, W = cam.height, cam.width
    out = (torch.empty((3, H, W), device=dev), torch.empty((H, W), device=dev),
           torch.empty((H, W), dtype=torch.int32, device=dev))

    def fwd(fr, timing=False):
        return R.forward(scene, cam, frame=fr, blend_variant=args.blend_variant, out=out, timing=timing,
                         sort_variant=args.sort_variant, sort_algo=args.sort_algo)

    def accumulate(acc, fr):
        for k, v in fr.stage_times().items():
            acc[k] = acc.get(k, 0.0) + v

    for i in range(max(2, args.warmup)):
        fwd(frames[i % 2])
    torch.cuda.synchronize()
    stage_acc = {}
    t0 = time.perf_counter()
    for i in range(args.steps):
        fwd(frames[i % 2], timing=True)
        if i > 0:
            accumulate(stage_acc, frames[(i - 1) % 2])
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.steps
    accumulate(stage_acc, frames[(args.steps - 1) % 2])
    stages = {k: v / args.steps for k, v in stage_acc.items()
              if not k.endswith("backward_ms") and k != "sort_first_pass_ms"}
    first_pass_ms = stage_acc.get("sort_first_pass_ms", 0.0) / args.steps
    info = frame.info()
    K, passes = int(info.num_keys), int(info.sort_passes)

    result_extra = {}
    if not args.no_backward:
        target = torch.from_numpy(S.target_image(40, W, H)).to(dev)
        grads = {k: torch.empty_like(getattr(scene, k)) for k in
                 ("means", "log_scales", "quats", "opacity_logits", "sh")}
        dl = torch.empty((3, H, W), device=dev)
        loss = torch.empty(1, device=dev)

        def fwdbwd(fr, timing=False):
            rgb, T, nc, _ = fwd(fr, timing)
            R.l1_loss_grad(rgb, target, dl, loss)
            R.backward(fr, scene, cam, T, nc, dl, grads)

        for i in range(max(2, args.warmup // 2)):
            fwdbwd(frames[i % 2])
        torch.cuda.synchronize()
        bw_acc = {}
        t0 = time.perf_counter()
        for i in range(args.steps):
            fwdbwd(frames[i % 2], timing=True)
            if i > 0:
                accumulate(bw_acc, frames[(i - 1) % 2])
        torch.cuda.synchronize()
        t_fb = (time.perf_counter() - t0) / args.steps
        accumulate(bw_acc, frames[(args.steps - 1) % 2])
        result_extra["fwd_bwd_fps"] = round(1.0 / t_fb, 3)
        result_extra["fwd_bwd_ms"] = round(t_fb * 1e3, 4)
        result_extra["backward_stage_ms"] = {k: round(v / args.steps, 4) for k, v in bw_acc.items()
                                             if k.endswith("backward_ms")}

    roof = roofline(stages, scene, K, passes, info, first_pass_ms, args.sort_variant, args.sort_algo)

    serving = None
    if not args.no_serving:
        try:
            from paper_2509_25626_amd import serve
            serving = serve.bench_serving(quick=True)
        except Exception as e:  # serving is reported when available
            serving = {"error": str(e)[:200]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene_np, cam, args.cpu_budget_s)

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
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {scene.n} Gaussians SH{scene.sh_degree}, {W}x{H}, 16x16 tiles, "
                               "forward render", "gaussians": scene.n, "width": W, "height": H,
                   "keys": K, "sort_passes": passes, "parallelism": "single GPU"},
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        **result_extra,
        "serving": serving,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    R.release_frame(frame)
    R.close()


if __name__ == "__main__":
    main()
