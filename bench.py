"""Throughput of the Gradient-SDF tracking + fusion loop on one MI355X.

Workload: the seeded synthetic room stream at 640x480 (fx = fy = 525,
cx = 319.5, cy = 239.5), 1 cm voxels, 5 cm truncation, 8^3 blocks,
3-level pyramid with 4/5/10 Gauss-Newton iterations (finest first), Huber
delta 1 cm.  Depth noise sigma(z) = 0.0012 + 0.0019 (z - 0.4)^2, range
0.4-4 m.  One step = one frame: track it against the map, then allocate and
integrate it at the estimated pose.  Frame 0 is fused at its ground-truth
pose before the warm-up.  All depth frames are resident in HBM before the
timed region starts.

Prints one JSON line (see the fields below).
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=89)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=12,
                    help="frames of the stream the oracle runs for the CPU baseline")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel event timing")
    return ap.parse_args()


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2111_13652_amd import _lib, synth
    from paper_2111_13652_amd.gsdf import GsdfMap

    cfg = synth.CONFIG_ROOM
    cam = cfg["cam"]
    n_frames = max(100, 1 + args.warmup + args.steps)
    t0 = time.time()
    stream = synth.make_stream(cam, n_frames, scene_seed=1, traj_seed=2, noise_seed=3)
    gen_s = time.time() - t0
    print(f"# generated {n_frames} frames in {gen_s:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    depth = torch.as_tensor(stream.depth).to(dev)                       # (F, H, W) float32
    gt = torch.as_tensor(stream.poses).to(dev)                          # (F, 3, 4) float64
    est = torch.zeros_like(gt)
    levels, iters, delta = 3, (4, 5, 10), 0.01
    m = GsdfMap(cfg["voxel_size"], cfg["truncation"], max_blocks=1 << 16, storage="fp32")
    s = torch.cuda.current_stream()

    def step(f):
        est[f].copy_(est[f - 1])
        m.track(depth[f], cam, est[f], levels=levels, iters=iters, delta=delta)
        m.allocate(depth[f], cam, est[f])
        m.integrate(depth[f], cam, est[f])

    est[0].copy_(gt[0])
    m.allocate(depth[0], cam, est[0])
    m.integrate(depth[0], cam, est[0])
    for f in range(1, 1 + args.warmup):
        step(f)
    torch.cuda.synchronize()

    lib = _lib.load()
    timing = not args.no_timing
    if timing:
        lib.gsdf_timing_enable(1)
    first = 1 + args.warmup
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(s)
    for f in range(first, first + args.steps):
        step(f)
    ev1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    fps = args.steps / (ms / 1e3)

    kernels = {}
    if timing:
        import ctypes as C
        for name, kid in (("track", _lib.K_TRACK), ("integrate", _lib.K_INTEGRATE),
                          ("allocate", _lib.K_ALLOCATE), ("pyramid", _lib.K_PYRAMID)):
            tot = C.c_double()
            n = C.c_int64()
            lib.gsdf_timing_read(kid, C.byref(tot), C.byref(n))
            kernels[name] = {"total_ms": tot.value, "launches": n.value,
                             "avg_us": 1e3 * tot.value / max(1, n.value)}
        lib.gsdf_timing_enable(0)

    # accuracy alongside throughput: ATE of the estimated trajectory
    E = est[: first + args.steps].cpu().numpy()
    G = stream.poses[: first + args.steps]
    ate = float(np.sqrt(np.mean(np.sum((E[:, :, 3] - G[:, :, 3]) ** 2, axis=1))))
    status = m.status_flags()

    # algorithmic bytes (per launch) of the kernels
    valid = (stream.depth[first:first + args.steps] > 0).sum(axis=(1, 2)).mean()
    npx = cam.width * cam.height
    report = {
        "metric": "tracked+fused frames/s at 640x480, 1 cm voxels; % of HBM peak GB/s",
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded room stream; stands in for TUM RGB-D 640x480 depth)",
        "config": {"workload": "room stream 640x480, 1 cm voxels, T 5 cm, 8^3 blocks, 3-level "
                               "pyramid (4/5/10 GN iterations), fp32 voxels",
                   "frames": n_frames, "wall_s": wall},
        "accuracy": {"ate_rmse_m": ate, "status": status},
        "kernels": kernels,
    }
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
