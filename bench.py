"""Throughput of the Gradient-SDF tracking + fusion loop on one MI355X.

Workload: the seeded synthetic room stream at 640x480 (fx = fy = 525,
cx = 319.5, cy = 239.5), 100 frames, 1 cm voxels, 5 cm truncation, 8^3
blocks, 3-level pyramid with 4/5/10 Gauss-Newton iterations (finest first),
Huber delta 1 cm.  Depth noise sigma(z) = 0.0012 + 0.0019 (z - 0.4)^2, range
0.4-4 m.  One step = one frame: track it against the map, then allocate and
integrate it at the estimated pose (gsdf_track_frame, gsdf_fuse_frame).
Frame 0 is fused at its ground-truth pose, frames 1..W are the warm-up and
frames W+1..W+K are timed.  All depth frames are resident in HBM before the
timed region starts.

Prints one JSON line.  Besides the contract's keys:
  "roofline"      the dominant kernel's algorithmic bytes per launch over its
                  mean launch time (HIP events recorded inside the library
                  around that kernel only, on its stream, in the timed region);
  "cpu_baseline"  the FP64 oracle on a bounded sample of the same stream;
  "kernels"       per-kernel event times from a second pass over the timed
                  frames with every kernel timed (not part of "value": events
                  around every launch cost about 9 % of the frame rate);
  "track_iterations"  where a tracking launch's time goes, per pyramid
                  level: work-group 0's wall-clock stamps after its pixel
                  sums, its part of the exchange, the total and the solve;
  "full_stream"   three passes over the whole 100-frame stream (median);
  "differentiation"  forward + adjoint over keyframes 0, 10, ..., 90 on the
                  100-frame map;
  "joint_refinement" one step of the joint geometry / colour / pose
                  refinement over 30 keyframes (bf16 map, colour stream);
  "comparison"    the paper's baseline system on the same frames: a map
                  without stored gradients tracked with the tri-linear
                  eight-voxel distance of Eq. (12)-(13), against the
                  gradient map with the Taylor distance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s

# Algorithmic bytes per unit of work.
#  tracking, per valid pixel-iteration: depth 4 + hash entry 16 + the voxel's
#    {psi, g} (16 B for float32, 8 B for the 16-bit pack); the float32 sum
#    form also reads W (4 B) to form psi, which the count leaves out;
#  fusion, per (pixel, voxel) update: read + write of the voxel record
#    (float4 + W = 20 B; 16-bit pack + W = 12 B; distance + W = 8 B);
#  allocation + normals, per pixel: depth 4 + {n_w, D} 16 written; plus a hash
#    entry (16 B) per distinct (16x16 tile, block) probe.
TRACK_BYTES = {"fp32": 36.0, "bf16": 28.0, "fp16": 28.0, "nograd": 36.0}
RECORD_BYTES = {"fp32": 20.0, "bf16": 12.0, "fp16": 12.0, "nograd": 8.0}
B_PIXEL_PREP = 4.0 + 16.0
B_ALLOC_PAIR = 16.0

# HBM-side bytes per launch from two rocprofv3 --pmc passes (FETCH_SIZE, then
# WRITE_SIZE) over this workload, each scaled by what the same counter reads
# for a plain 256 MiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).  A
# figure is reported only while the kernel's sources still hash to the
# values they had when the counters were taken.
MEASURED_TRAFFIC = {
    "track": {
        "bytes": 8625789,
        "sources": {
            "gsdf_track.hip": "7b0a13691000a5ba70cd6c2ebde83f0613147e67476830c5ff11efeacefeb93d",
            "gsdf_common.hpp": "5b726ce79643b29c9a682a0b6bcd966907429c824ecb04562facf2ef58d23989",
            "gsdf_host.hpp": "699a644f6155d591caffb7f5edc3cd6c971c32bc580d070b327d1d31c947ff6e",
            "gsdf_se3.hpp": "13c15ea94701e1129da7175cf338be9aa9cc57bf8857172577cef813f6209733"
        }
    }
}


def _traffic(kernel: str, storage: str):
    import hashlib
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or storage != "fp32":
        return None
    csrc = os.path.join(ROOT, "paper_2111_13652_amd", "csrc")
    for name, digest in m["sources"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return m["bytes"]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=89)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=27,
                    help="frames of the stream the oracle runs for the CPU baseline (27: about 12 s "
                         "on a recent server core, 10-30 s on most)")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--no-h2d", action="store_true", help="skip the PCIe-inclusive pass")
    ap.add_argument("--no-full", action="store_true", help="skip the three full-stream passes")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation measurement")
    ap.add_argument("--no-joint", action="store_true", help="skip the joint-refinement step")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the pass with the paper's baseline system")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times "
                         "(scale reference for hardware byte counters)")
    ap.add_argument("--workload", choices=("room640", "room1280"), default="room640",
                    help="room640: the headline workload; room1280: 1280x720, 5 mm voxels, T 2.5 cm")
    ap.add_argument("--storage", choices=("fp32", "bf16", "fp16"), default="fp32",
                    help="voxel storage: fp32 (plain path) or the 16-bit precision form")
    return ap.parse_args()


def _median(x):
    return float(np.median(np.asarray(x, np.float64)))


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(the design notes describe how it would shard)"}))
        sys.exit(2)
    import torch

    from paper_2111_13652_amd import _lib, synth
    from paper_2111_13652_amd.gsdf import GsdfMap

    hd = args.workload == "room1280"
    cfg = synth.CONFIG_ROOM_HD if hd else synth.CONFIG_ROOM
    cam = cfg["cam"]
    n_frames = max(100, 1 + args.warmup + args.steps)
    t0 = time.time()
    sc, tr, nz = cfg["seeds"]
    stream = synth.make_stream(cam, n_frames, scene_seed=sc, traj_seed=tr, noise_seed=nz)
    print(f"# generated {n_frames} frames in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    depth = torch.as_tensor(stream.depth).to(dev)                       # (F, H, W) float32
    gt = torch.as_tensor(stream.poses).to(dev)                          # (F, 3, 4) float64
    est = torch.zeros_like(gt)
    levels, iters, delta = 3, (4, 5, 10), 0.01
    max_blocks = 1 << (18 if hd else 16)
    m = GsdfMap(cfg["voxel_size"], cfg["truncation"], max_blocks=max_blocks, storage=args.storage)
    s = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def step(M, f, src=None, model="taylor"):
        d = depth[f] if src is None else src
        M.track(d, cam, est[f], levels=levels, iters=iters, delta=delta, init=est[f - 1], model=model)
        M.fuse(d, cam, est[f])

    def start(M, warm=args.warmup, model="taylor"):
        M.reset()
        est[0].copy_(gt[0])
        M.fuse(depth[0], cam, est[0])
        for f in range(1, 1 + warm):
            step(M, f, model=model)
        torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        ev0.record(s)
        fn()
        ev1.record(s)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def read_kernels(M):
        out = {}
        for name, kid in (("track", _lib.K_TRACK), ("fuse_blocks", _lib.K_INTEGRATE),
                          ("alloc_normals", _lib.K_ALLOC_NORMALS), ("pyramid", _lib.K_PYRAMID)):
            tot, n = M.timing_read(kid)
            if n:
                out[name] = {"total_ms": tot, "launches": n, "avg_us": 1e3 * tot / max(1, n)}
        return out

    if args.copy_mib > 0:
        n = args.copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy reference: 3 x {args.copy_mib} MiB read + written", file=sys.stderr, flush=True)
        del src, dst

    # ---- the timed region: frames first .. first + K - 1
    start(m)
    timing = not args.no_timing
    if timing:
        # inside the timed region only the roofline kernel (tracking) records
        # events (two per frame); the per-kernel breakdown is a second pass
        m.timing(1 << _lib.K_TRACK)
    first = 1 + args.warmup
    K = args.steps
    c0 = m.counters()
    ms = timed(lambda: [step(m, f) for f in range(first, first + K)])
    fps = K / (ms / 1e3)
    work = (m.counters() - c0).astype(np.float64)
    status = m.status_flags()
    E = est[: first + K].cpu().numpy()
    G = stream.poses[: first + K]
    ate = float(np.sqrt(np.mean(np.sum((E[:, :, 3] - G[:, :, 3]) ** 2, axis=1))))
    print(f"# timed {K} frames: {fps:.1f} frames/s", file=sys.stderr, flush=True)

    kernels, track_live = {}, None
    if timing:
        track_live = read_kernels(m).get("track")
        # breakdown pass: the same frames again with every kernel timed
        start(m)
        m.timing(0xffffffff)
        for f in range(first, first + K):
            step(m, f)
        torch.cuda.synchronize()
        kernels = read_kernels(m)
        m.timing(0)

    # ---- per-iteration breakdown of the tracking launch: the same frames
    # again, work-group 0 stamping the device wall clock after its pixel
    # sums, its part of the exchange, the total and the solve (outside the
    # timed region)
    iteration_clocks = None
    if timing:
        from paper_2111_13652_amd.gsdf import wall_clock_khz
        n_it = sum(iters[:levels])
        clk = torch.zeros((K, 4 * n_it), dtype=torch.int64, device=dev)
        start(m)
        for j, f in enumerate(range(first, first + K)):
            m.track(depth[f], cam, est[f], levels=levels, iters=iters, delta=delta, init=est[f - 1], clocks=clk[j])
            m.fuse(depth[f], cam, est[f])
        torch.cuda.synchronize()
        t = np.median(clk.cpu().numpy().reshape(K, n_it, 4).astype(np.float64), axis=0) * (1e3 / wall_clock_khz())
        prev = np.concatenate([[0.0], t[:-1, 3]])
        parts = np.stack([t[:, 0] - prev, t[:, 1] - t[:, 0], t[:, 2] - t[:, 1], t[:, 3] - t[:, 2]], axis=1)
        lv, i0 = [], 0
        for l in range(levels - 1, -1, -1):   # levels run coarse to fine
            n = iters[l]
            if n:
                mean = parts[i0:i0 + n].mean(axis=0)
                lv.append({"level": l, "iterations": n, "pixel_sums_us": mean[0], "exchange_us": mean[1],
                           "total_us": mean[2], "solve_us": mean[3]})
            i0 += n
        iteration_clocks = {"frames": K, "work_group": 0, "frame_us": float(t[-1, 3]), "levels": lv,
                            "meaning": "per iteration (mean over the level's iterations, median over frames): "
                                       "pixel sums = accumulate + the wait for the work-group's own waves; "
                                       "exchange = partial stored and (leaf leaders) the leaf's partials summed "
                                       "and stored; total = the leaf sums read; solve = 6x6 solve and pose update"}

    # ---- algorithmic bytes, from the live work counters
    npx = cam.width * cam.height
    per_kernel_bytes = {"track": TRACK_BYTES[args.storage] * work[5],
                        "fuse_blocks": 2.0 * RECORD_BYTES[args.storage] * work[0],
                        "alloc_normals": B_PIXEL_PREP * npx * K + B_ALLOC_PAIR * work[4]}
    total_bytes = sum(per_kernel_bytes.values())
    eff_gbs = total_bytes / (ms / 1e3) / 1e9

    roofline = None
    if kernels:
        dom = max(("track", "fuse_blocks", "alloc_normals"), key=lambda k: kernels[k]["total_ms"])
        # the dominant kernel's duration from the timed region when it is the
        # one timed there, else from the breakdown pass
        live = track_live if dom == "track" and track_live else kernels[dom]
        launches = max(1, live["launches"])
        avg_s = live["total_ms"] / 1e3 / launches
        bytes_per_launch = per_kernel_bytes[dom] / launches
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic(dom, args.storage),
                    "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6}

    # ---- three passes over the whole stream: frame 0 fused at its true pose,
    # frames 1 .. F-1 tracked and fused; the map of the last pass stays
    full = None
    if not args.no_full:
        F = depth.shape[0]
        rates = []
        for _ in range(3):
            start(m, warm=0)
            rates.append((F - 1) / (timed(lambda: [step(m, f) for f in range(1, F)]) / 1e3))
        Ef = est.cpu().numpy()
        full = {"frames_timed": f"1-{F - 1}", "passes": 3, "frames_per_s_median": _median(rates),
                "frames_per_s": rates, "blocks": m.num_blocks(), "status": m.status_flags(),
                "ate_rmse_m": float(np.sqrt(np.mean(np.sum((Ef[:, :, 3] - stream.poses[:, :, 3]) ** 2, axis=1))))}
        print(f"# full stream: {full['frames_per_s_median']:.1f} frames/s", file=sys.stderr, flush=True)

    # ---- differentiation: keyframe loss + adjoint over keyframes 0, 10, ...,
    # 90 (poses perturbed by 1 deg / 1 cm, seeds 4 + i) on the map of the
    # 100-frame stream (the last full pass; else the timed frames' map)
    diff = None
    if not args.no_adjoint:
        from paper_2111_13652_amd.gsdf import KeyframeLoss, keyframe_loss
        kf = list(range(0, 100, 10)) if full else list(range(first, first + K, max(1, K // 10)))[:10]
        T0 = torch.as_tensor(np.stack([synth.perturb_pose(stream.poses[f], 4 + i, 1.0, 0.01)
                                       for i, f in enumerate(kf)])).to(dev)
        D = depth[kf].contiguous()
        params = m.export_params().requires_grad_(True)
        xi = torch.zeros((len(kf), 6), dtype=torch.float64, device=dev, requires_grad=True)

        def fwd_bwd():
            params.grad = None
            xi.grad = None
            KeyframeLoss.apply(params, xi, m, D, cam, T0, delta).sum().backward()

        for _ in range(3):
            fwd_bwd()
        reps = 20
        if timing:
            m.timing(0xffffffff)
        dms = timed(lambda: [fwd_bwd() for _ in range(reps)]) / reps
        dk = {}
        if timing:
            for name, kid in (("loss", _lib.K_LOSS), ("backward", _lib.K_BACKWARD)):
                tot, n = m.timing_read(kid)
                dk[name] = {"avg_us": 1e3 * tot / max(1, n), "launches": n}
            m.timing(0)
        cnt = torch.zeros(len(kf), dtype=torch.float64, device=dev)
        keyframe_loss(m, params.detach(), xi.detach(), D, cam, T0, delta, count=cnt)
        used = float(cnt.sum().item())
        observed = int((m.weight[: m.num_blocks() * 512] > 0).sum().item())
        diff = {"keyframes": kf, "map": "100-frame stream" if full else "timed frames",
                "ms_per_forward_backward": dms, "pixels_used": used, "observed_voxels": observed,
                "param_blocks": int(params.shape[0]), "kernels": dk}
        if dk:
            # backward: depth 4 + hash entry 16 + W 4 + params 16 B read, 16 B of
            # gradient added per pixel used; 4 B depth per other pixel
            npx_all = len(kf) * npx
            bb = 4.0 * npx_all + (16 + 4 + 16 + 16) * used
            diff["backward_algorithmic_gbs"] = bb / (dk["backward"]["avg_us"] * 1e-6) / 1e9
        del params, xi

    # ---- joint refinement (the colour stream's configuration): one step =
    # the two adjoints (each also returns its loss), an Adam step on the
    # voxel parameters and colours, and one Gauss-Newton iteration of the
    # tracking kernel per keyframe on the bf16 map
    joint = None
    if not args.no_joint and not hd:
        from paper_2111_13652_amd.gsdf import refine_joint
        kj = list(range(0, 90, 3))                    # 30 keyframes
        t0 = time.time()
        rs = synth.make_rgbd_stream(cam, n_frames, sc, tr, nz, albedo_seed=7, frames=kj)
        print(f"# colour keyframes in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        J = GsdfMap(cfg["voxel_size"], cfg["truncation"], max_blocks=max_blocks, storage="bf16")
        for f in range(n_frames):
            J.fuse(depth[f], cam, gt[f])
        Dj = torch.as_tensor(rs.depth).to(dev)
        Cj = torch.as_tensor(rs.rgb).to(dev)
        Tj = torch.as_tensor(np.stack([synth.perturb_pose(stream.poses[f], 40 + i, 1.0, 0.01)
                                       for i, f in enumerate(kj)])).to(dev)
        refine_joint(J, Dj, Cj, cam, Tj.clone(), steps=2, write_back=False)   # warm-up
        t1 = timed(lambda: refine_joint(J, Dj, Cj, cam, Tj.clone(), steps=1, write_back=False))
        t6 = timed(lambda: refine_joint(J, Dj, Cj, cam, Tj.clone(), steps=6, write_back=False))
        joint = {"keyframes": len(kj), "storage": "bf16", "ms_per_step": (t6 - t1) / 5.0,
                 "ms_setup_and_first_step": t1,
                 "observed_voxels": int((J.weight[: J.num_blocks() * 512] > 0).sum().item())}
        del J, Dj, Cj

    # ---- PCIe-inclusive rate: each frame copied from pinned host memory first
    h2d = None
    if not args.no_h2d:
        host = torch.as_tensor(stream.depth[first:first + K]).pin_memory()
        buf = torch.empty_like(depth[0])
        start(m)

        def run():
            for i, f in enumerate(range(first, first + K)):
                buf.copy_(host[i], non_blocking=True)
                step(m, f, buf)
        h2d = K / (timed(run) / 1e3)

    # ---- CPU baseline: the FP64 oracle on the first frames of the same stream
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n_cpu = max(2, args.cpu_frames)
        t0 = time.perf_counter()
        oracle.track_stream(stream.depth[:n_cpu], cam, stream.poses[:n_cpu], cfg["voxel_size"],
                            cfg["truncation"], levels=levels, iters=iters, delta=delta)
        el = time.perf_counter() - t0
        cpu = {"value": (n_cpu - 1) / el, "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"frames 0-{n_cpu - 1} of the same stream: frame 0 fused at ground truth, "
                         f"{n_cpu - 1} frames tracked + allocated + fused, single-threaded FP64, "
                         f"{el:.1f} s on one core of {_cpu_model()} ({os.cpu_count()} visible)"}

    # ---- the paper's baseline system on the same frames (Sec. 5.3): a map
    # without stored gradients (Eq. (1)-(2) only) tracked with the
    # tri-linear distance (Eq. (12)-(13)); not part of "value"
    comparison = None
    if not args.no_comparison:
        B = GsdfMap(cfg["voxel_size"], cfg["truncation"], max_blocks=max_blocks, storage="nograd")
        start(B, model="trilinear")
        ms_b = timed(lambda: [step(B, f, model="trilinear") for f in range(first, first + K)])
        Eb = est[: first + K].cpu().numpy()
        bstat = B.status_flags()
        bk = {}
        if timing:
            start(B, model="trilinear")
            B.timing(0xffffffff)
            for f in range(first, first + K):
                step(B, f, model="trilinear")
            torch.cuda.synchronize()
            bk = read_kernels(B)
            B.timing(0)
        comparison = {
            "system": "map without stored gradients, tracked with the tri-linear distance of the 8 voxels "
                      "around each point (Eq. 12-13)",
            "frames_per_s": K / (ms_b / 1e3),
            "kernels": bk,
            "ate_rmse_m": float(np.sqrt(np.mean(np.sum((Eb[:, :, 3] - G[:, :, 3]) ** 2, axis=1)))),
            "status": bstat,
        }
        if bk and kernels:
            comparison["track_time_ratio"] = bk["track"]["avg_us"] / kernels["track"]["avg_us"]
            comparison["fusion_gradient_overhead"] = kernels["fuse_blocks"]["avg_us"] / bk["fuse_blocks"]["avg_us"] - 1
        del B

    report = {
        "metric": ("tracked+fused frames/s at 1280x720, 5 mm voxels; % of HBM peak GB/s" if hd else
                   "tracked+fused frames/s at 640x480, 1 cm voxels; % of HBM peak GB/s"),
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else f"{args.storage} storage, f32 compute",
        "data": ("synthetic (seeded room stream at 1280x720)" if hd else
                 "synthetic (seeded room stream standing in for TUM RGB-D 640x480 depth)"),
        "config": {"workload": ("room stream 1280x720, 5 mm voxels, T 2.5 cm" if hd else
                                "room stream 640x480, 1 cm voxels, T 5 cm") + ", 8^3 blocks, 3-level "
                               f"pyramid (4/5/10 GN iterations), {args.storage} voxels",
                   "stream_frames": n_frames, "frames_processed": first + K,
                   "frames_timed": f"{first}-{first + K - 1}", "seeds": list(cfg["seeds"])},
        "hbm_frac": eff_gbs / HBM_PEAK_GBS,
        "effective_gbs": eff_gbs,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fps_with_h2d": h2d,
        "accuracy": {"ate_rmse_m": ate, "status": status},
        "full_stream": full,
        "differentiation": diff,
        "joint_refinement": joint,
        "comparison": comparison,
        "work_per_frame": {"fusion_updates": work[0] / K, "fusion_pixel_visits": work[1] / K,
                           "fused_voxels": work[2] / K, "fused_blocks": work[3] / K,
                           "alloc_pairs": work[4] / K, "track_valid_px_iters": work[5] / K,
                           "track_used_px_iters": work[6] / K},
        "kernels": kernels,
        "track_iterations": iteration_clocks,
    }
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
