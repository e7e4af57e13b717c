#!/usr/bin/env python3
"""Benchmark of the pose-differentiable Gaussian splatting rasterizer on one
MI355X.

Workload (default): single-view pose estimation on a forward-facing synthetic
scene -- 200k Gaussians in a frustum slab at depth 1.5-8, SH degree 3,
1008x756 image, fx = fy = 815, initial pose error 5 deg / 0.1, Adam on the
pose only, FP32.  The scene, camera and target image are synthetic and
seeded (they stand in for the paper's LLFF pose-estimation scenes); the
target is rendered at the ground-truth pose.

A step is one pass of the whole hot path: preprocess, binning, radix sort,
tile ranges, per-tile depth order, forward rasterizer with the L1 loss
gradient in its epilogue (gsp_render_fwd_l1), backward rasterizer,
preprocess-backward with the pose reduction, and the tangent Adam update.
`--steps K` steps of one pose solve are timed with HIP events on the stream
the kernels run on, inputs already resident in HBM.

The JSON line also carries, for the dominant kernel, achieved vs peak
(`roofline`), and the FP64 CPU oracle timed on this host (`cpu_baseline`).

Serving (`serving` in the JSON line, skipped with --no-serve): a resident
1M-Gaussian SH-3 scene (the joint-reconstruction scene) and pose-estimation
requests of mixed sizes {320x240, 640x480, 1008x756}, starting errors
U(1, 5) deg / U(0.02, 0.1), 50 Adam iterations each, targets rendered at the
ground-truth poses.  The sequential rate mu_seq is measured on the first
100 requests solved one at a time, back to back; then, for Poisson arrival
rates of 0.5, 1 and 2 x mu_seq, the same arrival trace of all requests (500
by default) is served live twice: by the sequential server (one request at a
time, first come first served) and with continuous batching; latency =
completion - arrival.  Final poses of the two are compared bit for bit.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpix/s incl. pose grad; pose-solve requests/s + p50/p99 latency"
PEAK_HBM_GBS = 8000.0
# FP32 FMA peak of the unpacked VALU: 256 CU x 64 lanes x 2 flops x 2.4 GHz.
# (The published 157.3 TFLOP/s vector figure needs packed FP32 instructions,
# which this build disables.)
PEAK_FP32_TFLOPS = 78.6
# FP32 flops per (pixel, splat) pair of the compositing formulas (Eq. (3)-(4)
# forward; their adjoint backward), FMA counted as 2.
FWD_FLOPS_EVAL, FWD_FLOPS_BLEND = 19, 7
BWD_FLOPS_EVAL, BWD_FLOPS_BLEND = 16, 49
KERNEL_SOURCES = {
    "raster_fwd": ["raster_fwd.hip", "raster_common.h", "gsp_internal.h"],
    "raster_bwd": ["raster_bwd.hip", "raster_common.h", "gsp_internal.h"],
    "preprocess": ["preprocess.hip"],
    "tile_sort": ["sort.hip"],
    "depth_order": ["sort.hip"],
    "preprocess_bwd": ["preprocess_bwd.hip"],
}


def source_hash(stage):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(stage, []):
        with open(os.path.join(ROOT, "paper_2410_08743_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(stage, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{stage}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != source_hash(stage):
        return None
    return float(m_b.group(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-reps", type=int, default=15)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving measurement and print its JSON (for profiling)")
    ap.add_argument("--joint-only", action="store_true",
                    help="run only the joint-step measurement and print its JSON (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--no-joint", action="store_true", help="skip the joint-step measurement")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-scene measurement")
    ap.add_argument("--no-track", action="store_true", help="skip the tracking measurement")
    ap.add_argument("--no-relpose", action="store_true",
                    help="skip the relative-pose (two-frame) measurement")
    ap.add_argument("--relpose-only", action="store_true",
                    help="run only the relative-pose measurement and print its JSON")
    ap.add_argument("--track-only", action="store_true",
                    help="run only the tracking measurement and print its JSON")
    ap.add_argument("--track-frames", type=int, default=100)
    ap.add_argument("--track-frames-stored", type=int, default=10,
                    help="frames of the tracking run repeated with stored per-pixel lists")
    ap.add_argument("--joint-steps", type=int, default=20)
    ap.add_argument("--serve-rates", type=str, default="0.5,1,2",
                    help="arrival rates as multiples of the sequential rate")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="with --profile-only: also run a device-to-device copy of MIB MiB "
                         "(a plain copy of known size, to scale HBM counters)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed steps only (for rocprofv3), no JSON extras")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the "
              "path runs on one GPU (how it would shard across GPUs is a design note, not code)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_08743_amd import _native as N
    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    torch.cuda.set_device(0)
    dev = "cuda:0"
    if args.serve_only:
        print(json.dumps(serving_section(args, dev, with_cpu=False)), flush=True)
        return
    if args.track_only:
        print(json.dumps(tracking_section(args, dev)), flush=True)
        return
    if args.joint_only:
        print(json.dumps(joint_section(args, dev)), flush=True)
        return
    if args.relpose_only:
        print(json.dumps(relpose_section(args, dev)), flush=True)
        return
    wl = S.single_view()
    cam = wl.camera
    P = cam.width * cam.height
    g = R.GaussianParams.from_set(wl.scene, dev)
    gt = torch.tensor(wl.pose[None], device=dev)
    init = torch.tensor(wl.init_pose[None], device=dev)
    rast = R.Rasterizer(0)
    target = rast.forward(g, [cam], gt)[0].clone()
    print(f"[bench] workload {wl.name}: n={g.n}, {cam.width}x{cam.height}", file=sys.stderr, flush=True)

    # capacity from the starting pose, with room for the poses the solve visits
    rast.forward(g, [cam], init)
    m0, _ = rast.instances()
    rast.capacity = int(1.5 * m0) + 4096
    rast.ws = None
    dl = torch.empty(3 * P, dtype=torch.float32, device=dev)
    K = args.steps

    def new_state():
        return {"pose": init.clone(), "m": torch.zeros((1, 6), device=dev),
                "v": torch.zeros((1, 6), device=dev),
                "st": torch.zeros(1, dtype=torch.int32, device=dev),
                "dpose": torch.zeros((1, 6), device=dev)}

    def step(s, total):
        # render and L1 gradient in one pass (gsp_render_fwd_l1)
        rast.forward_l1(g, [cam], s["pose"], target, grad=dl, check=False)
        # pose-only backward whose final pose reduction applies the Adam step
        # (gsp_render_bwd_pose_step: bit-identical to backward + pose_adam)
        rast.backward_pose_step(g, [cam], s["pose"], dl, s["dpose"], s["m"], s["v"], s["st"],
                                1e-2, 1e-4, total)

    rast._ensure(g, N.view_array([cam]))
    s = new_state()
    for _ in range(args.warmup):
        step(s, max(args.warmup, 1))
    rast.reset_overflow()
    s = new_state()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        step(s, K)
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    M_last, overflow = rast.instances()
    if overflow:
        print("[bench] instance capacity overflowed during the timed solve", file=sys.stderr)
        sys.exit(3)
    ms_step = total_ms / K
    value = P * K / (total_ms * 1e-3) / 1e6
    rot_err, trans_err = S.pose_error(s["pose"][0].cpu().numpy(), wl.pose)
    rot0, trans0 = S.pose_error(wl.init_pose, wl.pose)
    print(f"[bench] {K} steps: {ms_step:.3f} ms/step, {value:.1f} Mpix/s; pose error "
          f"{rot0:.2f} deg/{trans0:.3f} -> {rot_err:.3f} deg/{trans_err:.4f}", file=sys.stderr, flush=True)
    # the 100-step solve of the workload, whatever --steps is
    s100 = new_state()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(100):
        step(s100, 100)
    e1.record()
    torch.cuda.synchronize()
    ms100 = e0.elapsed_time(e1)
    rot100, trans100 = S.pose_error(s100["pose"][0].cpu().numpy(), wl.pose)
    if rast.instances()[1]:
        print("[bench] instance capacity overflowed during the 100-step solve", file=sys.stderr)
        sys.exit(3)
    print(f"[bench] 100-step solve: {ms100:.1f} ms, error {rot0:.2f} deg/{trans0:.3f} -> "
          f"{rot100:.4f} deg/{trans100:.5f}", file=sys.stderr, flush=True)
    if args.profile_only:
        if args.calibrate_copy > 0:
            n = args.calibrate_copy << 18
            src = torch.ones(n, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            print(f"[bench] calibration copy: {args.calibrate_copy} MiB x 3", file=sys.stderr)
        return

    # per-stage timing pass (events bracket each stage on the same stream)
    R.profile_enable(0, R.PROFILE_TIMING)
    s = new_state()
    nprof = min(K, 50)
    for _ in range(nprof):
        step(s, nprof)
    stages = R.profile_read(0)
    R.profile_enable(0, 0)
    stage_ms = {k: ms / c for k, (c, ms) in stages.items()}

    # work counts at the starting pose: evaluated / blended pairs per pixel
    R.profile_enable(0, R.PROFILE_COUNTS)
    s = new_state()
    step(s, 1)
    R.profile_enable(0, 0)
    neval = rast.inspect(g, [cam], "neval", torch.int32).to(torch.int64).sum().item()
    nblend = rast.inspect(g, [cam], "nblend", torch.int32).to(torch.int64).sum().item()
    ncontrib = rast.inspect(g, [cam], "ncontrib", torch.int32).to(torch.int64).sum().item()
    M, _ = rast.instances()
    # lockstep cost: a tile's wave evaluates every pixel up to the tile's
    # largest stop position (forward) / contributor count (backward)
    tw, th = (cam.width + 15) // 16, (cam.height + 15) // 16

    def tile_max_sum(name):
        a = rast.inspect(g, [cam], name, torch.int32).view(cam.height, cam.width).cpu().numpy()
        pad = np.zeros((th * 16, tw * 16), np.int64)
        pad[:cam.height, :cam.width] = a
        return int(256 * pad.reshape(th, 16, tw, 16).max(axis=(1, 3)).sum())

    lockstep = {"fwd_pixel_evals": tile_max_sum("neval"), "bwd_pixel_evals": tile_max_sum("ncontrib")}
    n, S3 = g.n, (g.sh_degree + 1) ** 2
    param_bytes = 4 * (11 + 3 * S3)
    work = {
        "preprocess": ("hbm", (param_bytes + 64) * n),
        "duplicate": ("hbm", 20 * n + 12 * M),
        "tile_sort": ("hbm", 16 * M),
        "ranges": ("hbm", 8 * M + 8 * ((cam.width + 15) // 16) * ((cam.height + 15) // 16)),
        "depth_order": ("hbm", 12 * M),
        "raster_fwd": ("alu", FWD_FLOPS_EVAL * neval + FWD_FLOPS_BLEND * nblend),
        "raster_bwd": ("alu", BWD_FLOPS_EVAL * ncontrib + BWD_FLOPS_BLEND * nblend),
        "preprocess_bwd": ("hbm", (param_bytes - 4) * n + 36 * M + 8 * n),
        "pose_adam": ("hbm", 0),
    }
    stage_report = {}
    for k, ms in stage_ms.items():
        kind, amount = work.get(k, ("hbm", 0))
        if kind == "hbm":
            ach = amount / (ms * 1e-3) / 1e9
            stage_report[k] = {"ms": round(ms, 4), "bound": "hbm", "achieved_GBs": round(ach, 1),
                               "frac": round(ach / PEAK_HBM_GBS, 4)}
        else:
            ach = amount / (ms * 1e-3) / 1e12
            stage_report[k] = {"ms": round(ms, 4), "bound": "alu", "achieved_TFLOPs": round(ach, 2),
                               "frac": round(ach / PEAK_FP32_TFLOPS, 4)}
    dominant = max(stage_ms, key=stage_ms.get)
    kind, amount = work[dominant]
    dms = stage_ms[dominant]
    if kind == "alu":
        ach = amount / (dms * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "alu", "achieved": round(ach, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4)}
    else:
        ach = amount / (dms * 1e-3) / 1e9
        roof = {"kernel": dominant, "bound": "hbm", "achieved": round(ach, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4)}
    roof["avg_launch_ms"] = round(dms, 4)
    roof["algorithmic_per_launch"] = amount
    roof["traffic"] = traffic_from_profiles(dominant, "pose-200k-1008x756")
    if kind == "alu":
        roof["peak_note"] = ("unpacked FP32 FMA rate, 256 CU x 64 lanes x 2 flops x 2.4 GHz; the "
                             "published 157.3 TFLOP/s counts packed FP32 instructions, which this "
                             "build disables")
        roof["frac_of_published_157_3"] = round(ach / 157.3, 4)
    # roofline-bound time of the whole step: each stage at its own bound
    t_roof = 0.0
    for k, ms in stage_ms.items():
        kind_k, amt = work.get(k, ("hbm", 0))
        t_roof += amt / (PEAK_FP32_TFLOPS * 1e12) if kind_k == "alu" else amt / (PEAK_HBM_GBS * 1e9)
    step_roof = {"t_roof_ms": round(t_roof * 1e3, 4),
                 "rate_at_roof_mpix_s": round(P / t_roof / 1e6, 1) if t_roof > 0 else None,
                 "frac": round(t_roof * 1e3 / ms_step, 4)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, wl)

    tiny = None
    if not args.no_tiny:
        tiny = tiny_section(args, dev)
    joint = None
    if not args.no_joint:
        joint = joint_section(args, dev)
    track = None
    if not args.no_track:
        track = tracking_section(args, dev)
    relpose = None
    if not args.no_relpose:
        relpose = relpose_section(args, dev)
    hypotheses = multi_hypothesis_section(g, cam, target, wl, dev)
    serving = None
    if not args.no_serve:
        serving = serving_section(args, dev, with_cpu=not args.no_cpu)

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": g.n, "sh_degree": g.sh_degree,
                   "width": cam.width, "height": cam.height, "views_per_step": 1,
                   "step": "fwd+L1+bwd(pose)+adam", "parallelism": "single GPU"},
        "roofline": roof,
        "step_roofline": step_roof,
        "cpu_baseline": cpu,
        "tiny": tiny,
        "joint": joint,
        "tracking": track,
        "relative_pose": relpose,
        "multi_hypothesis": hypotheses,
        "serving": serving,
        "stages": stage_report,
        "work": {"instances": M, "evaluated_pairs": neval, "blended_pairs": nblend,
                 "backward_pairs": ncontrib, **lockstep},
        "pose_solve": {"steps": 100, "seconds": round(ms100 * 1e-3, 4),
                       "initial_error": [round(rot0, 3), round(trans0, 4)],
                       "final_error": [round(rot100, 4), round(trans100, 5)],
                       "timed_steps_final_error": [round(rot_err, 4), round(trans_err, 5)]},
    }
    print(json.dumps(line), flush=True)


def multi_hypothesis_section(g, cam, target, wl, dev):
    """Eight starting poses of the benchmark image solved at once (100
    steps, the hypotheses are the views of each launch), in SE(3) and in
    T x SO(3): the given start (5 deg / 0.1 off) and seven more, 10 deg /
    0.2 off in random directions; the best final loss picks the answer."""
    import numpy as np
    import torch

    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    rng = S.rng_for(1002, 9)
    inits = [wl.init_pose.astype(np.float64)] + [S.perturb_pose(wl.pose, 10.0, 0.2, rng)
                                                 for _ in range(7)]
    inits = torch.tensor(np.stack(inits).astype(np.float32), device=dev)
    out = {"hypotheses": 8, "steps": 100}
    for param in ("se3", "t_so3"):
        R.solve_multi_hypothesis(g, cam, target, inits, steps=10, parametrization=param)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, idx, losses, _ = R.solve_multi_hypothesis(g, cam, target, inits, steps=100,
                                                        parametrization=param)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        e = S.pose_error(best.cpu().numpy(), wl.pose)
        out[param] = {"ms": round(ms, 1), "best": idx, "final_error": [round(e[0], 4), round(e[1], 5)]}
    print(f"[bench] multi-hypothesis (8 starts, 100 steps): se3 {out['se3']['ms']} ms, "
          f"t_so3 {out['t_so3']['ms']} ms, errors {out['se3']['final_error']} / "
          f"{out['t_so3']['final_error']}", file=sys.stderr, flush=True)
    return out


def cpu_baseline(args, wl):
    """The FP64 CPU oracle timed on this host (a baseline, not the target):
    one forward render + one backward (every Gaussian gradient and the pose
    twist) of a seeded random upstream gradient.  `value` is the benchmark
    view (200k Gaussians, 1008x756) on all of the oracle's OpenMP threads;
    the same view on one thread, the tiny workload (1k Gaussians, 128x128)
    on all threads and on one, and one frame of the tracking room (500k
    Gaussians, 1200x680) on all threads are reported beside it.  Median of
    `cpu_reps` runs (of 3 for the room frame, 1 for the single-threaded
    benchmark view)."""
    import numpy as np

    import oracle
    from paper_2410_08743_amd import synthetic as S

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = oracle.max_threads()

    def timed(scene, cam, pose, reps, seed):
        h, w = cam.region()[3], cam.region()[2]
        up = S.upstream(seed, (3, h, w))
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.render(scene, cam, pose)
            oracle.backward(scene, cam, pose, up)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        return {"mpix_per_s": round(h * w / t / 1e6, 4), "seconds": round(t, 3), "runs": reps}

    cam = wl.camera
    main = timed(wl.scene, cam, wl.init_pose, args.cpu_reps, 111)
    tiny = S.tiny()
    out = {"value": main["mpix_per_s"], "unit": "Mpix/s", "cores": threads, "kind": "oracle",
           "sample": f"one fwd render + one bwd (pose and every Gaussian gradient, seeded random "
                     f"upstream gradient) of the full {cam.width}x{cam.height} view of the "
                     f"200k-Gaussian scene at the starting pose, FP64, median of {args.cpu_reps}",
           "seconds": main["seconds"], "cpu_model": model,
           "tiny_1k_128x128": timed(tiny.scene, tiny.camera, tiny.pose, 5, 112)}
    room = S.room(n_frames=61)
    out["room_500k_1200x680_frame"] = timed(room.scene, room.camera,
                                            room.extra["trajectory"][60], 3, 113)
    oracle.set_threads(1)
    try:
        out["single_thread"] = {
            "benchmark_view": timed(wl.scene, cam, wl.init_pose, 1, 111),
            "tiny_1k_128x128": timed(tiny.scene, tiny.camera, tiny.pose, 3, 112)}
    finally:
        oracle.set_threads(threads)
    print(f"[bench] cpu oracle ({model}, {threads} threads): {main['mpix_per_s']} Mpix/s; one "
          f"thread {out['single_thread']['benchmark_view']['mpix_per_s']} Mpix/s",
          file=sys.stderr, flush=True)
    return out


def tiny_section(args, dev):
    """The tiny correctness workload (1000 Gaussians, SH 0, 128x128): forward,
    L1 against the target pose's render, backward to every Gaussian
    parameter and the pose, Adam -- once with one view per launch (launch
    latency bound) and once with 32 copies of the view in one launch, each
    launched eagerly and as a replayed HIP graph of one step."""
    import numpy as np
    import torch

    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    wl = S.tiny()
    cam = wl.camera
    g = R.GaussianParams.from_set(wl.scene, dev)
    P = cam.width * cam.height
    out = {"workload": wl.name, "gaussians": g.n, "step": "fwd+L1+bwd(all params + pose)+adam"}
    for V in (1, 32):
        cams = [cam] * V
        rast = R.Rasterizer(0)
        tgt, _ = rast.forward(g, cams, torch.tensor(np.repeat(wl.init_pose[None], V, 0), device=dev))
        tgt = tgt.clone()
        pose = torch.tensor(np.repeat(wl.pose[None], V, 0), device=dev)
        m = torch.zeros((V, 6), device=dev)
        v = torch.zeros((V, 6), device=dev)
        st = torch.zeros(V, dtype=torch.int32, device=dev)
        img = torch.empty(3 * P * V, device=dev)
        dl = torch.empty_like(img)
        grads = {k: torch.empty(sh, device=dev) for k, sh in
                 (("means", (g.n, 3)), ("scales", (g.n, 3)), ("quats", (g.n, 4)),
                  ("opacities", (g.n,)), ("sh", tuple(g.sh.shape)))}
        grads["pose"] = torch.empty((V, 6), device=dev)
        rast.forward(g, cams, pose, images=img)
        rast.capacity = int(1.5 * rast.instances()[0]) + 1024
        rast.ws = None
        rast._ensure(g, R.N.view_array(cams))

        def step():
            rast.forward(g, cams, pose, check=False, images=img)
            R.loss_l1(cams, img, tgt, grad=dl, with_loss=False)
            rast.backward(g, cams, pose, dl, out=grads)
            R.pose_adam(pose, grads["pose"], m, v, st, 1e-2, 1e-4, 1000, guard=rast.ws)

        for _ in range(10):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        K = 200
        e0.record()
        for _ in range(K):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg, stream=side):
            step()
        for _ in range(10):
            cg.replay()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            cg.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_g = e0.elapsed_time(e1) / K
        out[f"views_{V}"] = {"ms_per_step": round(ms, 4), "mpix_per_s": round(V * P / (ms * 1e3), 2),
                             "graph_ms_per_step": round(ms_g, 4)}
    print(f"[bench] tiny: {out['views_1']['ms_per_step']:.3f} ms/step (1 view; graph "
          f"{out['views_1']['graph_ms_per_step']:.3f}), {out['views_32']['ms_per_step']:.3f} "
          f"ms/step (32 views, {out['views_32']['mpix_per_s']:.0f} Mpix/s; graph "
          f"{out['views_32']['graph_ms_per_step']:.3f})", file=sys.stderr, flush=True)
    return out


_JOINT = None


def joint_scene():
    global _JOINT
    if _JOINT is None:
        from paper_2410_08743_amd import synthetic as S
        _JOINT = S.joint()
    return _JOINT


def joint_section(args, dev):
    """Joint reconstruction and pose refinement step (Sec. III-C) at one GPU's
    share: 1M Gaussians (SH 3), 4 of the 20 arc views (1008x756) per step:
    forward, L_RGB = 0.8 L1 + 0.2 DSSIM with its gradient, backward to every
    Gaussian parameter and the 4 pose twists, Adam on the raw Gaussian
    parameters with the anisotropy hinge (r = 10), pose Adam.  The optimised
    scene is the ground-truth scene with mu += N(0, 0.01^2),
    log s += N(0, 0.1^2) and resampled colours; targets are rendered from the
    ground truth at the ground-truth poses; the views are visited in a fixed
    random order, four at a time."""
    import numpy as np
    import torch

    from paper_2410_08743_amd import joint as J
    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    wl = joint_scene()
    cam = wl.camera
    gt = R.GaussianParams.from_set(wl.scene, dev)
    rng = S.rng_for(1003, 5)
    sc = wl.scene
    noisy = S.GaussianSet((sc.means + rng.normal(0, 0.01, sc.means.shape)).astype(np.float32),
                          (sc.scales * np.exp(rng.normal(0, 0.1, sc.scales.shape))).astype(np.float32),
                          sc.quats, sc.opacities, S.colour_sh(rng, sc.n, 3), 3)
    V = 4
    nv = wl.extra["gt_poses"].shape[0]
    order = S.rng_for(1003, 6).permutation(nv)
    rast = R.Rasterizer(0)
    targets = []
    for k in range(nv):
        t, _ = rast.forward(gt, [cam], torch.tensor(wl.extra["gt_poses"][k:k + 1], device=dev))
        targets.append(t.clone().view(3, cam.height, cam.width))
    del rast
    raw = J.RawGaussians.from_set(noisy, dev)
    K = args.joint_steps
    ref = J.JointRefiner(raw, [cam] * nv, targets, torch.tensor(wl.extra["noisy_poses"], device=dev),
                         total_steps=3 + K, views_per_step=V, order=order)
    P = cam.width * cam.height
    for _ in range(3):
        ref.step()
    ref.rast.reset_overflow()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        ref.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    M, ovf = ref.rast.instances()
    if ovf:
        print("[bench] joint step overflowed its instance capacity", file=sys.stderr)
        return None
    # per-stage split from the library's own events, in a separate pass
    R.profile_enable(0, R.PROFILE_TIMING)
    R.profile_read(0)
    for _ in range(5):
        ref.step()
    stages = {k: round(ms_ / 5, 4) for k, (c, ms_) in R.profile_read(0).items()}
    R.profile_enable(0, 0)
    print(f"[bench] joint step: {ms:.3f} ms for {V} views ({V * P / (ms * 1e3):.1f} Mpix/s) {stages}",
          file=sys.stderr, flush=True)
    # work counters of one step (the forward's per-pixel evaluated and
    # blended pairs, the contributor counts, the instances)
    R.profile_enable(0, R.PROFILE_COUNTS)
    a, b = ref.batches[ref.k % len(ref.batches)]
    ref.step()
    R.profile_enable(0, 0)
    cams = ref.cams[a:b]
    cnt = lambda name: int(ref.rast.inspect(ref.g, cams, name, torch.int32).to(torch.int64).sum().item())
    neval, nblend, ncontrib = cnt("neval"), cnt("nblend"), cnt("ncontrib")
    Mj, _ = ref.rast.instances()
    n, S3 = raw.n, 16
    pb = 4 * (11 + 3 * S3)
    tiles = V * ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    work = {
        "preprocess": ("hbm", pb * n + 64 * V * n),
        "duplicate": ("hbm", 20 * V * n + 12 * Mj),
        "tile_sort": ("hbm", 16 * Mj),
        "ranges": ("hbm", 8 * Mj + 8 * tiles),
        "depth_order": ("hbm", 12 * Mj),
        "raster_fwd": ("alu", FWD_FLOPS_EVAL * neval + FWD_FLOPS_BLEND * nblend),
        "loss_rgb": ("hbm", 44 * 3 * P * V),
        "raster_bwd": ("alu", BWD_FLOPS_EVAL * ncontrib + BWD_FLOPS_BLEND * nblend),
        "preprocess_bwd": ("hbm", (pb - 4) * n + 36 * Mj + 8 * V * n + pb * n),
        "gaussian_adam": ("hbm", 28 * (pb // 4) * n + 16 * n),
        "pose_adam": ("hbm", 0),
    }
    report, t_roof = roofline_table(stages, work)
    dominant = max(stages, key=stages.get)
    return {"workload": "joint-1M-4x1008x756-sh3", "gaussians": raw.n, "views_per_step": V,
            "steps": K, "ms_per_step": round(ms, 4), "mpix_per_s": round(V * P / (ms * 1e3), 2),
            "instances": M, "stages": report,
            "work": {"instances": Mj, "evaluated_pairs": neval, "blended_pairs": nblend,
                     "backward_pairs": ncontrib},
            "roofline": {"kernel": dominant, **report[dominant]},
            "step_roofline": {"t_roof_ms": round(t_roof * 1e3, 4),
                              "rate_at_roof_mpix_s": round(V * P / t_roof / 1e6, 1),
                              "frac": round(t_roof * 1e3 / ms, 4)},
            "step": "fwd + (0.8 L1 + 0.2 DSSIM) + bwd(all Gaussian params + 4 poses) "
                    "+ Gaussian Adam with L_An + pose Adam"}


def roofline_table(stage_ms, work):
    """Per stage: achieved rate of its algorithmic work (bytes for HBM-bound
    stages, flops for ALU-bound ones) against its peak; and the roofline-
    bound time of all stages, each at its own bound (seconds)."""
    report, t_roof = {}, 0.0
    for k, ms in stage_ms.items():
        kind, amount = work.get(k, ("hbm", 0))
        if kind == "hbm":
            ach = amount / (ms * 1e-3) / 1e9
            report[k] = {"ms": round(ms, 4), "bound": "hbm", "achieved": round(ach, 1),
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4)}
            t_roof += amount / (PEAK_HBM_GBS * 1e9)
        else:
            ach = amount / (ms * 1e-3) / 1e12
            report[k] = {"ms": round(ms, 4), "bound": "alu", "achieved": round(ach, 2),
                         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(ach / PEAK_FP32_TFLOPS, 4)}
            t_roof += amount / (PEAK_FP32_TFLOPS * 1e12)
    return report, t_roof


def relpose_section(args, dev):
    """Relative pose between two consecutive frames (Sec. III-D) on the
    tracking room (500k Gaussians, SH 3, 1200x680): frames 60 and 61 of its
    trajectory; frame 60's depth map is the expected-depth render of the
    scene (the stand-in for a monocular estimate).  Timed, at the settings
    of Sec. IV: unprojection of every 4th pixel (51k points, the paper's
    50 000 per frame) with its three-nearest-neighbour scales, 100 fitting
    steps of the frame's scene (L_RGB, Gaussian Adam), 200 masked-L1 pose
    steps at 1e-3 -> 1e-4."""
    import numpy as np
    import torch

    from paper_2410_08743_amd import joint as J
    from paper_2410_08743_amd import relpose as RP
    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    wl = S.room(n_frames=63)
    cam = wl.camera
    g = R.GaussianParams.from_set(wl.scene, dev)
    traj = wl.extra["trajectory"]
    P0, P1 = traj[60].astype(np.float64), traj[61].astype(np.float64)
    rast = R.Rasterizer(0)
    t0 = torch.tensor(P0[None].astype(np.float32), device=dev)
    i0 = rast.forward(g, [cam], t0)[0].clone().view(3, cam.height, cam.width)
    i1 = rast.forward(g, [cam], torch.tensor(P1[None].astype(np.float32), device=dev))[0].clone()
    gz = R.GaussianParams.from_set(S.depth_coloured(wl.scene, P0), dev)
    dimg, al = R.Rasterizer(0).forward(gz, [cam], t0, alphas=True)
    depth = (dimg.view(3, cam.height, cam.width)[0] /
             al.view(cam.height, cam.width).clamp_min(1e-6)).contiguous()
    del rast, gz

    def run():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        raw = RP.unproject(cam, depth, i0, 4)
        ev[1].record()
        ref = J.JointRefiner(raw, [cam], [i0], RP.identity_poses(1, dev), 100, hp=RP.FIT_HYPER,
                             optimize_poses=False)
        for _ in range(100):
            ref.step()
        ev[2].record()
        pose = R.solve_poses(ref.g, [cam], i1.reshape(-1), RP.identity_poses(1, dev), steps=200,
                             lr=(1e-3, 1e-4), masked=True)
        ev[3].record()
        torch.cuda.synchronize()
        return raw.n, pose[0], [ev[k].elapsed_time(ev[k + 1]) for k in range(3)]

    run()                                     # warm-up (allocations, first launches)
    n, pose, (t_un, t_fit, t_pose) = run()
    H0 = np.vstack([P0, [0, 0, 0, 1]])
    H1 = np.vstack([P1, [0, 0, 0, 1]])
    gt = (H1 @ np.linalg.inv(H0))[:3]
    e0 = S.pose_error(np.hstack([np.eye(3), np.zeros((3, 1))]), gt)
    e1 = S.pose_error(pose.cpu().numpy(), gt)
    total = t_un + t_fit + t_pose
    print(f"[bench] relative pose: {n} Gaussians, unproject {t_un:.2f} ms, fit {t_fit:.1f} ms, "
          f"pose {t_pose:.1f} ms, error {e0[0]:.3f} deg / {e0[1]:.4f} -> {e1[0]:.4f} deg / "
          f"{e1[1]:.5f}", file=sys.stderr, flush=True)
    return {"workload": "relpose-room-1200x680-frames-60-61", "gaussians": n, "stride": 4,
            "unproject_ms": round(t_un, 3), "fit_ms_100_steps": round(t_fit, 2),
            "pose_ms_200_steps": round(t_pose, 2), "frame_pair_ms": round(total, 2),
            "initial_error": [round(e0[0], 4), round(e0[1], 5)],
            "final_error": [round(e1[0], 4), round(e1[1], 5)]}


def tracking_section(args, dev):
    """Sequential tracking through the torch.autograd.Function: the 500k-
    Gaussian room (SH 3), 1200x680, each frame starting from the previous
    frame's estimate (frame 0 from the ground truth turned by 1 deg and moved
    by 0.02) and running 50 pose-only Adam iterations on the L1 loss; the
    render and its backward are the library's, the loss and its gradient are
    torch's autograd.  The whole trajectory runs with the recomputing
    backward; then its first frames run again with stored per-pixel lists
    (GSP_STORE_LISTS: 12 B per blended pair).  For both, the peak HBM above
    what the scene and the target images hold is measured
    (torch.cuda.max_memory_allocated), as are the time per iteration and
    the pose errors."""
    import numpy as np
    import torch

    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import synthetic as S

    wl = S.room(n_frames=args.track_frames)
    cam = wl.camera
    traj = wl.extra["trajectory"]
    g = R.GaussianParams.from_set(wl.scene, dev)
    rast = R.Rasterizer(0)
    targets = []
    m0 = 0
    for k in range(len(traj)):
        t, _ = rast.forward(g, [cam], torch.tensor(traj[k:k + 1], device=dev))
        targets.append(t.clone())
        m0 = max(m0, rast.instances()[0])
    del rast
    iters = 50
    P = cam.width * cam.height
    start = S.perturb_pose(traj[0], 1.0, 0.02, S.rng_for(1004, 2))[None].astype(np.float32)

    def track(frames, store):
        rast = R.Rasterizer(0, capacity=int(1.5 * m0) + 4096, store_lists=store)
        pose = torch.tensor(start, device=dev)
        rast.forward(g, [cam], pose)             # sizes the buffers (and the pair capacity)
        if store:
            rast.pair_capacity = int(1.5 * rast.list_pairs()[0]) + 4096
            rast.lists = None
            rast.forward(g, [cam], pose)
        rast.reset_overflow()
        errs, pairs = [], 0
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        for k in range(frames):
            m = torch.zeros((1, 6), device=dev)
            v = torch.zeros((1, 6), device=dev)
            st = torch.zeros(1, dtype=torch.int32, device=dev)
            for _ in range(iters):
                tau = torch.zeros((1, 6), device=dev, requires_grad=True)
                img = R.render(g, [cam], pose, tau=tau, rast=rast, check=False)
                loss = (img - targets[k]).abs().mean()
                loss.backward()
                R.pose_adam(pose, tau.grad, m, v, st, 1e-2, 1e-4, iters, guard=rast.ws)
            errs.append(S.pose_error(pose[0].cpu().numpy(), traj[k]))
            if store:
                pairs = max(pairs, rast.list_pairs()[0])
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        peak = torch.cuda.max_memory_allocated()
        if rast.overflowed():
            return None
        ws = rast.ws.numel()
        lists = rast.lists.numel() if store else 0
        # the pose estimates feed the next frames: the stored run ends at
        # the recomputing run's errors up to FP32 rounding
        return {"seconds": sec, "ms_per_iteration": 1e3 * sec / (frames * iters),
                "errors": np.array(errs), "peak_above_scene_and_targets": int(peak - base),
                "peak_hbm_bytes": int(peak), "workspace_bytes": int(ws), "list_bytes": int(lists),
                "max_pairs": int(pairs)}

    rec = track(len(traj), False)
    if rec is None:
        print("[bench] tracking overflowed its instance capacity", file=sys.stderr)
        return None
    nst = min(args.track_frames_stored, len(traj))
    sto = track(nst, True)
    e = rec["errors"]
    sec = rec["seconds"]
    n_it = len(traj) * iters
    print(f"[bench] tracking: {len(traj)} frames x {iters} iterations in {sec:.2f} s "
          f"({rec['ms_per_iteration']:.3f} ms/iteration); median error {np.median(e[:, 0]):.3f} deg / "
          f"{np.median(e[:, 1]):.4f}; state above scene+targets {rec['peak_above_scene_and_targets'] / 1e9:.3f} GB",
          file=sys.stderr, flush=True)
    out = {"workload": wl.name, "gaussians": g.n, "frames": len(traj),
           "iterations_per_frame": iters, "seconds": round(sec, 3),
           "ms_per_iteration": round(rec["ms_per_iteration"], 4),
           "mpix_per_s": round(P * n_it / sec / 1e6, 2),
           "error_deg_median": round(float(np.median(e[:, 0])), 4),
           "error_deg_max": round(float(np.max(e[:, 0])), 4),
           "error_trans_median": round(float(np.median(e[:, 1])), 5),
           "error_trans_max": round(float(np.max(e[:, 1])), 5),
           "peak_hbm_bytes_recompute": rec["peak_hbm_bytes"],
           "state_bytes_recompute": rec["peak_above_scene_and_targets"],
           "workspace_bytes_recompute": rec["workspace_bytes"],
           "per_pixel_state_bytes_recompute": 8 * P,
           "note": "loss and its gradient in torch autograd; render, backward and Adam in the library"}
    if sto is not None:
        es = sto["errors"]
        same = float(np.max(np.abs(es - e[:nst])))
        print(f"[bench] tracking, stored lists: {nst} frames, {sto['ms_per_iteration']:.3f} ms/iteration, "
              f"state above scene+targets {sto['peak_above_scene_and_targets'] / 1e9:.3f} GB "
              f"(lists {sto['list_bytes'] / 1e9:.3f} GB, {sto['max_pairs']} pairs); "
              f"max |error difference| to the recomputing run {same:.2e}", file=sys.stderr, flush=True)
        out["stored_lists"] = {
            "frames": nst, "ms_per_iteration": round(sto["ms_per_iteration"], 4),
            "peak_hbm_bytes": sto["peak_hbm_bytes"],
            "state_bytes": sto["peak_above_scene_and_targets"],
            "list_bytes": sto["list_bytes"], "max_pairs_per_frame": sto["max_pairs"],
            "max_abs_error_difference_to_recompute": same,
            "ms_per_iteration_recompute_same_frames": round(
                1e3 * rec["seconds"] / n_it, 4)}
    return out


def serving_section(args, dev, with_cpu=True):
    import numpy as np
    import torch

    from paper_2410_08743_amd import render as R
    from paper_2410_08743_amd import serve as SV
    from paper_2410_08743_amd import synthetic as S

    iters = 50
    wl = joint_scene()
    g = R.GaussianParams.from_set(wl.scene, dev)
    specs = S.serving_requests(n_requests=args.serve_requests)
    rast = R.Rasterizer(0)
    reqs = []
    for sp in specs:
        cam = sp["camera"]
        tgt, _ = rast.forward(g, [cam], torch.tensor(sp["gt_pose"][None], device=dev))
        reqs.append(SV.PoseRequest(cam, tgt.clone().view(3, cam.height, cam.width),
                                   torch.tensor(sp["init_pose"], device=dev), 0.0, sp["rid"]))
    del rast
    torch.cuda.synchronize()
    print(f"[bench] serving: {g.n} Gaussians resident, {len(reqs)} requests", file=sys.stderr,
          flush=True)

    # sequential rate: one request at a time, back to back, on the first
    # requests of the trace
    seq_srv = SV.PoseServer(g, iters=iters, max_batch=1)
    seq_srv.run(reqs[:2])            # warm-up (calibration, allocations)
    n_cal = min(len(reqs), 100)
    cal = seq_srv.run(reqs[:n_cal])
    mu_seq = n_cal / cal[-1].completed
    print(f"[bench] sequential: {mu_seq:.2f} requests/s back to back", file=sys.stderr, flush=True)

    def errors(results):
        e = np.array([S.pose_error(r.pose, sp["gt_pose"]) for r, sp in zip(results, specs)])
        e0 = np.array([S.pose_error(sp["init_pose"], sp["gt_pose"]) for sp in specs])
        return {"rot_deg_p50": float(np.percentile(e[:, 0], 50)),
                "rot_deg_p99": float(np.percentile(e[:, 0], 99)),
                "trans_p50": float(np.percentile(e[:, 1], 50)),
                "trans_p99": float(np.percentile(e[:, 1], 99)),
                "initial_rot_deg_p50": float(np.percentile(e0[:, 0], 50)),
                "initial_trans_p50": float(np.percentile(e0[:, 1], 50))}

    def stats(res):
        st = SV.latency_stats(res)
        return {"requests_per_s": round(st["requests_per_s"], 3),
                "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
                "mean_batch": round(st["mean_batch"], 2)}

    gaps = np.array([sp["gap"] for sp in specs])
    rates = []
    srv = SV.PoseServer(g, iters=iters)
    srv.run(reqs[:4])                # warm-up
    seq_final = None
    for rel in [float(x) for x in args.serve_rates.split(",")]:
        lam = rel * mu_seq
        arr = np.cumsum(gaps) / lam
        arr -= arr[0]
        trace = [SV.PoseRequest(r.camera, r.target, r.init_pose, float(a), r.rid)
                 for r, a in zip(reqs, arr)]
        # both servers live on the same arrival trace
        seq = seq_srv.run(trace)
        batched = srv.run(trace)
        sb, ss = stats(batched), stats(seq)
        same = sum(bool(np.array_equal(a.pose, b.pose)) for a, b in zip(batched, seq))
        seq_final = seq
        rates.append({
            "arrival_rate_rel": rel, "arrival_rate": round(lam, 3),
            "batched": sb, "sequential": ss,
            "batched_final_error": errors(batched), "sequential_final_error": errors(seq),
            "identical_final_poses": f"{same}/{len(batched)}",
        })
        print(f"[bench] rate {rel} x mu_seq ({len(trace)} requests): batched {sb['requests_per_s']:.2f} "
              f"req/s p50 {sb['p50_ms']:.1f} ms p99 {sb['p99_ms']:.1f} ms (mean batch "
              f"{sb['mean_batch']:.1f}); sequential {ss['requests_per_s']:.2f} req/s p50 "
              f"{ss['p50_ms']:.1f} ms p99 {ss['p99_ms']:.1f} ms; identical {same}/{len(batched)}",
              file=sys.stderr, flush=True)

    out = {
        "workload": "serve-1M-sh3-mixed-320x240-640x480-1008x756",
        "gaussians": g.n, "requests": len(reqs), "iterations_per_request": iters,
        "sequential_requests_per_s_back_to_back": round(mu_seq, 3),
        "rates": rates,
        "final_error": errors(seq_final),
    }
    if with_cpu:
        import oracle
        per_size = {}
        for sp in specs:
            cam = sp["camera"]
            key = f"{cam.width}x{cam.height}"
            if key in per_size:
                continue
            t0 = time.perf_counter()
            oracle.render(wl.scene, cam, sp["init_pose"])
            oracle.backward(wl.scene, cam, sp["init_pose"],
                            np.zeros((3, cam.height, cam.width)))
            per_size[key] = round(iters * (time.perf_counter() - t0), 2)
        out["cpu_oracle_seconds_per_request"] = per_size
        out["cpu_oracle_cores"] = oracle.max_threads()
    return out


if __name__ == "__main__":
    main()
