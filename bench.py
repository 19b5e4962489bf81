"""Benchmark of the low-resolution 3DGS rasterizer with image gradients on one
MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c2_1080|c3_540|c3_1080]

A step is one whole forward frame: projection, depth sort, key emission, tile
sort, tile ranges and compositing with the Eq. 3-4 gradient buffers, on a
synthetic scene resident in HBM.  The default workload is 1M Gaussians in 64
anisotropic clusters (SH degree 3) at 960x540.  Prints one JSON line.

Roofline of the dominant stage: compositing is FP32-VALU bound; its
algorithmic work is 16 FLOP per evaluated (Gaussian, pixel) pair plus 44 FLOP
per blended pair, with the pair counts taken from the kernel's counting
variant on the same frame (identical to the oracle's away from threshold
ties).  Projection and sorting are HBM bound; their algorithmic bytes are
given per stage in the "stages" object.  The CPU baseline is the FP64 oracle
timed on this host on a bounded sample of the same frame.
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

METRIC = "Gaussian-pixel blends/s and frames/s at 960x540, 1M splats; p50/p99 latency"
PEAK_FP32 = 157.3e12      # MI355X vector FP32 (packed FMA), FLOP/s
PEAK_HBM = 8.0e12         # MI355X HBM3E, B/s
FLOP_EVAL = 16
FLOP_BLEND = 44


def workload(name):
    import synth
    if name == "c1":
        s, cam = synth.gen_cfg1()
        desc = "10k Gaussians uniform in [-1,1]^2x[2,6], SH deg 0, 256x256, forward + image gradients"
    elif name == "c2":
        s, cam = synth.gen_cfg2()
        desc = ("1M Gaussians in 64 anisotropic clusters, SH deg 3, 960x540, 16x16 tiles, "
                "forward + dC/dx, dC/dy + depth")
    elif name == "c2_1080":
        s, _ = synth.gen_cfg2()
        cam = synth.cfg2_camera(1920, 1080)
        desc = ("1M Gaussians in 64 anisotropic clusters, SH deg 3, 1920x1080, 16x16 tiles, "
                "forward + dC/dx, dC/dy + depth")
    elif name in ("c3_540", "c3_1080"):
        s, poses = synth.gen_cfg3()
        W, H = (960, 540) if name == "c3_540" else (1920, 1080)
        cam = synth.look_at_camera(poses[0], W, H)
        desc = f"6M Gaussians in 64 anisotropic clusters, SH deg 3, {W}x{H}, pose 0 of 60, forward + gradients"
    else:
        raise SystemExit(f"unknown workload {name}")
    return s, cam, desc


def stage_bytes(n_flat, n_real, sh_deg, keys, tiles, depth_passes=3, tile_passes=1):
    """Algorithmic HBM bytes per stage of one frame.
    project: per visible Gaussian its parameters (44 + 12 (deg+1)^2 B) in,
    the 48-B record, depth key, packed rectangle and tile count (60 B) out.
    depth sort: per flat Gaussian and pass the key read by the histogram, the
    key and value read and written by the scatter (20 B); the last pass also
    gathers and writes the packed rectangle (+8 B).
    emit: per flat Gaussian the rectangle read twice (chunk counts, emission)
    and its index (12 B); per pair the 16-bit tile id and the Gaussian index
    written (6 B).
    tile sort: one pass reads the 16-bit tile id twice and the index once and
    writes the index (12 B per pair) plus the tile ranges; more passes (32-bit
    global tile ids) move key and value per pass (20 B) and a boundary scan
    reads the tile ids (4 B)."""
    k = (sh_deg + 1) ** 2
    proj = n_real * (44 + 12 * k + 60)
    dsort = n_flat * (depth_passes * 20 + 8)
    emit = n_flat * 12 + keys * 6
    if tile_passes == 1:
        tsort = keys * 12 + tiles * 8
    else:
        tsort = keys * (20 * tile_passes + 4) + tiles * 8
    return dict(project=proj, depth_sort=dsort, emit=emit, tile_sort=tsort)


def _oracle_frame_legs(scene, cam, sample_tiles, workers):
    """One frame of the oracle: projection and binning (one process), then
    the compositing of `sample_tiles` random tiles in one process and of
    every tile over `workers` processes.  Blended pairs are the oracle's own
    count."""
    import oracle
    from oracle import binning, composite, parallel
    t0 = time.perf_counter()
    proj = oracle.project.project(scene, cam)
    t1 = time.perf_counter()
    _, vals, ranges = binning.bin_and_sort(proj)
    t2 = time.perf_counter()
    n_tiles = ranges.shape[0]
    W, H = int(cam.width), int(cam.height)
    res = {"project_s": t1 - t0, "binning_s": t2 - t1, "tiles": int(n_tiles)}
    if sample_tiles:
        rng = np.random.default_rng(0)
        tiles = (np.arange(n_tiles) if sample_tiles >= n_tiles
                 else rng.choice(n_tiles, size=sample_tiles, replace=False))
        blended = 0
        t3 = time.perf_counter()
        for t in tiles:
            blended += int(composite.composite_tile(proj, vals, ranges, int(t), W, H, np.zeros(3),
                                                    track=False).blended.sum())
        t4 = time.perf_counter()
        scale = n_tiles / len(tiles)
        res["single"] = {"composite_s": (t4 - t3) * scale, "sampled_tiles": int(len(tiles)),
                         "blended_pairs": int(round(blended * scale)),
                         "seconds_per_frame": (t2 - t0) + (t4 - t3) * scale}
    if workers:
        tm = {}
        img = parallel.composite_image_parallel(proj, vals, ranges, W, H, np.zeros(3), track=False,
                                                workers=workers, timing=tm)
        res["pool"] = {"composite_s": tm["composite_s"], "pool_start_s": tm["pool_start_s"],
                       "workers": tm["workers"], "blended_pairs": int(img.blended.sum()),
                       "seconds_per_frame": (t2 - t0) + tm["composite_s"]}
    return res


def cpu_baseline(workload_name, sample_tiles=600):
    """The FP64 oracle (plain NumPy, never tuned) timed on this host: the
    benchmark's frame with every tile composited over a process pool using
    all cores (the reported value), the same frame in one process with
    `sample_tiles` tiles composited and scaled to all, and the 10k-Gaussian
    256x256 frame in full in one process."""
    import synth
    from oracle import parallel
    workers = parallel.default_workers()
    scene, cam, _ = workload(workload_name)
    legs = _oracle_frame_legs(scene, cam, sample_tiles, workers)
    pool, single = legs["pool"], legs["single"]
    s1, c1 = synth.gen_cfg1()
    l1 = _oracle_frame_legs(s1, c1, 1 << 30, 0)["single"]
    return {"value": pool["blended_pairs"] / pool["seconds_per_frame"], "unit": "Gaussian-pixel blends/s",
            "cores": pool["workers"], "kind": "oracle",
            "sample": (f"the full frame: projection ({legs['project_s']:.2f} s) and binning "
                       f"({legs['binning_s']:.2f} s) in one process, all {legs['tiles']} tiles composited over "
                       f"{pool['workers']} processes ({pool['composite_s']:.2f} s wall, after "
                       f"{pool['pool_start_s']:.2f} s to start the pool); NumPy FP64"),
            "seconds_per_frame": pool["seconds_per_frame"], "blended_pairs": pool["blended_pairs"],
            "single_process": {"value": single["blended_pairs"] / single["seconds_per_frame"], "cores": 1,
                               "seconds_per_frame": single["seconds_per_frame"],
                               "sample": (f"projection and binning of the full frame, {single['sampled_tiles']} "
                                          f"random tiles of {legs['tiles']} composited "
                                          f"({single['composite_s'] * single['sampled_tiles'] / legs['tiles']:.2f} s) "
                                          "and scaled to all tiles")},
            "config1_full_frame": {"workload": "10k Gaussians, 256x256, SH deg 0, every tile", "cores": 1,
                                   "seconds_per_frame": l1["seconds_per_frame"],
                                   "blended_pairs": l1["blended_pairs"],
                                   "value": l1["blended_pairs"] / l1["seconds_per_frame"]},
            "cpu": _cpu_model(), "nproc": os.cpu_count(), "numpy": np.__version__}


def composite_traffic(workload_name):
    """HBM bytes per compositing launch from the committed rocprofv3 counter
    summary, if the compositing sources are unchanged since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_k_composite_{workload_name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_2605_11489_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("composite.hip", "composite_common.hpp", "gs_common.hpp"))
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    return rec["traffic_bytes"]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-opacity-overlap", action="store_true",
                    help="skip the extra timing of the same frame with opacity-aware tile overlap")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip the training-step timing (500k Gaussians, forward + L2 loss + backward)")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the extra timing of the 6M-Gaussian scene at 960x540 and 1920x1080")
    ap.add_argument("--no-warp", action="store_true",
                    help="skip the motion/warp timing (its graphs), e.g. under counter collection")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--frame-only", action="store_true",
                    help="only the workload's frame (no extra fields, CPU baseline or serving), e.g. under a profiler")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving comparison (Poisson trace, continuous batching vs one frame per launch)")
    ap.add_argument("--serve", action="store_true", help="serving benchmark instead of the frame benchmark")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-rates", default="200,700",
                    help="arrival rates of the serving object in the default line, requests/s")
    ap.add_argument("--serve-sizes", default="100000,1000000,3000000,6000000")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-work-queue", action="store_true",
                    help="--serve: also replay the trace against the server in work-queue mode")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the rasterizer runs on a single "
              "MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if a.serve:
        serve_bench(a)
        return
    if a.frame_only:
        a.no_cpu_baseline = a.no_opacity_overlap = a.no_backward = a.no_config3 = a.no_warp = a.no_serving = True

    # the oracle's CPU timing runs first, before anything touches the GPU
    cpu = None
    if not a.no_cpu_baseline:
        print("cpu baseline: the FP64 oracle on this host ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(a.workload)
        print(f"cpu baseline: done ({cpu['seconds_per_frame']:.2f} s per frame on {cpu['cores']} processes)",
              file=sys.stderr, flush=True)

    import torch
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    import ctypes as C

    torch.cuda.set_device(0)
    if a.copy_mib > 0:
        src = torch.ones(a.copy_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    scene, cam, desc = workload(a.workload)
    ds = R.DeviceScene.from_host(scene)
    W, H = cam.width, cam.height

    # one counting frame: exact key count, evaluated and blended pairs
    out_cnt = R.alloc_outputs(W, H)
    out_cnt["n_evaluated"] = torch.empty(H, W, dtype=torch.int32, device="cuda")
    out_cnt["n_blended"] = torch.empty(H, W, dtype=torch.int32, device="cuda")
    fr = R.render_batch([(ds, cam, R.opts_struct(), out_cnt)])
    rc, keys = R.forward_status(fr)
    abi.check(rc)
    E = int(out_cnt["n_evaluated"].to(torch.int64).sum().item())
    B = int(out_cnt["n_blended"].to(torch.int64).sum().item())
    key_capacity = fr.key_capacity
    ws = fr.workspace
    L = fr.layout
    del out_cnt

    out = R.alloc_outputs(W, H)
    jobs = R.make_jobs([(ds, cam, R.opts_struct(), out)])
    stream = R.current_stream_ptr()

    def step():
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), key_capacity, stream))

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: exactly `steps` frames back to back.  The library records
    # its stage events (HIP events on the launch stream) on every 10th frame
    # only: an event costs the stream a few microseconds.
    every = 10
    abi.check(abi.gs_profile_start((a.steps + every - 1) // every, every))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms = (C.c_double * abi.GS_N_STAGES)()
    nfr = C.c_int64(0)
    abi.check(abi.gs_profile_stop(stage_ms, C.byref(nfr)))
    rc, _ = R.forward_status(R.Frame(jobs, 1, [out], ws, L, key_capacity, None, []))
    abi.check(rc)
    ms = (t1 - t0) * 1e3 / a.steps

    # per-frame latency (outside the timed region): events around each of
    # at least 200 frames, whatever the number of timed steps
    n_lat = max(a.steps, 200)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    for i in range(n_lat):
        starts[i].record()
        step()
        ends[i].record()
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    fps = 1e3 / ms
    stages = {abi.STAGE_NAMES[i]: stage_ms[i] / max(nfr.value, 1) for i in range(abi.GS_N_STAGES)}
    n_flat = int(L.n_flat)
    # a single frame of any size takes one tile-sort pass (over 2048 tiles, one per band of tile rows)
    sb = stage_bytes(n_flat, scene.n, scene.sh_degree, keys, int(L.n_tiles), tile_passes=1)
    stage_info = {}
    for name, t in stages.items():
        info = {"ms": round(t, 5)}
        if name in sb:
            info.update(bound="hbm", algorithmic_bytes=sb[name], achieved_GBps=sb[name] / (t * 1e-3) / 1e9)
        else:
            flops = FLOP_EVAL * E + FLOP_BLEND * B
            info.update(bound="alu", algorithmic_flop=flops, achieved_TFLOPs=flops / (t * 1e-3) / 1e12)
        stage_info[name] = info
    # compositing is one kernel launch per frame; the other stages are chains
    # of short launches (sort passes), so the roofline is the compositing
    # kernel's whenever it is the longest single kernel of the frame
    dom = "composite"
    t_dom = stages[dom] * 1e-3
    if dom == "composite":
        flops = FLOP_EVAL * E + FLOP_BLEND * B
        roof = {"kernel": "k_composite", "bound": "alu", "achieved": flops / t_dom / 1e12, "peak": PEAK_FP32 / 1e12,
                "unit": "TFLOP/s", "frac": flops / t_dom / PEAK_FP32, "traffic": composite_traffic(a.workload),
                "per_launch": f"16 FLOP x {E} evaluated + 44 FLOP x {B} blended pairs"}
    else:
        by = sb[dom]
        roof = {"kernel": dom, "bound": "hbm", "achieved": by / t_dom / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": by / t_dom / PEAK_HBM, "traffic": None, "per_launch": f"{by} algorithmic bytes"}
    comp_flops = FLOP_EVAL * E + FLOP_BLEND * B
    result = {
        "metric": METRIC, "value": B * fps, "unit": "Gaussian-pixel blends/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "n_gaussians": scene.n, "width": W, "height": H, "keys": keys,
                   "evaluated_pairs": E, "blended_pairs": B},
        "frames_per_s": fps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "frames": int(lat.size),
                       "timing": "HIP events around each frame, frames back to back after the timed region"},
        "composite_blends_per_s": B / (stages["composite"] * 1e-3),
        "composite_frac_fp32_peak": comp_flops / (stages["composite"] * 1e-3) / PEAK_FP32,
        "stages": stage_info,
        "roofline": roof,
    }
    if not a.frame_only:
        result["gradient_upsample"] = upsample_run(out, a.steps, a.warmup)
    if not a.no_warp:
        result["motion_warp"] = warp_run(out, cam, a.steps, a.warmup)
    if not a.no_opacity_overlap:
        result["opacity_overlap"] = opacity_overlap_run(ds, cam, a.steps, a.warmup, B)
        from paper_2605_11489_amd import abi as _abi
        result["opacity_overlap"]["ellipse"] = opacity_overlap_run(ds, cam, a.steps, a.warmup, B,
                                                                   _abi.GS_OVERLAP_ELLIPSE)
    if not a.frame_only:
        result["with_normals"] = normals_run(ds, cam, a.steps, a.warmup)
        result["other_resolutions"] = resolutions_run(ds, a.steps, a.warmup)
        result["two_in_flight"] = two_in_flight_run(ds, cam, a.steps, a.warmup, B)
    if not a.no_backward:
        result["backward"] = backward_run(max(a.steps // 4, 20), max(a.warmup // 4, 5))
    if not a.no_config3:
        result["config3"] = config3_run(max(a.steps // 10, 10), max(a.warmup // 10, 3))
    if not a.no_serving:
        torch.cuda.empty_cache()
        result["serving"] = serving_run([float(x) for x in a.serve_rates.split(",")])
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def upsample_run(out, steps, warmup, scale=4):
    """Gradient-aware interpolation (Sec. 4.1, Eq. 5-7) of the frame's rgb and
    gradient buffers to scale x scale times the pixels; HBM-bound: per
    low-resolution pixel 36 B read (9 floats) and 12 scale^2 B written."""
    import torch
    from paper_2605_11489_amd import render as R
    rgb, gx, gy = out["rgb"], out["dcdx"], out["dcdy"]
    for _ in range(warmup):
        R.gradient_upsample(rgb, gx, gy, scale)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        R.gradient_upsample(rgb, gx, gy, scale)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    _, H, W = rgb.shape
    by = W * H * (36 + 12 * scale * scale)
    return {"scale": scale, "out": [3, H * scale, W * scale], "ms": ms, "bound": "hbm", "algorithmic_bytes": by,
            "achieved_GBps": by / (ms * 1e-3) / 1e9, "frac_hbm_peak": by / (ms * 1e-3) / PEAK_HBM}


def graph_ms(fn, steps, warmup, per_graph=10):
    """Milliseconds per call of `fn` (launches on the current stream): the
    calls are captured back to back in one HIP graph, per_graph of them, and
    the graph is replayed, so short kernels are timed without the host's
    launch overhead between them."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            fn()
    reps = max(1, steps // per_graph)
    for _ in range(max(1, warmup // per_graph)):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * per_graph)


def warp_run(out, cam, steps, warmup):
    """Motion vectors and forward warp (Sec. 4.2, Eq. 12-13) to the next pose
    of a 60-pose orbit (one 6 degree step), both frames the paper warps to the
    intermediate time: the low-resolution frame just rendered (colour, depth,
    gradients) and a 3840x2160 high-resolution frame (colour, depth, normal
    map; seeded synthetic planes, since the rasterizer renders at low
    resolution).  Three HBM-bound launches per warp.  Algorithmic bytes per
    source pixel 16 (alpha and depth read, motion written), per winning
    source its planes (36 B colour and gradients; 24 B colour and normal),
    per destination pixel the z-buffer (16 B filled and read) and the
    outputs (48 B; 36 B)."""
    import numpy as np
    import torch
    import synth
    from paper_2605_11489_amd import render as R
    eyes = synth.orbit_poses(60)
    res = {}
    # low resolution: the rendered frame
    src = cam
    dst = synth.look_at_camera(eyes[1], cam.width, cam.height)
    ws = R.alloc_workspace(R.warp_workspace_bytes(src, dst))
    o = R.alloc_warp_outputs(cam.width, cam.height, dst.width, dst.height)

    def lr():
        R.motion_warp(src, dst, out["rgb"], out["alpha"], out["depth"], out["dcdx"], out["dcdy"], ws, o)

    lr()
    torch.cuda.synchronize()
    winners = int((o["weight"] > 0).sum().item())
    ms = graph_ms(lr, steps, warmup)
    n_src, n_dst = cam.width * cam.height, dst.width * dst.height
    by = 16 * n_src + 36 * winners + 64 * n_dst
    res["low_res"] = {"size": [cam.width, cam.height], "planes": "rgb, depth, dcdx, dcdy", "winners": winners,
                      "ms": ms, "algorithmic_bytes": by, "achieved_GBps": by / (ms * 1e-3) / 1e9,
                      "frac_hbm_peak": by / (ms * 1e-3) / PEAK_HBM}
    # high resolution: 3840x2160 synthetic colour, depth and normal planes
    Wh, Hh = 3840, 2160
    srch = synth.look_at_camera(eyes[0], Wh, Hh)
    dsth = synth.look_at_camera(eyes[1], Wh, Hh)
    alpha, depth, rgb, _, _ = synth.frame_fields(3, Wh, Hh)
    nrm = np.random.default_rng(4).normal(size=(3, Hh, Wh)).astype(np.float32)
    t = {k: torch.from_numpy(v).cuda() for k, v in dict(alpha=alpha, depth=depth, rgb=rgb, normal=nrm).items()}
    wsh = R.alloc_workspace(R.warp_workspace_bytes(srch, dsth))
    oh = R.alloc_warp_outputs(Wh, Hh, Wh, Hh, planes=("rgb", "normal"))

    def hr():
        R.motion_warp(srch, dsth, t["rgb"], t["alpha"], t["depth"], None, None, wsh, oh, normal=t["normal"])

    hr()
    torch.cuda.synchronize()
    winners = int((oh["weight"] > 0).sum().item())
    ms = graph_ms(hr, max(steps // 4, 10), max(warmup // 4, 10))
    by = 16 * Wh * Hh + 24 * winners + 52 * Wh * Hh
    res["high_res"] = {"size": [Wh, Hh], "planes": "rgb, depth, normal", "winners": winners, "ms": ms,
                       "algorithmic_bytes": by, "achieved_GBps": by / (ms * 1e-3) / 1e9,
                       "frac_hbm_peak": by / (ms * 1e-3) / PEAK_HBM}
    res["timing"] = "HIP graph of 10 back-to-back warps, replayed"
    return res


def backward_run(steps, warmup):
    """One training step of the backward configuration (500k Gaussians, SH
    deg 3, 960x540, L2 loss against a seeded target) through the
    torch.autograd.Function: rasterize() (cached workspace, pair count
    checked in the backward), the loss, loss.backward() (adjoint of
    compositing and projection written into fresh gradient tensors).  Also
    the same step as a plain C-ABI loop with a pre-sized workspace (loss
    gradient by hand, gradients written in place), and the backward call
    alone with HIP events on its stream."""
    import ctypes as C
    import torch
    import synth
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    from paper_2605_11489_amd.autograd import rasterize
    scene, cam = synth.gen_cfg4()
    ds = R.DeviceScene.from_host(scene)
    W, H = cam.width, cam.height
    tgt = torch.from_numpy(synth.gen_target(1, H, W)).cuda()
    params = [t.clone().requires_grad_(True) for t in ds.tensors()]

    def step():
        for p in params:
            p.grad = None
        rgb = rasterize(*params, cam)[0]
        ((rgb - tgt) ** 2).sum().backward()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    finite = all(bool(torch.isfinite(p.grad).all()) for p in params)

    # the same step as a C-ABI loop: pre-sized workspace, no autograd
    out = R.alloc_outputs(W, H)
    opts = R.opts_struct()
    fr = R.render_batch([(ds, cam, opts, out)], with_backward=True)
    rc, keys = R.forward_status(fr)
    abi.check(rc)
    jobs = R.make_jobs([(ds, cam, opts, out)])
    ws, kc = fr.workspace, fr.key_capacity
    stream = R.current_stream_ptr()
    grads = [torch.zeros_like(t) for t in ds.tensors()]
    gs = abi.gs_grads(*[g.data_ptr() for g in grads], 1, 0)   # written, not accumulated: no clearing
    g_rgb = torch.empty_like(out["rgb"])
    sc, cs, outs = ds.c_struct(), R.camera_struct(cam), R.outputs_struct(out)

    def backward():
        abi.check(abi.gs_render_backward(C.byref(sc), C.byref(cs), C.byref(opts), C.byref(outs), ws.data_ptr(),
                                         ws.numel(), kc, g_rgb.data_ptr(), None, None, C.byref(gs), stream))

    def cabi_step():
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), kc, stream))
        torch.sub(out["rgb"], tgt, out=g_rgb)
        g_rgb.mul_(2.0)
        backward()

    for _ in range(warmup):
        cabi_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        cabi_step()
    torch.cuda.synchronize()
    ms_cabi = (time.perf_counter() - t0) * 1e3 / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record()
        backward()
        e1.record()
    torch.cuda.synchronize()
    bms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    return {"n_gaussians": scene.n, "size": [W, H], "keys": keys, "train_step_ms": ms,
            "train_steps_per_s": 1e3 / ms, "train_step_timing": "rasterize() + L2 loss + loss.backward(), "
            "parameter gradients formed by autograd each step", "c_abi_step_ms": ms_cabi,
            "backward_ms": bms, "grads_finite": finite,
            "backward_timing": "gs_render_backward alone (adjoint of compositing and projection), median of "
                               "per-call HIP events"}


def config3_run(steps, warmup):
    """The 6M-Gaussian scene of the same generator at 960x540 and 1920x1080
    (first pose of the 60-pose orbit): whole-frame time per resolution, and
    the whole orbit frame by frame at 960x540."""
    import torch
    import synth
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    scene, poses = synth.gen_cfg3()
    ds = R.DeviceScene.from_host(scene)
    res = {"n_gaussians": scene.n}
    for W, H in ((960, 540), (1920, 1080)):
        cam = synth.look_at_camera(poses[0], W, H)
        out = R.alloc_outputs(W, H)
        fr = R.render_batch([(ds, cam, R.opts_struct(), out)])
        rc, keys = R.forward_status(fr)
        abi.check(rc)
        jobs = R.make_jobs([(ds, cam, R.opts_struct(), out)])
        stream = R.current_stream_ptr()
        ws = fr.workspace

        def step():
            abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), fr.key_capacity, stream))

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[f"{W}x{H}"] = {"ms_per_step": ms, "frames_per_s": 1e3 / ms, "keys": keys}
        del fr, out, ws
    res["orbit_960x540"] = orbit_run(ds, poses, 960, 540)
    return res


def orbit_run(ds, poses, W, H):
    """Every pose of the 60-pose orbit once, in order, at W x H, each frame
    timed by HIP events on the launch stream; one workspace sized for the
    pose with the most pairs.  A warm-up lap precedes the timed lap."""
    import ctypes as C
    import torch
    import synth
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    out = R.alloc_outputs(W, H)
    jobs = [R.make_jobs([(ds, synth.look_at_camera(p, W, H), R.opts_struct(), out)]) for p in poses]
    keys = [R.count_keys(j, 1)[0] for j in jobs]
    cap = max(keys)
    L = R.layout_for(jobs[0], 1, cap)
    ws = R.alloc_workspace(L.total_bytes)
    stream = R.current_stream_ptr()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(jobs) + 1)]
    for lap in range(2):
        for k, j in enumerate(jobs):
            if lap:
                ev[k].record()
            abi.check(abi.gs_render_forward_batch(j, 1, ws.data_ptr(), ws.numel(), cap, stream))
        if lap:
            ev[-1].record()
    torch.cuda.synchronize()
    st = C.c_int64(0)
    abi.check(abi.gs_forward_status(ws.data_ptr(), C.byref(L), C.byref(st)))
    ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(len(jobs))])
    return {"poses": len(jobs), "ms_mean": float(ms.mean()), "ms_p50": float(np.percentile(ms, 50)),
            "ms_min": float(ms.min()), "ms_max": float(ms.max()), "frames_per_s": float(len(jobs) / ms.sum() * 1e3),
            "keys_min": int(min(keys)), "keys_max": int(cap),
            "timing": "each pose once per lap, HIP events between consecutive frames of the timed lap"}


def two_in_flight_run(ds, cam, steps, warmup, blends):
    """Sustained rendering of independent frames with two in flight: two
    workspaces and output sets, frames issued alternately on two streams
    (default priority), so that one frame's latency-bound sorts overlap the
    other's compositing.  `steps` frames in total; per-frame latency is the
    main line's, this is throughput only."""
    import torch
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctx = []
    for s in streams:
        out = R.alloc_outputs(cam.width, cam.height)
        fr = R.render_batch([(ds, cam, R.opts_struct(), out)])
        rc, _ = R.forward_status(fr)
        abi.check(rc)
        ctx.append((R.make_jobs([(ds, cam, R.opts_struct(), out)]), fr.workspace, fr.key_capacity, s.cuda_stream))
    torch.cuda.synchronize()

    def issue(k):
        jobs, ws, cap, st = ctx[k % 2]
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), cap, st))

    for k in range(warmup):
        issue(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        issue(k)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_frame": ms, "frames_per_s": 1e3 / ms, "blends_per_s": blends / (ms * 1e-3),
            "streams": 2, "timing": "wall clock over the frames, issued alternately on two streams"}


def resolutions_run(ds, steps, warmup):
    """The same 1M-Gaussian scene and camera pose at the paper's other
    low-resolution shape (2560x1440 / 4 = 640x360) and at 1920x1080:
    whole-frame time over `steps` frames, pairs and blends."""
    import torch
    import synth
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    res = {}
    for W, H in ((640, 360), (1920, 1080)):
        cam = synth.cfg2_camera(W, H)
        out = R.alloc_outputs(W, H)
        fr = R.render_batch([(ds, cam, R.opts_struct(), out)])
        rc, keys = R.forward_status(fr)
        abi.check(rc)
        jobs = R.make_jobs([(ds, cam, R.opts_struct(), out)])
        stream = R.current_stream_ptr()
        ws = fr.workspace

        def step():
            abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), fr.key_capacity, stream))

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[f"{W}x{H}"] = {"ms_per_step": ms, "frames_per_s": 1e3 / ms, "keys": keys}
        del fr, out, ws
    return res


def normals_run(ds, cam, steps, warmup):
    """The same frame with the normal map N and normal-view map Nv as extra
    outputs (Sec. 4.1, 4.2): the projection writes a 16 B normal per
    Gaussian and the normal-blending compositing variant runs (6 more FLOP
    per blended pair, 16 B more per pixel written).  Whole-frame and
    per-stage times from the library's stage events."""
    import ctypes as C
    import torch
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    out = R.alloc_outputs(cam.width, cam.height, normals=True)
    fr = R.render_batch([(ds, cam, R.opts_struct(), out)])
    rc, _ = R.forward_status(fr)
    abi.check(rc)
    jobs = R.make_jobs([(ds, cam, R.opts_struct(), out)])
    stream = R.current_stream_ptr()
    ws = fr.workspace

    def step():
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), fr.key_capacity, stream))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    abi.check(abi.gs_profile_start((steps + 9) // 10, 10))
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stage_ms = (C.c_double * abi.GS_N_STAGES)()
    nfr = C.c_int64(0)
    abi.check(abi.gs_profile_stop(stage_ms, C.byref(nfr)))
    return {"ms_per_step": ms, "frames_per_s": 1e3 / ms,
            "stages_ms": {abi.STAGE_NAMES[i]: stage_ms[i] / max(nfr.value, 1) for i in range(abi.GS_N_STAGES)}}


def opacity_overlap_run(ds, cam, steps, warmup, blended, mode=None):
    """The same frame with opacity-aware tile overlap (by default the
    ellipse's bounding box; GS_OVERLAP_ELLIPSE: the tiles the ellipse reaches,
    row by row): identical image buffers (tested bit for bit), fewer
    (tile, Gaussian) pairs.  Whole-frame time over `steps` frames."""
    import torch
    from paper_2605_11489_amd import abi
    from paper_2605_11489_amd import render as R
    out = R.alloc_outputs(cam.width, cam.height)
    opts = R.opts_struct(overlap=abi.GS_OVERLAP_OPACITY if mode is None else mode)
    fr = R.render_batch([(ds, cam, opts, out)])
    rc, keys = R.forward_status(fr)
    abi.check(rc)
    jobs = R.make_jobs([(ds, cam, opts, out)])
    stream = R.current_stream_ptr()
    ws = fr.workspace

    def step():
        abi.check(abi.gs_render_forward_batch(jobs, 1, ws.data_ptr(), ws.numel(), fr.key_capacity, stream))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"ms_per_step": ms, "frames_per_s": 1e3 / ms, "value": blended * 1e3 / ms, "keys": keys,
            "unit": "Gaussian-pixel blends/s"}



SERVE_METRIC = "served-frame p50/p99 latency and frames/s, Poisson 200 req/s over 4 resident scenes"
SERVE_SIZES = (100_000, 1_000_000, 3_000_000, 6_000_000)


def _serve_trace(srv, ids, trace, warm):
    """Replays `trace` against one server: submits each request at its
    arrival time, polls every outstanding ticket; latency is the server's
    poll-visible completion minus submission."""
    import synth
    outstanding = {}
    done = []
    rejected = 0
    start = time.perf_counter()

    def reap():
        for tk in list(outstanding):
            r = srv.poll(tk)
            if r is not None:
                done.append((outstanding.pop(tk), r.status, r.t_done - r.t_submit, r.batch_size, r.retries))
                srv.release(tk)

    for (ta, sidx, (W, H), eye) in trace:
        while True:
            now = time.perf_counter() - start
            reap()
            if now >= ta:
                break
            time.sleep(min(0.0005, ta - now))
        rc, tk = srv.submit_rc(ids[sidx], synth.look_at_camera(eye, W, H))
        if rc == 0:
            outstanding[tk] = ta
        else:
            rejected += 1
    while outstanding:
        reap()
        time.sleep(0.0005)
    end = time.perf_counter() - start
    meas = [d for d in done if d[0] >= warm]
    lat = np.array([d[2] for d in meas if d[1] == 0]) * 1e3
    return {"frames_per_s": len(meas) / max(end - warm, 1e-9),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean())},
            "completed": len(meas), "failed": sum(1 for d in meas if d[1] != 0), "rejected": rejected,
            "retries": int(sum(d[4] for d in meas)), "mean_batch": float(np.mean([d[3] for d in meas])),
            "wall_s": end}


def serving_run(rates, seconds=None, min_requests=3000, warm=1.0, budget_gb=32.0, sizes=SERVE_SIZES,
                max_batch=16, n_streams=3, heavy_ms=0.6, work_queue_leg=False, order=None):
    """The serving configuration: four resident scenes (the clustered
    generator, seeds 10-13, SH deg 3), Poisson arrivals (seed 20) at each
    rate, resolutions uniform over 320x180 .. 1920x1080, eyes on the sphere
    of radius 4.  The same trace is replayed against the continuous-batching
    server and against the one-frame-per-launch FIFO renderer (and, with
    work_queue_leg, against the server in work-queue mode), in the order
    `order` names (default: batched first); the measured part lasts
    `seconds` (default: long enough for `min_requests`)."""
    import torch
    import synth
    from paper_2605_11489_amd import render as R
    from paper_2605_11489_amd.serve import Server
    t0 = time.perf_counter()
    dev_scenes = [R.DeviceScene.from_host(synth.gen_clustered(seed, n, 3))
                  for seed, n in zip((10, 11, 12, 13), sizes)]
    print(f"serving: scenes generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    res = {"workload": (f"Poisson arrivals (seed 20) over resident scenes of {list(sizes)} Gaussians "
                        "(SH deg 3), resolutions uniform over 320x180, 640x360, 960x540, 1920x1080, eyes "
                        "uniform on the sphere of radius 4"),
           "budget_GB": budget_gb, "max_batch": max_batch, "streams": n_streams, "heavy_ms": heavy_ms,
           "rates": {}}
    for rate in rates:
        meas = seconds if seconds else max(min_requests / rate, 2.0)
        trace = synth.serving_trace(seed=20, rate=rate, duration=warm + meas, n_scenes=len(sizes))
        per = {"warmup_s": warm, "measured_s": meas, "requests": len(trace)}
        modes = order or (("batched", "work_queue", "fifo") if work_queue_leg else ("batched", "fifo"))
        for mode in modes:
            with Server(int(budget_gb * (1 << 30)), max_batch=max_batch, n_streams=n_streams,
                        fifo=(mode == "fifo"), key_factor=1.5, heavy_ms=heavy_ms,
                        work_queue=(mode == "work_queue")) as srv:
                ids = [srv.register(ds) for ds in dev_scenes]
                # one request per (scene, resolution) class primes the pair estimates
                for sidx in range(len(ids)):
                    for (W, H) in synth.SERVING_RESOLUTIONS:
                        tk = srv.submit(ids[sidx], synth.look_at_camera((0.0, 0.0, -4.0), W, H))
                        while srv.poll(tk) is None:
                            time.sleep(0.001)
                        srv.release(tk)
                r = _serve_trace(srv, ids, trace, warm)
                r["max_batch"] = srv.stats()["max_batch"]
                r["arena_peak_GB"] = srv.stats()["bytes_peak"] / 2 ** 30
                r["early_reports"] = srv.stats()["flag_done"]
            per[{"fifo": "fifo_one_frame_per_launch", "batched": "batched",
                 "work_queue": "batched_work_queue"}[mode]] = r
            print(f"serving: {rate:g} req/s {mode}: p50 {r['latency_ms']['p50']:.2f} ms, "
                  f"p99 {r['latency_ms']['p99']:.2f} ms, {r['frames_per_s']:.0f} frames/s",
                  file=sys.stderr, flush=True)
        b, f = per["batched"], per["fifo_one_frame_per_launch"]
        per["p99_ratio_fifo_over_batched"] = f["latency_ms"]["p99"] / b["latency_ms"]["p99"]
        per["p50_ratio_fifo_over_batched"] = f["latency_ms"]["p50"] / b["latency_ms"]["p50"]
        res["rates"][f"{rate:g}"] = per
    del dev_scenes
    torch.cuda.empty_cache()
    return res


def serve_bench(a):
    """The serving benchmark alone: the trace at --serve-rate for
    --serve-seconds measured seconds (the specified 30 s by default)."""
    import torch
    torch.cuda.set_device(0)
    sizes = tuple(int(x) for x in a.serve_sizes.split(","))
    res = serving_run([a.serve_rate], seconds=a.serve_seconds, warm=2.0, budget_gb=a.serve_budget_gb, sizes=sizes,
                      work_queue_leg=a.serve_work_queue)
    per = res["rates"][f"{a.serve_rate:g}"]
    b, f = per["batched"], per["fifo_one_frame_per_launch"]
    out = {"metric": SERVE_METRIC, "value": b["latency_ms"]["p99"], "unit": "ms (p99)", "n_gpus": 1,
           "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": res["workload"] + f", {a.serve_rate:g} req/s", "warmup_s": per["warmup_s"],
                      "measured_s": per["measured_s"], "budget_GB": a.serve_budget_gb},
           "batched": b, "fifo_one_frame_per_launch": f,
           "p99_speedup_vs_fifo": f["latency_ms"]["p99"] / b["latency_ms"]["p99"]}
    if "batched_work_queue" in per:
        out["batched_work_queue"] = per["batched_work_queue"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
