"""Throughput of the fisheye plane sweep on one MI355X.

A step is one whole pass of the hot path (level images, border marks, the
sweep, the epilogue) over one frame of the workload: the 1024x768 street
scene with 3 sources, 128 fronto + 64 ground planes, 9x9 ZNCC, mean of the
best 2 sources, winner-take-all with parabolic refinement, FP32.  Inputs are
resident in HBM before the timed region.

Prints one JSON line: plane-pixel evaluations per second (pixels x planes per
step / step time), the roofline of the sweep kernel (VALU-bound; achieved
algorithmic lane-ops per second over the chip's non-packed FP32 issue rate,
from the kernel's own HIP-event durations), and the FP64 CPU oracle timed on
a bounded sample of the same workload."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "plane-pixel evals/s (Gpix·planes/s) + depth maps/s vs plain FP32, 1 GPU"
# non-packed FP32 VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8e12   # bytes/s


def algorithmic_ops_per_plane_pixel(n_src: int) -> int:
    """Lane-ops of the method's own arithmetic per (pixel, plane) that meets
    its plane: per source 9 (plane-induced point) + 10 (projection) + 5
    (bounds) + 13 (bilinear from four 8-bit taps: 4 for the cell and its
    weights, 2 for the address, 6 for three lerps, 1 for centring) + 14
    (window sums) + 9 (ZNCC and cost) + 2 (aggregation), and 6 for the
    winner-take-all update."""
    return 62 * n_src + 6


def cpu_model() -> str:
    """The host CPU's model name (Linux)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


# HBM bytes per launch of the sweep kernel on the C2 workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of
# "python bench.py --steps 2 --warmup 1 --no-cpu --no-batched --copy-calibration"
# (the persistent sweep kernel of C2), each scaled by what the same counter
# reads for a 256 MiB device copy (FETCH_SIZE reads half the copied bytes,
# WRITE_SIZE all of them).  Valid only for the kernel code they were taken on:
# a hash of the sources' code (comments and whitespace left out) guards them.
COUNTED_TRAFFIC = {
    "sources_sha256": "8018443a063b5531241ade691a1f0373e21b4c1bab6e9effbf85dde7dff85cdc",
    "fetch_kib": 29729.6, "write_kib": 183417.4, "fetch_scale": 262144.0 / 131086.7, "write_scale": 1.0,
}
TRAFFIC_SOURCES = ["paper_1809_06132_amd/csrc/sweep_common.h", "paper_1809_06132_amd/csrc/psweep_internal.h",
                   "paper_1809_06132_amd/csrc/inst_persistent.hip", "paper_1809_06132_amd/csrc/api.cpp"]


def _code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed, so that
    a comment edit does not count as a kernel change (string literals are
    kept as they are)."""
    import re
    string = r'"(?:\\.|[^"\\])*"'
    no_comments = re.sub(string + r'|//[^\n]*|/\*.*?\*/',
                         lambda m: m.group(0) if m.group(0).startswith('"') else " ", text, flags=re.S)
    parts = re.split("(" + string + ")", no_comments)
    return "".join(p if i % 2 else re.sub(r"\s+", " ", p) for i, p in enumerate(parts)).strip()


def kernel_sources_sha256() -> str:
    """Hash of the code (not the comments) of the sources the counted traffic
    depends on."""
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def counted_traffic():
    """HBM bytes per sweep launch from the counters, or None when the kernel
    sources changed since they were taken."""
    c = COUNTED_TRAFFIC
    if c["sources_sha256"] is None or c["sources_sha256"] != kernel_sources_sha256():
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def cpu_baseline(fr, st, target_s=15.0, one_core_s=5.0):
    """The FP64 oracle on random pixels of the frame (every plane and source of
    each): median of three runs of about target_s / 3 seconds on all the
    oracle's threads, and one run of about one_core_s on a single thread."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(99)
    lv = st.levels[0]
    P = lv.n_fronto + lv.n_ground

    def sample(n):
        return np.stack([rng.integers(0, fr.ref.shape[1], n), rng.integers(0, fr.ref.shape[0], n)], 1).astype(np.int32)

    def timed(n):
        px = sample(n)
        t0 = time.perf_counter()
        oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, pixels=px)
        return time.perf_counter() - t0

    def sized(seconds, probe=1024):
        dt = timed(probe)
        return int(min(2_000_000, max(probe, probe * seconds / max(dt, 1e-3))))

    cores = oracle.threads()
    # share of (pixel, plane, source) evaluations with a usable window, from
    # the oracle's per-source costs on a seeded sample of pixels
    px = sample(4096)
    sv = oracle.sweep_level(lv, st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, pixels=px,
                            srcvol=True)["srcvol"]
    valid_share = float(np.isfinite(sv).mean())
    n = sized(target_s / 3)
    runs = sorted(timed(n) for _ in range(3))
    dt = runs[1]
    oracle.set_threads(1)
    try:
        n1 = sized(one_core_s, probe=256)
        dt1 = timed(n1)
    finally:
        oracle.set_threads(cores)
    return {"value": n * P / dt / 1e9, "unit": "Gpix·planes/s", "cores": cores, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"{n} random pixels of the 1024x768 frame, all {P} planes x 3 sources, FP64 two-pass "
                      f"ZNCC per window; median of 3 runs ({', '.join(f'{t:.1f}' for t in runs)} s)",
            "one_core": {"value": n1 * P / dt1 / 1e9, "cores": 1, "sample": f"{n1} random pixels, {dt1:.1f} s"},
            "valid_source_evaluation_share": valid_share}


class _C5:
    """C5: 16 frame sets of mixed size (1280x960 / 1024x768 / 640x480), 4
    sources, two levels of 192 + 64 planes, resident on the GPU."""

    def __init__(self):
        import scenegen
        from paper_1809_06132_amd.sweep import frame_to_device
        wl = scenegen.workload("C5")
        self.frames = wl.frames
        self.W, self.H = scenegen.C5_SIZES[0]
        self.st = scenegen.c5_settings(self.W, self.H)
        self.dev = []
        for i, fr in enumerate(self.frames):
            d = frame_to_device(fr)
            d["camera_set"] = i
            self.dev.append(d)

    def sweep(self, storage, launch, max_frames):
        from paper_1809_06132_amd.sweep import PlaneSweep
        ps = PlaneSweep(self.st, self.W, self.H, 4, max_frames=max_frames, max_camera_sets=len(self.frames),
                        storage=storage, launch=launch)
        for i, fr in enumerate(self.frames):
            ps.set_cameras(i, fr.ref_cam, fr.src_cams, fr.poses)
            w, h = fr.ref_cam.width, fr.ref_cam.height
            ps.set_crop(i, (w - w // 2) // 2, (h - h // 2) // 2, w // 2, h // 2)
        outs = [ps.alloc_outputs(camera_set=i) for i in range(len(self.frames))]
        return ps, outs

    def plain_ms(self, steps, warmup):
        """Plain form: one frame per run, FP32 staging, per-level grid launches."""
        import torch
        ps, outs = self.sweep("f32", "grid", 1)
        pp = sum(ps.plane_pixels([d]) for d in self.dev)
        for _ in range(warmup):
            for d, o in zip(self.dev, outs):
                ps.run([d], [o])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for d, o in zip(self.dev, outs):
                ps.run([d], [o])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        ps.close()
        return ms, pp

    def batched_ms(self, storage, launch, steps, warmup):
        """Batched form: every frame in one run captured as a HIP graph, the
        tile shape and plane chunks per level picked by the autotuner on this
        very batch (tuned afresh, no cache)."""
        import torch
        from paper_1809_06132_amd import autotune
        ps, outs = self.sweep(storage, launch, len(self.frames))
        choice = autotune.tune(ps, self.dev, outs, reps=3, cache_path=None)
        ps.capture_graph(self.dev, outs)
        for _ in range(warmup):
            ps.launch_graph()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ps.launch_graph()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        ps.close()
        return ms, {"tiles": choice["tiles"], "chunks": choice["chunks"]}


def bench_c5(args):
    """C5: the batched form (one persistent launch for every frame, level and
    tile, or one grid per frame and level; FP16 or FP32 staging; replayed as
    a HIP graph) against plain per-frame FP32 launches."""
    c5 = _C5()
    res, tuned = {}, {}
    res["plain_f32_ms"], pp = c5.plain_ms(args.steps, args.warmup)
    for storage, launch in (("f16", "persistent"), ("f32", "persistent"), ("f16", "grid"), ("f32", "grid")):
        ms, choice = c5.batched_ms(storage, launch, args.steps, args.warmup)
        res[f"batched_{launch}_{storage}_graph_ms"] = ms
        tuned[f"{launch}_{storage}"] = choice
    line = {"metric": METRIC, "workload": "C5", "plane_pixels_per_batch": pp, "maps_per_batch": len(c5.frames)}
    for k, v in res.items():
        line[k] = v
        line[k.replace("_ms", "_gpps")] = pp / (v * 1e-3) / 1e9
    best = min((k for k in res if k.startswith("batched")), key=res.get)
    line["autotuned"] = tuned
    line["best_batched"] = best
    line["best_batched_vs_plain_f32"] = res["plain_f32_ms"] / res[best]
    if not args.no_cpu:
        line["cpu_baseline"] = _c5_cpu_baseline(c5)
    print(json.dumps(line), flush=True)


def _c5_cpu_baseline(c5, seconds=10.0):
    """The FP64 oracle on random pixels of the batch's first frame (1280x960),
    both levels with all their planes: plane-pixel evaluations per second."""
    import numpy as np

    import oracle
    import scenegen
    fr = c5.frames[0]
    st = scenegen.c5_settings(fr.ref_cam.width, fr.ref_cam.height)
    rng = np.random.default_rng(7)
    done, t0, n = 0, time.perf_counter(), 256
    while time.perf_counter() - t0 < seconds:
        for lv in st.levels:
            rc, rimg, scs, simgs = oracle.level_inputs(fr, lv)
            h, w = rimg.shape
            px = np.stack([rng.integers(0, w, n), rng.integers(0, h, n)], 1).astype(np.int32)
            oracle.sweep_level(lv, st, rc, rimg, scs, simgs, fr.poses, pixels=px)
            done += n * (lv.n_fronto + lv.n_ground)
    dt = time.perf_counter() - t0
    return {"value": done / dt / 1e9, "unit": "Gpix·planes/s", "cores": oracle.threads(), "cpu": cpu_model(),
            "kind": "oracle", "sample": f"random pixels of both levels of the 1280x960 frame, all 256 planes x 4 "
                                        f"sources, FP64, {dt:.1f} s"}


def _time_runs(ps, frames, outs, steps, warmup):
    """Median, p10 and p90 of whole psweep_run calls, from HIP events on the
    launch stream (torch's current stream)."""
    import numpy as np
    import torch
    for _ in range(warmup):
        ps.run(frames, outs)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ps.run(frames, outs)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    p10, p50, p90 = (float(v) for v in np.percentile(ms, [10, 50, 90]))
    return p50, [p10, p50, p90]


def bench_levels(args):
    """Two-level maps: C3 (1024x768, 3 sources; low 512x384 with 96 planes at
    7x7, full-resolution 512x384 centre crop with 64 planes at 9x9) in every
    staging precision, and the paper's shape (1024x544; 64 + 30 planes on the
    512x272 level at 7x7 and on the 572x332 full-resolution crop at 9x9) with
    5 cameras (4 sources) and with 3 (the two nearest sources)."""
    import torch

    import scenegen
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device

    rows = []
    if args.workload == "C3":
        wl = scenegen.workload("C3")
        cases = [("C3", wl.frames[0], wl.settings, list(range(3)), st) for st in ("f32", "f16", "bf16")]
        # both levels in one persistent launch (their tiles balance each other)
        cases.append(("C3", wl.frames[0], wl.settings, list(range(3)), "f32", "persistent"))
    else:
        wl = scenegen.workload("paper")
        cases = [("paper", wl.frames[0], wl.settings, list(range(4)), "f32"),
                 ("paper", wl.frames[0], wl.settings, [0, 1], "f32")]
    for name, fr, st, srcs, storage, *launch in cases:
        launch = launch[0] if launch else "grid"
        W, H = fr.ref_cam.width, fr.ref_cam.height
        ps = PlaneSweep(st, W, H, len(srcs), storage=storage, launch=launch)
        ps.set_cameras(0, fr.ref_cam, [fr.src_cams[i] for i in srcs], [fr.poses[i] for i in srcs])
        d = frame_to_device(fr)
        d["srcs"] = [d["srcs"][i] for i in srcs]
        out = ps.alloc_outputs()
        pp = ps.plane_pixels([d])
        med, pct = _time_runs(ps, [d], [out], args.steps, args.warmup)
        torch.cuda.synchronize()
        maps = {k: v.cpu().numpy() for k, v in out["merged"].items()}
        ps.close()
        rows.append({"workload": name, "cameras": len(srcs) + 1, "storage": storage, "launch": launch,
                     "ms_per_map": med,
                     "ms_p10_p50_p90": pct, "maps_per_s": 1e3 / med, "plane_pixels_per_map": pp,
                     "gpix_planes_per_s": pp / (med * 1e-3) / 1e9})
        if name == "C3" and not args.no_cpu:
            rows[-1]["vs_oracle"] = _accuracy(maps, _c3_oracle(fr, st))
    line = {"metric": METRIC, "workload": args.workload, "results": rows}
    if args.workload == "C3" and not args.no_cpu:
        ref, secs = _c3_oracle.cache
        import oracle
        line["cpu_baseline"] = {"value": 1.0 / secs, "unit": "maps/s", "cores": oracle.threads(), "cpu": cpu_model(),
                                "kind": "oracle", "sample": "the whole two-level 1024x768 map (both levels at every "
                                "pixel, then the merge), FP64, one run"}
    if args.workload == "paper":
        line["context"] = ("the paper's multi-scale depth stage: 36 ms per frame with 5 cameras on a GTX 1080; "
                           "3 cameras about 17% less")
        line["three_vs_five_cameras_time_ratio"] = rows[1]["ms_per_map"] / rows[0]["ms_per_map"]
    print(json.dumps(line), flush=True)


def _c3_oracle(fr, st):
    """The FP64 oracle's two-level map of the frame (computed once, timed)."""
    if getattr(_c3_oracle, "cache", None) is None:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.run(fr, st)["merged"]
        _c3_oracle.cache = (ref, time.perf_counter() - t0)
    return _c3_oracle.cache[0]


def _accuracy(gpu, ref):
    """Merged map against the oracle's: level and index agreement over the
    oracle's valid pixels, and the range's relative error on the pixels
    whose level and index agree (p50, p99.9, max)."""
    import numpy as np
    ov = ref["level"] != 255
    same = ov & (gpu["level"] == ref["level"]) & (gpu["index"] == ref["index"])
    rel = np.abs(gpu["depth"][same] - ref["depth"][same]) / ref["depth"][same]
    return {"pixels": int(ov.sum()), "level_agreement": float((gpu["level"][ov] == ref["level"][ov]).mean()),
            "index_agreement": float(same.sum() / ov.sum()),
            "depth_rel_err_p50_p999_max": [float(np.quantile(rel, 0.5)), float(np.quantile(rel, 0.999)),
                                           float(rel.max())]}


def bench_c4(args):
    """C4: soft-argmin forward and backward (640x480, 2 sources, 64 fronto
    planes, 7x7, T = 0.1) on the GPU, and the FP64 oracle's backward on the
    64x48 crop the gradient checks use (timed on the host cores)."""
    import numpy as np
    import torch

    import oracle
    import scenegen
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device

    wl = scenegen.workload("C4")
    fr, st = wl.frames[0], wl.settings
    W, H, S = fr.ref_cam.width, fr.ref_cam.height, len(fr.srcs)
    ps = PlaneSweep(st, W, H, S)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    d = frame_to_device(fr)
    out = ps.alloc_outputs()
    pp = ps.plane_pixels([d])
    fwd, fwd_pct = _time_runs(ps, [d], [out], args.steps, args.warmup)
    g = torch.randn((H, W), device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    shapes = [s.shape for s in fr.srcs]
    def time_backward(image_grads):
        for _ in range(args.warmup):
            ps.soft_backward(g, shapes, image_grads=image_grads)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ps.soft_backward(g, shapes, image_grads=image_grads)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), [float(v) for v in np.percentile(ms, [10, 50, 90])]

    bwd, bwd_pct = time_backward(True)
    bwd_pose, bwd_pose_pct = time_backward(False)
    ps.close()
    line = {"metric": METRIC, "workload": "C4", "plane_pixels": pp, "forward_ms": fwd,
            "forward_ms_p10_p50_p90": fwd_pct, "forward_gpix_planes_per_s": pp / (fwd * 1e-3) / 1e9,
            "backward_ms": bwd, "backward_ms_p10_p50_p90": bwd_pct,
            "backward_pose_only_ms": bwd_pose, "backward_pose_only_ms_p10_p50_p90": bwd_pose_pct}
    if not args.no_cpu:
        rect = (288, 216, 64, 48)
        rng = np.random.default_rng(0)
        gg = rng.normal(size=(rect[3], rect[2]))
        t0 = time.perf_counter()
        oracle.soft_backward(st.levels[0], st, fr.ref_cam, fr.ref, fr.src_cams, fr.srcs, fr.poses, rect, gg)
        dt = time.perf_counter() - t0
        line["cpu_baseline_backward"] = {"seconds": dt, "cores": oracle.threads(), "kind": "oracle",
                                         "sample": "FP64 backward on the 64x48 crop at (288, 216), all 64 planes"}
    print(json.dumps(line), flush=True)


def bench_tsdf(args):
    """TSDF fusion (Sec. III-C) of 1024x768 fisheye depth maps into the
    paper's local map: a box of 75 x 4 x 75 blocks of 8^3 voxels at 0.1 m
    (60 m x 3.2 m x 60 m), mu = 0.3 m, following a vehicle that drives 0.5 m
    per frame through the street scene.  Per integration: all five kernels
    (HIP events around psweep_tsdf_integrate); the roofline of the
    integration kernel is HBM: 16 bytes per voxel of the visible blocks
    (read and write of TSDF value and weight) over its duration."""
    import numpy as np
    import torch

    import scenegen
    from paper_1809_06132_amd.tsdf import TsdfMap

    n = max(args.steps, 4)
    seq = scenegen.depth_sequence(n_frames=n, w=1024, h=768, f=360.0, step_m=0.5, seed=1009)
    depths = [torch.from_numpy(d).cuda() for d in seq.depths]
    tm = TsdfMap(voxel=0.1, mu=0.3, blocks=(75, 4, 75), w_max=100.0, min_obs=3, max_width=1024, max_height=768)
    centre = lambda k: (seq.centres[k][0], 0.0, seq.centres[k][2])
    for k in range(min(args.warmup, n)):
        tm.integrate(seq.cam, seq.poses[k], centre(k), depths[k])
    tm.reset()
    torch.cuda.synchronize()
    ms, vis = [], []
    for k in range(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tm.integrate(seq.cam, seq.poses[k], centre(k), depths[k])
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        vis.append(tm.stats()[1])
    out = tm.extract()
    torch.cuda.synchronize()
    kept = int(torch.isfinite(out["tsdf"]).sum())
    tm.close()
    med = float(np.median(ms))
    vox = float(np.median(vis)) * 512
    line = {"metric": "TSDF integrations/s (1024x768 fisheye depth maps)", "workload": "tsdf",
            "frames": n, "ms_per_integration": med,
            "ms_p10_p50_p90": [float(v) for v in np.percentile(ms, [10, 50, 90])],
            "integrations_per_s": 1e3 / med, "visible_blocks_median": float(np.median(vis)),
            "voxels_in_view_per_s": vox / (med * 1e-3), "extracted_voxels_after_run": kept,
            "map": "75 x 4 x 75 blocks of 8^3 voxels, 0.1 m, mu 0.3 m, w_max 100, >= 3 observations"}
    if not args.no_cpu:
        import oracle
        o = oracle.TsdfOracle(0.1, 0.3, (75, 4, 75), min_obs=3)
        t0 = time.perf_counter()
        o.integrate(seq.cam, seq.poses[0], seq.depths[0], centre(0))
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "integrations/s", "cores": 1, "kind": "oracle",
                                "sample": "one integration of the first depth map, FP64, single thread"}
    print(json.dumps(line), flush=True)


def bench_filter(args):
    """Depth-map filtering (Sec. III-A: best cost, uniqueness ratio, local
    continuity) and box masking (Sec. IV-B) of the C2 map (1024x768, the
    sweep's merged output).  Calls are timed back to back with HIP events on
    the current stream.  Both kernels are HBM-bound: the filter's algorithmic
    bytes are 17 per pixel (depth, cost1, cost2 read, kept range and code
    written), the mask's 5 per masked pixel (range and code written).  The
    filter codes are compared with the oracle's on the same maps."""
    import numpy as np
    import torch

    import scenegen
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device

    wl = scenegen.workload("C2")
    fr, st = wl.frames[0], wl.settings
    W, H = fr.ref_cam.width, fr.ref_cam.height
    ps = PlaneSweep(st, W, H, len(fr.srcs))
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    out = ps.alloc_outputs()
    ps.run([frame_to_device(fr)], [out])
    merged = out["merged"]
    rng = np.random.default_rng(31)
    boxes = [tuple(int(v) for v in (x, y, x + bw, y + bh)) for x, y, bw, bh in
             zip(rng.integers(0, W - 200, 12), rng.integers(H // 3, H - 200, 12),
                 rng.integers(40, 200, 12), rng.integers(40, 200, 12))]
    mask = np.zeros((H, W), bool)
    for x0, y0, x1, y1 in boxes:
        mask[y0:y1, x0:x1] = True
    n_masked = int(mask.sum())

    def timed(fn, n, reps=5):
        # n back-to-back calls between two events (the launches queue ahead
        # of the GPU, so host submission is not inside the figure), reps times
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / n)
        return ms

    for _ in range(args.warmup):
        d, c = ps.filter(merged)
        ps.mask_boxes(d, boxes, code=c)
    torch.cuda.synchronize()
    f_ms = timed(lambda: ps.filter(merged), args.steps)
    d, c = ps.filter(merged)
    torch.cuda.synchronize()
    gd, gc = d.cpu().numpy(), c.cpu().numpy()
    m_ms = timed(lambda: ps.mask_boxes(d, boxes, code=c), args.steps)
    m = {k: v.cpu().numpy() for k, v in merged.items()}
    ps.close()
    f_med, m_med = float(np.median(f_ms)), float(np.median(m_ms))
    f_bytes, m_bytes = 17.0 * W * H, 5.0 * n_masked
    line = {"metric": "depth-map filter and box mask, 1024x768 (C2 map)", "workload": "filter",
            "filter_ms": f_med, "filter_ms_min_max": [float(min(f_ms)), float(max(f_ms))],
            "filter_maps_per_s": 1e3 / f_med,
            "filter_roofline": {"bound": "hbm", "achieved": f_bytes / (f_med * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                                "unit": "GB/s", "frac": f_bytes / (f_med * 1e-3) / HBM_PEAK,
                                "algorithmic_bytes": f_bytes},
            "mask_ms": m_med, "mask_boxes": len(boxes), "masked_pixels": n_masked,
            "mask_roofline": {"bound": "hbm", "achieved": m_bytes / (m_med * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                              "unit": "GB/s", "frac": m_bytes / (m_med * 1e-3) / HBM_PEAK,
                              "algorithmic_bytes": m_bytes},
            "filter_codes": {str(k): int(v) for k, v in zip((0, 1, 2, 3, 255),
                                                          np.bincount(gc.ravel(), minlength=256)[[0, 1, 2, 3, 255]])}}
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        od, oc = oracle.depth_filter(fr.ref_cam, st.ground_n, m["depth"].astype(np.float64),
                                     m["cost1"].astype(np.float64), m["cost2"].astype(np.float64))
        dt = time.perf_counter() - t0
        c1, c2 = m["cost1"].astype(np.float64), m["cost2"].astype(np.float64)
        with np.errstate(invalid="ignore"):
            near = np.isfinite(c2) & (np.abs(c2 - 1.05 * c1) <= 1e-6 * np.abs(c2))
        line["codes_differing_off_threshold"] = int(((gc != oc) & ~near).sum())
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "filtered maps/s", "cores": 1,
                                "kind": "oracle", "sample": "the whole 1024x768 map, FP64"}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="default workload: skip the batched-vs-plain comparison on the 16-frame batch")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--launch", default="persistent", choices=["grid", "persistent"],
                    help="C2: one grid of tiles, or the persistent launch (resident workgroups taking tiles "
                         "from per-XCD queues)")
    ap.add_argument("--workload", default="C2", choices=["C2", "C3", "C4", "C5", "paper", "tsdf", "filter"],
                    help="C2 (default): the benchmark line; C3: two-level maps per staging precision; "
                         "C4: soft forward and backward; C5: batched vs plain; paper: the paper's shape "
                         "with 5 and 3 cameras; tsdf: depth-map fusion; filter: depth-map filter and box mask")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the sweep runs on one "
              "device (frames, or plane ranges, would shard across GPUs)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "C5":
        bench_c5(args)
        return
    if args.workload in ("C3", "paper"):
        bench_levels(args)
        return
    if args.workload == "C4":
        bench_c4(args)
        return
    if args.workload == "tsdf":
        bench_tsdf(args)
        return
    if args.workload == "filter":
        bench_filter(args)
        return

    import torch

    import scenegen
    from paper_1809_06132_amd.sweep import PlaneSweep, frame_to_device

    wl = scenegen.workload("C2")
    fr, st = wl.frames[0], wl.settings
    ps = PlaneSweep(st, fr.ref_cam.width, fr.ref_cam.height, len(fr.srcs), storage=args.storage,
                    launch=args.launch)
    ps.set_cameras(0, fr.ref_cam, fr.src_cams, fr.poses)
    frame = frame_to_device(fr)
    out = ps.alloc_outputs()
    plane_pixels = ps.plane_pixels([frame])
    met_pixels = ps.plane_pixels_met([frame])
    for _ in range(args.warmup):
        ps.run([frame], [out])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ps.run([frame], [out])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3

    # distribution of single steps (HIP events on the launch stream, which is
    # torch's current stream here), after the timed region
    import numpy as np
    step_ms = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ps.run([frame], [out])
        e1.record()
        torch.cuda.synchronize()
        step_ms.append(e0.elapsed_time(e1))
    p10, p50, p90 = (float(v) for v in np.percentile(step_ms, [10, 50, 90]))

    # sweep-kernel duration from HIP events recorded on the launch stream
    ps.set_timing(True)
    kms = []
    for _ in range(max(5, min(20, args.steps))):
        ps.run([frame], [out])
        torch.cuda.synchronize()
        kms.append(ps.sweep_kernel_ms()[0])
    ps.set_timing(False)
    kernel_ms = sorted(kms)[len(kms) // 2]
    # the algorithmic work is the (pixel, plane) pairs that take part in the
    # method: the pixel has a window and its ray meets the plane (the rest
    # have no cost at all); the nominal count (every pixel and plane) is
    # reported beside it
    ops_pp = algorithmic_ops_per_plane_pixel(len(fr.srcs))
    ops = met_pixels * ops_pp
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    nominal = plane_pixels * ops_pp / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    traffic = counted_traffic()
    # algorithmic HBM bytes of one map: the 8-bit reference and sources once,
    # and 24 B of outputs per pixel (index, offset, two costs, range, z)
    W, H = fr.ref_cam.width, fr.ref_cam.height
    alg_bytes = float((1 + len(fr.srcs)) * W * H + 24 * W * H)
    line = {
        "metric": METRIC,
        "value": plane_pixels / (ms * 1e-3) / 1e9,
        "unit": "Gpix·planes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "step_ms_p10_p50_p90": [p10, p50, p90],
        "maps_per_s": 1e3 / ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"{args.storage}-staged/f32",
        "data": "synthetic (seeded ray-cast street scene)",
        "config": {"workload": "C2: 1024x768 ref + 3 fisheye sources (xi 0.9), 128 fronto + 64 ground planes, "
                               "ZNCC 9x9, mean of best 2, WTA + parabola",
                   "plane_pixels_per_step": plane_pixels, "plane_pixels_met_per_step": met_pixels,
                   "launch": args.launch, "storage": args.storage},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-ops/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel_ms": kernel_ms,
                     "ops_per_plane_pixel": ops_pp,
                     "work": "(pixel, plane) pairs whose pixel has a window and whose ray meets the plane",
                     "pairs": met_pixels,
                     "nominal": {"pairs": plane_pixels, "achieved": nominal, "frac": nominal / peak},
                     # not binding: the HBM side of the same launch, as fractions of 8 TB/s
                     "hbm": {"algorithmic_bytes": alg_bytes,
                             "algorithmic_frac": alg_bytes / (kernel_ms * 1e-3) / HBM_PEAK,
                             "counted_frac": None if traffic is None else traffic / (kernel_ms * 1e-3) / HBM_PEAK}},
    }
    ps.close()
    if not args.no_batched:
        # the batched form against the plain FP32 form (the metric's second
        # half): 16 mixed-size frames, FP16 staging, one persistent launch in a
        # HIP graph, tiles and chunks autotuned on the batch
        c5 = _C5()
        plain, pp5 = c5.plain_ms(max(3, args.steps // 10), 2)
        batched, choice = c5.batched_ms("f16", "persistent", max(3, args.steps // 10), 2)
        line["batched_vs_plain_f32"] = {
            "workload": "C5: 16 frame sets (6 x 1280x960, 5 x 1024x768, 5 x 640x480), 4 sources, two levels of "
                        "192 + 64 planes (7x7 low level, 9x9 centre crop)",
            "plain_f32_ms_per_batch": plain, "batched_ms_per_batch": batched,
            "batched_form": "persistent launch, FP16 staging, HIP graph", "autotuned": choice,
            "maps_per_s_plain": 16e3 / plain, "maps_per_s_batched": 16e3 / batched,
            "gpix_planes_per_s_batched": pp5 / (batched * 1e-3) / 1e9, "ratio": plain / batched}
    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(fr, st)
        # nominal plane-pixels count every pixel and plane; this many (pixel,
        # plane, source) windows were usable (estimated by the oracle sample)
        share = line["cpu_baseline"]["valid_source_evaluation_share"]
        line["config"]["valid_plane_pixel_source_evals_per_step"] = share * plane_pixels * len(fr.srcs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
