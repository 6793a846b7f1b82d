#!/usr/bin/env python3
"""Throughput of transient path tracing on one MI355X.

One step = one transient render of the whole workload (every path sample
traced with BVH traversal, BSDF sampling and next-event estimation, every
contribution histogrammed into the pixel x time film), inputs resident in
HBM.  Default workload: confocal NLOS, 64x64 scan points on a 1x1 m relay
wall, 9,680-triangle hidden blob, 512 bins of 2.4 mm from 0.9 m, 4096 spp,
3 bounces (16,777,216 path samples per step).

Prints one JSON line: Mpath-samples/s, the backward/forward time ratio of
the differentiable box-room workload, the roofline of the render kernel and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T VALU lane-ops/s
# (non-packed FP32 / INT32; an FMA counts as one op).
PEAK_VALU_LANE_OPS = 256 * 64 * 2.4e9

# Algorithmic lane-ops per counted event, from the operation counts of the
# formulas the kernel evaluates (one add / mul / fma / min / max / compare /
# select / divide / square root / integer op = 1).
OPS_PER = {
    "nodes": 46,          # two slab tests (12 fma, 12 min/max, 8 reductions, 6 compares) + ordering
    "tris": 46,           # Moller-Trumbore + box-entry acceptance + closest/tie update
    "rays": 15,           # reciprocal direction (3 guards, 3 divides) and o/d (3 mul)
    "shadow_rays": 15,
    "vertices": 170,      # hit point, NEE geometry, normal, frame, BSDF, bin, continuation, offsets
    "draws": 112,         # Philox4x32-10 (10 rounds x 10 ops) + 4 uniform conversions
    "contributions": 12,  # contribution product, transmittance/scale, LDS add
}

WORKLOADS = {
    "confocal": dict(desc="confocal NLOS 64x64 scan, 9,682 tris (9,680-tri blob + 2-tri wall), 512 bins x 2.4 mm "
                          "from 0.9 m, 4096 spp, 3 bounces, FP32",
                     traffic="k_render_deferred_confocal_nlos_64x64x512_4096spp_hbm_traffic.txt"),
    "box": dict(desc="box room 34 tris, 64x64 pinhole, 256 bins x 0.01 m from 0, 16 spp, max depth 4, FP32"),
    "large": dict(desc="terrain + 49 displaced spheres 998,608 tris, fog sigma_t 0.1, 512x512, 1024 bins x 5 mm "
                       "from 4.5 m, 64 spp, max depth 8, FP32"),
    "glass": dict(desc="box room 34 tris with a glass box (index 1.5) and fluorescent room walls (scattering delay "
                       "mean 5 cm), 64x64 pinhole, 256 bins x 0.01 m from 0, 16 spp, max depth 8, FP32"),
    "batched": dict(desc="256 confocal NLOS scenes: blob triangles log-uniform 1k-50k, scan grids 16^2-64^2, "
                         "256-1024 bins x 2.4 mm from 0.9 m, 256 spp, 3 bounces, one graph launch, FP32"),
}


KERNEL_SOURCES = ["paper_2510_25660_amd/csrc/render.hip", "paper_2510_25660_amd/csrc/device_math.h",
                  "paper_2510_25660_amd/csrc/scene_view.h", "paper_2510_25660_amd/csrc/bvh.hip"]


def active_lanes(counts):
    """Mean active lanes (of 64) when a wave runs a node visit, a triangle
    test or a vertex, from the counting build's per-lane and per-wave counts."""
    return {k: round(counts[k] / counts["wave_" + w], 2) if counts["wave_" + w] else None
            for k, w in (("nodes", "nodes"), ("tris", "tris"), ("vertices", "vertices"))}


def measured_traffic(workload):
    """HBM bytes per launch of the render kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or the kernel
    sources changed after the counters were taken."""
    import hashlib
    name = WORKLOADS[workload].get("traffic")
    if not name:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    if fields.get("kernel_sources_sha1", "").strip() != h.hexdigest():
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def make_scene(name):
    from paper_2510_25660_amd import scenes
    if name == "confocal":
        return scenes.confocal_nlos()
    if name == "box":
        return scenes.box_scene()
    if name == "large":
        return scenes.large_scene()
    if name == "glass":
        return scenes.glass_box_scene(delay_mean=0.05)
    raise ValueError(name)


def time_launches(fn, steps, warmup):
    """Per-launch durations (ms) with HIP events on the launch stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_all0.record(stream)
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    return t_all0.elapsed_time(t_all1), per


def film_atomic_rate(film, sc, launch_ms, reps=20):
    """The deferred form splits a pixel's 4096 samples over two workgroups
    (2048-sample chunks) that add their partial films with HBM atomics: at
    most one float add per chunk and non-zero bin.  Their rate against a
    scatter-add (torch index_add_) of as many float adds at the same bins."""
    import torch
    chunks = max(1, -(-sc.spp // 2048))
    nz = torch.nonzero(film.reshape(-1)).reshape(-1)
    idx = nz.repeat(chunks)
    vals = torch.ones(idx.numel(), device="cuda", dtype=torch.float32)
    buf = torch.zeros(film.numel(), device="cuda", dtype=torch.float32)
    ms, _ = time_launches(lambda: buf.index_add_(0, idx, vals), reps, 3)
    per_launch = int(idx.numel())
    rate = per_launch / (launch_ms * 1e-3)
    peak = per_launch / (ms / reps * 1e-3)
    return {"per_launch_at_most": per_launch, "rate_per_s": round(rate, 1), "scatter_add_rate_per_s": round(peak, 1),
            "frac": round(rate / peak, 4)}


def backward_forward_ratio(tr, steps=5, warmup=1):
    """Backward (path-replay adjoint) over forward time on the differentiable
    box room (9,826 triangles, 64x64, 256 bins, 1024 spp, depth 4)."""
    import torch
    from paper_2510_25660_amd import scenes
    sc = scenes.diff_scene()
    with tr.upload(sc) as dev:
        a = torch.from_numpy(sc.albedo).cuda()
        r = torch.from_numpy(sc.roughness).cuda()
        _, film = tr.render_transient(dev, albedo=a, roughness=r)
        delta = torch.randn_like(film) * 1e-3
        fwd_ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, albedo=a, roughness=r), steps, warmup)
        bwd_ms, _ = time_launches(lambda: tr.render_transient_backward(dev, delta, albedo=a, roughness=r), steps,
                                  warmup)
        rep_ms, _ = time_launches(lambda: tr.render_transient_backward(dev, delta, albedo=a, roughness=r,
                                                                       kernel="path"), steps, warmup)
        # forward mode along one parameter: the roughness of the two boxes
        v = (torch.from_numpy(sc.mat_type) == scenes.MAT_GGX).float().cuda()
        dfilm = torch.empty_like(film)
        tan_ms, _ = time_launches(lambda: tr.render_transient_tangent(dev, None, v, film=film, dfilm=dfilm, albedo=a,
                                                                      roughness=r), steps, warmup)
    return bwd_ms / fwd_ms, fwd_ms / steps, bwd_ms / steps, rep_ms / steps, tan_ms / steps


def run_batched(args, tr):
    """The batched workload: one graph launch renders all 256 scenes."""
    import torch
    from paper_2510_25660_amd import scenes
    scs = scenes.batched_nlos()
    devs = [tr.upload(s) for s in scs]
    try:
        b = tr.Batch(devs, autotune=True)
        info = b.info()
        total_ms, per = time_launches(b.render, args.steps, args.warmup)
        seq = None
        if args.compare_kernels:
            films = b.films
            seq_ms, _ = time_launches(lambda: [tr.render_transient(d, film=f) for d, f in zip(devs, films)],
                                      max(1, args.steps // 4), 1)
            seq = seq_ms / max(1, args.steps // 4)
        b.destroy()
    finally:
        for d in devs:
            d.destroy()
    paths = sum(s.n_pixels * s.spp for s in scs)
    ms = total_ms / args.steps
    out = {
        "metric": "Mpath-samples/s into transient film at 1 GPU; backward/forward time ratio",
        "value": round(paths / (ms * 1e-3) / 1e6, 3), "unit": "Mpath-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded scene generators)",
        "config": {"workload": WORKLOADS["batched"]["desc"], "paths_per_step": paths,
                   "triangles": int(sum(s.n_tris for s in scs)), "batch": info},
    }
    if seq is not None:
        out["sequential_single_scene_ms"] = round(seq, 3)
    return out


def box_room_graph(tr, replays=200):
    """The box-room workload (65,536 paths: too small to fill the GPU, so
    launch overhead matters): one render captured in a hipGraph, GPU time of
    each of `replays` replays; median and per-render latency."""
    import torch
    sc = make_scene("box")
    with tr.upload(sc) as dev:
        film = torch.empty((sc.height, sc.width, sc.n_bins), device="cuda", dtype=torch.float32)
        steady = torch.empty((sc.height, sc.width), device="cuda", dtype=torch.float32)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(3):
                tr.render_transient(dev, film=film, steady=steady)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            tr.render_transient(dev, film=film, steady=steady)
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(replays)]
        for _ in range(5):
            graph.replay()
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            graph.replay()
            b.record(stream)
        torch.cuda.synchronize()
        per_us = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
        del graph
    med = per_us[len(per_us) // 2]
    return {"workload": WORKLOADS["box"]["desc"], "replays": replays, "median_us": round(med, 2),
            "min_us": round(per_us[0], 2), "max_us": round(per_us[-1], 2),
            "mpaths_per_s": round(sc.n_pixels * sc.spp / (med * 1e-6) / 1e6, 3)}


def glass_room(tr, steps, warmup):
    """The glass-box room (dielectric interfaces, Eq. 3; scattering delays,
    Eq. 10): Mpath-samples/s of the path form."""
    import torch
    sc = make_scene("glass")
    with tr.upload(sc) as dev:
        film = torch.empty((sc.height, sc.width, sc.n_bins), device="cuda", dtype=torch.float32)
        steady = torch.empty((sc.height, sc.width), device="cuda", dtype=torch.float32)
        ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady), 4 * steps, warmup)
        _, _, counts = tr.render_transient_counted(dev)
    ms /= 4 * steps
    return {"workload": WORKLOADS["glass"]["desc"], "ms_per_step": round(ms, 4),
            "mpaths_per_s": round(sc.n_pixels * sc.spp / (ms * 1e-3) / 1e6, 3), "counts": counts}


def cpu_baseline(sc, max_threads=16):
    """The oracle on the host cores over a bounded sample of the workload."""
    import oracle
    threads = max(1, min(max_threads, os.cpu_count() or 1))
    O = oracle.Oracle(sc)
    if sc.sensor == 1:
        pix = np.arange(sc.n_pixels, dtype=np.int32)
        spp = sc.spp
        sample = f"the whole workload: all {sc.n_pixels} scan points at the full {spp} spp"
    else:
        pix = np.arange(0, sc.n_pixels, max(1, sc.n_pixels // 4096), dtype=np.int32)
        spp = min(sc.spp, 16)
        sample = f"{len(pix)} of {sc.n_pixels} pixels at {spp} spp"
    t0 = time.perf_counter()
    O.render(pixels=pix, spp=spp, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(len(pix) * spp / dt / 1e6, 4), "unit": "Mpath-samples/s", "cores": threads,
            "kind": "oracle", "sample": sample, "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="confocal", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--tile-pixels", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--kernel", default="auto", choices=["auto", "path", "deferred", "wavefront"])
    ap.add_argument("--compare-kernels", action="store_true", help="also time each kernel form")
    ap.add_argument("--builder", default="ploc", choices=["ploc", "lbvh"])
    ap.add_argument("--phasor-freqs", type=int, default=16,
                    help="also time the frequency-space film with this many frequencies (0: skip)")
    ap.add_argument("--no-nlos-area", action="store_true", help="skip the NLOS area-sampling measurement")
    ap.add_argument("--no-glass", action="store_true", help="skip the glass-room measurement")
    ap.add_argument("--no-box-graph", action="store_true", help="skip the graph-replayed box-room latency")
    ap.add_argument("--atomic-calibration", action="store_true",
                    help="compare the render's film atomics with a scatter-add of as many float adds at the same bins")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a device copy of this many MiB (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the renderer runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the path would shard by pixel tiles or sample ranges)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_25660_amd as tr
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batched":
        print(json.dumps(run_batched(args, tr)), flush=True)
        return
    sc = make_scene(args.workload)
    shape = dict(tile_pixels=args.tile_pixels, block_size=args.block_size, kernel=args.kernel)
    paths = sc.n_pixels * sc.spp
    # scene upload + BVH build (off the timed loop; the first build also warms the runtime, so time a second one)
    tr.upload(sc, builder=args.builder).destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev0 = tr.upload(sc, builder=args.builder)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    dev0.destroy()
    with tr.upload(sc, builder=args.builder) as dev:
        info = dev.info()
        steady = torch.empty((sc.height, sc.width), device="cuda", dtype=torch.float32)
        film = torch.empty((sc.height, sc.width, sc.n_bins), device="cuda", dtype=torch.float32)
        step = lambda: tr.render_transient(dev, film=film, steady=steady, **shape)
        total_ms, per = time_launches(step, args.steps, args.warmup)
        _, _, counts = tr.render_transient_counted(dev, **shape)
        forms = {}
        if args.compare_kernels:
            for form in ("path", "deferred", "wavefront"):
                sh = dict(shape, kernel=form)
                ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady, **sh), args.steps,
                                      args.warmup)
                forms[form] = round(paths / (ms / args.steps * 1e-3) / 1e6, 3)
        phasor = None
        if args.phasor_freqs:
            # the same paths into a phasor film (Sec. 4.3) instead of the histogram
            freqs = list(np.linspace(0.5, 16.6, args.phasor_freqs))
            ph = torch.empty((sc.height, sc.width, len(freqs), 2), device="cuda", dtype=torch.float32)
            ms, _ = time_launches(lambda: tr.render_phasor(dev, freqs, phasor=ph, steady=steady, **shape),
                                  args.steps, args.warmup)
            phasor = {"n_freq": len(freqs), "freq_range_per_m": [0.5, 16.6], "ms_per_step": round(ms / args.steps, 4),
                      "mpaths_per_s": round(paths / (ms / args.steps * 1e-3) / 1e6, 3)}
        nlos = None
        if sc.sensor == 1 and sc.max_depth == 4 and not args.no_nlos_area:
            # NLOS area sampling of the hidden vertex (Sec. 4.5) on the same
            # scan: its rate, and the variance of the steady image relative
            # to the default cosine sampling at equal spp (from the squared
            # differences of two independent renders of each estimator)
            ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady, nlos_area=True),
                                  args.steps, args.warmup)
            ms_path, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady, nlos_area=True,
                                                                   kernel="path"), args.steps, args.warmup)
            _, _, area_counts = tr.render_transient_counted(dev, nlos_area=True)
            diff = []
            for area in (True, False):
                a = tr.render_transient(dev, seed=11, nlos_area=area)[0].double()
                b = tr.render_transient(dev, seed=12, nlos_area=area)[0].double()
                diff.append(float(((a - b) ** 2).mean()))
            nlos = {"ms_per_step": round(ms / args.steps, 4),
                    "mpaths_per_s": round(paths / (ms / args.steps * 1e-3) / 1e6, 3),
                    "path_form_mpaths_per_s": round(paths / (ms_path / args.steps * 1e-3) / 1e6, 3),
                    "variance_vs_cosine": round(diff[0] / diff[1], 5),
                    "efficiency_vs_cosine": round((diff[1] / diff[0]) * (total_ms / ms), 3),
                    "counts": area_counts}
    ms_per_step = total_ms / args.steps
    value = paths / (ms_per_step * 1e-3) / 1e6
    launch_ms = float(np.mean(per))
    # the deferred form adds split pixels' partial films with HBM atomics
    form = args.kernel if args.kernel != "auto" else ("deferred" if sc.sensor == 1 else "path")
    atomics = (film_atomic_rate(film, sc, launch_ms)
               if args.atomic_calibration and form == "deferred" and sc.spp > 2048 else None)
    ops = sum(OPS_PER[k] * counts[k] for k in OPS_PER)
    # the kernel the automatic choice runs: the deferred form for the confocal sensor
    kernel_name = {"path": "k_render", "deferred": "k_render_deferred", "wavefront": "k_render_wf"}[form]
    achieved = ops / (launch_ms * 1e-3)
    out = {
        "metric": "Mpath-samples/s into transient film at 1 GPU; backward/forward time ratio",
        "value": round(value, 3),
        "unit": "Mpath-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scene generators)",
        "config": {"workload": WORKLOADS[args.workload]["desc"], "paths_per_step": paths,
                   "triangles": info["n_triangles"], "bvh_depth": info["bvh_depth"]},
        "scene_upload_and_bvh_build_ms": round(upload_ms, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(PEAK_VALU_LANE_OPS / 1e12, 2),
                     "unit": "T lane-ops/s", "frac": round(achieved / PEAK_VALU_LANE_OPS, 4),
                     "traffic": measured_traffic(args.workload), "traffic_unit": "bytes/launch",
                     "kernel": kernel_name, "launch_ms": round(launch_ms, 4),
                     "ops_per_launch": int(ops), "counts": counts,
                     "active_lanes_per_wave": active_lanes(counts)},
    }
    if forms:
        out["kernel_forms_mpaths_per_s"] = forms
    if atomics:
        out["film_atomics"] = atomics
    if phasor:
        out["phasor_film"] = phasor
    if nlos:
        out["nlos_area_sampling"] = nlos
    if args.workload == "confocal" and not args.no_glass:
        out["glass_room"] = glass_room(tr, args.steps, args.warmup)
    if args.workload == "confocal" and not args.no_box_graph:
        out["box_room_graph"] = box_room_graph(tr)
    if not args.no_backward:
        ratio, f_ms, b_ms, rep_ms, t_ms = backward_forward_ratio(tr)
        out["backward_forward_ratio"] = round(ratio, 3)
        out["backward_forward_ms"] = [round(f_ms, 3), round(b_ms, 3)]
        out["backward_replay_ms"] = round(rep_ms, 3)
        out["forward_mode_ms"] = round(t_ms, 3)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
