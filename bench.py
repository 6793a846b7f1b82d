#!/usr/bin/env python3
"""Throughput of transient path tracing on one MI355X.

One step = one transient render of the whole workload (every path sample
traced with BVH traversal, BSDF sampling and next-event estimation, every
contribution histogrammed into the pixel x time film), inputs resident in
HBM.  Headline workload (the largest configuration): the 998,608-triangle
fogged terrain with 49 displaced Lambertian / GGX spheres, 512x512 pinhole
film, 1024 bins of 5 mm from 4.5 m, 64 spp, max depth 8 (16,777,216 path
samples per step).

The JSON line also carries, each with its own rate and roofline, the
confocal NLOS scan (64x64 scan points, 9,680-triangle blob, 512 bins of
2.4 mm, 4096 spp; with its phasor film and NLOS area sampling), the batch of
256 confocal scenes rendered by one graph launch, the box room's latency
(graph replays), the glass room, and the backward/forward time ratio of the
differentiable box room; then the CPU oracle timed on a bounded sample of
the headline workload.
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
HBM_PEAK_GBPS = 8000.0

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
                       "from 4.5 m, 64 spp, max depth 8, FP32",
                  traffic="k_render_hbm_split_large_terrain_spheres_fog_512x512x1024_64spp_hbm_traffic.txt"),
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


def profile_fields(name):
    """The `key: value` lines of a committed rocprofv3 summary in profiles/,
    or None when there is none or the kernel sources changed after the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    fields = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    if fields.get("kernel_sources_sha1", "").strip() != h.hexdigest():
        return None
    return fields


def measured_traffic(workload):
    """HBM bytes per launch of the render kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (None when stale or absent)."""
    name = WORKLOADS[workload].get("traffic")
    fields = profile_fields(name) if name else None
    return int(float(fields["traffic_bytes_per_launch"])) if fields else None


def measured_issue(workload):
    """VALU issue of the render kernel from the committed SQ and memory-pipe
    summaries: the fraction of SIMD cycles issuing a VALU instruction
    (4 cycles per wave64 instruction on a 16-lane SIMD, 1,024 SIMDs,
    GRBM_GUI_ACTIVE / 8 cycles per XCD) and the fraction of lanes active in
    them; None when stale or absent."""
    name = WORKLOADS[workload].get("traffic")
    if not name:
        return None
    sq = profile_fields(name.replace("_hbm_traffic.txt", "_sq_counters.txt"))
    mem = profile_fields(name.replace("_hbm_traffic.txt", "_memory_pipe.txt"))
    if not sq or not mem:
        return None
    num = lambda f, k: float(f[k].split()[0])
    active = num(sq, "SQ_ACTIVE_INST_VALU")
    cycles = num(mem, "GRBM_GUI_ACTIVE") / 8
    return {"valu_issue_frac": round(4 * active / (1024 * cycles), 3),
            "active_lane_frac": round(num(sq, "SQ_THREAD_CYCLES_VALU") / (64 * active), 3),
            "source": "profiles/ (rocprofv3 SQ and GRBM counters of the same kernel sources)"}


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


def host_cpu():
    """Cores this process may run on, all cores of the host, and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return usable, os.cpu_count() or 1, model


def cpu_baseline(sc, stride_all=1, stride_one=16):
    """The unchanged oracle on the host cores over a bounded sample of the
    workload: one pixel (or scan point) in `stride_all` at the full spp on
    all usable cores, and one in `stride_one` on one thread."""
    import oracle
    usable, total, model = host_cpu()
    O = oracle.Oracle(sc)
    out = {}
    for label, stride, threads in (("all", stride_all, usable), ("one", stride_one, 1)):
        pix = np.arange(0, sc.n_pixels, stride, dtype=np.int32)
        t0 = time.perf_counter()
        O.render(pixels=pix, spp=sc.spp, threads=threads)
        dt = time.perf_counter() - t0
        out[label] = (len(pix), dt, threads)
    n_all, dt_all, th = out["all"]
    n_one, dt_one, _ = out["one"]

    def sample(stride, n):
        which = f"all {n} pixels" if stride == 1 else f"one pixel in {stride} ({n} of {sc.n_pixels})"
        return f"{which} at the full {sc.spp} spp"

    return {"value": round(n_all * sc.spp / dt_all / 1e6, 4), "unit": "Mpath-samples/s", "cores": th,
            "kind": "oracle", "sample": sample(stride_all, n_all) + ", threads over pixels",
            "seconds": round(dt_all, 2), "host_nproc": total, "host_usable_cores": usable, "host_cpu_model": model,
            "one_thread": {"value": round(n_one * sc.spp / dt_one / 1e6, 4), "unit": "Mpath-samples/s",
                           "sample": sample(stride_one, n_one), "seconds": round(dt_one, 2)}}


def roofline_of(counts, launch_ms, kernel, traffic=None, algorithmic_bytes=None):
    """VALU roofline of a render launch: algorithmic lane-ops (counted work x
    per-event cost) over the launch time, against 39.3 T lane-ops/s; with the
    HBM bytes per launch measured by rocprofv3 when they are current."""
    ops = sum(OPS_PER[k] * counts[k] for k in OPS_PER)
    achieved = ops / (launch_ms * 1e-3)
    r = {"bound": "alu", "achieved": round(achieved / 1e12, 4), "peak": round(PEAK_VALU_LANE_OPS / 1e12, 2),
         "unit": "T lane-ops/s", "frac": round(achieved / PEAK_VALU_LANE_OPS, 4), "traffic": traffic,
         "traffic_unit": "bytes/launch", "kernel": kernel, "launch_ms": round(launch_ms, 4), "ops_per_launch": int(ops),
         "counts": counts}
    if "wave_nodes" in counts:
        r["active_lanes_per_wave"] = active_lanes(counts)
    if algorithmic_bytes is not None:
        hb = {"algorithmic_bytes_per_launch": int(algorithmic_bytes),
              "algorithmic_gbps": round(algorithmic_bytes / (launch_ms * 1e-3) / 1e9, 2),
              "peak_gbps": HBM_PEAK_GBPS}
        hb["algorithmic_frac"] = round(hb["algorithmic_gbps"] / HBM_PEAK_GBPS, 5)
        if traffic:
            hb["measured_gbps"] = round(traffic / (launch_ms * 1e-3) / 1e9, 2)
            hb["measured_frac"] = round(hb["measured_gbps"] / HBM_PEAK_GBPS, 4)
            hb["measured_over_algorithmic"] = round(traffic / algorithmic_bytes, 2)
        r["hbm"] = hb
    return r


def algorithmic_bytes(sc, info):
    """Bytes the method itself must move per render: the film (and the steady
    image) written once, the scene (BVH nodes, triangle records, materials)
    read once."""
    film = sc.n_pixels * (sc.n_bins + 1) * 4
    return film + int(info["device_bytes"])


def measure_single(tr, name, args, shape, extras):
    """One workload: its rate, its counted work and its roofline (+ the
    workload's extra measurements when `extras`)."""
    import torch
    sc = make_scene(name)
    paths = sc.n_pixels * sc.spp
    # scene upload + BVH build (off the timed loop; the first build also warms the runtime, so time a second one)
    tr.upload(sc, builder=args.builder).destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev0 = tr.upload(sc, builder=args.builder)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t0) * 1e3
    dev0.destroy()
    out = {}
    with tr.upload(sc, builder=args.builder) as dev:
        info = dev.info()
        steady = torch.empty((sc.height, sc.width), device="cuda", dtype=torch.float32)
        film = torch.empty((sc.height, sc.width, sc.n_bins), device="cuda", dtype=torch.float32)
        step = lambda: tr.render_transient(dev, film=film, steady=steady, **shape)
        total_ms, per = time_launches(step, args.steps, args.warmup)
        _, _, counts = tr.render_transient_counted(dev, **shape)
        if args.compare_kernels:
            forms = {}
            for form in ("path", "deferred", "wavefront"):
                sh = dict(shape, kernel=form)
                ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady, **sh), args.steps,
                                      args.warmup)
                forms[form] = round(paths / (ms / args.steps * 1e-3) / 1e6, 3)
            out["kernel_forms_mpaths_per_s"] = forms
        if extras and not args.no_deterministic:
            # TRHIP_FLAG_DETERMINISTIC on the same workload (fixed-point sums,
            # bit-reproducible): a few renders
            n_det = max(2, args.steps // 4)
            ms, _ = time_launches(lambda: tr.render_transient(dev, film=film, steady=steady, deterministic=True),
                                  n_det, 1)
            out["deterministic"] = {"ms_per_step": round(ms / n_det, 4),
                                    "mpaths_per_s": round(paths / (ms / n_det * 1e-3) / 1e6, 3)}
        if extras and args.phasor_freqs and sc.sensor == 1:
            # the same paths into a phasor film (Sec. 4.3) instead of the histogram
            freqs = list(np.linspace(0.5, 16.6, args.phasor_freqs))
            ph = torch.empty((sc.height, sc.width, len(freqs), 2), device="cuda", dtype=torch.float32)
            ms, _ = time_launches(lambda: tr.render_phasor(dev, freqs, phasor=ph, steady=steady, **shape),
                                  args.steps, args.warmup)
            out["phasor_film"] = {"n_freq": len(freqs), "freq_range_per_m": [0.5, 16.6],
                                  "ms_per_step": round(ms / args.steps, 4),
                                  "mpaths_per_s": round(paths / (ms / args.steps * 1e-3) / 1e6, 3)}
        if extras and sc.sensor == 1 and sc.max_depth == 4 and not args.no_nlos_area:
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
            out["nlos_area_sampling"] = {
                "ms_per_step": round(ms / args.steps, 4),
                "mpaths_per_s": round(paths / (ms / args.steps * 1e-3) / 1e6, 3),
                "path_form_mpaths_per_s": round(paths / (ms_path / args.steps * 1e-3) / 1e6, 3),
                "variance_vs_cosine": round(diff[0] / diff[1], 5),
                "efficiency_vs_cosine": round((diff[1] / diff[0]) * (total_ms / ms), 3),
                "counts": area_counts}
    ms_per_step = total_ms / args.steps
    launch_ms = float(np.mean(per))
    form = args.kernel if args.kernel != "auto" else ("deferred" if sc.sensor == 1 else "path")
    kernel_name = {"path": "k_render", "deferred": "k_render_deferred", "wavefront": "k_render_wf"}[form]
    if form == "path" and sc.sensor == 0 and sc.n_bins >= 512 and sc.n_tris > 32768:
        # the path form keeps long films of large scenes in HBM, with split stacks up to 64 levels
        kernel_name = "k_render_hbm_split" if info["bvh_depth"] <= 64 else "k_render_hbm"
    res = {"value": round(paths / (ms_per_step * 1e-3) / 1e6, 3), "ms_per_step": round(ms_per_step, 4),
           "config": {"workload": WORKLOADS[name]["desc"], "paths_per_step": paths,
                      "triangles": info["n_triangles"], "bvh_depth": info["bvh_depth"]},
           "scene_upload_and_bvh_build_ms": round(upload_ms, 2),
           "roofline": roofline_of(counts, launch_ms, kernel_name, measured_traffic(name),
                                   algorithmic_bytes(sc, info))}
    issue = measured_issue(name)
    if issue:
        res["roofline"]["issue"] = issue
    res.update(out)
    return res, sc


def run_batched(args, tr, counted=True):
    """The batched workload: one graph launch renders all 256 scenes; its
    work counts are those of the scenes' single renders (same paths)."""
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
        counts = None
        if counted:
            counts = {}
            for d in devs:
                _, _, c = tr.render_transient_counted(d)
                for k, v in c.items():
                    counts[k] = counts.get(k, 0) + v
    finally:
        for d in devs:
            d.destroy()
    paths = sum(s.n_pixels * s.spp for s in scs)
    ms = total_ms / args.steps
    out = {"value": round(paths / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4),
           "config": {"workload": WORKLOADS["batched"]["desc"], "paths_per_step": paths,
                      "triangles": int(sum(s.n_tris for s in scs)), "batch": info}}
    if counts:
        out["roofline"] = roofline_of(counts, float(np.mean(per)), "k_batch")
    if seq is not None:
        out["sequential_single_scene_ms"] = round(seq, 3)
    return out


def json_line(value, ms, args, config, unit="Mpath-samples/s"):
    return {"metric": "Mpath-samples/s into transient film at 1 GPU; backward/forward time ratio",
            "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded scene generators)", "config": config}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS),
                    help="headline workload (default: the large scene, the largest configuration)")
    ap.add_argument("--only", action="store_true", help="measure the headline workload alone")
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
    ap.add_argument("--no-deterministic", action="store_true", help="skip the deterministic-sums measurement")
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
        b = run_batched(args, tr, counted=not args.only)
        out = json_line(b.pop("value"), b.pop("ms_per_step"), args, b.pop("config"))
        out.update(b)
        print(json.dumps(out), flush=True)
        return
    shape = dict(tile_pixels=args.tile_pixels, block_size=args.block_size, kernel=args.kernel)
    head, sc = measure_single(tr, args.workload, args, shape, extras=True)
    out = json_line(head.pop("value"), head.pop("ms_per_step"), args, head.pop("config"))
    out.update(head)
    if not args.only:
        if args.workload != "confocal":
            conf, _ = measure_single(tr, "confocal", args, dict(tile_pixels=0, block_size=0, kernel="auto"),
                                     extras=True)
            out["confocal"] = conf
        out["batched"] = run_batched(args, tr)
        out["glass_room"] = glass_room(tr, args.steps, args.warmup)
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
