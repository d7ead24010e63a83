"""Benchmark: exact order-independent transparency of quad scenes on one
MI355X.

A step is one whole frame of the path -- setup, binning, sorted
rasterization (block sort + per-pixel sorter, depth slices for dense blocks)
and the exact per-pixel pass -- over a scene resident in HBM.  The headline
frame is the 1920x1080 one with 1M quads in a Gaussian cloud (106 M
fragments), at the tuning the library's rule table picks for it.  The
unsorted compute blend (the "1.00" reference of the paper's comparison) is
timed the same way on the same GPU.  Side legs: the 1280x720 200k-quad frame
(rule table and online-tuned), a 64-frame mixed batch and the serving loop.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mfrags/s & frames/s vs unsorted compute blend; p50/p99 ms; ≤1 LSB vs oracle"
HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_2405_13364_amd", "csrc", "lr_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

WORKLOADS = {
    "c2": "1280x720, 200k quads 2-8 px uniform on screen, z U[1,50], alpha U[0.1,0.9], seed 1",
    "c2b": "1280x720, 200k quads 4-16 px uniform on screen, z U[1,50], alpha U[0.1,0.9], seed 1",
    "c3": "1920x1080, 1M quads 1-30 px in a Gaussian cloud (sigma 0.15 screen), z U[1,10], "
          "alpha U[0.05,0.5], seed 2",
    "c1": "256x256, 1k quads 4-40 px, z U[1,10], alpha U[0.2,0.8], seed 0",
    "c3o": "1920x1080, 1M quads 1-30 px in a Gaussian cloud (sigma 0.15 screen), z U[1,10], "
           "alpha U[0.8,1.0], seed 2",
}

KERNELS = {"setup": "k_setup", "bin_count": "k_bin_count4 (k_bin_count past 8192 bins)", "bin_scan": "k_bin_scan",
           "bin_scatter": "k_bin_scatter4 (k_bin_scatter past 8192 bins)", "raster": "k_raster",
           "fallback": "k_fallback"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(stage, n, visible, pairs, W, H):
    """Bytes the method must move per launch of a stage: quads are 52 bytes
    in, setup records 72 bytes (snapped vertices, plane, bbox, colour, id),
    bboxes 8 bytes, bin list entries 4 bytes, RGBA8 pixels 4 bytes."""
    if stage == "setup":
        return 52 * n + 72 * visible
    if stage == "bin_count":
        return 8 * visible
    if stage == "bin_scatter":
        return 8 * visible + 4 * pairs
    if stage == "raster":
        return pairs * (4 + 72) + 4 * W * H
    return None


def algorithmic_lane_ops(fragments, entries):
    """VALU lane operations the sorted raster needs per frame: about 40 per
    fragment (plane key, K-sorter insert, front-to-back blend) and about 4
    per block entry and pixel lane (coverage bit tests and mask handling)."""
    return 40 * fragments + 4 * 64 * entries


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(workload, stage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, and
    the tuning the counters were taken on, if they were taken on the current
    kernel source; else (None, None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    entry = t.get(workload, {}).get(stage)
    if not entry or entry.get("kernel_source_sha") != kernel_source_hash():
        return None, None
    return entry.get("bytes_per_launch"), entry.get("tuning")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, min_seconds):
    """The oracle (test infrastructure, untuned) on the host: whole frames on
    all the cores this process may use (row bands, at most 16 threads), then
    one whole frame on one core."""
    import oracle
    oracle.build(force=False)
    threads = oracle.default_threads()
    reps, t0, total = 0, time.perf_counter(), 0
    ref = None
    while True:
        res = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False, threads=threads)
        reps += 1
        total += res["total"]
        ref = res
        if time.perf_counter() - t0 >= min_seconds:
            break
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    one = oracle.render(sc.v, sc.rgba, sc.camera, sc.width, sc.height, want_order=False, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": round(total / dt / 1e6, 3), "unit": "Mfrags/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} full {sc.width}x{sc.height} frame(s) of the bench workload on {threads} threads "
                      f"({dt:.1f} s), then 1 full frame on 1 thread ({dt1:.1f} s)",
            "all_cores": {"cores": threads, "value": round(total / dt / 1e6, 3),
                          "frames_per_s": round(reps / dt, 4)},
            "one_core": {"cores": 1, "value": round(one["total"] / dt1 / 1e6, 3),
                         "frames_per_s": round(1.0 / dt1, 4)},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}, ref


def time_steps(torch, fn, steps, warmup):
    """Milliseconds for `steps` back-to-back calls, one event pair around all of them."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t_begin = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_begin.record()
    for _ in range(steps):
        fn()
    t_end.record()
    torch.cuda.synchronize()
    return t_begin.elapsed_time(t_end)


def step_latencies(torch, fn, steps):
    """Per-call device milliseconds (an event pair around each call)."""
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        starts[k].record()
        fn()
        ends[k].record()
    torch.cuda.synchronize()
    return np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])


def calibrate_copy(mib):
    """A plain device-to-device copy of known size, run under rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters to scale them to bytes."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": n, "bytes_written": n, "launches": 4}),
          flush=True)


def mixed_batch_leg(torch, lucidraster, scenes, rules, reps, log):
    """64 frames of uneven size, count and shape (seeds 1000..1063): one
    batched call (graph replay, and direct launches) against 64 sequential
    renders with the same tuning."""
    frames = [scenes.mixed_scene(1000 + i) for i in range(64)]
    res = {"frames": 64, "quads": int(sum(s.n for s in frames)), "tuning": "autotuned" if rules else "default",
           "workload": "64 frames, seeds 1000-1063: size from {256x256, 640x480, 1280x720, 1920x1080}, "
                       "quads log-uniform 1k-500k, shape of the 256x256, 1280x720 or 1920x1080 workload"}
    arena = 24 << 30
    ctxs = {"graph": lucidraster.Context(arena_bytes=arena, tuning=rules, graphs=True),
            "direct": lucidraster.Context(arena_bytes=arena, tuning=rules, graphs=False)}
    outs_seq = None
    for mode, ctx in ctxs.items():
        hs = [ctx.upload(s.v, s.rgba) for s in frames]
        outs = [ctx.new_image(s.width, s.height) for s in frames]
        reqs = [(h, s.camera, s.width, s.height, o) for h, s, o in zip(hs, frames, outs)]
        ctx.render_batch(reqs)  # plans capacities, captures the graph
        ctx.render_batch(reqs)
        frags = ctx.stats()["fragments"]
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            ctx.render_batch(reqs, check=False)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ctx.sync()
        ms = float(np.median(ts))
        res[f"batch_{mode}"] = {"ms": round(ms, 4), "frames_per_s": round(64e3 / ms, 2),
                                "Mfrags_per_s": round(frags / (ms * 1e-3) / 1e6, 3)}
        if mode == "graph":
            # the same 64 frames rendered one at a time
            seq = [ctx.new_image(s.width, s.height) for s in frames]
            for h, s, o in zip(hs, frames, seq):
                ctx.render(h, s.camera, s.width, s.height, out=o)
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for h, s, o in zip(hs, frames, seq):
                    ctx.render(h, s.camera, s.width, s.height, out=o, check=False)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b))
            ctx.sync()
            ms_s = float(np.median(ts))
            res["sequential"] = {"ms": round(ms_s, 4), "frames_per_s": round(64e3 / ms_s, 2),
                                 "Mfrags_per_s": round(frags / (ms_s * 1e-3) / 1e6, 3)}
            res["batch_equals_single"] = all(bool((o == q).all()) for o, q in zip(outs, seq))
            res["fragments"] = int(frags)
        log(f"batch {mode}: {ms:.3f} ms for 64 frames")
        ctx.close()
    res["batch_over_sequential"] = round(res["sequential"]["ms"] / res["batch_graph"]["ms"], 3)
    return res


def serving_leg(torch, lucidraster, scenes, rules, n_scenes, n_req, log):
    """Poisson arrivals over resident mixed scenes: continuous batching on two
    stream slots vs one-at-a-time, at fractions of the one-at-a-time capacity."""
    from paper_2405_13364_amd import serving
    ctx = lucidraster.Context(arena_bytes=40 << 30, tuning=rules, graphs=False, batch_slots=2)
    meta = []
    for s in range(n_scenes):
        sc = scenes.mixed_scene(2000 + s)
        meta.append((ctx.upload(sc.v, sc.rgba), sc.width, sc.height))
    cam = scenes.Camera()
    for h, W, H in meta:  # warm-up and capacity planning
        ctx.render(h, cam, W, H)
    # one-at-a-time service time: every scene once, back to back
    outs = {(W, H): ctx.new_image(W, H) for _, W, H in meta}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, W, H in meta:
        ctx.render(h, cam, W, H, out=outs[(W, H)], check=False)
    torch.cuda.synchronize()
    service_ms = (time.perf_counter() - t0) * 1e3 / len(meta)
    cap = 1e3 / service_ms
    res = {"scenes": n_scenes, "requests_per_rate": n_req, "service_ms_alone": round(service_ms, 4),
           "capacity_frames_per_s": round(cap, 2), "budget_bytes": 8 << 30,
           "workload": f"{n_scenes} resident scenes (seeds 2000+), Poisson arrivals (seed 3000), camera "
                       "yaw/pitch jitter U[-2, 2] deg"}
    modes = {"one_at_a_time": (1, 1), "continuous": (2, 16)}
    for mode, (slots, mb) in modes.items():
        rows = []
        for frac in (0.5, 0.8, 0.95, 1.1):
            trace = serving.poisson_trace(frac * cap, n_req, meta, seed=3000)
            be = serving.GpuBackend(ctx, slots, keep_every=97 if mode == "continuous" and frac == 0.95 else 0)
            srv = serving.Server(be, 8 << 30, slots=slots, max_batch=mb)
            be.start_clock()
            done = srv.run(trace)
            ctx.sync()
            row = {"rate_frac": frac, "offered_per_s": round(frac * cap, 2)}
            row.update(serving.summarize(done))
            rows.append(row)
            if be.outputs:
                ok = True
                for r in trace:
                    if r.rid in be.outputs:
                        alone = ctx.render(r.scene, r.camera, r.width, r.height)
                        ok = ok and bool((alone == be.outputs[r.rid]).all())
                res["served_equal_alone"] = {"checked": len(be.outputs), "equal": ok}
            log(f"serving {mode} at {frac:.2f} x capacity: {row['frames_per_s']} frames/s, "
                f"p50 {row['p50_ms']} ms, p99 {row['p99_ms']} ms, {row['batches']} batches")
        # saturation: every request present at t = 0
        trace = serving.poisson_trace(1e9, n_req, meta, seed=3001)
        be = serving.GpuBackend(ctx, slots)
        be.start_clock()
        done = serving.Server(be, 8 << 30, slots=slots, max_batch=mb).run(trace)
        ctx.sync()
        res[mode] = {"rates": rows, "saturated": serving.summarize(done)}
    res["saturated_speedup"] = round(res["continuous"]["saturated"]["frames_per_s"] /
                                     res["one_at_a_time"]["saturated"]["frames_per_s"], 3)
    ctx.close()
    return res


def variant_rows(torch, lucidraster, sc, tune, variants, steps, warmup, arena):
    """Frame time and statistics of one frame under several context options
    (same tuning), each timed back to back like the headline."""
    b, k, bh = tune
    rows = {}
    for label, opts in variants.items():
        ctx = lucidraster.Context(arena_bytes=arena, bin_size=b, sorter_depth=k, block_h=bh, **opts)
        h = ctx.upload(sc.v, sc.rgba)
        out = ctx.new_image(sc.width, sc.height)
        ctx.render(h, sc.camera, sc.width, sc.height, out=out)
        st = ctx.stats()
        ms = time_steps(torch, lambda: ctx.render(h, sc.camera, sc.width, sc.height, out=out, check=False),
                        steps, warmup) / steps
        ctx.sync()
        rows[label] = {"ms_per_frame": round(ms, 5), "frames_per_s": round(1000.0 / ms, 2),
                       "bin_pairs": int(st["bin_pairs"]), "fragments_processed": int(st["fragments"]),
                       "flagged_pixels": int(st["flagged_pixels"]), "image": out.cpu()}
        ctx.close()
    ref = next(iter(rows.values()))["image"]
    for row in rows.values():
        row["max_lsb_vs_first"] = int((row.pop("image").to(torch.int32) - ref.to(torch.int32)).abs().max().item())
    return rows


def large_quads_leg(torch, lucidraster, autotune, rules, steps, warmup, arena, log):
    """The large-primitive path: the 1280x720 frame plus 4,000 long thin
    quads (2% of the quads, 300-700 px by 3-8 px, turned in the screen plane),
    binned by their kept bins vs by their whole bbox (LR_FLAG_BBOX_BINNING)."""
    from paper_2405_13364_amd import scenes
    sc = scenes.with_long_quads(scenes.scene("c2"), 4000, 7)
    tune = tuple(autotune.resolve(rules, sc.width, sc.height, sc.n))
    rows = variant_rows(torch, lucidraster, sc, tune, {"large_path": {}, "bbox_binning": {"bbox_binning": True}},
                        steps, warmup, arena)
    res = {"workload": "1280x720: the 200k-quad frame plus 4,000 quads of 300-700 x 3-8 px turned in the screen "
                       "plane (seed 7)", "tuning": f"bin {tune[0]}, K {tune[1]}, 8x{tune[2]}", **rows,
           "speedup": round(rows["bbox_binning"]["ms_per_frame"] / rows["large_path"]["ms_per_frame"], 3)}
    log(f"large quads: {rows['large_path']['ms_per_frame']:.4f} ms vs bbox binning "
        f"{rows['bbox_binning']['ms_per_frame']:.4f} ms")
    return res


def classes_leg(torch, lucidraster, steps, warmup, arena, log):
    """Density classes (LR_FLAG_DENSITY_CLASSES, off by default) on the
    1920x1080 cloud at bin 16 and bin 32, sorter depth 8."""
    from paper_2405_13364_amd import scenes
    sc = scenes.scene("c3")
    res = {"workload": f"c3: {WORKLOADS['c3']}"}
    for tune in ((16, 8, 8), (32, 8, 8)):
        rows = variant_rows(torch, lucidraster, sc, tune, {"one_class": {}, "classes": {"density_classes": True}},
                            steps, warmup, arena)
        res[f"bin {tune[0]}, K {tune[1]}, 8x{tune[2]}"] = rows
        log(f"density classes at bin {tune[0]}: {rows['classes']['ms_per_frame']:.4f} ms vs one class "
            f"{rows['one_class']['ms_per_frame']:.4f} ms")
    return res


def cutoff_leg(torch, lucidraster, autotune, rules, steps, warmup, arena, log):
    """The transmittance cutoff (LR_FLAG_ALPHA_CUTOFF) against the exact
    blend, at the rule-table tuning: the 1920x1080 cloud (alpha U[0.05, 0.5])
    and the same cloud with alpha U[0.8, 1.0]."""
    from paper_2405_13364_amd import scenes
    res = {"note": "ms per frame, exact blend vs transmittance cutoff (stop below 2^-20); fragments = "
                   "fragments processed by the raster and the exact pass"}
    for name in ("c3", "c3o"):
        sc = scenes.scene(name)
        b, k, bh = autotune.resolve(rules, sc.width, sc.height, sc.n)
        row = {"workload": f"{name}: {WORKLOADS[name]}", "tuning": f"bin {b}, K {k}, 8x{bh}"}
        for mode in ("exact", "cutoff"):
            ctx = lucidraster.Context(arena_bytes=arena, bin_size=b, sorter_depth=k, block_h=bh,
                                      alpha_cutoff=(mode == "cutoff"))
            h = ctx.upload(sc.v, sc.rgba)
            out = ctx.new_image(sc.width, sc.height)
            ctx.render(h, sc.camera, sc.width, sc.height, out=out)
            st = ctx.stats()
            ms = time_steps(torch, lambda: ctx.render(h, sc.camera, sc.width, sc.height, out=out, check=False),
                            steps, warmup) / steps
            ctx.sync()
            row[mode] = {"ms_per_frame": round(ms, 5), "frames_per_s": round(1000.0 / ms, 2),
                         "fragments_processed": int(st["fragments"]),
                         "flagged_pixels": int(st["flagged_pixels"])}
            if mode == "cutoff":
                row["max_lsb_vs_exact"] = int((out.to(torch.int32) - ref_img.to(torch.int32)).abs().max().item())
            else:
                ref_img = out.clone()
            ctx.close()
        row["speedup"] = round(row["exact"]["ms_per_frame"] / row["cutoff"]["ms_per_frame"], 3)
        log(f"cutoff {name}: exact {row['exact']['ms_per_frame']:.4f} ms, cutoff {row['cutoff']['ms_per_frame']:.4f} ms")
        res[name] = row
    return res


def frame_leg(torch, lucidraster, autotune, sc, workload, tune, tuning_note, steps, warmup, arena):
    """Sorted and unsorted frame times of one workload at one tuning, and the
    dominant kernel's roofline from a pass with events between stages."""
    W, H = sc.width, sc.height
    b, k, bh = tune
    ctx = lucidraster.Context(arena_bytes=arena, bin_size=b, sorter_depth=k, block_h=bh)
    h = ctx.upload(sc.v, sc.rgba)
    out = ctx.new_image(W, H)
    # first frame sizes the workspace (and re-plans bin capacity if needed)
    ctx.render(h, sc.camera, W, H, out=out)
    st = ctx.stats()
    log(f"{workload}: {st['fragments']} fragments, {st['bin_pairs']} bin pairs, {st['block_entries']} block "
        f"entries, {st['flagged_pixels']} flagged pixels, {st['dense_blocks']} blocks in depth slices")
    sorted_fn = lambda: ctx.render(h, sc.camera, W, H, out=out, check=False)
    log(f"{workload}: timing sorted render, {warmup} warmup + {steps} steps")
    ms = time_steps(torch, sorted_fn, steps, warmup) / steps
    ctx.sync()
    per = step_latencies(torch, sorted_fn, steps)
    ctx.sync()
    st = ctx.stats()
    frags = st["fragments"]
    log(f"{workload}: timing unsorted compute blend")
    out_u = ctx.new_image(W, H)
    unsorted_fn = lambda: ctx.render_unsorted(h, sc.camera, W, H, out=out_u, check=False)
    ms_u = time_steps(torch, unsorted_fn, steps, warmup) / steps
    ctx.sync()
    per_u = step_latencies(torch, unsorted_fn, steps)
    ctx.sync()
    ctx.close()

    # per-stage times: HIP events recorded on the launch stream around every
    # stage of each timed frame (a separate pass: the events themselves add
    # time between kernels, so the frame times above are measured without them)
    log(f"{workload}: timing stages")
    ctx_t = lucidraster.Context(arena_bytes=arena, bin_size=b, sorter_depth=k, block_h=bh, timing=True)
    h_t = ctx_t.upload(sc.v, sc.rgba)
    ctx_t.render(h_t, sc.camera, W, H, out=out)
    time_steps(torch, lambda: ctx_t.render(h_t, sc.camera, W, H, out=out, check=False), steps, warmup)
    ctx_t.sync()
    stage = ctx_t.stage_times(steps)  # the timed frames
    ctx_t.close()
    ms_staged = float(stage[:, 7].mean()) / 1e3
    names = lucidraster.STAGES[:7]
    avg_us = {nm: float(stage[:, i].mean()) for i, nm in enumerate(names) if nm != "unused"}
    dom = max(avg_us, key=avg_us.get)
    if algorithmic_bytes(dom, sc.n, st["visible"], st["bin_pairs"], W, H) is None:
        dom = "raster"
    nbytes = algorithmic_bytes(dom, sc.n, st["visible"], st["bin_pairs"], W, H)
    achieved = nbytes / (avg_us[dom] * 1e-6) / 1e9
    hbm = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 5), "algorithmic_bytes": int(nbytes)}
    traffic, traffic_tuning = measured_traffic(workload, dom)
    if traffic is not None and traffic_tuning != f"bin {b}, K {k}, 8x{bh}":
        traffic, traffic_tuning = None, None
    if dom == "raster":
        # the raster is bound by VALU issue, not by HBM: its roofline is the
        # ALU one, with the HBM view beside it
        ops = algorithmic_lane_ops(frags, st["block_entries"])
        a_ops = ops / (avg_us[dom] * 1e-6) / 1e12
        roofline = {"bound": "alu", "achieved": round(a_ops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                    "unit": "T lane-op/s", "frac": round(a_ops / ALU_PEAK_TOPS, 5),
                    "traffic": traffic, "traffic_tuning": traffic_tuning,
                    "kernel": KERNELS[dom], "kernel_avg_us": round(avg_us[dom], 3),
                    "algorithmic_lane_ops": int(ops), "fragments": int(frags),
                    "block_entries": int(st["block_entries"]), "bin_pairs": int(st["bin_pairs"]),
                    "hbm_view": hbm}
    else:
        roofline = dict(hbm, traffic=traffic, traffic_tuning=traffic_tuning, kernel=KERNELS[dom],
                        kernel_avg_us=round(avg_us[dom], 3))
    return {
        "ms": ms, "frags": int(frags), "stats": st, "out": out,
        "line": {
            "workload": f"{workload}: {WORKLOADS[workload]}", "tuning": f"bin {b}, K {k}, 8x{bh}",
            "tuning_note": tuning_note, "fragments": int(frags), "visible_quads": int(st["visible"]),
            "ms_per_frame": round(ms, 5), "Mfrags_per_s": round(frags / (ms * 1e-3) / 1e6, 3),
            "frames_per_s": round(1000.0 / ms, 2),
            "p50_ms": round(float(np.percentile(per, 50)), 5), "p99_ms": round(float(np.percentile(per, 99)), 5),
            "unsorted": {"ms_per_step": round(ms_u, 5), "Mfrags_per_s": round(frags / (ms_u * 1e-3) / 1e6, 3),
                         "frames_per_s": round(1000.0 / ms_u, 2),
                         "p50_ms": round(float(np.percentile(per_u, 50)), 5),
                         "p99_ms": round(float(np.percentile(per_u, 99)), 5)},
            "sorted_over_unsorted": round(ms / ms_u, 3),
            "stage_us": {kk: round(v, 3) for kk, v in avg_us.items()},
            "stage_note": "stage times from a pass with HIP events between stages; that pass's frames take "
                          f"{ms_staged:.4f} ms",
            "flagged_pixels": int(st["flagged_pixels"]), "sliced_blocks": int(st["dense_blocks"]),
            "roofline": roofline,
        },
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--tuning", default="rules", choices=("rules", "online"),
                    help="rules: the library's rule table (default); online: fastest tuning timed on the frame")
    ap.add_argument("--bin-size", type=int, default=0, help="override the tuning's bin size")
    ap.add_argument("--sorter-depth", type=int, default=0, help="override the tuning's sorter depth")
    ap.add_argument("--block-h", type=int, default=0, help="override the tuning's block height")
    ap.add_argument("--cpu-seconds", type=float, default=6.0,
                    help="minimum seconds of all-core oracle frames (one single-core frame follows)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the 1280x720 side leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-frame mixed batch")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving loop")
    ap.add_argument("--no-cutoff", action="store_true", help="skip the transmittance-cutoff leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the large-quad binning and density-class comparisons")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--serve-scenes", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (a frame would shard by screen "
              "region across GPUs; that is a design, not code); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return

    import torch
    from paper_2405_13364_amd import autotune, lucidraster, scenes

    rules = autotune.load_rules()
    arena = 2 << 30

    def pick_tuning(sc, mode):
        if mode == "online":
            log(f"{sc.name}: online tuning on the frame")
            tctx = lucidraster.Context(arena_bytes=arena)
            th_ = tctx.upload(sc.v, sc.rgba)
            best, ttimes = autotune.tune_frame(tctx, th_, sc.camera, sc.width, sc.height)
            tctx.close()
            return tuple(best), (f"online: fastest of {len(ttimes)} tunings timed on this frame (rule table "
                                 f"pick {'/'.join(map(str, autotune.resolve(rules, sc.width, sc.height, sc.n)))})")
        return tuple(autotune.resolve(rules, sc.width, sc.height, sc.n)), "rule table (lr_set_tuning rules)"

    log(f"generating workload {args.workload}")
    sc = scenes.scene(args.workload)
    tune, note = pick_tuning(sc, args.tuning)
    tune = (args.bin_size or tune[0], args.sorter_depth or tune[1], args.block_h or tune[2])
    if args.bin_size or args.sorter_depth or args.block_h:
        note += " with command-line overrides"
    log(f"tuning: bin {tune[0]}, sorter depth {tune[1]}, block 8x{tune[2]} ({note})")
    head = frame_leg(torch, lucidraster, autotune, sc, args.workload, tune, note, args.steps, args.warmup, arena)
    line = head["line"]
    ms, frags = head["ms"], head["frags"]
    res = {
        "metric": METRIC,
        "value": line["Mfrags_per_s"],
        "unit": "Mfrags/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": line["workload"], "width": sc.width, "height": sc.height,
                   "quads": sc.n, "visible_quads": line["visible_quads"], "fragments": int(frags),
                   "bin_size": tune[0],
                   "block": f"8x{tune[2]}", "sorter_depth": tune[1], "tuning": note,
                   "arithmetic": "i32 coverage, f64 depth plane, f32 blend"},
        "frames_per_s": line["frames_per_s"],
        "p50_ms": line["p50_ms"],
        "p99_ms": line["p99_ms"],
        "unsorted": line["unsorted"],
        "sorted_over_unsorted": line["sorted_over_unsorted"],
        "paper_sw_over_hw": 3.30,
        "stage_us": line["stage_us"],
        "stage_note": line["stage_note"],
        "flagged_pixels": line["flagged_pixels"],
        "sliced_blocks": line["sliced_blocks"],
        "roofline": line["roofline"],
    }
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle: about {args.cpu_seconds:.0f} s on all cores, then one frame on one core")
        cb, ref = cpu_baseline(sc, args.cpu_seconds)
        res["cpu_baseline"] = cb
        got = head["out"].cpu().numpy().astype(np.int32)
        res["max_lsb_vs_oracle"] = int(np.abs(got - ref["rgba8"].astype(np.int32)).max())
        res["fragments_equal_oracle"] = bool(ref["total"] == frags)
    else:
        res["cpu_baseline"] = None
    if not args.no_side and args.workload != "c2":
        side = {}
        sc2 = scenes.scene("c2")
        for mode in ("rules", "online"):
            t2, n2 = pick_tuning(sc2, mode)
            side[mode] = frame_leg(torch, lucidraster, autotune, sc2, "c2", t2, n2, args.steps, args.warmup,
                                   arena)["line"]
        res["side_c2"] = side
    if not args.no_cutoff:
        log("transmittance cutoff leg")
        res["alpha_cutoff"] = cutoff_leg(torch, lucidraster, autotune, rules, args.steps, args.warmup, arena, log)
    if not args.no_variants:
        log("large-quad binning and density classes")
        res["large_quads"] = large_quads_leg(torch, lucidraster, autotune, rules, args.steps, args.warmup, arena, log)
        res["density_classes"] = classes_leg(torch, lucidraster, args.steps, args.warmup, arena, log)
    if not args.no_batch:
        log("64-frame mixed batch")
        res["batch"] = mixed_batch_leg(torch, lucidraster, scenes, rules, args.batch_reps, log)
    if not args.no_serving:
        log("serving loop")
        res["serving"] = serving_leg(torch, lucidraster, scenes, rules, args.serve_scenes, args.serve_requests, log)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
