"""Autotuner: per-frame-shape choice of bin size, block shape and sorter depth.

The sweep renders sample frames of every class (frame size x quads-per-pixel
bucket), each drawn from the three base workload shapes, under every tuning
(bin 16/32/64 x 8x8 or 8x4 blocks x sorter depth 4..32), and keeps for each
class the tuning with the least mean slowdown over the class's frames (each
frame's time divided by its own best time, so a dense frame does not decide
for the light ones).  The result is a list of
``lr_tune_rule`` records (first match wins), written as JSON beside this
module; ``Context(tuning=load_rules())`` installs it.

Every tuning gives the same image (the renderer is exact), so the sweep only
measures time.
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
RULES_PATH = os.path.join(HERE, "tuning.json")

BINS = (16, 32, 64)
BLOCKS = (8, 4)
DEPTHS = (4, 8, 12, 16, 24, 32)
# The online tuner also tries depth 2.  It pays only on frames whose pixels
# hold a couple of fragments; a rule chosen on a class's sample frames would
# also apply it to denser frames of the class, whose extra flagged pixels
# cost more than the shallower sorter saves (measured on the mixed batch).
ONLINE_DEPTHS = (2,) + DEPTHS
# quads-per-pixel bucket upper bounds and the value sampled in each bucket
QPP_BUCKETS = ((0.01, 0.005), (0.05, 0.022), (0.15, 0.08), (0.3, 0.2), (0.6, 0.4), (1.2, 0.8), (1e9, 2.0))


def tunings(depths=DEPTHS):
    return list(itertools.product(BINS, depths, BLOCKS))


def sample_frames(W: int, H: int, qpp: float, seed: int):
    """One frame per base workload shape at this size and density (at most
    1M quads, the largest single-frame workload)."""
    from . import scenes
    n = int(min(1_000_000, max(1_000, round(qpp * W * H))))
    out = []
    for k, base in enumerate(("c1", "c2", "c3")):
        b = scenes.RECIPES[base]
        rc = scenes.Recipe(W, H, n, seed + k, b.gaussian, b.sigma, b.z, b.side, b.alpha)
        out.append(scenes.generate(rc, f"tune-{base}-{W}x{H}-{n}"))
    return out


def time_frame(ctx, h, sc, tune, reps: int) -> float:
    """Median GPU milliseconds of one frame rendered as a one-frame batch."""
    import torch
    out = ctx.new_image(sc.width, sc.height)
    req = [(h, sc.camera, sc.width, sc.height, out) + tuple(tune)]
    ctx.render_batch(req)  # warm-up (and capacity planning)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.render_batch(req, check=False)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ctx.sync()
    return float(np.median(ts))


def sweep(resolutions=None, reps: int = 5, log=print) -> Dict[str, object]:
    from . import lucidraster, scenes
    resolutions = resolutions or scenes.RESOLUTIONS
    ctx = lucidraster.Context(arena_bytes=8 << 30, graphs=False)
    rules, table = [], []
    t0 = time.perf_counter()
    for W, H in sorted(resolutions, key=lambda r: r[0] * r[1]):
        for qmax, qpp in QPP_BUCKETS:
            frames = sample_frames(W, H, qpp, seed=4000 + W + H)
            hs = [ctx.upload(s.v, s.rgba) for s in frames]
            times = {}
            for tune in tunings():
                times[tune] = [time_frame(ctx, h, s, tune, reps) for h, s in zip(hs, frames)]
            for h in hs:
                ctx.release(h)
            fastest = [min(t[i] for t in times.values()) for i in range(len(frames))]
            slowdown = {tune: float(np.mean([t[i] / fastest[i] for i in range(len(frames))]))
                        for tune, t in times.items()}
            best = min(slowdown, key=slowdown.get)
            default = (32, 8, 8)
            table.append({"width": W, "height": H, "qpp": qpp, "quads": frames[0].n,
                          "best": list(best), "best_slowdown": round(slowdown[best], 4),
                          "best_ms": [round(x, 4) for x in times[best]],
                          "default_ms": [round(x, 4) for x in times[default]],
                          "fastest_ms": [round(x, 4) for x in fastest]})
            rules.append({"max_pixels": W * H, "max_quads_per_pixel": qmax, "bin_size": best[0],
                          "sorter_depth": best[1], "block_h": best[2]})
            log(f"[autotune] {W}x{H} qpp {qpp}: best bin {best[0]} K {best[1]} block 8x{best[2]} "
                f"(mean slowdown {slowdown[best]:.3f}) ms per shape {[round(x, 3) for x in times[best]]}; "
                f"bin 32 K 8 8x8: {[round(x, 3) for x in times[default]]}")
    ctx.close()
    return {"rules": rules, "sweep": table, "reps": reps, "seconds": round(time.perf_counter() - t0, 1)}


def tune_frame(ctx, h, cam, W: int, H: int, reps: int = 10, candidates=None):
    """Online tuning of one frame: every tuning timed on this very frame (as
    one-frame batches, median of `reps`); returns the fastest (bin_size,
    sorter_depth, block_h) and the table of times."""
    times = {}
    sc = type("F", (), {"width": W, "height": H, "camera": cam})
    for tune in candidates or tunings(ONLINE_DEPTHS):
        times[tune] = time_frame(ctx, h, sc, tune, reps)
    best = min(times, key=times.get)
    return best, times


def load_rules(path: str = RULES_PATH) -> Optional[List[dict]]:
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)["rules"]


def resolve(rules: Optional[List[dict]], W: int, H: int, n: int, default=(32, 8, 8)):
    """(bin_size, sorter_depth, block_h) the library picks for a frame: the
    first rule matching its pixel count and quads per pixel."""
    px = W * H
    for u in rules or []:
        if px <= u["max_pixels"] and n / px <= u["max_quads_per_pixel"]:
            return (u["bin_size"], u["sorter_depth"], u["block_h"])
    return default


def main():
    import argparse
    ap = argparse.ArgumentParser(description="sweep tunings on the GPU and write the rule table")
    ap.add_argument("--out", default=RULES_PATH)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    res = sweep(reps=args.reps)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(f"wrote {args.out}: {len(res['rules'])} rules in {res['seconds']} s")


if __name__ == "__main__":
    main()
