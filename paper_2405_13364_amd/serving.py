"""Continuous-batching render server over the C ABI.

Requests (a resident scene, a camera and a frame size) arrive over time.  The
server keeps every scene resident in HBM and runs a small number of stream
slots, each with its own batch workspace in the context's arena.  As soon as
a slot is free it takes the waiting requests in arrival order, as many as fit
the device-memory budget (the sum of the footprints of everything in flight,
``lr_request_bytes``) and the batch-size limit, and renders them with one
``lr_render_batch`` on that slot's stream.  Requests that arrive while other
batches are on the GPU are admitted as soon as a slot and memory free up, so
work from different batches overlaps on the device.

One-at-a-time rendering is the same loop with one slot and batches of one.

The scheduling logic is independent of the GPU: ``Server`` talks to a backend
with four calls (footprint, submit, done, wait), so the host policy is
tested on the CPU with a simulated backend, and ``GpuBackend`` drives the
real library.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds since the start of the trace
    scene: int                     # resident scene handle
    camera: object                 # scenes.Camera
    width: int
    height: int
    tune: Tuple = ()               # optional (bin_size, sorter_depth, block_h)


@dataclasses.dataclass
class Completion:
    rid: int
    arrival: float
    submit: float
    finish: float
    batch: int
    slot: int

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Server:
    """Admission and continuous batching over `slots` concurrent stream slots."""

    def __init__(self, backend, budget_bytes: int, slots: int = 2, max_batch: int = 16):
        if slots < 1 or max_batch < 1:
            raise ValueError("slots and max_batch must be at least 1")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.slots = slots
        self.max_batch = max_batch
        # admission statistics of the last run: batches closed early because
        # the next request would not fit the budget, times a free slot waited
        # for memory, and the most bytes ever in flight
        self.stats = {"budget_cut_batches": 0, "memory_waits": 0, "max_inflight": 0}

    def run(self, requests: Sequence[Request]) -> List[Completion]:
        be = self.backend
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: deque = deque()
        busy: Dict[int, Tuple[object, List[Request], int, float]] = {}
        inflight = 0
        done: List[Completion] = []
        nbatch = 0
        fp_cache: Dict[Tuple, int] = {}
        self.stats = {"budget_cut_batches": 0, "memory_waits": 0, "max_inflight": 0}

        def footprint(r: Request) -> int:
            key = (r.scene, r.width, r.height, tuple(r.tune))
            if key not in fp_cache:
                fp_cache[key] = int(be.footprint(r))
            return fp_cache[key]

        while pending or waiting or busy:
            now = be.now()
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if footprint(r) > self.budget:
                    raise ValueError(f"request {r.rid} needs {footprint(r)} bytes, over the budget {self.budget}")
                waiting.append(r)
            # retire finished batches
            for slot in list(busy):
                token, reqs, fp, t_sub = busy[slot]
                if be.done(token):
                    t_fin = be.now()
                    for r in reqs:
                        done.append(Completion(r.rid, r.arrival, t_sub, t_fin, token_batch(token), slot))
                    be.release(token)
                    inflight -= fp
                    del busy[slot]
            # admit into free slots
            free = [s for s in range(self.slots) if s not in busy]
            while free and waiting:
                batch, fp = [], 0
                while (waiting and len(batch) < self.max_batch
                       and inflight + fp + footprint(waiting[0]) <= self.budget):
                    r = waiting.popleft()
                    batch.append(r)
                    fp += footprint(r)
                if not batch:
                    self.stats["memory_waits"] += 1
                    break  # wait for memory
                if waiting and len(batch) < self.max_batch:
                    self.stats["budget_cut_batches"] += 1
                slot = free.pop(0)
                t_sub = be.now()
                token = be.submit(slot, batch, nbatch)
                busy[slot] = (token, batch, fp, t_sub)
                inflight += fp
                self.stats["max_inflight"] = max(self.stats["max_inflight"], inflight)
                nbatch += 1
            if not (pending or waiting or busy):
                break
            next_arrival = pending[0].arrival if pending else math.inf
            be.wait(next_arrival, [busy[s][0] for s in busy])
        return done


def token_batch(token) -> int:
    return token["batch"]


class GpuBackend:
    """Drives the library: one torch stream per slot, output buffers pooled
    per frame size (or kept, for checking), completion by stream events.

    Every batch also reports each frame's error bits (lr_request.status) into
    a device tensor, copied to pinned host memory on the slot's stream before
    the completion event.  A frame whose bin lists overflowed (its image was
    not written) is rendered again once its batch is done: the library's
    capacity hint is raised (lr_sync) and the failed frames are re-submitted
    on the same slot, so the request completes only with its exact image."""

    def __init__(self, ctx, slots: int, keep_outputs: bool = False, keep_every: int = 0,
                 max_retries: int = 2):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.streams = [torch.cuda.Stream(device=ctx.device) for _ in range(slots)]
        self.keep = keep_outputs
        self.keep_every = keep_every
        self.max_retries = max_retries
        self.outputs: Dict[int, object] = {}
        self.pool: Dict[Tuple[int, int], List[object]] = {}
        self.retried: List[int] = []     # request ids rendered again after a capacity error
        self.t0 = time.perf_counter()

    def start_clock(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def footprint(self, r: Request) -> int:
        t = tuple(r.tune) + (None,) * (3 - len(r.tune))
        return self.ctx.request_bytes(r.scene, r.camera, r.width, r.height, *t)

    def _kept(self, rid: int) -> bool:
        return self.keep or (self.keep_every > 0 and rid % self.keep_every == 0)

    def _image(self, W, H, rid):
        free = self.pool.get((W, H))
        if free and not self._kept(rid):
            return free.pop()
        return self.ctx.new_image(W, H)

    def _launch(self, slot: int, reqs: List[Request], outs: List[object]):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            status_dev = torch.empty(len(reqs), dtype=torch.int32, device=f"cuda:{self.ctx.device}")
            self.ctx.render_batch([(r.scene, r.camera, r.width, r.height, o) + tuple(r.tune)
                                   for r, o in zip(reqs, outs)], stream=st, check=False, status=status_dev)
            status_host = torch.empty(len(reqs), dtype=torch.int32, pin_memory=True)
            status_host.copy_(status_dev, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(st)
        return ev, status_dev, status_host

    def submit(self, slot: int, reqs: List[Request], batch_id: int):
        outs = [self._image(r.width, r.height, r.rid) for r in reqs]
        ev, sd, sh = self._launch(slot, reqs, outs)
        # 'idx': the requests of this token whose frames the last launch covered
        return {"event": ev, "outs": outs, "reqs": reqs, "batch": batch_id, "slot": slot,
                "status_dev": sd, "status": sh, "idx": list(range(len(reqs))), "tries": 0}

    def done(self, token) -> bool:
        if not token["event"].query():
            return False
        from .lucidraster import LR_ERR_CAPACITY, LR_FRAME_ERR_CAPACITY, LRError
        st = token["status"].numpy()
        bad = [token["idx"][k] for k in range(len(token["idx"])) if int(st[k]) & LR_FRAME_ERR_CAPACITY]
        if not bad:
            return True
        if token["tries"] >= self.max_retries:
            raise RuntimeError(f"requests {[token['reqs'][k].rid for k in bad]} overflowed their bin lists "
                               f"{token['tries'] + 1} times")
        # raise the capacity hints (waits for the device), then render the
        # failed frames again on the same slot
        try:
            self.ctx.sync()
        except LRError as e:
            if e.status != LR_ERR_CAPACITY:
                raise
        reqs = [token["reqs"][k] for k in bad]
        outs = [token["outs"][k] for k in bad]
        self.retried.extend(r.rid for r in reqs)
        ev, sd, sh = self._launch(token["slot"], reqs, outs)
        token.update(event=ev, status_dev=sd, status=sh, idx=bad, tries=token["tries"] + 1)
        return False

    def release(self, token):
        for r, o in zip(token["reqs"], token["outs"]):
            if self._kept(r.rid):
                self.outputs[r.rid] = o
            else:
                self.pool.setdefault((r.width, r.height), []).append(o)

    def wait(self, next_arrival: float, tokens):
        # spin briefly: completions and arrivals are microseconds apart
        time.sleep(0)


class SimBackend:
    """A simulated GPU for host-side tests: a batch of frames on a slot takes
    setup + sum(frame costs) seconds, slots run in parallel."""

    def __init__(self, cost: Dict[int, float], footprint_bytes: Dict[int, int], setup: float = 1e-4):
        self.cost = cost
        self.fp = footprint_bytes
        self.setup = setup
        self.t = 0.0
        self.log: List[Tuple[float, int, List[int]]] = []

    def now(self) -> float:
        return self.t

    def footprint(self, r: Request) -> int:
        return self.fp[r.rid]

    def submit(self, slot, reqs, batch_id):
        fin = self.t + self.setup + sum(self.cost[r.rid] for r in reqs)
        self.log.append((self.t, slot, [r.rid for r in reqs]))
        return {"finish": fin, "batch": batch_id}

    def done(self, token) -> bool:
        return self.t >= token["finish"]

    def release(self, token):
        pass

    def wait(self, next_arrival: float, tokens):
        nxt = min([next_arrival] + [t["finish"] for t in tokens])
        if nxt == math.inf:
            raise RuntimeError("server waits with nothing pending")
        self.t = max(self.t, nxt)


def poisson_trace(rate: float, n: int, scenes_meta: Sequence[Tuple[int, int, int]], seed: int,
                  jitter_deg: float = 2.0) -> List[Request]:
    """n requests with exponential inter-arrival times at `rate` per second;
    each picks a resident scene uniformly (scenes_meta: handle, width, height)
    and a camera turned by yaw and pitch uniform in +-jitter_deg."""
    from . import scenes
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    which = rng.integers(0, len(scenes_meta), n)
    yaw = rng.uniform(-jitter_deg, jitter_deg, n)
    pitch = rng.uniform(-jitter_deg, jitter_deg, n)
    t = np.cumsum(gaps)
    out = []
    for i in range(n):
        h, W, H = scenes_meta[int(which[i])]
        out.append(Request(i, float(t[i]), h, scenes.Camera.jittered(float(yaw[i]), float(pitch[i])), W, H))
    return out


def summarize(done: List[Completion]) -> Dict[str, float]:
    lat = np.array([c.latency for c in done]) * 1e3
    span = max(c.finish for c in done) - min(c.arrival for c in done)
    return {"requests": len(done), "frames_per_s": round(len(done) / span, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4), "batches": len({c.batch for c in done})}
