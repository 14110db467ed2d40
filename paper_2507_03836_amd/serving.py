"""Continuous-batching request server for trained F-Hash models.

Rendering a trained representation is ray marching whose samples are decoded
by the encoding + MLP, with the adaptive marching pace of Sec. 3.3 (ARM,
Algorithm 1): every iteration a sample budget is divided over the rays still
alive.  This
module serves many such renders, and batches of point queries (x, y, z, t),
against models that stay resident on the device:

* requests arrive at any time and wait in a FIFO queue;
* a request is admitted when a slot is free and its device footprint (render
  state + image, or query outputs) fits the memory budget next to the
  resident models; it then joins the running batch at the next iteration, so
  work of requests that arrived at different times overlaps on the device;
* one iteration marches every admitted render request, appends a chunk of
  pending point queries, and decodes all samples of one model with a single
  fused encode + MLP launch; then every render composites its own samples.
  The iteration's sample budget is handed out oldest request first.  Default
  ("backfill"): the oldest render takes the ARM pace the whole budget allows,
  younger ones only what it leaves, and a render waits for a turn when that
  is less than one sample per alive ray.  "oldest_first" reserves one sample
  per alive ray of every younger render, so all of them move every
  iteration; "shared" gives every render the pace of the budget over all
  alive rays;
* a request leaves the batch when its last ray terminates or its last point
  is decoded, and its latency (arrival to completion) is recorded.

The decoded value of a sample depends only on its position and the model, and
the ARM pace changes how many lattice samples a ray takes per iteration but
not which ones or their compositing order, so each result is the same alone
and in any mix.

`Scheduler` holds the host logic only and drives an executor.  `GpuExecutor`
issues the libfhash calls (render step API and fused forward); tests drive
the scheduler with a host-only executor as well.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np


@dataclasses.dataclass(eq=False)   # requests compare by identity
class Request:
    """A render request (view, t, W, H) or a point-query request (pos)."""
    model: str
    kind: str                      # "render" or "points"
    arrival: float = 0.0           # seconds on the scheduler clock
    view: object = None            # 14 float32 (eye, fwd, right, up, tan(fovy/2), aspect)
    t: float = 0.0                 # render time in [0, T-1] (voxel time units)
    W: int = 0
    H: int = 0
    pos: object = None             # device float32 [n][4] positions in [0,1]^4
    n: int = 0                     # number of point queries
    # filled by the server
    rid: int = -1
    result: object = None          # rgba [H][W][4] or y [n]
    t_admit: float = -1.0
    t_done: float = -1.0
    iterations: int = 0
    samples: int = 0
    # scheduler-private
    alive: int = 0
    done: int = 0
    chunk: tuple = (0, 0)
    state: object = None
    ws: object = None

    @property
    def rays(self) -> int:
        return self.W * self.H if self.kind == "render" else 0

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Scheduler:
    """Iteration-level scheduler: FIFO admission by slots and memory,
    one shared ARM pace, model-grouped decode, per-request completion.

    sample_budget  samples decoded per iteration (size of the shared buffer);
                   admitted renders hold at most half of it in rays, so pace
                   >= 1 always fits and point queries always get a share
    mem_budget     device bytes available to requests (after resident models)
    max_active     request slots
    policy         "oldest_first", "shared" or "backfill" division of the sample budget
    """

    def __init__(self, executor, sample_budget: int = 1 << 22, mem_budget: int = 1 << 36,
                 max_active: int = 64, arm_max: int = 64, policy: str = "backfill"):
        if sample_budget < 2:
            raise ValueError("sample budget must be at least 2")
        if policy not in ("oldest_first", "shared", "backfill"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        self.ex = executor
        self.C = int(sample_budget)
        self.mem_budget = int(mem_budget)
        self.max_active = int(max_active)
        self.arm_max = int(arm_max)
        self.queue: deque[Request] = deque()
        self.active: list[Request] = []
        self.finished: list[Request] = []
        self.mem_used = 0
        self.rays_used = 0
        self.iterations = 0
        self.samples = 0
        self.peak_mem = 0
        self.peak_active = 0
        self._next_id = 0

    # ------------------------------------------------------------------ queue
    def submit(self, req: Request) -> Request:
        if req.kind == "render":
            if req.W < 1 or req.H < 1 or req.rays > self.C // 2:
                raise ValueError(f"render {req.W}x{req.H} exceeds half the sample budget {self.C}")
        elif req.kind == "points":
            if req.n < 0:
                raise ValueError("negative point count")
        else:
            raise ValueError(f"unknown request kind {req.kind!r}")
        if not self.ex.has_model(req.model):
            raise KeyError(f"model {req.model!r} is not resident")
        if self.ex.request_bytes(req) > self.mem_budget:
            raise ValueError("request footprint exceeds the memory budget")
        req.rid = self._next_id
        self._next_id += 1
        self.queue.append(req)
        return req

    def busy(self) -> bool:
        return bool(self.queue or self.active)

    def _admit(self):
        # strict FIFO: the head waits for memory / slots, nothing overtakes it
        while self.queue and len(self.active) < self.max_active:
            r = self.queue[0]
            need = self.ex.request_bytes(r)
            if self.mem_used + need > self.mem_budget:
                break
            if r.kind == "render" and self.rays_used + r.rays > self.C // 2:
                break
            self.queue.popleft()
            self.mem_used += need
            self.rays_used += r.rays
            self.peak_mem = max(self.peak_mem, self.mem_used)
            r.t_admit = self.ex.now()
            if r.kind == "render":
                r.alive = self.ex.begin(r)
            else:
                self.ex.begin(r)
                r.done = 0
            self.active.append(r)
            if (r.kind == "render" and r.alive == 0) or (r.kind == "points" and r.n == 0):
                self._retire(r)
        self.peak_active = max(self.peak_active, len(self.active))

    def _retire(self, r: Request):
        self.active.remove(r)
        self.mem_used -= self.ex.request_bytes(r)
        self.rays_used -= r.rays
        r.t_done = self.ex.now()
        self.ex.finish(r)
        self.finished.append(r)

    # ------------------------------------------------------------- iteration
    def paces(self) -> list[int]:
        """ARM pace of every admitted render (admission order) this iteration."""
        renders = [r for r in self.active if r.kind == "render"]
        pending = sum(r.n - r.done for r in self.active if r.kind == "points")
        budget = self.C - min(pending, self.C // 2)
        alive = sum(r.alive for r in renders)
        if self.policy == "shared":
            p = self.ex.pace(budget, alive, self.arm_max)
            return [p] * len(renders)
        out = []
        if self.policy == "backfill":
            for i, r in enumerate(renders):
                p = 0 if (i > 0 and budget < r.alive) else self.ex.pace(budget, r.alive,
                                                                         self.arm_max)
                out.append(p)
                budget -= p * r.alive
            return out
        reserve = alive
        for r in renders:
            reserve -= r.alive
            p = self.ex.pace(budget - reserve, r.alive, self.arm_max)
            out.append(p)
            budget -= p * r.alive
        return out

    def step(self) -> int:
        """One iteration over the running batch; returns samples decoded."""
        self._admit()
        if not self.active:
            return 0
        renders = [r for r in self.active if r.kind == "render"]
        points = [r for r in self.active if r.kind == "points"]
        paces = self.paces()
        used = sum(p * r.alive for p, r in zip(paces, renders))
        assert used <= self.C
        pt_budget = self.C - used
        pace_of = {id(r): p for p, r in zip(paces, renders)}
        renders = [r for r in renders if pace_of[id(r)] > 0]  # the others wait a turn
        models = list(dict.fromkeys(r.model for r in self.active))
        off = 0
        for m in models:
            start = off
            group = [r for r in renders if r.model == m]
            if group:
                # one march over the model's renders: their samples share
                # [start, off) of the buffer, interleaved
                counts = self.ex.march_batch(group, [pace_of[id(r)] for r in group], off)
                for r, ns in zip(group, counts):
                    r.samples += ns
                    off += ns
                assert off <= self.C
            for r in points:
                if r.model != m:
                    continue
                k = min(r.n - r.done, pt_budget)
                r.chunk = (off, k)
                if k > 0:
                    self.ex.load_points(r, r.done, k, off)
                    off += k
                    pt_budget -= k
            if off > start:
                self.ex.decode(m, start, off)
        if renders:
            for r, alive in zip(renders, self.ex.composite_batch(renders)):
                r.alive = alive
                r.iterations += 1
        completed = []
        for r in points:
            o, k = r.chunk
            if k > 0:
                self.ex.store_points(r, r.done, k, o)
                r.done += k
                r.iterations += 1
            if r.done == r.n:
                completed.append(r)
        if completed:
            self.ex.sync()
        for r in renders:
            if r.alive == 0:
                self._retire(r)
        for r in completed:
            self._retire(r)
        self.iterations += 1
        self.samples += off
        return off

    # ------------------------------------------------------------- driving
    def run(self, arrivals: list[Request], realtime: bool = True) -> list[Request]:
        """Serve requests whose `arrival` fields are offsets (s) from the start.

        realtime: wait for arrivals on the wall clock; otherwise every request
        is submitted at once (closed-loop saturation measurement)."""
        order = sorted(arrivals, key=lambda r: r.arrival)
        t0 = self.ex.now()
        i = 0
        n_done0 = len(self.finished)
        while i < len(order) or self.busy():
            now = self.ex.now() - t0
            while i < len(order) and (not realtime or order[i].arrival <= now):
                r = order[i]
                r.arrival = t0 + (r.arrival if realtime else 0.0)
                self.submit(r)
                i += 1
            if not self.busy():
                self.ex.wait_until(t0 + order[i].arrival)
                continue
            self.step()
        return self.finished[n_done0:]


def latency_stats(reqs: list[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    span = max(r.t_done for r in reqs) - min(r.arrival for r in reqs)
    rays = sum(r.rays for r in reqs)
    pts = sum(r.n for r in reqs if r.kind == "points")
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "span_s": span, "rays_per_s": rays / span if span > 0 else 0.0,
            "points_per_s": pts / span if span > 0 else 0.0,
            "requests_per_s": len(reqs) / span if span > 0 else 0.0}


# --------------------------------------------------------------------- GPU side
@dataclasses.dataclass
class ResidentModel:
    """A trained model kept on the device: index, decoder table (f32 or f16),
    MLP parameters, the occupancy for rendering and TF.  occ: the coreset's
    occupancy grid (fhash_occupancy_grid), which renders start from; without
    it, the voxel feature mask rows mask_bits."""
    index: object
    mlp: object
    table: object
    params: object
    mask_bits: object
    dims: list
    tf: object
    keep: tuple = ()               # tensors the index views (directory)
    occ: object = None

    def nbytes(self) -> int:
        tot = 0
        occ = self.occ if self.occ is not None else self.mask_bits
        for t in (self.table, self.params, occ, self.tf) + tuple(self.keep):
            tot += t.numel() * t.element_size()
        return tot


class GpuExecutor:
    """libfhash calls for the scheduler, on torch's current stream."""

    def __init__(self, sample_budget: int = 1 << 22, ds: float = 0.5, alpha_stop: float = 0.99,
                 arm_max: int = 64, max_steps: int = 1 << 20):
        import torch

        from . import _lib as fl
        self.torch, self.fl = torch, fl
        fl.lib()
        self.models: dict[str, ResidentModel] = {}
        self.opts = fl.render_opts(ds=ds, alpha_stop=alpha_stop, arm_max=arm_max,
                                   max_steps=max_steps)
        self.pos = torch.empty(sample_budget, 4, dtype=torch.float32, device="cuda")
        self.y = torch.empty(sample_budget, dtype=torch.float32, device="cuda")
        self.counts = torch.empty(1 + fl.RENDER_BATCH_MAX, dtype=torch.int32, device="cuda")

    def add_model(self, name: str, m: ResidentModel):
        self.models[name] = m

    def has_model(self, name: str) -> bool:
        return name in self.models

    def resident_bytes(self) -> int:
        return sum(m.nbytes() for m in self.models.values()) + \
            self.pos.numel() * 4 + self.y.numel() * 4

    def request_bytes(self, r: Request) -> int:
        if r.kind == "render":
            m = self.models[r.model]
            st = self.fl.fhash_render_state_bytes(r.W, r.H, m.dims)
            return st + r.W * r.H * 16
        return r.n * 4

    def now(self) -> float:
        return time.perf_counter()

    def wait_until(self, t: float):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)

    def pace(self, budget, alive, arm_max) -> int:
        return self.fl.fhash_render_pace(budget, alive, arm_max)

    def begin(self, r: Request) -> int:
        torch, fl = self.torch, self.fl
        m = self.models[r.model]
        if r.kind == "points":
            if r.n and (r.pos is None or tuple(r.pos.shape) != (r.n, 4)
                        or r.pos.dtype != torch.float32 or not r.pos.is_contiguous()):
                raise ValueError("point queries need contiguous float32 [n][4] positions")
            r.result = torch.empty(r.n, dtype=torch.float32, device="cuda")
            return 0
        nb = fl.fhash_render_state_bytes(r.W, r.H, m.dims)
        r.ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        r.result = torch.empty(r.H, r.W, 4, dtype=torch.float32, device="cuda")
        view = r.view if isinstance(r.view, fl.View) else fl.view_struct(r.view)
        if m.occ is not None:
            r.state = fl.fhash_render_begin_grid(view, r.t, r.W, r.H, m.occ, m.dims, r.ws,
                                                 r.result)
        else:
            r.state = fl.fhash_render_begin(view, r.t, r.W, r.H, m.mask_bits, m.dims, r.ws,
                                            r.result)
        return int(r.state.n_alive)

    def march_batch(self, rs: list, paces: list, off: int) -> list:
        """One march launch per FHASH_RENDER_BATCH_MAX renders; their samples
        go to pos[off:], interleaved, each ray's at offsets it keeps."""
        B, out = self.fl.RENDER_BATCH_MAX, []
        for i in range(0, len(rs), B):
            ns = self.fl.fhash_render_march_batch([r.state for r in rs[i: i + B]],
                                                  paces[i: i + B], self.opts, self.pos, off,
                                                  self.pos.shape[0], self.counts)
            out += ns
            off += sum(ns)
        return out

    def load_points(self, r: Request, start: int, k: int, off: int):
        self.pos[off: off + k].copy_(r.pos[start: start + k])

    def decode(self, model: str, start: int, end: int):
        m = self.models[model]
        self.fl.fhash_fused_fwd(m.index, m.mlp, self.pos[start:end], end - start, m.table,
                                m.params, self.y[start:end])

    def composite_batch(self, rs: list) -> list:
        """One composite launch per FHASH_RENDER_BATCH_MAX renders; returns the
        alive-ray counts."""
        B, out = self.fl.RENDER_BATCH_MAX, []
        for i in range(0, len(rs), B):
            ch = rs[i: i + B]
            out += self.fl.fhash_render_composite_batch(
                [r.state for r in ch], self.y, [self.models[r.model].tf for r in ch], self.opts,
                [r.result for r in ch], self.counts)
        return out

    def store_points(self, r: Request, start: int, k: int, off: int):
        r.result[start: start + k].copy_(self.y[off: off + k])

    def sync(self):
        self.torch.cuda.synchronize()

    def finish(self, r: Request):
        r.ws = None
        r.state = None


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """n arrival offsets (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
