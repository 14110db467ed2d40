"""Host logic of the continuous-batching server, driven by a host-only executor.

The executor below models a render as rays of known lengths (lattice samples
that pass the occupancy test) and a decoder as a fixed function of the sample,
and moves every sample through one shared buffer exactly like the device
executor does (one march per model group writes the requests' samples
interleaved, one decode per model over a range, composite reads each ray's run
back).  A bookkeeping mistake (wrong offset, a chunk decoded by the wrong
model, a request retired early, a budget overrun) changes a result or trips an
assertion.
"""
import numpy as np
import pytest

from paper_2507_03836_amd.serving import Request, Scheduler, latency_stats, poisson_arrivals


def _ray_len(rid, ray):
    return (rid * 7 + ray * 13) % 23  # 0..22 samples, some rays empty


def _decode(model, a, b):
    return (model + 1) * 1.5 + np.sin(a * 0.37 + b * 0.011)


class HostExecutor:
    def __init__(self, C, models=("m0", "m1")):
        self.C = C
        self.models = {m: i for i, m in enumerate(models)}
        self.buf = np.full((C, 2), np.nan)
        self.y = np.full(C, np.nan)
        self.clock = 0.0
        self.decoded = []       # (model, start, end) per decode launch
        self.paces = []

    def has_model(self, m):
        return m in self.models

    def request_bytes(self, r):
        return r.W * r.H * 100 if r.kind == "render" else r.n * 4

    def now(self):
        return self.clock

    def wait_until(self, t):
        self.clock = max(self.clock, t)

    def pace(self, budget, alive, arm_max):
        self.paces.append((budget, alive))
        return 1 if alive == 0 else int(min(max(budget // alive, 1), arm_max))

    def begin(self, r):
        if r.kind == "points":
            r.result = np.full(r.n, np.nan)
            return 0
        n = r.W * r.H
        r.state = {"k": np.zeros(n, int), "len": np.array([_ray_len(r.rid, i) for i in range(n)]),
                   "acc": np.zeros(n), "alive": [i for i in range(n) if _ray_len(r.rid, i) > 0],
                   "taken": None}
        r.result = r.state["acc"]
        return len(r.state["alive"])

    def march_batch(self, rs, paces, off):
        # like the device: one launch for the group, the requests' samples
        # interleaved ray by ray, each ray's run contiguous at an offset it keeps
        queues = []
        for r, pace in zip(rs, paces):
            s = r.state
            assert pace >= 1
            s["taken"] = []
            queues.append([(r, pace, ray) for ray in s["alive"]])
        counts = [0] * len(rs)
        o = off
        for j in range(max((len(q) for q in queues), default=0)):
            for i, q in enumerate(queues):
                if j >= len(q):
                    continue
                r, pace, ray = q[j]
                s = r.state
                c = min(pace, s["len"][ray] - s["k"][ray])
                for t in range(c):
                    self.buf[o + t] = (r.rid * 100000 + ray, s["k"][ray] + t)
                s["taken"].append((ray, o, c))
                s["k"][ray] += c
                o += c
                counts[i] += c
        assert o <= self.C
        self.clock += 1e-6 * (o - off)
        return counts

    def load_points(self, r, start, k, off):
        self.buf[off: off + k, 0] = r.pos[start: start + k]
        self.buf[off: off + k, 1] = -1.0

    def decode(self, model, start, end):
        self.decoded.append((model, start, end))
        i = self.models[model]
        self.y[start:end] = _decode(i, self.buf[start:end, 0], self.buf[start:end, 1])
        self.buf[start:end] = np.nan
        self.clock += 1e-4

    def composite_batch(self, rs):
        out = []
        for r in rs:
            s = r.state
            alive = []
            for ray, o, c in s["taken"]:
                for j in range(c):
                    v = self.y[o + j]
                    assert np.isfinite(v)
                    s["acc"][ray] += v
                    self.y[o + j] = np.nan
                if s["k"][ray] < s["len"][ray]:
                    alive.append(ray)
            s["alive"] = alive
            out.append(len(alive))
        return out

    def store_points(self, r, start, k, off):
        assert np.isfinite(self.y[off: off + k]).all()
        r.result[start: start + k] = self.y[off: off + k]
        self.y[off: off + k] = np.nan

    def sync(self):
        pass

    def finish(self, r):
        r.state = None


def _expected_render(r):
    i = {"m0": 0, "m1": 1}[r.model]
    out = np.zeros(r.W * r.H)
    for ray in range(r.W * r.H):
        for k in range(_ray_len(r.rid, ray)):
            out[ray] += _decode(i, r.rid * 100000 + ray, k)
    return out


def _expected_points(r):
    i = {"m0": 0, "m1": 1}[r.model]
    return _decode(i, r.pos, -1.0)


def _mixed_requests(rng, n):
    reqs = []
    for j in range(n):
        m = "m0" if rng.random() < 0.5 else "m1"
        if rng.random() < 0.6:
            reqs.append(Request(model=m, kind="render", W=int(rng.integers(1, 9)),
                                H=int(rng.integers(1, 7)), arrival=float(j) * 1e-4))
        else:
            k = int(rng.integers(0, 150))
            reqs.append(Request(model=m, kind="points", n=k, pos=rng.uniform(0, 1, k),
                                arrival=float(j) * 1e-4))
    return reqs


@pytest.mark.parametrize("C,max_active", [(100, 64), (200, 3), (1000, 1)])
def test_every_result_equals_its_alone_value(C, max_active):
    rng = np.random.default_rng(C)
    reqs = _mixed_requests(rng, 30)
    ex = HostExecutor(C)
    sch = Scheduler(ex, sample_budget=C, mem_budget=10 ** 9, max_active=max_active, arm_max=8)
    done = sch.run(reqs, realtime=True)
    assert len(done) == len(reqs) and not sch.busy()
    for r in reqs:
        exp = _expected_render(r) if r.kind == "render" else _expected_points(r)
        np.testing.assert_allclose(r.result, exp, rtol=0, atol=1e-12)
        assert r.t_done >= r.t_admit >= r.arrival
    assert sch.peak_active <= max_active
    assert sch.mem_used == 0 and sch.rays_used == 0


def test_one_decode_per_model_per_iteration_over_disjoint_ranges():
    rng = np.random.default_rng(5)
    reqs = _mixed_requests(rng, 20)
    for r in reqs:
        r.arrival = 0.0
    ex = HostExecutor(256)
    sch = Scheduler(ex, sample_budget=256, arm_max=4)
    sch.run(reqs, realtime=False)
    # ranges of one iteration never overlap and stay inside the buffer
    for model, a, b in ex.decoded:
        assert 0 <= a < b <= 256
    assert sch.samples == sum(b - a for _, a, b in ex.decoded)


def test_admission_respects_memory_slots_and_ray_budget():
    ex = HostExecutor(128)
    # each 4x4 render costs 1600 bytes; budget admits two at a time
    sch = Scheduler(ex, sample_budget=128, mem_budget=3500, max_active=8)
    reqs = [Request(model="m0", kind="render", W=4, H=4) for _ in range(6)]
    order = []
    real_begin = ex.begin

    def begin(r):
        order.append(r.rid)
        assert sch.mem_used <= 3500
        return real_begin(r)

    ex.begin = begin
    sch.run(reqs, realtime=False)
    assert order == sorted(order)               # FIFO admission
    assert sch.peak_mem <= 3500 and sch.peak_active == 2
    # the ray budget: renders hold at most half the samples in rays
    sch2 = Scheduler(HostExecutor(64), sample_budget=64, mem_budget=10 ** 9)
    reqs2 = [Request(model="m1", kind="render", W=4, H=4) for _ in range(5)]
    for r in reqs2:
        sch2.submit(r)
    sch2._admit()
    assert sch2.rays_used <= 32 and len(sch2.active) == 2


def test_submit_validation():
    ex = HostExecutor(64)
    sch = Scheduler(ex, sample_budget=64, mem_budget=2000)
    with pytest.raises(KeyError):
        sch.submit(Request(model="nope", kind="points", n=1, pos=np.zeros(1)))
    with pytest.raises(ValueError):
        sch.submit(Request(model="m0", kind="render", W=8, H=5))   # 40 rays > 64 / 2
    with pytest.raises(ValueError):
        sch.submit(Request(model="m0", kind="points", n=501, pos=np.zeros(501)))  # > 2000 B
    with pytest.raises(ValueError):
        sch.submit(Request(model="m0", kind="video"))
    with pytest.raises(ValueError):
        Scheduler(ex, sample_budget=1)


def test_pace_policies_and_point_share():
    ex = HostExecutor(100)
    sch = Scheduler(ex, sample_budget=100, arm_max=64, policy="shared")
    a = sch.submit(Request(model="m0", kind="render", W=5, H=2))
    b = sch.submit(Request(model="m1", kind="render", W=4, H=2))
    sch._admit()
    alive = a.alive + b.alive
    assert sch.paces() == [min(64, 100 // alive)] * 2
    sch.policy = "oldest_first"
    pa = min(64, (100 - b.alive) // a.alive)
    pb = min(64, max(1, (100 - pa * a.alive) // b.alive))
    assert sch.paces() == [pa, pb]
    # pending points take up to half of the budget away from the renders
    p = sch.submit(Request(model="m0", kind="points", n=300, pos=np.zeros(300)))
    sch._admit()
    pa = min(64, (50 - b.alive) // a.alive)
    pb = min(64, max(1, (50 - pa * a.alive) // b.alive))
    assert sch.paces() == [pa, pb]
    used = pa * a.alive + pb * b.alive
    sch.step()
    assert p.done == 100 - used
    # backfill: the oldest takes what it can use alone, younger ones the rest or wait
    sch.policy = "backfill"
    pa = min(64, 50 // a.alive)
    left = 50 - pa * a.alive
    pb = 0 if left < b.alive else min(64, left // b.alive)
    assert sch.paces() == [pa, pb]
    with pytest.raises(ValueError):
        Scheduler(ex, policy="lifo")


@pytest.mark.parametrize("policy", ["oldest_first", "shared", "backfill"])
def test_oldest_first_never_starves_and_budget_holds(policy):
    rng = np.random.default_rng(77)
    reqs = _mixed_requests(rng, 25)
    ex = HostExecutor(120)
    sch = Scheduler(ex, sample_budget=120, arm_max=16, policy=policy)
    real = ex.march_batch

    def march_batch(rs, paces, off):
        assert all(p >= 1 for p in paces) and len(rs) == len(paces)
        return real(rs, paces, off)

    ex.march_batch = march_batch
    sch.run(reqs, realtime=True)
    for r in reqs:
        exp = _expected_render(r) if r.kind == "render" else _expected_points(r)
        np.testing.assert_allclose(r.result, exp, rtol=0, atol=1e-12)


def test_large_point_request_is_chunked():
    ex = HostExecutor(64)
    sch = Scheduler(ex, sample_budget=64)
    pos = np.linspace(0, 1, 1000)
    r = Request(model="m1", kind="points", n=1000, pos=pos)
    sch.run([r], realtime=False)
    assert r.iterations == (1000 + 63) // 64
    np.testing.assert_allclose(r.result, _expected_points(r), atol=1e-12)


def test_poisson_arrivals_and_stats():
    a = poisson_arrivals(50.0, 4000, seed=5004)
    assert np.all(np.diff(a) > 0)
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0
    reqs = [Request(model="m0", kind="render", W=2, H=2, arrival=float(i)) for i in range(10)]
    for i, r in enumerate(reqs):
        r.t_done = r.arrival + 0.001 * (i + 1)
    s = latency_stats(reqs)
    assert abs(s["p50_ms"] - 5.5) < 1e-9 and s["requests"] == 10
    assert abs(s["rays_per_s"] - 40 / 9.01) < 1e-9


def test_requests_with_array_fields_retire_in_any_order():
    # requests compare by identity, so array-valued fields never reach ==
    ex = HostExecutor(400)
    sch = Scheduler(ex, sample_budget=400)
    reqs = [Request(model="m0", kind="render", W=9 - k, H=3, view=np.arange(14.0))
            for k in range(5)]
    sch.run(reqs, realtime=False)
    assert len(sch.finished) == 5
