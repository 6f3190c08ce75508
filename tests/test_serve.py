"""Scheduler of the serving loop on the CPU, with a simulated engine and clock."""
import numpy as np
import pytest

from paper_1712_06758_amd.serve import Server, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeEngine:
    """Simulated engine: every sample needs `iters` iterations; one step advances
    all busy slots by `poll` iterations and costs `step_cost` seconds."""

    def __init__(self, n, slots, clock, iters=40, poll=8, step_cost=1e-3):
        self.n, self.slots, self.clock = n, slots, clock
        self.free = list(range(slots - 1, -1, -1))
        self.busy = {}
        self.slot_bytes = 100 * n ** 3
        self.iters, self.poll_iters, self.step_cost = iters, poll, step_cost
        self.max_busy = 0
        self.started = []

    def has_free(self):
        return bool(self.free)

    def start(self, part, xi):
        slot = self.free.pop()
        part.slot = slot
        part.left = self.iters
        part.xi = xi
        self.busy[slot] = part
        self.max_busy = max(self.max_busy, len(self.busy))
        self.started.append(part)

    def step(self):
        for p in self.busy.values():
            p.left -= self.poll_iters
        self.clock.t += self.step_cost

    def ready(self):
        return True

    def poll(self):
        out = []
        for p in self.busy.values():
            if p.left <= 0:
                p.iters = self.iters
                out.append(p)
        return out

    def finish(self, part, mesh):
        del self.busy[part.slot]
        self.free.append(part.slot)
        part.result = (mesh, part.kind, part.xi)
        return part.result

    def sync(self):
        pass


def make(levels=(32, 64, 128), slots=None, budget=10 ** 12, keep=True):
    clock = FakeClock()
    sizes = sorted(set(levels) | {n // 2 for n in levels if n != min(levels)})
    slots = slots or {n: 4 for n in sizes}
    engines = {n: FakeEngine(n, slots[n], clock) for n in sizes}
    srv = Server(engines, levels, noise_fn=lambda level, seed: ("xi", level, seed),
                 restrict_fn=lambda xi, n: ("xc",) + xi[1:], hbm_budget=budget, clock=clock,
                 keep_results=keep)
    return srv, engines, clock


def arrivals(spec):
    return sorted(spec)


def test_all_requests_complete_with_coupled_parts():
    srv, eng, clock = make()
    arr = arrivals([(0.001 * i, (32, 64, 128)[i % 3], i) for i in range(60)])
    rep = srv.run(arr)
    assert rep["completed"] == 60
    for r in srv.done:
        kinds = sorted(p.kind for p in r.parts)
        if r.level == 32:
            assert kinds == ["fine"]
        else:
            assert kinds == ["coarse", "fine"]
            assert r.parts[1].box_n == r.level // 2
            # the coarse part is driven by the restricted fine noise of the same request
            assert r.parts[1].result[2] == ("xc", r.level, (r.level, r.rid))
        assert r.t_done >= r.t_admit >= r.t_arrival - 1e-12


def test_fifo_per_level_and_slot_reuse():
    srv, eng, clock = make(levels=(32,), slots={32: 2})
    arr = arrivals([(0.0, 32, i) for i in range(10)])
    srv.run(arr)
    order = [r.rid for r in sorted(srv.done, key=lambda r: r.t_admit)]
    assert order == sorted(order)
    assert eng[32].max_busy == 2                    # slots were reused, never over-filled
    assert len(eng[32].started) == 10


def test_hbm_budget_bounds_in_flight_work():
    srv, eng, clock = make(levels=(32, 64))
    fp64 = srv.footprint(srv.submit(64, (64, -1), 0.0, -1)); srv.queues[64].clear()
    srv2, eng2, _ = make(levels=(32, 64), budget=fp64 + 10)
    arr = arrivals([(0.0, 64, i) for i in range(6)] + [(0.0, 32, 100 + i) for i in range(6)])
    rep = srv2.run(arr)
    assert rep["completed"] == 12
    assert srv2.peak_in_flight <= fp64 + 10
    # with room for one level-64 request at a time, at most one is in flight
    assert eng2[64].max_busy == 1


def test_oversized_request_is_refused():
    srv, eng, clock = make(levels=(32, 64), budget=1000)
    rep = srv.run(arrivals([(0.0, 64, 0), (0.0, 32, 1)]))
    assert rep["refused"] == 2 and rep["completed"] == 0


def test_large_request_is_not_starved_by_small_ones():
    srv, eng, clock = make(levels=(32, 128), slots={32: 8, 64: 2, 128: 1})
    f128 = 100 * (128 ** 3 + 64 ** 3) + 16 * (128 ** 3 + 64 ** 3)
    srv.hbm_budget = f128 + 100 * 32 ** 3 * 2
    arr = [(0.0, 32, i) for i in range(3)] + [(0.0005, 128, 99)] + [(0.0006 + 1e-4 * i, 32, 200 + i) for i in range(50)]
    srv.run(sorted(arr))
    big = [r for r in srv.done if r.level == 128][0]
    later_small = [r for r in srv.done if r.level == 32 and r.t_arrival > big.t_arrival]
    assert all(r.t_admit >= big.t_admit for r in later_small)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert percentile([5, 1, 3], 50) == 3


def test_report_fields():
    srv, eng, clock = make()
    rep = srv.run(arrivals([(0.0, n, i) for i, n in enumerate((32, 64, 128) * 5)]))
    for n in (32, 64, 128):
        lv = rep["levels"][n]
        assert lv["requests"] == 5 and lv["p99_ms"] >= lv["p50_ms"] > 0
    assert rep["samples_per_s"] > 0


def test_big_level_cu_mask_keeps_every_xcd_populated():
    from paper_1712_06758_amd.serve import big_level_cu_mask
    w = big_level_cu_mask(256, 32)
    assert w.dtype == np.uint32 and w.size == 8
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")
    assert bits.sum() == 224 and bits[:224].all() and not bits[224:].any()
    # mask bits go to the 8 XCDs in turn: each keeps 28 units and frees 4
    assert all(bits[x::8].sum() == 28 for x in range(8))
    with pytest.raises(ValueError):
        big_level_cu_mask(256, 0)
    with pytest.raises(ValueError):
        big_level_cu_mask(256, 256)
