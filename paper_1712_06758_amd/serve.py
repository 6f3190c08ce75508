"""Continuous-batching request loop for a multilevel Monte Carlo driver.

A request at level n asks for a coupled pair of Gaussian-field samples of the
same random event (Sec. "Hierarchical SPDE sampler with non-matching mesh
embedding"): the fine sample on the n^3 box and, unless n is the coarsest
level, the coarse sample on the (n/2)^3 box driven by the restricted noise of
eq. ml-linsys.  Both are projected onto the level's tet mesh.

Each box size has one resident engine: a sampler handle (operators and
multigrid hierarchy stay on the device), its own HIP stream and a pool of
slots.  The loop
  * moves arrived requests into per-engine FIFO queues,
  * admits queued work into free slots while the HBM footprint of in-flight
    work stays within the budget (continuous batching: slots are refilled
    while the other slots keep iterating),
  * enqueues a few MINRES iterations on every engine (the engines' streams run
    concurrently on the device),
  * polls, retires converged slots (field -> projection), and completes a
    request when all its parts are done.
The engine interface is small so that the scheduler can be exercised on the
CPU with a simulated engine (tests/test_serve.py).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import sys
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import _abi


# ---------------------------------------------------------------------------
# request bookkeeping


@dataclass
class Part:
    req: "Request"
    box_n: int                 # box edge this part is solved on
    kind: str                  # "fine" or "coarse"
    slot: int = -1
    iters: int = 0
    result: object = None      # u_tet tensor (GPU engine) or None
    done_event: object = None  # marks the end of the part's projection on its engine's stream


@dataclass
class Request:
    rid: int
    level: int
    seed: tuple
    t_arrival: float
    parts: list = field(default_factory=list)
    t_admit: float = -1.0
    t_done: float = -1.0
    footprint: int = 0
    pending: int = 0
    noise: object = None       # fine noise (tensor or NoiseKey), kept for verification when asked


@dataclass(frozen=True)
class NoiseKey:
    """Noise of a request part, drawn on the device by the counter-based
    generator: the event's own field (coupled = 0) or the restriction of the
    event's field on the twice finer box (coupled = 1, the coarse part)."""
    seed: int
    event: int
    coupled: int = 0


def request_event(seed) -> int:
    """Generator event of a request (level, index): unique per request."""
    level, r = seed
    return (int(level) << 40) | int(r)


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


# ---------------------------------------------------------------------------
# GPU engine


class GpuEngine:
    """One box size: a resident sampler handle, a stream and a slot pool."""

    STATE_ACTIVE, STATE_DONE, STATE_NOTCONV, STATE_FAILED, STATE_IDLE = 0, 1, 2, 3, 4

    def __init__(self, n, kappa, g, precision, slots, device, rtol=None, meshes=None, poll=4, transfers=None,
                 cu_mask=None):
        import torch
        from . import Box
        self.torch = torch
        self.n = n
        self.slots = slots
        self.device = device
        self.box = Box(n, kappa, g, precision=precision, rtol=rtol, max_batch=slots, device=device)
        self.box.set_poll_interval(poll)
        self.poll_iters = poll
        if cu_mask is None:
            self.stream = torch.cuda.Stream(device=device)
        else:   # a stream confined to the compute units of the mask
            self.stream = masked_stream(device, cu_mask, n)
        self.free = list(range(slots - 1, -1, -1))
        self.busy = {}
        self.transfers = {}           # mesh name -> (n_tet, nnz, rp, ci, cv)
        self.host_transfers = {}
        for name, (xyz, tets) in (meshes or {}).items():
            self.host_transfers[name] = self.add_mesh(name, xyz, tets)
        for name, (rp, ci, cv) in (transfers or {}).items():
            self.add_transfer(name, rp, ci, cv)
        L = _abi.lib()
        with torch.cuda.device(device), torch.cuda.stream(self.stream):
            _abi.check(L.spde_slots_reset(self.box._hh.h, slots, self._sp()))
        self.slot_bytes = self.box.info()["workspace_bytes"] // slots
        self._state = np.zeros(slots, dtype=np.int32)
        self._iters = np.zeros(slots, dtype=np.int32)
        self._event = None

    def _sp(self):
        return C.c_void_p(self.stream.cuda_stream)

    def add_mesh(self, name, xyz, tets):
        """Pi of this box onto a tet mesh, built from the geometry (host clipper);
        returns the host CSR."""
        from . import build_transfer_host
        rp, ci, cv = build_transfer_host(self.n, xyz, tets)
        self.add_transfer(name, rp, ci, cv)
        return rp, ci, cv

    def add_transfer(self, name, rp, ci, cv):
        """Register a host CSR Pi of this box onto the tet mesh `name`."""
        from . import transfer_chunk_order
        torch = self.torch
        d = self.device
        self.transfers[name] = (rp.size - 1, ci.size, torch.as_tensor(rp).to(d),
                                torch.as_tensor(ci).to(d), torch.as_tensor(cv).to(d),
                                torch.as_tensor(transfer_chunk_order(self.n, rp, ci)).to(d))

    def has_free(self):
        return bool(self.free)

    def start(self, part, xi):
        """Start `part` in a free slot from a noise tensor [n^3] on the device or
        from a NoiseKey (noise drawn inside the initialisation kernel)."""
        slot = self.free.pop()
        part.slot = slot
        self.busy[slot] = part
        L = _abi.lib()
        with self.torch.cuda.device(self.device):
            if isinstance(xi, NoiseKey):
                _abi.check(L.spde_slot_start_seeded(self.box._hh.h, slot, xi.seed, xi.event, xi.coupled,
                                                    self._sp()))
                return
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            xi.record_stream(self.stream)
            _abi.check(L.spde_slot_start(self.box._hh.h, slot, C.c_void_p(xi.data_ptr()), self._sp()))

    def step(self):
        if not self.busy:
            return
        with self.torch.cuda.device(self.device):
            _abi.check(_abi.lib().spde_slots_step(self.box._hh.h, self.slots, self.poll_iters, self._sp()))
            self._event = self.torch.cuda.Event()
            self._event.record(self.stream)

    def ready(self):
        """True when the last enqueued step has finished on the device."""
        return self._event is None or self._event.query()

    def poll(self):
        """Finished parts (state != active) after the enqueued work."""
        if not self.busy:
            return []
        L = _abi.lib()
        with self.torch.cuda.device(self.device):
            _abi.check(L.spde_slots_poll(self.box._hh.h, self.slots, self._state.ctypes.data,
                                         self._iters.ctypes.data, self._sp()))
        out = []
        for slot, part in list(self.busy.items()):
            st = int(self._state[slot])
            if st != self.STATE_ACTIVE:
                part.iters = int(self._iters[slot])
                part.status = st
                out.append(part)
        return out

    def finish(self, part, mesh):
        """Field of a finished part projected onto `mesh`; frees the slot."""
        torch = self.torch
        L = _abi.lib()
        n_tet, nnz, rp, ci, cv, od = self.transfers[mesh]
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            u = torch.empty(self.n ** 3, dtype=torch.float64, device=self.device)
            ut = torch.empty(n_tet, dtype=torch.float64, device=self.device)
            _abi.check(L.spde_slot_finish(self.box._hh.h, part.slot, C.c_void_p(u.data_ptr()), self._sp()))
            # one sample: the product needs no work buffer
            _abi.check(L.spde_csr_apply(n_tet, nnz, C.c_void_p(rp.data_ptr()), C.c_void_p(ci.data_ptr()),
                                        C.c_void_p(cv.data_ptr()), self.n ** 3, 1, C.c_void_p(u.data_ptr()),
                                        C.c_void_p(ut.data_ptr()), C.c_void_p(od.data_ptr()), None, 0,
                                        self._sp()))
            part.done_event = torch.cuda.Event()
            part.done_event.record(self.stream)
        del self.busy[part.slot]
        self.free.append(part.slot)
        part.result = ut
        return ut


# ---------------------------------------------------------------------------
# the server


class Server:
    """Continuous-batching MLMC request loop over per-box-size engines.

    engines: {box_n: engine}; every level n needs engines n and n/2 (except the
    coarsest level).  hbm_budget: bytes of device memory that in-flight work may
    claim (slot workspace share plus per-request noise and outputs).  A request
    is admitted when its parts find free slots and its footprint fits the
    budget; build_gpu_server derives the budget from the device memory left
    free after the engines are built, so with the default slot pools the slot
    count is what binds."""

    def __init__(self, engines, levels, noise_fn, restrict_fn, hbm_budget, clock=time.perf_counter,
                 keep_results=False):
        self.engines = engines
        self.levels = sorted(levels)
        self.coarsest = self.levels[0]
        self.noise_fn = noise_fn
        self.restrict_fn = restrict_fn
        self.hbm_budget = hbm_budget
        self.clock = clock
        self.keep_results = keep_results
        self.queues = {n: deque() for n in engines}
        self.in_flight = 0
        self.peak_in_flight = 0
        self.done = []
        self.refused = 0
        self.queue_depth = []

    def parts_of(self, req):
        parts = [Part(req, req.level, "fine")]
        if req.level != self.coarsest:
            parts.append(Part(req, req.level // 2, "coarse"))
        return parts

    def footprint(self, req):
        b = 0
        for p in req.parts:
            e = self.engines[p.box_n]
            b += e.slot_bytes + 2 * 8 * p.box_n ** 3
        return b

    def submit(self, level, seed, t_arrival, rid):
        req = Request(rid, level, seed, t_arrival)
        req.parts = self.parts_of(req)
        req.footprint = self.footprint(req)
        if req.footprint > self.hbm_budget:
            self.refused += 1
            return None
        req.pending = len(req.parts)
        # requests are admitted whole: queue the request at its fine engine
        self.queues[level].append(req)
        return req

    def _slots_available(self, req):
        need = {}
        for p in req.parts:
            need[p.box_n] = need.get(p.box_n, 0) + 1
        return all(len(self.engines[n].free) >= k for n, k in need.items())

    def _admit(self, now):
        """Admit queued requests oldest-first across levels.  A request that does
        not fit the HBM budget blocks admission (it is not bypassed, so large
        requests cannot starve); one whose engine has no free slot lets younger
        requests of other levels through."""
        while True:
            heads = sorted((q[0] for q in self.queues.values() if q), key=lambda r: (r.t_arrival, r.rid))
            admitted = False
            for req in heads:
                if self.in_flight + req.footprint > self.hbm_budget:
                    return
                if not self._slots_available(req):
                    continue
                self.queues[req.level].popleft()
                xi = self.noise_fn(req.level, req.seed)
                if self.keep_results:
                    req.noise = xi
                self.engines[req.level].start(req.parts[0], xi)
                if len(req.parts) == 2:
                    xc = self.restrict_fn(xi, req.level)
                    self.engines[req.level // 2].start(req.parts[1], xc)
                req.t_admit = now
                self.in_flight += req.footprint
                self.peak_in_flight = max(self.peak_in_flight, self.in_flight)
                admitted = True
                break
            if not admitted:
                return

    def _retire(self, e, t0):
        for part in e.poll():
            req = part.req
            e.finish(part, req.level)
            if not self.keep_results:
                part.result = None
            req.pending -= 1
            if req.pending == 0:
                # the parts ran on different engines' streams: the request is
                # done when the last projection of every part has finished
                for p in req.parts:
                    if p.done_event is not None:
                        p.done_event.synchronize()
                req.t_done = self.clock() - t0
                self.in_flight -= req.footprint
                self.done.append(req)

    def run(self, arrivals, time_limit=None, progress_every=None):
        """Serve `arrivals`, a list of (t, level, request_index) sorted by t
        (seconds after the start).  Each engine is polled, refilled and stepped
        again as soon as its previous step has finished on the device, so small
        boxes cycle at their own pace beside large ones."""
        t0 = self.clock()
        ai = 0
        total = len(arrivals)
        n_done0 = len(self.done)
        next_report = progress_every
        while len(self.done) - n_done0 < total - self.refused:
            now = self.clock() - t0
            if next_report is not None and now >= next_report:
                print(f"[serve] t={now:.1f}s arrived={ai} done={len(self.done) - n_done0} "
                      f"queued={sum(len(q) for q in self.queues.values())}", file=sys.stderr, flush=True)
                next_report += progress_every
            if time_limit is not None and now > time_limit:
                break
            while ai < total and arrivals[ai][0] <= now:
                t, level, r = arrivals[ai]
                self.submit(level, (level, r), t, ai)
                ai += 1
            progressed = False
            for e in self.engines.values():
                if e.busy and e.ready():
                    self._retire(e, t0)
                    progressed = True
            self._admit(self.clock() - t0)
            self.queue_depth.append((now, sum(len(q) for q in self.queues.values())))
            for e in self.engines.values():
                if e.busy and e.ready():
                    e.step()
                    progressed = True
            if not progressed:
                if ai < total and not any(e.busy for e in self.engines.values()) and \
                        not any(self.queues.values()):
                    wait = arrivals[ai][0] - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.005))
                else:
                    time.sleep(2e-5)
        return self.report(self.clock() - t0, n_done0)

    def report(self, wall, first=0):
        done = self.done[first:]
        out = {"wall_s": round(wall, 3), "completed": len(done), "refused": self.refused,
               "peak_in_flight_bytes": self.peak_in_flight, "levels": {}}
        samples = 0
        for n in self.levels:
            reqs = [r for r in done if r.level == n]
            if not reqs:
                continue
            lat = [r.t_done - r.t_arrival for r in reqs]
            wait = [r.t_admit - r.t_arrival for r in reqs]
            it = [p.iters for r in reqs for p in r.parts]
            samples += sum(len(r.parts) for r in reqs)
            out["levels"][n] = {"requests": len(reqs), "p50_ms": round(1e3 * percentile(lat, 50), 3),
                                "p99_ms": round(1e3 * percentile(lat, 99), 3),
                                "mean_queue_wait_ms": round(1e3 * float(np.mean(wait)), 3),
                                "mean_iters": round(float(np.mean(it)), 2),
                                "requests_per_s": round(len(reqs) / wall, 2) if wall > 0 else 0.0}
        # a request is one coupled pair (fine + coarse part, fine only on the
        # coarsest level); samples count the parts
        out["requests_per_s"] = round(len(done) / wall, 2) if wall > 0 else 0.0
        out["samples_per_s"] = round(samples / wall, 2) if wall > 0 else 0.0
        out["max_queue_depth"] = max((d for _, d in self.queue_depth), default=0)
        return out


# ---------------------------------------------------------------------------
# GPU server construction and the command-line load run


# Slots per box size.  Small levels get many: a request then never waits for a
# free slot, and its latency is set by how fast its engine steps while sharing
# the GPU.  (More slots on the small levels raise the sustainable request rate
# at the cost of latency.)
DEFAULT_SLOTS = {16: 128, 32: 128, 64: 64, 128: 16, 256: 4}
# compute units kept free of the 128^3 / 256^3 engines' kernels (4 per XCD of 256)
DEFAULT_RESERVE_CUS = 32


_MASKED_STREAMS = {}


def masked_stream(device, cu_mask, tag):
    """A stream whose kernels run only on the compute units of cu_mask (bit i of
    word w: unit 32 w + i), one per (device, mask, tag) for the life of the
    process, like torch's own stream pool: tensors whose memory was last used on
    it (results, noise marked with record_stream) may outlive any engine."""
    import torch
    words = np.ascontiguousarray(cu_mask, dtype=np.uint32)
    device = torch.device(device)
    key = (device.index, words.tobytes(), tag)
    st = _MASKED_STREAMS.get(key)
    if st is None:
        ptr = C.c_void_p()
        with torch.cuda.device(device):
            _abi.check(_abi.lib().spde_stream_create_cu_mask(words.size, words.ctypes.data, C.byref(ptr)))
        st = _MASKED_STREAMS[key] = torch.cuda.ExternalStream(ptr.value, device=device)
    return st


def big_level_cu_mask(n_cu, reserve):
    """CU mask words for the long-kernel engines: the first n_cu - reserve mask
    bits set.  The runtime deals consecutive mask bits out to the XCDs in turn
    (it rejects a mask that leaves one XCD with no compute unit), so the top
    bits are the last compute units of every XCD: with reserve a multiple of 8
    each XCD keeps reserve / 8 of its units for the short kernels of the small
    levels."""
    if not 0 < reserve < n_cu:
        raise ValueError(f"reserve must lie in (0, {n_cu})")
    words = np.zeros((n_cu + 31) // 32, dtype=np.uint32)
    for i in range(n_cu - reserve):
        words[i // 32] |= np.uint32(1 << (i % 32))
    return words


def build_gpu_server(levels=(32, 64, 128, 256), corr_len=0.05, precision="mixed", slots=None,
                     hbm_budget=None, device=None, keep_results=False, poll=4, noise_seed=2024,
                     reserve_cus=DEFAULT_RESERVE_CUS, big_level=128):
    """Engines for the levels and their coupled coarse boxes.  A request's noise
    is the generator field of (noise_seed, request_event(request seed)); its
    coarse part draws the restriction of that field.  reserve_cus > 0: the
    engines of boxes of big_level^3 and above run on streams that leave that many
    compute units to the smaller boxes, whose kernels then need not wait for a
    long kernel to finish."""
    import torch
    from . import coarsen_transfer_host, g_unit_variance
    from workloads import serve_mesh
    device = torch.device(device or "cuda:0")
    kappa = 1.0 / corr_len
    g = g_unit_variance(kappa)
    levels = sorted(levels)
    sizes = sorted(set(levels) | {n // 2 for n in levels if n != levels[0]})
    slots = slots or {n: DEFAULT_SLOTS.get(n, 8) for n in sizes}
    engines = {}
    meshes = {n: serve_mesh(n) for n in levels}
    big_mask = None
    if reserve_cus > 0:
        n_cu = torch.cuda.get_device_properties(device).multi_processor_count
        big_mask = big_level_cu_mask(n_cu, reserve_cus)
    # finest first: the coarse part of level n projects with Pi of the (n/2)^3 box
    # onto level n's mesh, coarsened from the fine engine's Pi (children summed,
    # eq. recursive_l2_projection) instead of clipped again
    for n in sorted(sizes, reverse=True):
        need = {n: meshes[n]} if n in levels else {}
        coarse = {}
        if 2 * n in levels:
            coarse[2 * n] = coarsen_transfer_host(2 * n, *engines[2 * n].host_transfers[2 * n])
        engines[n] = GpuEngine(n, kappa, g, precision, slots[n], device, meshes=need, poll=poll,
                               transfers=coarse, cu_mask=big_mask if n >= big_level else None)
        if 2 * n in engines:
            engines[2 * n].host_transfers.clear()     # device copies are registered
    if hbm_budget is None:
        # the slot workspaces are bound already; what in-flight requests may add
        # (noise and output buffers) is the device memory still free, less a
        # reserve of 4 GiB.  On a 288 GB device the slot pools bind long before
        # this budget does, so admission is in practice by free slots.
        free, _ = torch.cuda.mem_get_info(device)
        hbm_budget = sum(e.slot_bytes * e.slots for e in engines.values()) + max(0, free - (4 << 30))

    def noise_fn(level, seed):
        return NoiseKey(int(noise_seed), request_event(seed))

    def restrict_fn(key, n):
        return NoiseKey(key.seed, key.event, 1)

    return Server(engines, levels, noise_fn, restrict_fn, hbm_budget, keep_results=keep_results)


def main(argv=None):
    ap = argparse.ArgumentParser(description="MLMC serving load run (continuous batching)")
    ap.add_argument("--duration", type=float, default=10.0, help="arrival window in seconds")
    ap.add_argument("--scale", type=float, default=1.0, help="multiplier of the request rates")
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--levels", default="32,64,128,256")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--reserve-cus", type=int, default=DEFAULT_RESERVE_CUS,
                    help="compute units kept free of the 128^3 and 256^3 engines' kernels (0: none)")
    ap.add_argument("--slots", default="",
                    help="slots per box size overriding the defaults, e.g. 32:512,64:128,256:8")
    args = ap.parse_args(argv)
    from workloads import SERVE_LEVELS, SERVE_CORR_LEN, poisson_arrivals
    levels = [int(x) for x in args.levels.split(",")]
    rates = {n: SERVE_LEVELS[n] * args.scale for n in levels}
    slots = None
    if args.slots:
        over = {int(k): int(v) for k, v in (item.split(":") for item in args.slots.split(","))}
        sizes = sorted(set(levels) | {n // 2 for n in levels if n != min(levels)})
        slots = {n: over.get(n, DEFAULT_SLOTS.get(n, 8)) for n in sizes}
    srv = build_gpu_server(levels, SERVE_CORR_LEN, args.precision, slots=slots, reserve_cus=args.reserve_cus)
    # warm-up: one request per level, not timed
    warm = [(0.0, n, 10 ** 6 + i) for i, n in enumerate(levels)]
    srv.run(warm)
    srv.done.clear()
    srv.queue_depth.clear()
    arrivals = poisson_arrivals(rates, args.duration, seed=args.seed)
    print(f"[serve] {len(arrivals)} requests over {args.duration} s at rate scale {args.scale}",
          file=sys.stderr, flush=True)
    rep = srv.run(arrivals, time_limit=args.duration * 4 + 30, progress_every=2.0)
    rep["rates_per_s"] = rates
    rep["precision"] = args.precision
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
