"""Continuous-batching SpMM server over the C ABI.

Requests (matrix id from a resident pool, N, B type, B seed, arrival time)
arrive on a Poisson clock.  The scheduler:

* admits waiting requests in arrival order while their HBM footprint fits
  the budget: the plan (resident, or built on admission) plus what the
  library reports one batched execution occupies (``spmm_run_bytes``: B, C
  and the request's share of the submission's workspace); a request that
  does not fit now lets later, smaller ones pass (no head-of-line blocking),
  and one that can never fit -- the library answers BUDGET for the whole
  budget less its plan -- is rejected;
* keeps plans resident in an LRU cache charged to the same budget, evicting
  only plans no in-flight request uses;
* forms a batch as soon as one of its streams is free and launches it with
  one ``spmm_submit`` (one graph replay of the persistent kernels), so
  batches on different streams overlap on the device while new requests keep
  being admitted as earlier ones complete.  Requests are sized by their
  plan's algorithmic bytes: a large one (estimated above ``large_ms`` at
  ``est_rate`` bytes/s) runs alone, as an ``spmm_run`` (one workgroup per
  item, so the device interleaves other streams' work with it, which the
  persistent batched kernels would lock out), on at most ``large_streams``
  streams at once (one by default: measured at 0.7x saturation with four
  streams, two large streams left small requests a p99 of 13.5 ms against
  5.6 ms with one, for 3% less throughput), so small requests always have a
  stream; small ones batch together
  (up to ``max_batch``), overtaking large ones that wait for a stream;
* polls tickets (an event for a large request) and retires finished
  requests immediately, freeing their memory, and records latency =
  completion - arrival on the host monotonic clock.

The arithmetic of every request is fixed by its plan and N, so a request's
result is bitwise the same alone and in any mix.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from . import api

GiB = 1 << 30


@dataclass
class Request:
    rid: int
    matrix: int
    n: int
    b_kind: str
    seed: int
    arrival: float                      # seconds from the start of the stream
    admitted_at: float = -1.0
    done_at: float = -1.0
    status: str = "waiting"            # waiting | admitted | running | done | rejected
    footprint: int = 0                 # bytes of its execution (B, C, workspace share)
    need: int = 0                      # footprint plus its plan's bytes, checked at admission
    large: bool = False                # runs in a batch of its own (see Server)
    B: object = None
    C: object = None


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    small_latencies_ms: list = field(default_factory=list)
    large_latencies_ms: list = field(default_factory=list)
    rejected: int = 0
    batches: int = 0
    batch_sizes: list = field(default_factory=list)
    max_queue: int = 0
    flops: float = 0.0
    wall_s: float = 0.0
    plan_builds: int = 0
    plan_evictions: int = 0

    def summary(self) -> dict:
        def arr(x):
            return np.array(x) if x else np.zeros(1)
        lat, small, large = arr(self.latencies_ms), arr(self.small_latencies_ms), arr(self.large_latencies_ms)
        done = len(self.latencies_ms)
        return {
            "completed": done,
            "rejected": self.rejected,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "large": len(self.large_latencies_ms),
            "p50_small_ms": float(np.percentile(small, 50)),
            "p99_small_ms": float(np.percentile(small, 99)),
            "p50_large_ms": float(np.percentile(large, 50)),
            "p99_large_ms": float(np.percentile(large, 99)),
            "mean_ms": float(lat.mean()),
            "throughput_req_s": done / self.wall_s if self.wall_s > 0 else 0.0,
            "gflops": self.flops / self.wall_s / 1e9 if self.wall_s > 0 else 0.0,
            "batches": self.batches,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "max_queue": self.max_queue,
            "plan_builds": self.plan_builds,
            "plan_evictions": self.plan_evictions,
            "wall_s": self.wall_s,
        }


class PlanCache:
    """Resident plans keyed by (matrix, N, B type), LRU, charged to the budget."""

    def __init__(self, pool, opts_for):
        self.pool = pool
        self.opts_for = opts_for
        self.plans = collections.OrderedDict()   # key -> (plan, bytes)
        self.users = collections.Counter()
        self.alg = {}                            # key -> algorithmic bytes of one run

    def bytes_of(self, key) -> int:
        return self.plans[key][1] if key in self.plans else 0

    def alg_bytes(self, key) -> float:
        return self.alg.get(key, 0.0)

    def get(self, key, stats: Stats):
        if key in self.plans:
            self.plans.move_to_end(key)
            return self.plans[key][0]
        mid, n, b_kind = key
        A = self.pool[mid]["A"]
        opts = self.opts_for(self.pool[mid], n, b_kind)
        if hasattr(A, "host_rows"):
            # a matrix held on the device: the plan is built there (spmm_plan_device)
            plan = api.Plan.on_device(A.rowptr, A.colidx, A.vals, A.m, A.k, n, b_kind, opts)
        else:
            plan = api.Plan(A, n, b_kind, opts)
        st = plan.stats()
        self.plans[key] = (plan, st["device_bytes"])
        self.alg[key] = float(st["algorithmic_bytes"])
        stats.plan_builds += 1
        return plan

    def evictable_bytes(self, keep=None) -> int:
        return sum(b for k, (p, b) in self.plans.items() if self.users[k] == 0 and k != keep)

    def evict(self, need: int, stats: Stats, keep=None) -> int:
        freed = 0
        for k in list(self.plans.keys()):
            if freed >= need:
                break
            if self.users[k] == 0 and k != keep:
                plan, b = self.plans.pop(k)
                plan.destroy()
                freed += b
                stats.plan_evictions += 1
        return freed

    def resident_bytes(self) -> int:
        return sum(b for _, b in self.plans.values())


def default_opts_for(item, n, b_kind):
    """Plan options per matrix kind: block masks use aligned windows of 64
    rows (one window per 64-row block-row, whose dense 64x64 blocks fill its
    tiles, so each block-row stages its B rows once), graphs the
    tuned/heuristic default."""
    if item["kind"] == "mask":
        return api.default_opts(mode="mixed", row_order="original_ranges", window_h=64)
    return api.default_opts(mode="auto")


class Server:
    def __init__(self, pool, budget_bytes=200 * GiB, n_streams=4, max_batch=64,
                 opts_for=default_opts_for, keep_results=False, large_ms=1.0, est_rate=1.5e12,
                 large_streams=None):
        import torch
        self.torch = torch
        self.pool = pool
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.plans = PlanCache(pool, opts_for)
        self.keep_results = keep_results
        self.used = 0
        self.large_ms = large_ms
        # streams that may run a large request at once (at least one stays for small ones)
        self.large_streams = max(1, min(n_streams - 1, 1 if large_streams is None
                                        else large_streams)) if n_streams > 1 else 1
        self.large_bytes = large_ms * 1e-3 * est_rate

    def _plan_key(self, r: Request):
        return (r.matrix, r.n, r.b_kind)

    # --- main loop ----------------------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Serve ``requests`` (list of dicts from synth.serving_requests).
        With ``realtime`` the arrival times are honoured on the host clock;
        otherwise every request is available at once (closed loop)."""
        torch = self.torch
        reqs = [Request(**{k: d[k] for k in ("rid", "matrix", "n", "b_kind", "seed", "arrival")})
                for d in requests]
        stats = Stats()
        waiting = collections.deque()
        inflight = {}          # stream index -> (ticket, [requests], large batch)
        free_streams = list(range(len(self.streams)))
        t0 = time.monotonic()
        nxt = 0
        finished = 0
        total = len(reqs)
        while finished < total:
            now = time.monotonic() - t0
            # arrivals
            while nxt < total and (not realtime or reqs[nxt].arrival <= now):
                if not realtime:
                    reqs[nxt].arrival = now
                waiting.append(reqs[nxt])
                nxt += 1
            stats.max_queue = max(stats.max_queue, len(waiting))
            # completions
            for si in list(inflight.keys()):
                done, batch, _ = inflight[si]
                if done():
                    tdone = time.monotonic() - t0
                    for r in batch:
                        r.done_at = tdone
                        r.status = "done"
                        stats.latencies_ms.append((tdone - r.arrival) * 1e3)
                        (stats.large_latencies_ms if r.large else
                         stats.small_latencies_ms).append((tdone - r.arrival) * 1e3)
                        A = self.pool[r.matrix]["A"]
                        stats.flops += 2.0 * A.nnz * r.n
                        self.used -= r.footprint
                        self.plans.users[self._plan_key(r)] -= 1
                        if not self.keep_results:
                            r.B = None
                            r.C = None
                        finished += 1
                    del inflight[si]
                    free_streams.append(si)
            # admission + batch formation on a free stream
            if free_streams and waiting:
                si = free_streams[0]
                stream = self.streams[si]
                batch = []
                big_batch = False
                keep = collections.deque()
                # a large request may take this stream while fewer than
                # large_streams run (so small ones always keep a stream)
                large_ok = sum(1 for v in inflight.values() if v[2]) < self.large_streams
                while waiting and len(batch) < self.max_batch:
                    r = waiting.popleft()
                    key = self._plan_key(r)
                    plan = self.plans.get(key, stats)
                    big = self.plans.alg_bytes(key) > self.large_bytes
                    if big and (batch or not large_ok):
                        keep.append(r)             # alone, on a later stream
                        continue
                    pbytes = self.plans.bytes_of(key)
                    # the library's footprint of one batched execution, checked
                    # against the whole budget less the plan: BUDGET = never fits
                    st, io = plan.run_bytes(batched=not big, budget=max(0, self.budget - pbytes))
                    r.footprint, r.need = io, io + pbytes
                    if st == L.SPMM_ERR_BUDGET:
                        r.status = "rejected"
                        stats.rejected += 1
                        finished += 1
                        continue
                    occupied = self.used + self.plans.resident_bytes() + io
                    if occupied > self.budget:
                        over = occupied - self.budget
                        if self.plans.evictable_bytes(keep=key) >= over:
                            self.plans.evict(over, stats, keep=key)
                        else:
                            keep.append(r)         # wait for memory; let smaller ones pass
                            continue
                    self.plans.users[key] += 1
                    self.used += r.footprint
                    A = self.pool[r.matrix]["A"]
                    dt = torch.float32 if r.b_kind == "f32" else torch.bfloat16
                    with torch.cuda.stream(stream):
                        g = torch.Generator(device="cuda")
                        g.manual_seed(r.seed)
                        r.B = torch.randn((A.k, r.n), generator=g, device="cuda",
                                          dtype=torch.float32).to(dt)
                        r.C = torch.empty((A.m, r.n), device="cuda", dtype=torch.float32)
                    r.status = "running"
                    r.admitted_at = time.monotonic() - t0
                    r.large = big
                    batch.append((r, plan))
                    if big:
                        big_batch = True
                        break
                keep.extend(waiting)
                waiting = keep
                if batch:
                    free_streams.pop(0)
                    if big_batch:
                        # one large request: spmm_run, whose grids hold one
                        # item per workgroup, so the device keeps dispatching
                        # other streams' work between its workgroups (the
                        # batched kernels are persistent and would hold every
                        # CU until they finish)
                        (r, plan), = batch
                        plan.run(r.B, r.C, stream=stream)
                        ev = torch.cuda.Event()
                        ev.record(stream)
                        done = ev.query
                    else:
                        items = [api.WorkItem(plan, r.B, r.C) for r, plan in batch]
                        ticket = api.spmm_submit(items, stream=stream)
                        done = (lambda t: lambda: api.spmm_poll(t))(ticket)
                    inflight[si] = (done, [r for r, _ in batch], big_batch)
                    stats.batches += 1
                    stats.batch_sizes.append(len(batch))
            elif not inflight and not waiting and nxt < total and realtime:
                time.sleep(max(0.0, min(0.001, reqs[nxt].arrival - now)))
            else:
                time.sleep(20e-6)
        torch.cuda.synchronize()
        stats.wall_s = time.monotonic() - t0
        self.requests = reqs
        return stats

    def solo(self, request: dict):
        """Run one request alone on the default stream (for the mix test)."""
        torch = self.torch
        r = Request(**{k: request[k] for k in ("rid", "matrix", "n", "b_kind", "seed", "arrival")})
        plan = self.plans.get(self._plan_key(r), Stats())
        A = self.pool[r.matrix]["A"]
        dt = torch.float32 if r.b_kind == "f32" else torch.bfloat16
        g = torch.Generator(device="cuda")
        g.manual_seed(r.seed)
        B = torch.randn((A.k, r.n), generator=g, device="cuda", dtype=torch.float32).to(dt)
        C = torch.empty((A.m, r.n), device="cuda", dtype=torch.float32)
        plan.run(B, C)
        torch.cuda.synchronize()
        return B, C
