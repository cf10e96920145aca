"""Continuous-batching request loop over the transform library.

A request asks for the inverse then the forward transform of its own batch of
maps at its own (L, spin) -- one "transform" per map, as in the throughput
benchmark.  The loop

* admits arrived requests in arrival order while their device-memory footprint
  fits in a fixed budget and a stream slot is free (admission by HBM
  footprint);
* groups the waiting requests that share (L, spin) with the oldest one into a
  single batched call (up to the library's batch limit), so one launch
  sequence serves all of them;
* runs each group on its own HIP stream, so groups admitted while others are
  still on the GPU overlap with them on the device;
* frees a group's memory and slot when its completion event fires, and times
  every request from its arrival to that event.

Plans (Wigner seed and spin tables, FFT tables) are built for every (L, spin)
before the loop starts and stay resident.  The scheduling logic
(``Scheduler``) is pure Python and runs without a GPU; ``GpuServer`` drives
the library through its C ABI on torch streams.
"""

from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

BATCH_MAX = 64   # the library's per-call batch limit


def footprint_bytes(L: int, batch: int, workspace: int, cbytes: int = 8) -> int:
    """Device bytes a group holds while in flight: its input coefficients, the
    maps, the output coefficients (``cbytes`` per complex) and one workspace."""
    N = 2 * L - 1
    return batch * (2 * L * L + L * N) * cbytes + workspace


@dataclasses.dataclass
class Group:
    L: int
    spin: int
    requests: list
    batch: int
    nbytes: int
    admitted_s: float = 0.0


class Scheduler:
    """FIFO admission with same-(L, spin) grouping under a memory budget.

    ``workspace(L, spin, batch)`` gives the library's workspace size for one
    batched call.  ``next_group`` takes the oldest waiting request and every
    later waiting request with the same (L, spin) that still fits the batch
    limit and the free memory; it returns None when the oldest request does not
    fit (head-of-line order is kept, so no request starves).
    """

    def __init__(self, budget_bytes: int, workspace: Callable[[int, int, int], int],
                 max_batch: int = BATCH_MAX, cbytes: int = 8):
        self.budget = int(budget_bytes)
        self.used = 0
        self.workspace = workspace
        self.max_batch = max_batch
        self.cbytes = cbytes
        self.waiting: collections.deque = collections.deque()

    def arrive(self, req) -> None:
        if req.batch > self.max_batch:
            raise ValueError(f"request {req.rid}: batch {req.batch} exceeds {self.max_batch}")
        need = footprint_bytes(req.L, req.batch, self.workspace(req.L, req.spin, req.batch), self.cbytes)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} bytes, more than the whole budget {self.budget}")
        self.waiting.append(req)

    def group_bytes(self, L: int, spin: int, batch: int) -> int:
        return footprint_bytes(L, batch, self.workspace(L, spin, batch), self.cbytes)

    def next_group(self) -> Optional[Group]:
        if not self.waiting:
            return None
        head = self.waiting[0]
        free = self.budget - self.used
        batch = head.batch
        need = self.group_bytes(head.L, head.spin, batch)
        if need > free:
            return None
        members = [head]
        for req in list(self.waiting)[1:]:
            if (req.L, req.spin) != (head.L, head.spin) or batch + req.batch > self.max_batch:
                continue
            more = self.group_bytes(head.L, head.spin, batch + req.batch)
            if more > free:
                continue
            members.append(req)
            batch += req.batch
            need = more
        for req in members:
            self.waiting.remove(req)
        self.used += need
        return Group(head.L, head.spin, members, batch, need)

    def release(self, group: Group) -> None:
        self.used -= group.nbytes
        assert self.used >= 0


@dataclasses.dataclass
class Result:
    rid: int
    L: int
    spin: int
    batch: int
    arrival_s: float
    done_s: float
    group_size: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not xs:
        return float("nan")
    ys = sorted(xs)
    k = max(0, min(len(ys) - 1, int(math.ceil(q / 100.0 * len(ys))) - 1))
    return ys[k]


class GpuServer:
    """Runs a request stream on one GPU (see the module docstring).

    ``precision`` is the library precision of every call ("fp32", "bf16x3" or
    "fp64"); ``streams`` the number of concurrent groups; ``budget_bytes`` the
    admission budget.  Inputs are drawn on the device from each request's seed
    (complex Gaussian, variance C_l = 1/(l+1)^2, zero for l < |spin|) inside
    the request's own buffers when its group is admitted.

    ``graphs`` > 0 keeps up to that many captured transforms (``sht.Graph``,
    one per (L, spin, batch) shape, each at most ``graph_bytes`` of device
    memory): a shape seen for the ``graph_after``-th time is captured (the
    least used idle graph makes room), and later groups of a cached shape
    replay its graph instead of launching the stages one by one, unless that
    graph is still in flight.  Graph buffers are outside the
    admission budget (the budget still reserves each request's own
    footprint).
    """

    def __init__(self, precision: str = "fp32", streams: int = 4, budget_bytes: int = 16 << 30,
                 device: int = 0, graphs: int = 0, graph_bytes: int = 1 << 30, graph_after: int = 3):
        import torch
        from . import sht
        self.torch = torch
        self.sht = sht
        self.precision = precision
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.budget = budget_bytes
        self.cdtype = sht.io_dtype(precision)
        self.cbytes = 16 if precision == "fp64" else 8
        self._ws_cache: Dict[Tuple[int, int, int], int] = {}
        self._scale: Dict[Tuple[int, int], "torch.Tensor"] = {}
        self.graph_cap = graphs
        self.graph_bytes = graph_bytes
        self.graph_after = graph_after
        self._graphs: "Dict[Tuple[int, int, int], list]" = {}   # shape -> [Graph, busy event or None]
        self._seen: Dict[Tuple[int, int, int], int] = {}
        self.graph_launches = 0
        self.graph_captures = 0

    def workspace(self, L: int, spin: int, batch: int) -> int:
        key = (L, spin, batch)
        if key not in self._ws_cache:
            self._ws_cache[key] = self.sht.workspace_bytes(L, spin, batch, self.precision)
        return self._ws_cache[key]

    def warm(self, keys: Iterable[Tuple[int, int]]) -> None:
        """Build the plan of every (L, spin) before serving."""
        for L, s in sorted(set(keys)):
            self.sht.plan_warmup(L, s, self.precision, self.dev)
            self._spectrum(L, s)
        self.torch.cuda.synchronize(self.dev)

    def _spectrum(self, L: int, spin: int):
        key = (L, spin)
        if key not in self._scale:
            torch = self.torch
            l_of = torch.repeat_interleave(torch.arange(L, dtype=torch.float64), 2 * torch.arange(L) + 1)
            sc = 1.0 / (l_of + 1.0)
            sc[l_of < abs(spin)] = 0.0
            self._scale[key] = sc.to(self.dev, torch.float32 if self.cbytes == 8 else torch.float64)
        return self._scale[key]

    def fill_input(self, req, out) -> None:
        """Seeded device draw of one request's coefficients into ``out`` [batch, L*L]."""
        torch = self.torch
        g = torch.Generator(device=self.dev)
        g.manual_seed(int(req.seed))
        out.copy_(torch.randn(out.shape, generator=g, device=self.dev, dtype=self.cdtype))
        out.mul_(self._spectrum(req.L, req.spin))

    def _graph_for(self, L: int, s: int, B: int):
        """The cached graph of this shape if it is idle (capturing it on the
        shape's second sighting), else None."""
        key = (L, s, B)
        self._seen[key] = self._seen.get(key, 0) + 1
        ent = self._graphs.get(key)
        if ent is not None:
            if ent[1] is not None and not ent[1].query():
                return None
            return ent
        foot = (2 * B * L * L + B * L * (2 * L - 1)) * self.cbytes + self.workspace(L, s, B)
        if self._seen[key] < self.graph_after or foot > self.graph_bytes:
            return None
        if len(self._graphs) >= self.graph_cap:
            idle = [k for k, e in self._graphs.items() if e[1] is None or e[1].query()]
            if not idle:
                return None
            victim = min(idle, key=lambda k: self._seen[k])
            if self._seen[victim] >= self._seen[key]:
                return None
            self._graphs.pop(victim)[0].close()
        ent = [self.sht.Graph(L, s, B, self.precision, device=self.dev), None]
        self._graphs[key] = ent
        self.graph_captures += 1
        return ent

    def close_graphs(self) -> None:
        for g, _ in self._graphs.values():
            g.close()
        self._graphs.clear()

    def _launch(self, group: Group, stream, keep: Optional[set]):
        torch = self.torch
        L, s, B = group.L, group.spin, group.batch
        ent = self._graph_for(L, s, B) if self.graph_cap > 0 else None
        if ent is not None:
            g = ent[0]
            with torch.cuda.stream(stream):
                off = 0
                slices = []
                for req in group.requests:
                    self.fill_input(req, g.flm_in[off:off + req.batch])
                    slices.append((req, off))
                    off += req.batch
                g.launch(stream)
                kept = {}
                if keep:
                    for req, o in slices:
                        if req.rid in keep:
                            sl = slice(o, o + req.batch)
                            kept[req.rid] = (g.flm_in[sl].clone(), g.map[sl].clone(), g.flm_out[sl].clone())
                done = torch.cuda.Event(enable_timing=True)
                done.record(stream)
            ent[1] = done
            self.graph_launches += 1
            return done, (), kept
        with torch.cuda.stream(stream):
            flm = torch.empty((B, L * L), dtype=self.cdtype, device=self.dev)
            fmap = torch.empty((B, L, 2 * L - 1), dtype=self.cdtype, device=self.dev)
            back = torch.empty_like(flm)
            ws = torch.empty(self.workspace(L, s, B), dtype=torch.uint8, device=self.dev)
            off = 0
            slices = []
            for req in group.requests:
                self.fill_input(req, flm[off:off + req.batch])
                slices.append((req, off))
                off += req.batch
            self.sht.inverse(flm, L, s, self.precision, out=fmap, workspace=ws)
            self.sht.forward(fmap, L, s, self.precision, out=back, workspace=ws)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        kept = {}
        if keep:
            for req, o in slices:
                if req.rid in keep:
                    kept[req.rid] = (flm[o:o + req.batch], fmap[o:o + req.batch], back[o:o + req.batch])
        return done, (flm, fmap, back, ws), kept

    def run(self, requests: Sequence, keep: Optional[Iterable[int]] = None, closed_loop: bool = False,
            poll_s: float = 20e-6):
        """Serve ``requests`` (each with rid, arrival_s, L, spin, batch, seed).

        Arrival times are honoured in real time from the start of the call
        (all arrive at once with ``closed_loop``).  Returns (results, kept,
        stats): per-request results, the device outputs of the ``keep`` rids
        as (flm, map, back) views, and summary statistics.
        """
        torch = self.torch
        keep = set(keep or ())
        g_launch0, g_capture0 = self.graph_launches, self.graph_captures
        reqs = sorted(requests, key=lambda r: (0.0 if closed_loop else r.arrival_s, r.rid))
        sched = Scheduler(self.budget, self.workspace, cbytes=self.cbytes)
        free = list(range(len(self.streams)))
        inflight = []   # (group, stream index, done event, buffers)
        results: List[Result] = []
        kept_all = {}
        torch.cuda.synchronize(self.dev)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.streams[0])
        t0 = time.perf_counter()
        i = 0
        peak_used = 0
        max_inflight = 0
        while i < len(reqs) or sched.waiting or inflight:
            now = time.perf_counter() - t0
            while i < len(reqs) and (closed_loop or reqs[i].arrival_s <= now):
                sched.arrive(reqs[i])
                i += 1
            progressed = False
            still = []
            for grp, si, done, bufs in inflight:
                if done.query():
                    t_done = ref.elapsed_time(done) / 1e3
                    for req in grp.requests:
                        arr = 0.0 if closed_loop else req.arrival_s
                        results.append(Result(req.rid, req.L, req.spin, req.batch, arr, t_done,
                                              len(grp.requests)))
                    sched.release(grp)
                    free.append(si)
                    progressed = True
                else:
                    still.append((grp, si, done, bufs))
            inflight = still
            while free:
                grp = sched.next_group()
                if grp is None:
                    break
                si = free.pop(0)
                grp.admitted_s = time.perf_counter() - t0
                done, bufs, kept = self._launch(grp, self.streams[si], keep)
                kept_all.update(kept)
                inflight.append((grp, si, done, bufs))
                peak_used = max(peak_used, sched.used)
                max_inflight = max(max_inflight, len(inflight))
                progressed = True
            if not progressed:
                time.sleep(poll_s)
        torch.cuda.synchronize(self.dev)
        makespan = max(r.done_s for r in results) if results else 0.0
        lat = [r.latency_s for r in results]
        maps = sum(r.batch for r in results)
        stats = {"requests": len(results), "maps": maps, "makespan_s": makespan,
                 "transforms_per_s": maps / makespan if makespan > 0 else float("nan"),
                 "requests_per_s": len(results) / makespan if makespan > 0 else float("nan"),
                 "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
                 "mean_group_size": sum(r.group_size for r in results) / max(1, len(results)),
                 "peak_admitted_bytes": peak_used, "max_inflight_groups": max_inflight,
                 "budget_bytes": self.budget, "streams": len(self.streams),
                 "graph_launches": self.graph_launches - g_launch0,
                 "graph_captures": self.graph_captures - g_capture0}
        return results, kept_all, stats
