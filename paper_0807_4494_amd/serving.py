"""Continuous-batching request loop over the transform library.

A request asks for the inverse then the forward transform of its own batch of
maps at its own (L, spin) -- one "transform" per map, as in the throughput
benchmark.  The loop

* admits arrived requests in arrival order while their device-memory footprint
  fits in a fixed budget and a stream slot is free (admission by HBM
  footprint);
* groups the waiting requests that share the oldest one's L into one call,
  whatever their spins (``sht_inverse_multi`` / ``sht_forward_multi``: one
  contraction launch serves every spin segment of the group), up to the
  library's batch and segment limits; ``by_spin=True`` restricts a group to
  one (L, spin);
* runs each group on its own HIP stream, so groups admitted while others are
  still on the GPU overlap with them on the device;
* frees a group's memory and slot when its completion event fires, and times
  every request from its arrival to that event;
* drops a waiting request whose ``timeout_s`` has passed (status
  ``"timeout"``) and honours ``cancel(rid)``: a waiting request is removed, an
  in-flight one finishes on the device but is reported ``"cancelled"``;
* marks every request of a group whose launch or completion fails as
  ``"failed"`` and keeps serving the others.

Plans (Wigner seed and spin tables, FFT tables) are built for every (L, spin)
before the loop starts and stay resident.  The loop itself (``Server``,
``Scheduler``) is pure Python over an executor interface: ``GpuExecutor``
drives the library through its C ABI on torch streams, and the CPU tests
drive the same loop with a simulated executor (timing, failures).
"""

from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

BATCH_MAX = 64   # the library's per-call batch limit
SEG_MAX = 8      # spin segments per call (SHT_MULTI_SEG_MAX)


def footprint_bytes(L: int, batch: int, workspace: int, cbytes: int = 8) -> int:
    """Device bytes a group holds while in flight: its input coefficients, the
    maps, the output coefficients (``cbytes`` per complex) and one workspace."""
    N = 2 * L - 1
    return batch * (2 * L * L + L * N) * cbytes + workspace


@dataclasses.dataclass
class Group:
    """One call: ``segments`` [(spin, maps)] in call order, ``requests`` in
    the same order (segment 0's requests first)."""
    L: int
    requests: list
    segments: List[Tuple[int, int]]
    batch: int
    nbytes: int
    admitted_s: float = 0.0

    @property
    def spin(self) -> Optional[int]:
        return self.segments[0][0] if len(self.segments) == 1 else None

    @property
    def shape(self) -> tuple:
        return (self.L, tuple(self.segments))


def pair_order(spins: List[int]) -> List[int]:
    """Spins in order of first appearance, except that -s is moved right
    after s (s != 0): the library then runs the two segments as one
    contraction, with one Wigner generation for both (Eq. (wignerd_sym6))."""
    out: List[int] = []
    for s in spins:
        if s in out:
            continue
        out.append(s)
        if s != 0 and -s in spins:
            out.append(-s)
    return out


class Scheduler:
    """FIFO admission with same-L grouping under a memory budget.

    ``workspace(L, spin, batch)`` gives the library's workspace size for one
    batched call.  ``next_group`` takes the oldest waiting request and every
    later waiting request with the same L (and the same spin if
    ``by_spin``) that still fits the batch limit, the segment limit and the
    free memory; it returns None when the oldest request does not fit
    (head-of-line order is kept, so no request starves).
    """

    def __init__(self, budget_bytes: int, workspace: Callable[[int, int, int], int],
                 max_batch: int = BATCH_MAX, cbytes: int = 8, by_spin: bool = False, max_segments: int = SEG_MAX):
        self.budget = int(budget_bytes)
        self.used = 0
        self.workspace = workspace
        self.max_batch = max_batch
        self.cbytes = cbytes
        self.by_spin = by_spin
        self.max_segments = max_segments
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
        spins = [head.spin]
        for req in list(self.waiting)[1:]:
            if req.L != head.L or batch + req.batch > self.max_batch:
                continue
            if self.by_spin and req.spin != head.spin:
                continue
            if req.spin not in spins and len(spins) >= self.max_segments:
                continue
            more = self.group_bytes(head.L, head.spin, batch + req.batch)
            if more > free:
                continue
            members.append(req)
            if req.spin not in spins:
                spins.append(req.spin)
            batch += req.batch
            need = more
        for req in members:
            self.waiting.remove(req)
        self.used += need
        spins = pair_order(spins)
        ordered = [r for s in spins for r in members if r.spin == s]
        segments = [(s, sum(r.batch for r in members if r.spin == s)) for s in spins]
        return Group(head.L, ordered, segments, batch, need)

    def release(self, group: Group) -> None:
        self.used -= group.nbytes
        assert self.used >= 0

    def expire(self, now_s: float, arrival: Callable = lambda r: r.arrival_s) -> list:
        """Remove and return the waiting requests whose deadline
        (``arrival(r)`` + ``timeout_s``, when the request has one) has passed."""
        gone = [r for r in self.waiting
                if getattr(r, "timeout_s", None) is not None and now_s > arrival(r) + r.timeout_s]
        for r in gone:
            self.waiting.remove(r)
        return gone

    def cancel(self, rid: int):
        """Remove a waiting request; returns it, or None if it is not waiting."""
        for r in self.waiting:
            if r.rid == rid:
                self.waiting.remove(r)
                return r
        return None


@dataclasses.dataclass
class Result:
    rid: int
    L: int
    spin: int
    batch: int
    arrival_s: float
    done_s: float
    group_size: int
    status: str = "ok"        # ok, timeout, cancelled, failed
    segments: int = 1         # spin segments of the request's call

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


class Server:
    """The serving loop over an executor (see the module docstring).

    The executor provides ``workspace(L, spin, batch)``, ``cbytes``,
    ``begin()`` (start of a run; its clock starts at 0), ``now()`` (seconds
    on that clock), ``idle()`` (nothing progressed: wait a little),
    ``launch(group, slot, keep)`` -> (handle, kept outputs) (raises on a
    failed launch), ``poll(handle)`` -> None while running, else
    ("ok", completion time) or ("failed", message), and ``end()``.
    """

    def __init__(self, executor, streams: int = 4, budget_bytes: int = 16 << 30, by_spin: bool = False):
        self.ex = executor
        self.nstreams = streams
        self.budget = budget_bytes
        self.by_spin = by_spin
        self._cancel_lock = threading.Lock()
        self._cancel: set = set()

    def cancel(self, rid: int) -> None:
        """Ask for request ``rid`` to be cancelled (thread-safe; takes effect
        at the loop's next turn)."""
        with self._cancel_lock:
            self._cancel.add(rid)

    def run(self, requests: Sequence, keep: Optional[Iterable[int]] = None, closed_loop: bool = False,
            on_tick: Optional[Callable[[float], None]] = None):
        """Serve ``requests`` (each with rid, arrival_s, L, spin, batch, seed
        and optionally timeout_s).  Arrival times are honoured on the
        executor's clock from the start of the call (all arrive at once with
        ``closed_loop``).  ``on_tick(now)`` runs at every turn of the loop.
        Returns (results, kept, stats): per-request results, the device
        outputs of the ``keep`` rids (as the executor returns them), and
        summary statistics over the requests served."""
        keep = set(keep or ())
        ex = self.ex
        reqs = sorted(requests, key=lambda r: (0.0 if closed_loop else r.arrival_s, r.rid))
        sched = Scheduler(self.budget, ex.workspace, cbytes=ex.cbytes, by_spin=self.by_spin)
        free = list(range(self.nstreams))
        inflight = []   # (group, slot, handle)
        results: List[Result] = []
        kept_all = {}
        cancelled_inflight: set = set()
        ex.begin()
        i = 0
        peak_used = 0
        max_inflight = 0

        def arrival(req):
            return 0.0 if closed_loop else req.arrival_s

        def finish(grp, t, status):
            for req in grp.requests:
                st = "cancelled" if req.rid in cancelled_inflight else status
                results.append(Result(req.rid, req.L, req.spin, req.batch, arrival(req), t,
                                      len(grp.requests), st, len(grp.segments)))
                if st != "ok":
                    kept_all.pop(req.rid, None)

        while i < len(reqs) or sched.waiting or inflight:
            now = ex.now()
            if on_tick is not None:
                on_tick(now)
            while i < len(reqs) and (closed_loop or reqs[i].arrival_s <= now):
                sched.arrive(reqs[i])
                i += 1
            progressed = False
            for req in sched.expire(now, arrival):
                results.append(Result(req.rid, req.L, req.spin, req.batch, arrival(req), now, 0, "timeout"))
                progressed = True
            with self._cancel_lock:
                pending, self._cancel = self._cancel, set()
            for rid in pending:
                req = sched.cancel(rid)
                if req is not None:
                    results.append(Result(req.rid, req.L, req.spin, req.batch, arrival(req), now, 0, "cancelled"))
                    progressed = True
                elif any(r.rid == rid for g, _, _ in inflight for r in g.requests):
                    cancelled_inflight.add(rid)
                elif not any(r.rid == rid for r in results) and any(r.rid == rid for r in reqs[i:]):
                    # not arrived yet: cancelled on arrival
                    with self._cancel_lock:
                        self._cancel.add(rid)
            still = []
            for grp, si, h in inflight:
                try:
                    st = ex.poll(h)
                except Exception as e:       # a failed completion fails its group only
                    st = ("failed", str(e))
                if st is None:
                    still.append((grp, si, h))
                    continue
                status, t = st[0], (st[1] if st[0] == "ok" else now)
                finish(grp, t, "ok" if status == "ok" else "failed")
                sched.release(grp)
                free.append(si)
                progressed = True
            inflight = still
            while free:
                grp = sched.next_group()
                if grp is None:
                    break
                si = free.pop(0)
                grp.admitted_s = now
                try:
                    h, kept = ex.launch(grp, si, keep)
                except Exception:            # a failed launch fails its group only
                    finish(grp, now, "failed")
                    sched.release(grp)
                    free.append(si)
                    progressed = True
                    continue
                kept_all.update(kept)
                inflight.append((grp, si, h))
                peak_used = max(peak_used, sched.used)
                max_inflight = max(max_inflight, len(inflight))
                progressed = True
            if not progressed:
                ex.idle()
        ex.end()
        ok = [r for r in results if r.status == "ok"]
        makespan = max((r.done_s for r in ok), default=0.0)
        lat = [r.latency_s for r in ok]
        maps = sum(r.batch for r in ok)
        counts = collections.Counter(r.status for r in results)
        stats = {"requests": len(ok), "maps": maps, "makespan_s": makespan,
                 "transforms_per_s": maps / makespan if makespan > 0 else float("nan"),
                 "requests_per_s": len(ok) / makespan if makespan > 0 else float("nan"),
                 "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
                 "mean_group_size": sum(r.group_size for r in ok) / max(1, len(ok)),
                 "mean_segments": sum(r.segments for r in ok) / max(1, len(ok)),
                 "peak_admitted_bytes": peak_used, "max_inflight_groups": max_inflight,
                 "budget_bytes": self.budget, "streams": self.nstreams,
                 "timeouts": counts.get("timeout", 0), "cancelled": counts.get("cancelled", 0),
                 "failed": counts.get("failed", 0)}
        return results, kept_all, stats


class GpuExecutor:
    """Runs groups through the library on torch streams of one GPU.

    ``precision`` is the library precision of every call ("fp32", "bf16x3" or
    "fp64").  Inputs are drawn on the device from each request's seed
    (complex Gaussian, variance C_l = 1/(l+1)^2, zero for l < |spin|) inside
    the request's own buffers when its group is admitted.

    ``graphs`` > 0 keeps up to that many captured transforms (``sht.Graph``,
    one per single-spin (L, spin, batch) group shape, each at most
    ``graph_bytes`` of device memory): a shape seen for the ``graph_after``-th
    time is captured (the least used idle graph makes room), and later groups
    of a cached shape replay its graph instead of launching the stages one by
    one, unless that graph is still in flight.  Graph buffers are outside the
    admission budget.  Groups of several spins always launch eagerly.
    """

    def __init__(self, precision: str = "fp32", streams: int = 4, device: int = 0, graphs: int = 0,
                 graph_bytes: int = 1 << 30, graph_after: int = 3, poll_s: float = 20e-6):
        import torch
        from . import sht
        self.torch = torch
        self.sht = sht
        self.precision = precision
        self.dev = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.cdtype = sht.io_dtype(precision)
        self.cbytes = 16 if precision == "fp64" else 8
        self.poll_s = poll_s
        self._ws_cache: Dict[Tuple[int, int], int] = {}
        self._scale: Dict[Tuple[int, int], "torch.Tensor"] = {}
        self.graph_cap = graphs
        self.graph_bytes = graph_bytes
        self.graph_after = graph_after
        self._graphs: "Dict[Tuple[int, int, int], list]" = {}   # shape -> [Graph, busy event or None]
        self._seen: Dict[Tuple[int, int, int], int] = {}
        self.graph_launches = 0
        self.graph_captures = 0

    def workspace(self, L: int, spin: int, batch: int) -> int:
        key = (L, batch)     # the workspace does not depend on the spin
        if key not in self._ws_cache:
            self._ws_cache[key] = self.sht.workspace_bytes(L, 0, batch, self.precision)
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

    # ---- the clock: seconds since begin() on the host, completion times
    # from GPU events against a reference event recorded at begin() ----
    def begin(self) -> None:
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record(self.streams[0])
        self._t0 = time.perf_counter()
        self._g0 = (self.graph_launches, self.graph_captures)

    def now(self) -> float:
        return time.perf_counter() - self._t0

    def idle(self) -> None:
        time.sleep(self.poll_s)

    def end(self) -> None:
        self.torch.cuda.synchronize(self.dev)

    def poll(self, handle):
        done = handle[0]
        if not done.query():
            return None
        return ("ok", self._ref.elapsed_time(done) / 1e3)

    def _graph_for(self, L: int, s: int, B: int):
        """The cached graph of this shape if it is idle (capturing it on the
        shape's graph_after-th sighting), else None."""
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

    def launch(self, group: Group, slot: int, keep: set):
        torch = self.torch
        stream = self.streams[slot]
        L, B = group.L, group.batch
        single = len(group.segments) == 1
        ent = self._graph_for(L, group.segments[0][0], B) if (self.graph_cap > 0 and single) else None
        if ent is not None:
            g = ent[0]
            # the graph's buffers were made on the creating stream: order
            # this stream after it before writing them
            stream.wait_stream(torch.cuda.current_stream(self.dev))
            with torch.cuda.stream(stream):
                off = 0
                slices = []
                for req in group.requests:
                    self.fill_input(req, g.flm_in[off:off + req.batch])
                    slices.append((req, off))
                    off += req.batch
                g.launch(stream)
                kept = {}
                for req, o in slices:
                    if req.rid in keep:
                        sl = slice(o, o + req.batch)
                        kept[req.rid] = (g.flm_in[sl].clone(), g.map[sl].clone(), g.flm_out[sl].clone())
                done = torch.cuda.Event(enable_timing=True)
                done.record(stream)
            ent[1] = done
            self.graph_launches += 1
            return (done, ()), kept
        with torch.cuda.stream(stream):
            flm = torch.empty((B, L * L), dtype=self.cdtype, device=self.dev)
            fmap = torch.empty((B, L, 2 * L - 1), dtype=self.cdtype, device=self.dev)
            back = torch.empty_like(flm)
            ws = torch.empty(self.workspace(L, 0, B), dtype=torch.uint8, device=self.dev)
            off = 0
            slices = []
            for req in group.requests:
                self.fill_input(req, flm[off:off + req.batch])
                slices.append((req, off))
                off += req.batch
            spins = [s for s, _ in group.segments]
            batches = [n for _, n in group.segments]
            if single:
                self.sht.inverse(flm, L, spins[0], self.precision, out=fmap, workspace=ws)
                self.sht.forward(fmap, L, spins[0], self.precision, out=back, workspace=ws)
            else:
                self.sht.inverse_multi(flm, L, spins, batches, self.precision, out=fmap, workspace=ws)
                self.sht.forward_multi(fmap, L, spins, batches, self.precision, out=back, workspace=ws)
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
        kept = {}
        with torch.cuda.stream(stream):
            # copies, so that the group's buffers are freed with the group
            for req, o in slices:
                if req.rid in keep:
                    sl = slice(o, o + req.batch)
                    kept[req.rid] = (flm[sl].clone(), fmap[sl].clone(), back[sl].clone())
        return (done, (flm, fmap, back, ws)), kept


class GpuServer(Server):
    """The serving loop on one GPU (``Server`` over a ``GpuExecutor``).

    ``by_spin`` (default False) groups by (L, spin) instead of by L.  The
    remaining arguments are the executor's.
    """

    def __init__(self, precision: str = "fp32", streams: int = 4, budget_bytes: int = 16 << 30,
                 device: int = 0, graphs: int = 0, graph_bytes: int = 1 << 30, graph_after: int = 3,
                 by_spin: bool = False):
        ex = GpuExecutor(precision, streams, device, graphs, graph_bytes, graph_after)
        super().__init__(ex, streams, budget_bytes, by_spin)
        self.precision = precision

    def warm(self, keys) -> None:
        self.ex.warm(keys)

    def close_graphs(self) -> None:
        self.ex.close_graphs()

    def run(self, requests, keep=None, closed_loop=False, on_tick=None):
        g0 = (self.ex.graph_launches, self.ex.graph_captures)
        res, kept, stats = super().run(requests, keep, closed_loop, on_tick)
        stats["graph_launches"] = self.ex.graph_launches - g0[0]
        stats["graph_captures"] = self.ex.graph_captures - g0[1]
        return res, kept, stats
