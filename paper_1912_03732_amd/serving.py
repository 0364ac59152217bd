"""Serving: continuous batching of S-box evaluations on one GPU.

Requests (an n x m table each) arrive at arbitrary times.  The server keeps a
bounded FIFO of waiting requests and, every scheduling pass, (1) retires the
batches whose completion event has fired and frees their device memory,
(2) forms a new batch from the head of the FIFO as long as the batch fits in
the device-memory arena and in the batch size cap, and launches it at once on
the next of several HIP streams -- so requests that arrive while other
batches run are admitted as memory frees up and their work overlaps on the
device.  A request larger than the whole arena is refused at submission.

A batch owns one arena block holding, contiguously, the library workspace
(queue counters, job descriptors, bit-sliced tables), the staged tables and
the outputs (per request: max |W| per mask, then NL).  Tables go up in one
host-to-device copy from pinned memory, results come back in one
device-to-host copy, and the batch itself is one ``sbox_walsh_nl_batched``
call, i.e. a persistent launch per size class pulling (box, mask range)
items from a device work queue.

The executor is the seam between scheduling and the device: ``Server`` only
calls ``footprint``, ``capacity``, ``try_launch``, ``poll`` and ``finish``, so
the scheduling logic can be exercised with any object providing them.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import time
from typing import Deque, Dict, List, Optional

import numpy as np

_ALIGN = 256


def _al(v: int) -> int:
    return (v + _ALIGN - 1) & ~(_ALIGN - 1)


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    m: int
    table: np.ndarray
    t_arrival: float = 0.0
    t_launch: Optional[float] = None
    t_done: Optional[float] = None
    nl: Optional[int] = None
    maxabs: Optional[np.ndarray] = None
    status: str = "new"        # new -> waiting -> running -> done | rejected
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrival


class FirstFit:
    """First-fit allocator over [0, size) with 256-byte granularity."""

    def __init__(self, size: int):
        self.size = size - size % _ALIGN
        self.free: List[List[int]] = [[0, self.size]]   # sorted [offset, length]
        self.used = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        nbytes = _al(max(nbytes, 1))
        for i, (off, ln) in enumerate(self.free):
            if ln >= nbytes:
                if ln == nbytes:
                    self.free.pop(i)
                else:
                    self.free[i] = [off + nbytes, ln - nbytes]
                self.used += nbytes
                return off
        return None

    def release(self, off: int, nbytes: int) -> None:
        nbytes = _al(max(nbytes, 1))
        i = bisect.bisect_left(self.free, [off, 0])
        self.free.insert(i, [off, nbytes])
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i][1] += self.free[i + 1][1]
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1][1] += self.free[i][1]
            self.free.pop(i)
        self.used -= nbytes

    def largest(self) -> int:
        return max((ln for _, ln in self.free), default=0)


def table_bytes(n: int, m: int) -> int:
    eb = 1 if m <= 8 else (2 if m <= 16 else 4)
    return eb << n


def request_bytes(n: int, m: int) -> int:
    """Device bytes one request adds to a batch block (table, bit-sliced words,
    descriptor, outputs)."""
    f = _al(m * (1 << max(0, n - 5)) * 4)
    return _al(table_bytes(n, m)) + f + 96 + _al(4 * (1 << m) + 4)


class GpuExecutor:
    """Runs batches through libsboxwalsh.so on one GPU."""

    def __init__(self, arena_bytes: int = 1 << 30, streams: int = 2, device: str = "cuda"):
        import torch

        from . import binding as B
        self.torch = torch
        self.B = B
        B.load()
        self.device = torch.device(device)
        self.arena = torch.empty(arena_bytes + _ALIGN, dtype=torch.uint8, device=self.device)
        self.base = (self.arena.data_ptr() + _ALIGN - 1) & ~(_ALIGN - 1)
        self.alloc = FirstFit(arena_bytes)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        self.next_stream = 0

    def capacity(self) -> int:
        return self.alloc.size

    def footprint(self, reqs) -> int:
        return 512 + sum(request_bytes(r.n, r.m) for r in reqs)

    def try_launch(self, reqs):
        torch, B = self.torch, self.B
        count = len(reqs)
        # layout: [workspace][tables][outputs]
        t_off, tsz = [], 0
        for r in reqs:
            t_off.append(tsz)
            tsz += _al(table_bytes(r.n, r.m))
        o_off, osz = [], 0
        for r in reqs:
            o_off.append(osz)
            osz += _al(4 * (1 << r.m) + 4)
        jobs = (B.sbox_job * count)()
        for i, r in enumerate(reqs):
            jobs[i].S, jobs[i].nl = 1, 1  # placeholders for the size query
            jobs[i].n, jobs[i].m = r.n, r.m
            jobs[i].s_elem_bytes = 1 if r.m <= 8 else (2 if r.m <= 16 else 4)
            jobs[i].layout = 0
        ws_bytes = B.sbox_batched_workspace_bytes(jobs, count)
        if ws_bytes == 0:
            raise B.SboxError(B.SBOX_ERR_UNSUPPORTED, B.last_error())
        ws_bytes = _al(ws_bytes)
        total = ws_bytes + tsz + osz
        off = self.alloc.alloc(total)
        if off is None:
            return None
        base = self.base + off
        tab_base, out_base = base + ws_bytes, base + ws_bytes + tsz
        # stage all tables in one pinned buffer, one copy
        host = torch.empty(tsz, dtype=torch.uint8, pin_memory=True)
        hv = host.numpy()
        for i, r in enumerate(reqs):
            eb = jobs[i].s_elem_bytes
            dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[eb]
            hv[t_off[i]:t_off[i] + (eb << r.n)] = np.ascontiguousarray(r.table, dtype=dt).view(np.uint8)
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        dev_view = self.arena[off + (self.base - self.arena.data_ptr()):][: total]
        with torch.cuda.stream(s):
            dev_view[ws_bytes:ws_bytes + tsz].copy_(host, non_blocking=True)
        for i, r in enumerate(reqs):
            jobs[i].S = tab_base + t_off[i]
            jobs[i].maxabs_per_b = out_base + o_off[i]
            jobs[i].nl = out_base + o_off[i] + 4 * (1 << r.m)
            jobs[i].spectrum = None
        st = B.sbox_walsh_nl_batched(jobs, count, base, ws_bytes, int(s.cuda_stream))
        if st != B.SBOX_OK:
            self.alloc.release(off, total)
            raise B.SboxError(st, B.last_error())
        out_host = torch.empty(osz, dtype=torch.uint8, pin_memory=True)
        with torch.cuda.stream(s):
            out_host.copy_(dev_view[ws_bytes + tsz:ws_bytes + tsz + osz], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"event": ev, "off": off, "total": total, "host_in": host, "host_out": out_host,
                "o_off": o_off, "reqs": reqs}

    def poll(self, h) -> bool:
        return h["event"].query()

    def finish(self, h):
        h["event"].synchronize()
        out = h["host_out"].numpy()
        res = []
        for i, r in enumerate(h["reqs"]):
            mx = out[h["o_off"][i]: h["o_off"][i] + 4 * (1 << r.m)].view(np.int32).copy()
            nl = int(out[h["o_off"][i] + 4 * (1 << r.m): h["o_off"][i] + 4 * (1 << r.m) + 4].view(np.int32)[0])
            res.append((nl, mx))
        self.alloc.release(h["off"], h["total"])
        return res


class Server:
    """Bounded FIFO + continuous batching over an executor."""

    def __init__(self, executor, max_batch: int = 512, max_waiting: int = 100000, max_inflight: int = 4,
                 clock=time.perf_counter):
        self.ex = executor
        self.max_batch = max_batch
        self.max_waiting = max_waiting
        self.max_inflight = max_inflight
        self.clock = clock
        self.waiting: Deque[Request] = collections.deque()
        self.inflight: Deque = collections.deque()
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self.batches = 0
        self.batch_sizes: List[int] = []

    def submit(self, req: Request) -> bool:
        if req.t_arrival == 0.0:
            req.t_arrival = self.clock()
        if self.ex.footprint([req]) > self.ex.capacity():
            req.status, req.error = "rejected", "larger than the device arena"
            self.rejected.append(req)
            return False
        if len(self.waiting) >= self.max_waiting:
            req.status, req.error = "rejected", "waiting queue full"
            self.rejected.append(req)
            return False
        req.status = "waiting"
        self.waiting.append(req)
        return True

    def _retire(self) -> int:
        k = 0
        while self.inflight and self.ex.poll(self.inflight[0]):
            h = self.inflight.popleft()
            now = self.clock()
            for r, (nl, mx) in zip(h["reqs"], self.ex.finish(h)):
                r.nl, r.maxabs, r.t_done, r.status = nl, mx, now, "done"
                self.done.append(r)
                k += 1
        return k

    def _launch(self) -> bool:
        if not self.waiting or len(self.inflight) >= self.max_inflight:
            return False
        batch: List[Request] = []
        budget = self.ex.footprint([])
        limit = self.ex.capacity()
        for r in self.waiting:  # FIFO prefix that fits
            need = self.ex.footprint([r]) - self.ex.footprint([])
            if len(batch) >= self.max_batch or budget + need > limit:
                break
            batch.append(r)
            budget += need
        if not batch:
            return False
        h = self.ex.try_launch(batch)
        while h is None and len(batch) > 1:  # fragmentation: shrink the batch
            batch = batch[: len(batch) // 2]
            h = self.ex.try_launch(batch)
        if h is None:
            return False
        now = self.clock()
        for _ in batch:
            r = self.waiting.popleft()
            r.t_launch, r.status = now, "running"
        self.inflight.append(h)
        self.batches += 1
        self.batch_sizes.append(len(batch))
        return True

    def pump(self) -> int:
        """One scheduling pass; returns the number of requests completed."""
        k = self._retire()
        while self._launch():
            k += self._retire()
        return k

    def drain(self, timeout: float = 60.0) -> None:
        t0 = self.clock()
        while (self.waiting or self.inflight) and self.clock() - t0 < timeout:
            self.pump()
        if self.waiting or self.inflight:
            raise TimeoutError("serving loop did not drain")


def run_open_loop(server: Server, arrivals, reqs: List[Request], clock=time.perf_counter) -> Dict:
    """Submit reqs[i] at time arrivals[i] (seconds from start, sorted), pump
    the server between arrivals, drain, and summarise latency/throughput."""
    t0 = clock()
    i = 0
    N = len(reqs)
    while i < N:
        now = clock() - t0
        while i < N and arrivals[i] <= now:
            reqs[i].t_arrival = t0 + arrivals[i]
            server.submit(reqs[i])
            i += 1
        server.pump()
    server.drain()
    return summarize(server, t0)


def summarize(server: Server, t0: float) -> Dict:
    lat = np.array([r.latency for r in server.done], dtype=np.float64)
    t_end = max((r.t_done for r in server.done), default=t0)
    out = {"completed": len(server.done), "rejected": len(server.rejected), "batches": server.batches,
           "mean_batch": float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0}
    if lat.size:
        out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                    "mean_ms": float(lat.mean() * 1e3),
                    "throughput_rps": len(server.done) / max(t_end - t0, 1e-9)})
    return out


def sweep(rates=(1000, 2000, 5000, 10000, 20000, 50000), count: int = 20000, arena_bytes: int = 1 << 30,
          streams: int = 2, seed_offset: int = 0) -> List[Dict]:
    """Open-loop Poisson rate sweep of the serving workload (sizes 8/12/16)."""
    from . import inputs
    ex = GpuExecutor(arena_bytes=arena_bytes, streams=streams)
    rows = []
    for rate in rates:
        t, ns, pick, pools = inputs.workload_serving(rate, count=count,
                                                     seed=inputs.SEED_BASE + 5 + seed_offset)
        reqs = [Request(i, int(n), int(n), pools[int(n)][int(p)]) for i, (n, p) in enumerate(zip(ns, pick))]
        srv = Server(ex)
        # warm the kernels for each size class once
        for n in (8, 12, 16):
            srv.submit(Request(-1, n, n, pools[n][0]))
        srv.drain()
        srv = Server(ex)
        row = run_open_loop(srv, t, reqs)
        row["rate"] = rate
        rows.append(row)
    return rows


if __name__ == "__main__":
    import json
    import sys
    rates = [float(x) for x in sys.argv[1:]] or [1000, 2000, 5000, 10000, 20000, 50000]
    for row in sweep(rates):
        print(json.dumps(row), flush=True)
