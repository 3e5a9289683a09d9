"""Serving loop with continuous batching over the batched C ABI.

Requests (compress a resident field, or decompress a resident stream) arrive
over time.  The server admits arrived requests while the device memory held
by everything in flight stays under a limit, groups the admitted requests of
one step into a batch (one batched compress call and one batched decompress
call), and launches it on the next free HIP stream.  Batches therefore run
while others are still on the device, and requests that arrive meanwhile
join the next batch as streams and memory free up.  Every request's result
is the one a one-field call gives: the batched calls run the same kernels
per field.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import List, Optional

import paper_2602_17552_amd as tsz


@dataclass
class Request:
    rid: int
    op: str                    # "compress" or "decompress"
    arrival: float             # seconds on the server's clock
    src: object = None         # compress: float32 CUDA field; decompress: uint8 CUDA stream
    shape: tuple = ()          # field shape (decompress: of the reconstruction)
    eb: float = 1e-3
    mode: str = "rel"
    nbytes: int = 0            # field bytes (the throughput unit)
    mem: int = 0               # device bytes held while in flight
    admitted: float = -1.0
    done: float = -1.0
    status: int = -100
    result: object = None      # compress: uint8 stream view; decompress: float32 field
    batch: int = -1            # batch it ran in
    tag: object = None         # the caller's label


@dataclass
class _Batch:
    bid: int
    stream: object
    reqs: List[Request]
    comp: Optional[object] = None
    dec: Optional[object] = None
    event: object = None
    mem: int = 0
    launched: float = 0.0


def request_mem(op: str, shape, stream_bytes: int = 0) -> int:
    """Device bytes a request holds in flight: outputs plus its workspace."""
    n = 1
    for d in shape:
        n *= int(d)
    ws = tsz.workspace_size(tuple(shape))
    if op == "compress":
        return tsz.compress_bound(tuple(shape)) + ws + 16
    return 4 * n + ws + stream_bytes + 16


class Server:
    """Continuous-batching server on one GPU.

    mem_limit: device bytes that in-flight requests may hold together;
    max_batch: requests per batch; streams: batches in flight at once;
    keep_results: keep each finished request's output (else only its status
    and timing)."""

    def __init__(self, mem_limit: int = 64 << 30, max_batch: int = 64, streams: int = 4, device=None,
                 clock=time.perf_counter, keep_results: bool = True, **params):
        import torch
        self.device = device or torch.device("cuda:0")
        self.mem_limit = int(mem_limit)
        self.max_batch = int(max_batch)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, int(streams)))]
        self.params = params
        self.keep_results = keep_results
        self.clock = clock
        self.t0 = clock()
        self.waiting: collections.deque = collections.deque()
        self.inflight: List[_Batch] = []
        self.mem_in_use = 0
        self.peak_mem = 0
        self.peak_inflight = 0
        self.done: List[Request] = []
        self._bid = 0
        self._next_stream = 0
        self.batch_sizes: List[int] = []

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request):
        if not req.mem:
            sb = req.src.numel() if req.op == "decompress" else 0
            req.mem = request_mem(req.op, req.shape, sb)
        if req.mem > self.mem_limit:
            raise ValueError("request %d needs more device memory than the admission limit" % req.rid)
        self.waiting.append(req)

    def _free_stream(self):
        busy = {id(b.stream) for b in self.inflight}
        for k in range(len(self.streams)):
            s = self.streams[(self._next_stream + k) % len(self.streams)]
            if id(s) not in busy:
                self._next_stream = (self._next_stream + k + 1) % len(self.streams)
                return s
        return None

    def _launch(self):
        """Admits waiting requests (arrival order) into one batch on a free
        stream, within the memory limit."""
        import torch
        if not self.waiting:
            return False
        s = self._free_stream()
        if s is None:
            return False
        reqs, mem = [], 0
        while self.waiting and len(reqs) < self.max_batch:
            r = self.waiting[0]
            if self.mem_in_use + mem + r.mem > self.mem_limit:
                break
            reqs.append(self.waiting.popleft())
            mem += r.mem
        if not reqs:
            return False
        t = self.now()
        b = _Batch(self._bid, s, reqs, mem=mem, launched=t)
        self._bid += 1
        comp = [r for r in reqs if r.op == "compress"]
        dec = [r for r in reqs if r.op == "decompress"]
        # the batch's inputs may still be in production on the submitting
        # stream: order the batch after it, and tell the allocator that the
        # inputs are in use on this stream until the batch ends
        s.wait_stream(torch.cuda.current_stream(self.device))
        for r in reqs:
            r.src.record_stream(s)
        with torch.cuda.stream(s):
            if comp:
                b.comp = tsz.CompressBatch([r.src for r in comp], [r.eb for r in comp], [r.mode for r in comp],
                                           device=self.device, **self.params)
                b.comp.run(stream=s)
            if dec:
                b.dec = tsz.DecompressBatch([r.src for r in dec], [r.shape for r in dec], device=self.device)
                b.dec.run(stream=s)
            b.event = torch.cuda.Event()
            b.event.record(s)
        for r in reqs:
            r.admitted = t
            r.batch = b.bid
        self.mem_in_use += mem
        self.peak_mem = max(self.peak_mem, self.mem_in_use)
        self.inflight.append(b)
        self.peak_inflight = max(self.peak_inflight, len(self.inflight))
        self.batch_sizes.append(len(reqs))
        return True

    def _complete(self, b: _Batch, t: float):
        import torch
        comp = [r for r in b.reqs if r.op == "compress"]
        dec = [r for r in b.reqs if r.op == "decompress"]
        # results were made on the batch's stream; the caller uses them on
        # its own, so the allocator must not reuse them for the batch stream
        # while work the caller enqueues there may still read them
        consumer = torch.cuda.current_stream(self.device)
        if b.comp is not None:
            st, streams = b.comp.results()
            for r, s_, out in zip(comp, st, streams):
                r.status, r.result = int(s_), out
                if self.keep_results:
                    out.record_stream(consumer)
        if b.dec is not None:
            st = b.dec.status.cpu().tolist()
            for r, s_, rec in zip(dec, st, b.dec.recs):
                r.status, r.result = int(s_), rec
                if self.keep_results:
                    rec.record_stream(consumer)
        for r in b.reqs:
            r.done = t
            if not self.keep_results:
                r.result = None  # the batch's buffers return to the allocator
            self.done.append(r)
        self.mem_in_use -= b.mem

    def step(self) -> int:
        """Retires finished batches, then launches while streams, memory and
        waiting requests allow.  Returns the number of requests retired."""
        n = 0
        keep = []
        for b in self.inflight:
            if b.event.query():
                self._complete(b, self.now())
                n += len(b.reqs)
            else:
                keep.append(b)
        self.inflight = keep
        while self._launch():
            pass
        return n

    def drain(self):
        while self.waiting or self.inflight:
            self.step()

    def stats(self):
        import numpy as np
        lat = np.array([r.done - r.arrival for r in self.done]) * 1e3
        q = np.array([r.admitted - r.arrival for r in self.done]) * 1e3
        out = {"requests": len(self.done),
               "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
               "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
               "mean_ms": round(float(lat.mean()), 3) if lat.size else None,
               "queue_p99_ms": round(float(np.percentile(q, 99)), 3) if q.size else None,
               "batches": len(self.batch_sizes),
               "mean_batch": round(float(np.mean(self.batch_sizes)), 2) if self.batch_sizes else 0,
               "max_batch": max(self.batch_sizes) if self.batch_sizes else 0,
               "peak_inflight_batches": self.peak_inflight,
               "peak_mem_bytes": self.peak_mem,
               "failed": sum(1 for r in self.done if r.status != 0)}
        return out


def run_trace(server: Server, trace, make_request, realtime: bool = True, deadline: float = None):
    """Feeds (arrival_s, op) pairs to the server as their arrival times pass
    (or all at once, realtime=False) and serves until every request is done.
    make_request(i, arrival, op) builds the Request."""
    reqs = [make_request(i, t, op) for i, (t, op) in enumerate(trace)]
    k = 0
    server.t0 = server.clock()
    while k < len(reqs) or server.waiting or server.inflight:
        now = server.now()
        while k < len(reqs) and (not realtime or reqs[k].arrival <= now):
            if not realtime:
                reqs[k].arrival = now
            server.submit(reqs[k])
            k += 1
        server.step()
        if deadline is not None and now > deadline:
            raise TimeoutError("serving did not finish in time")
    return reqs
