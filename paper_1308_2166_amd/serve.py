"""Continuous-batching ingest of many edge streams on one GPU.

A request is one chunk of one stream: a batch of that stream's edges,
already resident in device memory.  The loop

* admits a stream (gives it a bank slot of r estimators) when its first
  chunk arrives and a slot is free; the number of slots is what a device
  memory budget allows: the banks' bytes plus the step scratch of the
  largest step the loop launches (at most one chunk per slot and at most
  `max_step_edges` edges), both as the library accounts them
  (tc_bank_bytes, tc_step_bytes_max), and that scratch is reserved up
  front, so serving never allocates; later streams wait;
* keeps every admitted stream's estimator state resident in HBM;
* whenever fewer than `depth` steps are in flight, launches one step that
  takes the oldest waiting chunk of admitted streams, oldest first, up to
  `max_step_edges` edges (never two chunks of a stream in one step: a
  chunk is a batch, and the random key depends on the batch index);
* records each step's completion with a GPU event, so a chunk's ingest
  latency is its step's completion time minus its arrival time;
* frees a stream's slot once its last chunk is done and its estimate read.

Every stream therefore gets exactly the result it would get alone (each
chunk processed as one batch of its own bank, in order), whatever the mix.
All arithmetic runs in the kernels behind tc_multi_process.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import torch

from . import (MultiBank, tc_bank_bytes, tc_multi_assign, tc_multi_device_bytes,
               tc_multi_estimate, tc_multi_get_tuning, tc_multi_reserve_max,
               tc_multi_set_vertex_bound, tc_step_bytes_max)


@dataclasses.dataclass
class Chunk:
    t: float            # arrival time (seconds from the start of the run)
    stream: int         # stream id
    edges: torch.Tensor  # (w, 2) int32 device tensor
    last: bool          # the stream's final chunk


@dataclasses.dataclass
class Result:
    S: int
    m: int
    tau: float


def server_bytes(slots: int, r: int, max_step_edges: int) -> int:
    """Device bytes of a server with `slots` banks of r estimators whose
    steps hold at most `slots` chunks and `max_step_edges` edges."""
    return slots * tc_bank_bytes(r) + 16 + tc_step_bytes_max(slots, r, max_step_edges)


def slots_for_budget(budget_bytes: int, r: int, max_step_edges: int,
                     most: int = 1 << 20) -> int:
    """The largest number of bank slots (at most `most`) whose server fits
    the budget (0 if not even one does)."""
    lo, hi = 0, most
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if server_bytes(mid, r, max_step_edges) <= budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    return lo


def poisson_arrivals(chunks_per_stream, rate_per_s: float, seed: int):
    """Merge per-stream chunk lists (each in stream order) into one arrival
    sequence: aggregate Poisson arrivals at `rate_per_s` (rate 0: everything
    at time 0), each arrival taking the next chunk of a stream drawn with
    probability proportional to its remaining chunks.  Returns Chunk list."""
    import numpy as np
    rng = np.random.default_rng(seed)
    left = np.array([len(c) for c in chunks_per_stream], dtype=np.int64)
    total = int(left.sum())
    times = (np.cumsum(rng.exponential(1.0 / rate_per_s, total)) if rate_per_s > 0
             else np.zeros(total))
    nxt = [0] * len(left)
    out = []
    for k in range(total):
        cum = np.cumsum(left)
        s = int(np.searchsorted(cum, rng.random() * cum[-1], side="right"))
        s = min(s, len(left) - 1)
        while left[s] == 0:
            s = (s + 1) % len(left)
        i = nxt[s]
        nxt[s] += 1
        left[s] -= 1
        out.append(Chunk(float(times[k]), s, chunks_per_stream[s][i],
                         nxt[s] == len(chunks_per_stream[s])))
    return out


class Server:
    """Admission, continuous batching and latency bookkeeping."""

    def __init__(self, r: int, max_step_edges: int, slots: int | None = None,
                 budget_bytes: int | None = None, depth: int = 2,
                 stream: torch.cuda.Stream | None = None,
                 vertex_bound: int | None = None, max_slots: int = 1 << 20):
        """Banks of r estimators; every step holds at most max_step_edges
        edges (no chunk may be larger).  The slot count is `slots`, or the
        most that `budget_bytes` of device memory allows (at most
        max_slots).  The step scratch is reserved here for the largest
        step, so serving allocates nothing; every run reassigns the slots it
        uses, so a Server serves many runs.  vertex_bound: every vertex id
        of every stream is below it (fewer radix passes; an id at or above
        it fails the run)."""
        if slots is None:
            if budget_bytes is None:
                raise ValueError("give slots or budget_bytes")
            slots = slots_for_budget(budget_bytes, r, max_step_edges, max_slots)
        if slots < 1:
            raise ValueError("the memory budget leaves no bank slot")
        self.slots, self.r, self.depth = slots, r, depth
        self.max_step_edges = max_step_edges
        self.budget_bytes = budget_bytes
        self.bank = MultiBank([r] * slots, [0] * slots)
        if vertex_bound is not None:
            tc_multi_set_vertex_bound(self.bank.h, vertex_bound)
        tc_multi_reserve_max(self.bank.h, slots, max_step_edges)
        self.stream = stream or torch.cuda.current_stream()

    def device_bytes(self) -> int:
        """Device bytes the server's banks and scratch hold now."""
        return tc_multi_device_bytes(self.bank.h)

    def run(self, arrivals, seeds, spin_s: float = 2e-5):
        """arrivals: list of Chunk sorted by time.  Returns (latencies in
        seconds per chunk, results per stream, elapsed seconds, r*w done).
        Afterwards self.steps is the number of steps launched and
        self.fused_steps those whose chunks all took the fused single-launch
        step (every chunk at most the tuning's fused_edges)."""
        st = self.stream
        fused_edges = tc_multi_get_tuning(self.bank.h)["fused_edges"]
        self.steps = self.fused_steps = 0
        pending = collections.deque(arrivals)
        ready = collections.defaultdict(collections.deque)
        slot_of, waitlist, free = {}, collections.deque(), list(range(self.slots))[::-1]
        done_streams, results, lat = [], {}, []
        inflight = collections.deque()
        rw = 0
        torch.cuda.synchronize()
        # the GPU clock's origin: an event that has completed before the
        # host clock starts, so a GPU time after it never reads as earlier
        # than the host time of the same instant (latencies err high by the
        # few microseconds the synchronisation takes to return, never low)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(st)
        ref.synchronize()
        t0 = time.perf_counter()
        while pending or inflight or waitlist or any(ready.values()):
            now = time.perf_counter() - t0
            while pending and pending[0].t <= now:
                c = pending.popleft()
                if c.stream not in slot_of and not ready[c.stream]:
                    waitlist.append(c.stream)
                ready[c.stream].append(c)
            # retire finished steps (in order)
            while inflight and inflight[0][0].query():
                ev, items = inflight.popleft()
                t_done = ref.elapsed_time(ev) / 1e3
                for c in items:
                    lat.append(t_done - c.t)
                    if c.last:
                        done_streams.append(c.stream)
            # a finished stream's slot is read out and freed only when needed
            if waitlist and not free and done_streams:
                S, m, tau = tc_multi_estimate(self.bank.h)
                for sid in done_streams:
                    b = slot_of.pop(sid)
                    results[sid] = Result(int(S[b]), int(m[b]), float(tau[b]))
                    free.append(b)
                done_streams = []
            while waitlist and free:
                sid = waitlist.popleft()
                b = free.pop()
                tc_multi_assign(self.bank.h, b, seeds[sid], st)
                slot_of[sid] = b
            if len(inflight) < self.depth:
                ids, chunks, items = [], [], []
                # oldest waiting chunks first, up to the step's edge cap
                heads = sorted((ready[sid][0].t, sid) for sid in slot_of if ready[sid])
                room = self.max_step_edges
                for _, sid in heads:
                    w = int(ready[sid][0].edges.shape[0])
                    if w > self.max_step_edges:
                        raise ValueError(f"a chunk of {w} edges exceeds the step cap")
                    if w > room:
                        continue
                    room -= w
                    c = ready[sid].popleft()
                    ids.append(slot_of[sid])
                    chunks.append(c.edges)
                    items.append(c)
                    rw += self.r * w
                if ids:
                    self.bank.process(ids, chunks, st)
                    self.steps += 1
                    self.fused_steps += all(int(c.shape[0]) <= fused_edges for c in chunks)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(st)
                    inflight.append((ev, items))
                    continue
            if inflight or pending:
                time.sleep(spin_s)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        S, m, tau = tc_multi_estimate(self.bank.h)
        for sid in done_streams:
            b = slot_of.pop(sid)
            results[sid] = Result(int(S[b]), int(m[b]), float(tau[b]))
        return lat, results, elapsed, rw

    def close(self):
        self.bank.close()


def chunk_streams(streams, seed: int, lo: int = 1000, hi: int = 1_000_000):
    """Cut every stream into chunks of log-uniform size in [lo, hi] pairs."""
    g = torch.Generator().manual_seed(seed)
    out = []
    for e in streams:
        m = e.shape[0]
        pieces, j = [], 0
        while j < m:
            u = float(torch.rand(1, generator=g, dtype=torch.float64))
            w = int(round(lo * (hi / lo) ** u))
            pieces.append(e[j:j + w])
            j += w
        out.append(pieces)
    return out
