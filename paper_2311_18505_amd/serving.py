"""Continuous-batching synthesis server over the C ABI.

Requests (one string each: physical parameters, excitation, duration) arrive
over time.  A request is admitted into a free device slot as soon as one is
free and its memory fits the budget (strings beyond the largest size class are
refused); its state then stays on the device until it finishes.  Every loop
iteration advances all admitted strings by one chunk (480 samples = 10 ms at
48 kHz) in one batched launch, gathers the new chunk of every active string in
one copy and hands it to the caller, so requests that arrive while others are
being stepped join the next launch and overlap with them on the GPU.

Latencies are measured on the host clock from a request's arrival: the first
chunk (its first samples on the host) and completion (its last samples on the
host).  A request whose string the device flags (energy monitor or solver)
fails alone: its slot is freed, its audio is not delivered past the last
sample it produced, and it counts neither as done nor in the latencies.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import binding

CHUNK = 480


@dataclasses.dataclass
class Request:
    rid: int
    params: dict
    excitation: dict
    arrival: float          # seconds after the start of the run
    nbytes: int = 0         # device memory charged to the budget while admitted


@dataclasses.dataclass
class ServeStats:
    first_chunk_s: dict
    completion_s: dict
    refused: list
    failed: list
    wall_s: float
    audio_s: float
    chunks: int
    max_active: int
    step_ms: list

    def summary(self) -> dict:
        def pct(d, q):
            v = np.fromiter(d.values(), dtype=np.float64)
            return float(np.percentile(v, q)) * 1e3 if len(v) else None
        return {
            "requests_done": len(self.completion_s),
            "refused": len(self.refused),
            "failed": len(self.failed),
            "first_chunk_ms": {"p50": pct(self.first_chunk_s, 50), "p99": pct(self.first_chunk_s, 99)},
            "completion_ms": {"p50": pct(self.completion_s, 50), "p99": pct(self.completion_s, 99)},
            "audio_s_per_s": self.audio_s / self.wall_s if self.wall_s > 0 else None,
            "wall_s": self.wall_s,
            "chunks": self.chunks,
            "max_active": self.max_active,
            "chunk_ms_mean": float(np.mean(self.step_ms)) if self.step_ms else None,
        }


def _estimate_bytes(params: dict, esz: int) -> int:
    """Device bytes of one request in a batch of element size esz (4 for
    FP32C, 8 for FP64): its output (two channels with the zeta readout) plus
    state, its excitation copy and tables (at most ~16 elements and 12 bytes
    of indices per grid point, lane padding included) and alignment."""
    nt, nl = binding.plan_grid(params)
    channels = 2 if params.get("readout_zeta", 0) else 1
    return channels * esz * (int(params["n_samples"]) + 64) + (16 * esz + 12) * (nt + nl) + 8 * 256


class Server:
    def __init__(self, capacity: int = 8192, precision: str = "fp32c", chunk: int = CHUNK,
                 mem_budget: int = 32 << 30):
        self.b = binding.StringBatch(capacity, precision)
        self.esz = 4 if precision == "fp32c" else 8
        self.capacity = capacity
        self.chunk = chunk
        self.mem_budget = mem_budget
        self.free = list(range(capacity - 1, -1, -1))   # pop() gives the lowest slot

    def close(self):
        self.b.close()

    def _admit(self, batch):
        """set_params + excite for (slot, request) pairs, one call per run of
        consecutive slots; returns the requests refused by the planner."""
        refused = []
        batch.sort(key=lambda x: x[0])
        i = 0
        while i < len(batch):
            j = i + 1
            while j < len(batch) and batch[j][0] == batch[j - 1][0] + 1:
                j += 1
            run = batch[i:j]
            try:
                self.b.set_params(run[0][0], [r.params for _, r in run])
                self.b.excite(run[0][0], [r.excitation for _, r in run])
            except binding.SbError:
                # admit the run one by one to isolate the refused requests
                for slot, r in run:
                    try:
                        self.b.set_params(slot, [r.params])
                        self.b.excite(slot, [r.excitation])
                    except binding.SbError:
                        refused.append((slot, r))
            i = j
        return refused

    def run(self, requests, keep=(), clock=time.perf_counter, on_chunk=None, log=None,
            log_every: float = 10.0) -> tuple:
        """Serve `requests` (arrival times relative to the start) in real time.
        Returns (ServeStats, {rid: samples} for the rids in `keep` that did not
        fail).  `log`, if
        given, receives a progress line every `log_every` seconds."""
        reqs = {r.rid: r for r in requests}
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        active = {}        # slot -> [request, samples_done, samples delivered]
        keep = set(keep)
        outputs = {rid: [] for rid in keep}
        first, done, refused, failed, step_ms = {}, {}, [], [], []
        mem_used, max_active, chunks = 0, 0, 0
        t0 = clock()
        next_log = log_every
        while pending or waiting or active:
            now = clock() - t0
            if log is not None and now >= next_log:
                log("t=%.0f s: %d done, %d active, %d waiting, %d chunks" % (now, len(done), len(active),
                                                                             len(waiting), chunks))
                next_log += log_every
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            new = []
            while waiting and self.free:
                r = waiting[0]
                need = _estimate_bytes(r.params, self.esz)
                if mem_used + need > self.mem_budget and (active or new):
                    break
                waiting.popleft()
                new.append((self.free.pop(), r))
                mem_used += need
                r.nbytes = need
            if new:
                for slot, r in self._admit(new):
                    refused.append(r.rid)
                    mem_used -= r.nbytes
                    self.free.append(slot)
                    new.remove((slot, r))
                for slot, r in new:
                    active[slot] = [r, 2, 0]
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            max_active = max(max_active, len(active))
            ts = clock()
            self.b.step(self.chunk)
            slots = sorted(active)
            rows, sdone, flags = self.b.gather_output(slots, [active[s][2] for s in slots], self.chunk + 2,
                                                      status=True)
            t_avail = clock() - t0
            step_ms.append((clock() - ts) * 1e3)
            chunks += 1
            for i, s in enumerate(slots):
                r, sd, dl = active[s]
                ns = int(r.params["n_samples"])
                if flags[i]:
                    # the device stopped this string: the request fails alone
                    failed.append(r.rid)
                    outputs.pop(r.rid, None)
                    del active[s]
                    self.free.append(s)
                    mem_used -= r.nbytes
                    continue
                sd = min(ns, int(sdone[i]))
                cnt = sd - dl
                if r.rid in outputs:
                    outputs[r.rid].append(rows[i, :cnt].copy())
                if on_chunk is not None:
                    on_chunk(r.rid, rows[i, :cnt])
                if dl == 0:
                    first[r.rid] = t_avail - r.arrival
                active[s] = [r, sd, sd]
                if sd >= ns:
                    done[r.rid] = t_avail - r.arrival
                    del active[s]
                    self.free.append(s)
                    mem_used -= r.nbytes
            self.free.sort(reverse=True)
        wall = clock() - t0
        audio = sum(int(reqs[rid].params["n_samples"]) / reqs[rid].params["fs"] for rid in done)
        stats = ServeStats(first, done, refused, failed, wall, audio, chunks, max_active, step_ms)
        return stats, {rid: np.concatenate(v) if v else np.empty(0) for rid, v in outputs.items()}


def requests_from(arrivals, items):
    """Requests from arrival times and (params, excitation) pairs."""
    return [Request(i, p, e, float(a)) for i, ((p, e), a) in enumerate(zip(items, arrivals))]
