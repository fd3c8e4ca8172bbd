"""Serving loop over the continuous-batching server of libpms.

Keyframe densification requests arrive over time (as a SLAM front end emits
keyframes); each is submitted to a ``Server`` the moment its arrival time
has passed, and the loop keeps stepping the server -- one tick advances
every admitted job by one half-sweep -- until every request is done.
Latency is measured per request from its arrival time to the host seeing
it done (polled after every tick, so at most about one tick late).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from ._binding import JobDesc, Server


@dataclasses.dataclass
class Request:
    arrival_s: float   # seconds after the start of the run
    job: object        # a JobDesc, or a callable that makes one at submission
    tag: object = None  # caller's label, returned with the result


@dataclasses.dataclass
class Result:
    tag: object
    arrival_s: float
    submit_s: float
    done_s: float

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def run(server: Server, requests: list[Request], stream=None, on_done=None,
        progress_every_s: float = 10.0, log=None, keep_jobs: bool = True, ready=None) -> dict:
    """Serves `requests` in real time; returns the per-request results and
    the summary (throughput, p50/p99 latency, mean batch occupancy).

    ``on_done(request, result)`` is called once per request when it is done
    (the job's output tensors are final then). With ``keep_jobs`` False the
    request drops its job after that call, which frees its tensors.
    ``ready(request)``, if given, holds an arrived request back until it
    returns True (e.g. until the keyframe it starts from is done); held
    requests are submitted in arrival order, and their latency still counts
    from arrival."""
    reqs = sorted(requests, key=lambda r: r.arrival_s)
    inflight: dict[int, tuple[Request, float]] = {}
    results: list[Result] = []
    i = 0
    t0 = time.perf_counter()
    next_report = progress_every_s
    held: list[Request] = []
    while i < len(reqs) or inflight or held:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i].arrival_s <= now:
            held.append(reqs[i])
            i += 1
        still = []
        for rq in held:
            if ready is not None and not ready(rq):
                still.append(rq)
                continue
            if not isinstance(rq.job, JobDesc):
                rq.job = rq.job()
            tk = server.submit(rq.job)
            inflight[tk] = (rq, now)
        held = still
        if not inflight:
            nxt = reqs[i].arrival_s - now if i < len(reqs) else 0.001
            time.sleep(max(0.0, min(nxt, 0.05)))
            continue
        active, _ = server.step(stream)
        now = time.perf_counter() - t0
        for tk in list(inflight):
            if server.poll(tk) == Server.DONE:
                rq, sub = inflight.pop(tk)
                res = Result(rq.tag, rq.arrival_s, sub, now)
                results.append(res)
                if on_done is not None:
                    on_done(rq, res)
                if not keep_jobs:
                    rq.job = None
        if active == 0 and inflight:
            time.sleep(0.0005)
        if log is not None and now >= next_report:
            log(f"t={now:.0f}s submitted {i}/{len(reqs)} done {len(results)} in flight {len(inflight)}")
            next_report += progress_every_s
    wall = time.perf_counter() - t0
    lat = np.array([r.latency_s for r in results]) if results else np.zeros(1)
    st = server.stats()
    return {
        "results": results,
        "requests": len(reqs),
        "wall_s": wall,
        "keyframes_per_s": len(results) / wall if wall > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "mean_occupancy": st["mean_occupancy"],
        "ticks": st["ticks"],
        "arena_peak_bytes": st["arena_peak"],
    }
