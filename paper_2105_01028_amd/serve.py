"""Replay a stream of forward-solve requests through the batched server.

Requests arrive at their (Poisson) arrival times on the wall clock; the loop
submits each one as it arrives and keeps the server advancing, so requests
that arrive while others run join the batch as soon as a slot and device
memory are free.  Latency of a request = completion time - arrival time
(queueing included)."""
import time
from typing import List

import numpy as np

from . import trinity as T


def run_stream(server: "T.Server", requests: List, chunk_steps: int = 64, time_scale: float = 1.0,
               keep_results: bool = False, deadline_s: float = None):
    """requests: list of workloads.Request (arrival_s, problem).  time_scale
    stretches arrival times (e.g. to offer a fraction of the server's capacity).
    Returns dict with per-request latency (s), wall time and, optionally,
    results."""
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival_s)
    ids = {}
    arrive = {}
    done_t = {}
    results = {}
    t0 = time.perf_counter()
    nxt = 0
    while len(done_t) < len(requests):
        now = time.perf_counter() - t0
        while nxt < len(order) and requests[order[nxt]].arrival_s * time_scale <= now:
            i = order[nxt]
            ids[i] = server.submit(requests[i].problem)
            arrive[i] = requests[i].arrival_s * time_scale
            nxt += 1
        running, queued = server.advance(chunk_steps)
        now = time.perf_counter() - t0
        for i, rid in ids.items():
            if i in done_t:
                continue
            st = server.info(rid).status
            if st in (T.REQ_DONE, T.REQ_FAILED, T.REQ_CANCELLED):
                done_t[i] = now
                if keep_results and st == T.REQ_DONE:
                    results[i] = server.result(rid)
        if running == 0 and queued == 0 and nxt < len(order):
            # idle until the next arrival
            wait = requests[order[nxt]].arrival_s * time_scale - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
        if deadline_s is not None and time.perf_counter() - t0 > deadline_s:
            break
    lat = np.array([done_t[i] - arrive[i] for i in sorted(done_t)])
    return {"latency_s": lat, "wall_s": time.perf_counter() - t0, "ids": ids,
            "results": results, "completed": len(done_t)}
