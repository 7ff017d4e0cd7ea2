"""Request loop for the continuous-batching engine.

Requests arrive at given times (seconds from the start); each is admitted
to the engine as soon as its device footprint fits (otherwise it waits in a
FIFO queue).  Every engine step decomposes the short requests admitted since
the last step whole on chip and advances every long (streaming) request by
one sift (several steps per call when the engine is lightly loaded); a
request's latency runs from its arrival to the poll that reports its outputs
complete.  The plain comparator serves the same arrivals one request
at a time, each with its own launch sequence (semd_decompose_ex).

Inputs and outputs are device tensors allocated before the loop starts.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

import torch

from . import Engine, semd_decompose_ex


# steps per engine call when nothing waits for admission and at most
# BURST_MAX_RESIDENT requests are resident
BURST_STEPS = 8
BURST_MAX_RESIDENT = 4


@dataclass
class Request:
    signal: torch.Tensor   # device, M*N column-major
    dims: tuple            # (M, N)
    out: torch.Tensor      # device, (K+1) x M*N
    n_imfs: torch.Tensor   # device, 1 int32
    D: int
    K: int
    S: int


def serve_engine(reqs: list[Request], arrivals: list[float], budget: int, max_requests: int,
                 stream=None) -> dict:
    """Continuous batching.  Returns per-request latencies (s), the wall time
    from the first arrival to the last completion, and the steps taken."""
    eng = Engine(budget, max_requests)
    n = len(reqs)
    lat = [0.0] * n
    queue: deque[int] = deque()
    owner: dict[int, int] = {}
    nxt = done = steps = 0
    max_resident = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            while queue:
                j = queue[0]
                r = reqs[j]
                t = eng.admit(r.signal, r.dims, r.out, r.n_imfs, r.D, r.K, r.S)
                if t is None:
                    break
                owner[t] = j
                queue.popleft()
            resident = eng.resident()
            max_resident = max(max_resident, resident)
            if resident == 0:
                if nxt < n:
                    wait = arrivals[nxt] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.002))
                continue
            # With no request waiting for admission and few resident, a step
            # is shorter on the device than its host round trip: take
            # BURST_STEPS steps in one call.  Otherwise one, so that
            # admissions and retirements happen at every step.
            burst = BURST_STEPS if not queue and resident <= BURST_MAX_RESIDENT else 1
            if burst > 1:
                eng.step_n(burst, stream)
            else:
                eng.step(stream)
            steps += burst
            fin = eng.poll()
            if fin:
                now = time.perf_counter() - t0
                for t in fin:
                    j = owner.pop(t)
                    lat[j] = now - arrivals[j]
                    done += 1
        wall = time.perf_counter() - t0
    finally:
        eng.close()
    return {"latency": lat, "wall": wall, "steps": steps, "max_resident": max_resident}


def serve_plain(reqs: list[Request], arrivals: list[float], path: int, stream=None) -> dict:
    """One request at a time in arrival order, each decomposed by its own
    launch sequence and waited for before the next starts."""
    n = len(reqs)
    lat = [0.0] * n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, r in enumerate(reqs):
        wait = arrivals[j] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        semd_decompose_ex(r.signal, list(r.dims), r.D, r.K, r.S, r.out, r.n_imfs, stream=stream,
                          path=path)
        torch.cuda.synchronize()
        lat[j] = time.perf_counter() - t0 - arrivals[j]
    wall = time.perf_counter() - t0
    return {"latency": lat, "wall": wall}
