"""Request loop over an ``xrt.Server``: open-loop arrivals, latency statistics.

``run_stream`` submits shots at their arrival times (seconds from the start),
drives ``progress()`` continuously, and reports per-shot latency from the
server's own clock (submit -> seen finished), images/s and terms/s.  Shots
that arrive while others run are admitted as memory and slots free up and
join the running persistent kernel.
"""
from __future__ import annotations

import time

import numpy as np


def poisson_arrivals(rng: np.random.Generator, n: int, rate: float) -> np.ndarray:
    """Arrival times of a Poisson process of the given rate (1/s)."""
    return np.cumsum(rng.exponential(1.0 / rate, n))


def run_stream(server, shots, arrivals, keep=None, on_done=None, timeout=600.0, sink=None, writers=0):
    """Serve ``shots`` arriving at ``arrivals`` (seconds, nondecreasing).

    keep:     indices whose images are copied out before release (returned:
              device tensors, or host arrays from a write-out server).
    on_done:  callback(index, ticket) run when a shot finishes, before release.
    sink:     callback(index, host image) for every shot (writing it out, say),
              then the release; run in the loop, or by ``writers`` threads
              while the loop keeps driving the server.
    Returns a dict with per-shot latency, admission wait and the makespan
    (which includes the sinks)."""
    keep = set(keep or ())
    n = len(shots)
    tickets = [None] * n
    latency = np.full(n, np.nan)
    wait = np.full(n, np.nan)
    images = {}
    pending = {}
    nxt = 0
    done = 0
    pool = None
    jobs = []
    if sink is not None and writers > 0:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=writers)

    def finish(i, t):
        sink(i, fetch(server, t))
        server.release(t)

    t0 = time.perf_counter()
    while done < n:
        now = time.perf_counter() - t0
        if now > timeout:
            raise TimeoutError(f"{n - done} shots still running after {timeout} s")
        while nxt < n and arrivals[nxt] <= now:
            tickets[nxt] = server.submit(shots[nxt])
            pending[tickets[nxt]] = nxt
            nxt += 1
        finished = []
        if server.progress() > 0:  # shots seen finishing in this call: find them
            for t, i in pending.items():
                info = server.info(t)
                if info.state == 2:
                    finished.append((t, i, info))
        for t, i, info in finished:
            latency[i] = info.t_done - info.t_submit
            wait[i] = info.t_admit - info.t_submit
            if i in keep:
                images[i] = server.host_image(t) if getattr(server, "writes_out", False) else server.image(t)
            if on_done is not None:
                on_done(i, t)
            if sink is None:
                server.release(t)
            elif pool is None:
                finish(i, t)
            else:
                jobs.append(pool.submit(finish, i, t))
            del pending[t]
            done += 1
        if not finished and nxt < n and not pending:
            # idle until the next arrival
            time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 0.001)))
    if pool is not None:
        for j in jobs:
            j.result()
        pool.shutdown()
    makespan = time.perf_counter() - t0
    return {"latency": latency, "admission_wait": wait, "makespan": makespan, "images": images,
            "tickets": tickets}


def fetch(server, ticket) -> np.ndarray:
    """A finished image on the host: read from the server's pinned host
    memory (write-out servers) or copied from the device arena."""
    if getattr(server, "writes_out", False):
        return server.host_image(ticket)
    return server.image(ticket, copy=False).cpu().numpy()


def summarize(result, shots, offered_rate=None):
    lat = result["latency"]
    terms = float(sum(s.n_terms for s in shots))
    out = {
        "shots": len(shots),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(np.mean(lat) * 1e3),
        "images_per_s": len(shots) / result["makespan"],
        "Gterm_per_s": terms / result["makespan"] / 1e9,
        "makespan_s": result["makespan"],
        "admission_wait_p99_ms": float(np.percentile(result["admission_wait"], 99) * 1e3),
    }
    if offered_rate is not None:
        out["offered_rate_per_s"] = offered_rate
    return out
