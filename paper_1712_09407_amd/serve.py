"""Poisson-arrival driver of the serving loop: p50/p99 event latency and
sustained events/s for a given arrival rate and server configuration."""
from __future__ import annotations

import time

import numpy as np


def run(server, events, rate_hz: float, n_events: int, seed: int = 4, keep=None):
    """Submit n_events events (cycling through `events`, HostEvent list) at
    Poisson arrival times of mean rate rate_hz.  Latency of an event = time
    its results are on the host - its scheduled arrival (waiting for
    admission included).  keep: set of indices whose results are fetched."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, n_events)
    t0 = server.now() + 0.05
    arrive = t0 + np.cumsum(gaps)
    lat = np.zeros(n_events)
    t_last = [0.0]
    done_n = 0
    busy_retries = 0
    fetched = {}
    i = 0

    def drain(timeout_ms=0):
        nonlocal done_n
        for d in server.poll(timeout_ms):
            k = int(d["tag"])
            if d["status"] != 0:
                raise RuntimeError(f"event {k} failed with {d['status']}")
            lat[k] = d["t_done"] - arrive[k]
            t_last[0] = max(t_last[0], d["t_done"])
            done_n += 1
            if keep is not None and k in keep:
                fetched[k] = server.fetch(d, events[k % len(events)].n_clusters)
            elif server.cfg.keep_results:
                server.fetch(d, events[k % len(events)].n_clusters)

    while i < n_events:
        now = server.now()
        if now < arrive[i]:
            drain(0)
            dt = arrive[i] - server.now()
            if dt > 2e-4:
                time.sleep(min(dt - 1e-4, 2e-3))
            continue
        rc = server.submit(events[i % len(events)], i)
        if rc == 0:
            i += 1
        else:
            busy_retries += 1
            drain(1)
    while done_n < n_events:
        drain(50)
    span = float(arrive[-1] - arrive[0]) if n_events > 1 else 1.0
    return dict(rate_hz=rate_hz, events=n_events,
                p50_ms=round(float(np.percentile(lat, 50) * 1e3), 3),
                p99_ms=round(float(np.percentile(lat, 99) * 1e3), 3),
                mean_ms=round(float(lat.mean() * 1e3), 3),
                offered_events_per_s=round((n_events - 1) / span, 1),
                sustained_events_per_s=round(n_events / (t_last[0] - arrive[0]), 1),
                busy_retries=busy_retries, stats=server.stats(), lat_ms=lat * 1e3), fetched
