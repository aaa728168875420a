"""Replay a job-arrival trace through the libkk job server in real time.

Arrivals follow the trace's own times (seconds from its start, scaled by
`time_scale`); the host thread submits every job whose arrival has passed,
then runs one server step (one chunk of sweeps for every admitted job) and
collects finished results.  When nothing is admitted or waiting it sleeps
until the next arrival.  Latency is completion minus scheduled arrival, both
on the server's clock, so time a job spends waiting for the current step to
end counts against it.
"""
from __future__ import annotations

import time
from typing import Iterable, List, Optional

import numpy as np

from . import kk


def replay(jobs: Iterable, server: "kk.Server", time_scale: float = 1.0, log=None) -> dict:
    jobs = sorted(jobs, key=lambda j: j.arrival)
    n = len(jobs)
    results: List[dict] = []
    t0 = server.now()
    i = 0
    submitted = 0
    while i < n or len(results) < submitted:
        now = server.now() - t0
        while i < n and jobs[i].arrival * time_scale <= now:
            server.submit(jobs[i], arrival=t0 + jobs[i].arrival * time_scale)
            i += 1
            submitted += 1
        if len(results) == submitted:
            # idle: wait for the next arrival
            if i < n:
                time.sleep(max(0.0, min(0.05, jobs[i].arrival * time_scale - now)))
            continue
        server.step()
        done = server.poll(1024)
        for r in done:
            server.release(r["id"])
        results.extend(done)
        if log and done:
            log(f"[serve] {len(results)}/{n} jobs done at t={server.now() - t0:.2f}s")
    return summarize(jobs, results, t0, server.stats(), time_scale)


def summarize(jobs, results: List[dict], t0: float, stats: dict, time_scale: float = 1.0) -> dict:
    failed = [r for r in results if r["status"] != kk.KK_OK]
    lat = np.array([r["t_done"] - r["t_arrival"] for r in results])
    wait = np.array([r["t_admit"] - r["t_arrival"] for r in results])
    first = min(j.arrival for j in jobs) * time_scale
    last_arrival = max(j.arrival for j in jobs) * time_scale
    end = max(r["t_done"] for r in results) - t0
    attempts = sum(r["attempts"] for r in results)
    offered_attempts = sum(j.L * j.L * j.sweeps for j in jobs)
    span = max(last_arrival - first, 1e-9)
    offered_rate = offered_attempts / span
    served_rate = attempts / max(end - first, 1e-9)
    return {
        "jobs": len(results), "failed": len(failed),
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()), "admission_wait_p50_s": float(np.percentile(wait, 50)),
        "admission_wait_p99_s": float(np.percentile(wait, 99)),
        "makespan_s": end - first, "attempts": attempts,
        "served_attempts_per_s": served_rate,
        "offered_jobs_per_s": (len(jobs) - 1) / span if len(jobs) > 1 else None,
        "offered_attempts_per_s": offered_rate,
        "served_over_offered": served_rate / offered_rate,
        "steps": stats["steps"], "peak_bytes": stats["peak_bytes"], "budget": stats["budget"],
        "gpu_busy_frac": stats["gpu_busy_s"] / max(end - first, 1e-9),
    }


def run_trace(jobs, chunk_sweeps: int = 1000, hbm_budget_bytes: int = 0, max_active: int = 0,
              time_scale: float = 1.0, log=None) -> dict:
    """Replay `jobs` through a fresh server and return the summary."""
    srv = kk.Server(hbm_budget_bytes=hbm_budget_bytes, max_active=max_active, chunk_sweeps=chunk_sweeps)
    try:
        return replay(jobs, srv, time_scale=time_scale, log=log)
    finally:
        srv.close()
