"""Drivers of the scan-job server (pic_server_* in libpic): a closed batch of
jobs submitted at once, and an open stream of jobs submitted at their arrival
times.  Scheduling, admission and batched stepping happen inside the library;
this module only submits on time, runs rounds and collects results.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding


def _summary(results, t_first, t_last, jobs):
    lat = np.array([r["t_finish"] - r["t_submit"] for r in results])
    esteps = sum(int(r["stats"]["electron_steps"]) for r in results)
    span = max(t_last - t_first, 1e-9)
    spans = [(r["t_admit"], r["t_finish"]) for r in results if r["t_admit"] >= 0]
    most = max((sum(1 for a, f in spans if a <= t0 < f) for t0, _ in spans), default=0)
    bad = [r for r in results if r["status"] not in ("PIC_OK", "PIC_ERR_OVERFLOW")]
    return dict(jobs=len(results), failed=len(bad), electron_steps=esteps, wall_s=span,
                electron_steps_per_s=esteps / span,
                latency_p50_s=float(np.percentile(lat, 50)) if lat.size else None,
                latency_p99_s=float(np.percentile(lat, 99)) if lat.size else None,
                latency_max_s=float(lat.max()) if lat.size else None,
                max_resident=most,
                kept_photons=int(sum(sum(r["stats"]["kept"]) for r in results)))


def run_batch(jobs, tables_by_z, max_jobs=64, quantum_steps=16, hbm_reserve_bytes=8 << 30):
    """Submit every job at t = 0 and serve until all are done."""
    srv = binding.Server(max_jobs=max_jobs, quantum_steps=quantum_steps,
                         hbm_reserve_bytes=hbm_reserve_bytes)
    t0 = srv.clock()
    for w in jobs:
        srv.submit(w, tables_by_z[int(w["Z"])], int(w["steps"]), t_arrival=t0)
    results = []
    while len(results) < len(jobs):
        r, q = srv.run()
        results += srv.poll()
        if r == 0 and q == 0 and len(results) < len(jobs):
            raise RuntimeError("server idle with jobs outstanding")
    t1 = max(r["t_finish"] for r in results)
    srv.close()
    return results, _summary(results, t0, t1, jobs)


def run_stream(arrivals, tables_by_z, max_jobs=64, quantum_steps=16,
               hbm_reserve_bytes=8 << 30, log=None):
    """Serve (arrival_s, job) pairs: each job is submitted once the server
    clock passes its arrival time, with that time as its arrival stamp."""
    srv = binding.Server(max_jobs=max_jobs, quantum_steps=quantum_steps,
                         hbm_reserve_bytes=hbm_reserve_bytes)
    pending = sorted(arrivals, key=lambda a: a[0])
    n = len(pending)
    t0 = srv.clock()
    results = []
    rounds = 0
    while len(results) < n:
        now = srv.clock() - t0
        while pending and pending[0][0] <= now:
            ta, w = pending.pop(0)
            srv.submit(w, tables_by_z[int(w["Z"])], int(w["steps"]), t_arrival=t0 + ta)
        r, q = srv.run()
        done = srv.poll()
        results += done
        rounds += 1
        if log and (done or rounds % 50 == 0):
            log(f"t={srv.clock() - t0:7.2f}s resident={r} queued={q} done={len(results)}/{n}")
        if r == 0 and q == 0 and pending:
            time.sleep(max(0.0, pending[0][0] - (srv.clock() - t0)))
    t1 = max(r["t_finish"] for r in results)
    srv.close()
    s = _summary(results, t0, t1, [w for _, w in arrivals])
    s["rounds"] = rounds
    return results, s


def run_sequential(jobs, tables_by_z):
    """The same jobs one after another with pic_step (no batching)."""
    t0 = time.perf_counter()
    esteps = 0
    lat = []
    for w in jobs:
        s = binding.Sim(w, tables_by_z[int(w["Z"])])
        s.pic_step(int(w["steps"]))
        s.synchronize()
        esteps += int(s.pic_emission_stats()["electron_steps"])
        s.pic_destroy()
        lat.append(time.perf_counter() - t0)
    t1 = time.perf_counter()
    return dict(jobs=len(jobs), electron_steps=esteps, wall_s=t1 - t0,
                electron_steps_per_s=esteps / (t1 - t0),
                latency_p50_s=float(np.percentile(lat, 50)),
                latency_p99_s=float(np.percentile(lat, 99)))
