"""Poisson request stream for the serving form (driver side).

Requests mix several processes, have log-uniform batch sizes and arrive with
exponential gaps; each is submitted to the C ABI server (me_server_*) as its
arrival time comes, so requests arrive while others are on the GPU.  Latency
is submit -> completion seen by the server loop (device-to-host copy
included).  Reading of an unspecified point: the process of each request is
drawn uniformly from the list.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B
from .inputs import CONFIGS, process_events


def make_stream(names, nreq, rate_hz, seed=5, nmin=256, nmax=65536):
    """Arrival times, process names and momenta of a seeded request stream."""
    ss = np.random.SeedSequence(seed)
    r_arr, r_proc, r_size, r_mom = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]
    gaps = r_arr.exponential(1.0 / rate_hz, size=nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    procs = [names[i] for i in r_proc.integers(0, len(names), size=nreq)]
    sizes = np.floor(np.exp(r_size.uniform(np.log(nmin), np.log(nmax), size=nreq))).astype(np.int64)
    moms = []
    for name, n in zip(procs, sizes):
        process, sqrt_s, _, _ = CONFIGS[name]
        from .inputs import PROCESS_LEGS, rambo
        moms.append(rambo(int(n), sqrt_s, PROCESS_LEGS[process][2:], seed=0, rng=r_mom))
    return arrivals, procs, moms


def run_stream(handles, arrivals, procs, moms, budget_bytes=1 << 30, n_slots=8, timeout_s=120.0, times=None,
               on_created=None):
    """Replay the stream against a server; returns per-request latencies,
    outputs and the wall time.  If `times` is a list, it receives the
    (queue_s, service_s) split of every request; on_created(server) runs
    once the server exists, before the first submission."""
    srv = B.me_server_create(budget_bytes, n_slots)
    if on_created is not None:
        on_created(srv)
    outs = [np.empty(m.shape[0], dtype=np.float64) for m in moms]
    tickets = []
    t0 = time.perf_counter()
    try:
        for i, (ta, name, m) in enumerate(zip(arrivals, procs, moms)):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            tickets.append(B.me_server_submit(srv, handles[name], m, outs[i]))
        lat = np.empty(len(tickets))
        status = np.empty(len(tickets), dtype=np.int64)
        for i, t in enumerate(tickets):
            st, l = B.me_server_wait(srv, t, timeout_s)
            status[i], lat[i] = st, l
            if times is not None:
                times.append(B.me_server_times(srv, t))
        wall = time.perf_counter() - t0
        stats = B.me_server_stats(srv)
    finally:
        B.me_server_destroy(srv)
    return lat, status, outs, wall, stats
