"""Serving loop over the continuous-batching server of libhjb.

Requests arrive on a Poisson clock; a request is submitted when its arrival
time has passed, admitted by the server when its HBM footprint fits,
prepared (coarse solve, feedback, colours, labels) and then joins the live
sweep rounds while other requests are running.  Latency = completion time
minus arrival time.  Every result is the bits of the same request solved
alone (the tests check it).
"""
from __future__ import annotations

import time
from typing import Iterable, List, Optional

import numpy as np

from . import hjb


def run(requests: Iterable, hbm_budget: int, precision: int = hjb.HJB_F32, tol: float = 1e-5,
        rounds_per_step: int = 4, opts: Optional[hjb.hjb_solve_opts] = None,
        closed_loop: bool = False, keep_results: bool = False, verbose: bool = False) -> dict:
    """Runs the server over `requests` (ServingRequest with arrival_s, fine,
    coarse).  closed_loop=True submits everything at t = 0 (capacity run).
    Returns latencies, throughput and optionally the results."""
    reqs: List = list(requests)
    reqs.sort(key=lambda r: r.arrival_s)
    S = hjb.hjb_server_create(hbm_budget, precision, tol, 0, opts)
    t0 = time.perf_counter()
    arrival = {r.rid: (0.0 if closed_loop else r.arrival_s) for r in reqs}
    tickets = {}
    done = {}
    stats = {}
    results = {}
    nxt = 0
    live = queued = 0
    steps = 0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrival[reqs[nxt].rid] <= now:
            r = reqs[nxt]
            tickets[r.rid] = (S.submit(r.fine, r.coarse), r)
            nxt += 1
        if not tickets and nxt < len(reqs):
            time.sleep(max(0.0, arrival[reqs[nxt].rid] - now))
            continue
        live, queued = S.step(rounds_per_step)
        steps += 1
        t_now = time.perf_counter() - t0
        for rid, (t, r) in list(tickets.items()):
            out, st = S.poll(t)
            if out is not None:
                done[rid] = t_now
                stats[rid] = st
                if keep_results:
                    results[rid] = out
                del tickets[rid]
        if verbose and steps % 20 == 0:
            import sys
            print(f"[serve] t={t_now:.2f}s done {len(done)}/{len(reqs)} live {live} "
                  f"queued {queued}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    S.free()
    lat = np.array([done[r.rid] - arrival[r.rid] for r in reqs])
    upd = sum(s["updates"] for s in stats.values())
    out = {
        "requests": len(reqs), "wall_s": wall, "steps": steps,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3),
        "requests_per_s": len(reqs) / wall, "updates": int(upd), "updates_per_s": upd / wall,
    }
    if keep_results:
        out["results"] = results
    return out


def run_stream(requests: Iterable, hbm_budget: int, precision: int = hjb.HJB_F32,
               tol: float = 1e-5, rounds_per_step: int = 4,
               opts: Optional[hjb.hjb_solve_opts] = None, progress_every: int = 0) -> dict:
    """Runs the server over a stream of requests in arrival order (arrival_s
    from the start of the run), holding only the requests in flight: each
    one is submitted when its arrival time has passed (the server copies its
    arrays) and dropped once its result is collected.  For long request
    streams whose arrays would not fit host memory all at once.  Returns
    latency percentiles and throughput."""
    S = hjb.hjb_server_create(hbm_budget, precision, tol, 0, opts)
    it = iter(requests)
    nxt = next(it, None)
    t0 = time.perf_counter()
    pending = {}
    lat: List[float] = []
    late: List[float] = []
    upd = 0
    done = 0
    while nxt is not None or pending:
        now = time.perf_counter() - t0
        while nxt is not None and nxt.arrival_s <= now:
            late.append(now - nxt.arrival_s)
            pending[nxt.rid] = (S.submit(nxt.fine, nxt.coarse), nxt.arrival_s)
            nxt = next(it, None)
            now = time.perf_counter() - t0
        if not pending:
            if nxt is not None:
                time.sleep(max(0.0, nxt.arrival_s - now))
            continue
        S.step(rounds_per_step)
        t_now = time.perf_counter() - t0
        for rid, (t, arr) in list(pending.items()):
            out, st = S.poll(t)
            if out is not None:
                lat.append(t_now - arr)
                upd += st["updates"]
                done += 1
                del pending[rid]
                if progress_every and done % progress_every == 0:
                    import sys
                    print(f"[serve] t={t_now:.1f}s done {done}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    S.free()
    L = np.array(lat)
    return {"requests": len(lat), "wall_s": wall,
            "p50_ms": float(np.percentile(L, 50) * 1e3), "p99_ms": float(np.percentile(L, 99) * 1e3),
            "mean_ms": float(L.mean() * 1e3), "max_ms": float(L.max() * 1e3),
            "requests_per_s": len(lat) / wall, "updates": int(upd), "updates_per_s": upd / wall,
            "submit_late_max_ms": float(max(late) * 1e3) if late else 0.0}
