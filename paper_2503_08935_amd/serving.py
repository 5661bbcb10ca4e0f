"""Request loop over the continuous-batching server (poisson_server_*).

A synthetic stream of Poisson solves arrives in real time; each request is
submitted when it arrives (its right-hand side generated on the device with the
counter-based generator), and the loop keeps calling poisson_server_step, which
retires finished requests, admits queued ones by HBM footprint and advances the
running ones in batches, one size class per stream. Latency is arrival to
observed completion.

Stream recipe (seeded, host side): request i has grid edge
n_i = sizes[floor(len(sizes) * u_i)] with u_i the i-th uniform of
workloads.uniform(seed) mapped to [0, 1), exponential inter-arrival gaps
-ln(1 - v_i) / rate from the uniforms of seed + 1, and f ~ U[-1, 1) with seed
1000 + i on the unit cube (h = 1/(n+1)).
"""
import collections
import time

import numpy as np

from . import _binding as B
from . import workloads


def make_stream(n_requests, sizes, rate, seed):
    u = (workloads.uniform(seed, n_requests) + 1.0) / 2.0
    idx = np.minimum((u * len(sizes)).astype(np.int64), len(sizes) - 1)
    edges = np.asarray(sizes)[idx]
    v = (workloads.uniform(seed + 1, n_requests) + 1.0) / 2.0
    gaps = -np.log1p(-v) / rate
    arrivals = np.cumsum(gaps)
    return edges, arrivals


def run_stream(n_requests=2000, sizes=(32, 48, 64, 96, 128, 192, 256), rate=200.0, seed=5,
               precond=B.PC_CHEBYSHEV, degree=4, precision=B.MIXED, tol=1e-8, maxit=5000,
               budget_bytes=64 << 30, max_slots=64, iters=4, queue_extra=16, use_graph=True,
               size_classes=None, fuse_updates=None, four_steps=None, progress=None):
    """Run the stream; returns a dict of latency / throughput metrics."""
    import torch
    dev = torch.device("cuda:0")
    edges, arrivals = make_stream(n_requests, sizes, rate, seed)
    stream = torch.cuda.Stream()
    srv = B.Server(budget_bytes, max_slots, stream=stream, use_graph=use_graph,
                   fuse_updates=fuse_updates, four_steps=four_steps,
                   size_classes=size_classes)
    waiting = collections.deque()           # arrived, not yet submitted
    inflight = {}                           # ticket -> (request id, rhs, x)
    lat = np.full(n_requests, np.nan)
    iters_done = np.zeros(n_requests, dtype=np.int64)
    status = np.zeros(n_requests, dtype=np.int64)
    relres = np.zeros(n_requests)
    next_id = 0
    done = 0
    cap = max_slots + queue_extra
    t0 = time.perf_counter()
    last_report = t0
    while done < n_requests:
        now = time.perf_counter() - t0
        while next_id < n_requests and arrivals[next_id] <= now:
            waiting.append(next_id)
            next_id += 1
        while waiting and len(inflight) < cap:
            i = waiting.popleft()
            n = int(edges[i])
            with torch.cuda.stream(stream):
                b = torch.empty(n ** 3, dtype=torch.float64, device=dev)
                x = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
            B.fill_uniform(b, 1000 + i, stream)
            t = srv.submit(b, x, (n, n, n), workloads.spacing(n), precond, degree, precision, tol,
                           maxit)
            inflight[t] = (i, b, x)
        if not inflight:
            if next_id < n_requests:
                time.sleep(max(0.0, min(arrivals[next_id] - (time.perf_counter() - t0), 0.05)))
            continue
        srv.step(iters)
        tnow = time.perf_counter() - t0
        for t in list(inflight):
            st, stats = srv.poll(t)
            if st == B.PENDING:
                continue
            i = inflight.pop(t)[0]
            lat[i] = tnow - arrivals[i]
            status[i] = st
            iters_done[i] = stats["iterations"]
            relres[i] = stats["relres_true"]
            done += 1
        if progress and time.perf_counter() - last_report > 5.0:
            last_report = time.perf_counter()
            progress(f"served {done}/{n_requests}, in flight {len(inflight)}, "
                     f"waiting {len(waiting)}, t={tnow:.1f}s")
    makespan = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    unknowns = edges.astype(np.float64) ** 3
    ms = lat * 1e3
    by_size = {int(n): {"count": int((edges == n).sum()),
                        "p50_ms": float(np.percentile(ms[edges == n], 50)),
                        "p99_ms": float(np.percentile(ms[edges == n], 99))}
               for n in sorted(set(int(e) for e in edges))}
    return {
        "requests": n_requests, "rate_per_s": rate, "sizes": list(sizes), "degree": degree,
        "precision": "mixed" if precision == B.MIXED else "fp64", "tol": tol,
        "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
        "max_ms": float(ms.max()), "mean_ms": float(ms.mean()),
        "makespan_s": makespan, "solves_per_s": n_requests / makespan,
        "unknown_iters_per_s": float((unknowns * iters_done).sum() / makespan),
        # device time of the batches summed over the size classes (whose batches
        # overlap), over the makespan: above 1 when classes ran side by side
        "utilization": info["busy_ms"] / (makespan * 1e3),
        "latency_by_grid": by_size,
        "all_ok": bool(np.all(status == B.OK)), "max_relres_true": float(relres.max()),
        "mean_iterations": float(iters_done.mean()), "peak_arena_bytes": info["peak_bytes"],
        "budget_bytes": info["budget_bytes"], "steps": info["steps"],
    }
