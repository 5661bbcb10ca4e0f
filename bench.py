#!/usr/bin/env python3
"""Benchmark: preconditioned Bi-CGSTAB for the 3D Poisson equation on one MI355X.

One step = one full solve (setup, iterations, true residual) of the 512^3 FP64
Chebyshev-8 Bi-CGSTAB on the unit cube, f ~ U[-1,1) (seed 4), x0 = 0, stopping at
relative residual 1e-8. The right-hand side is generated on the device with the
same counter-based generator as the host-side workloads, so inputs are resident
in HBM before the timed region. Printed as one JSON line:
  value        iterations per second over the timed solves (whole solves)
  loop_iter_per_s  iterations per second of the iteration loops' device time
               (HIP events); outside_loop_ms_per_solve is the rest of a solve
               (initial residual, interval and coefficients, true residual, host)
  hbm_gbps     algorithmic bytes of the iteration loop / loop device time
  tts_*        time to 1e-8 of the FP64 solve (median over the timed solves) and of
               the mixed solve (FP32 Chebyshev inside FP64 Bi-CGSTAB; median of 5),
               same right-hand side; fp64_x_is_oracle_x compares the FP64 x with the
               sha256 of the oracle's x stored under tests/golden/
  tol_1e-10, noisy_manufactured_tol_1e-10
               the other 512^3 configurations: FP64 and mixed to 1e-10, and the noisy
               manufactured problem with Block-Jacobi(CI) 64^3 vs Chebyshev-8 to 1e-10
               (median of 3 each)
  mixed_over_seeds_tol_1e-8
               mixed vs FP64 time to 1e-8 on five more right-hand sides (seeds 3, 5-8)
               and the median speed-up over them and seed 4
  solvers_256_tol_1e-8
               256^3, f ~ U[-1,1) seed 2, FP64 to 1e-8: no preconditioner, point Jacobi,
               Block-Jacobi(CI) 64^3 x 8, Chebyshev 4 and 8 (median of 3), each x checked
               against the sha256 of the oracle's stored solve
  roofline     dominant kernel (three fused interior Chebyshev steps, FP64),
               timed with HIP events on the stream it runs on
  cpu_baseline the CPU oracle on a bounded sample (2 iterations vs 1 iteration
               of the same 512^3 solve, median of 3; the difference is one
               iteration), all threads, plus one thread at 128^3, the host's CPU
               model, sockets, cores and memory, and the oracle's GB/s
  p99_solve_ms the serving stream: 2000 requests of n^3 grids, n uniform over
               {32,48,64,96,128,192,256}, Poisson arrivals at 200/s, mixed
               Chebyshev-4 to 1e-8, admitted by HBM footprint (serving.py);
               serving_below_saturation: 400 requests at 10/s
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "512³ Bi-CGSTAB iter/s + HBM GB/s; mixed vs FP64 time-to-1e-8; p99 solve ms"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="grid edge (n^3 interior unknowns)")
    ap.add_argument("--degree", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision solve")
    ap.add_argument("--no-unfused", action="store_true",
                    help="skip the comparison solve with one Chebyshev step per pass")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra 512^3 configurations (tol 1e-10 FP64 and mixed, Block-"
                         "Jacobi vs Chebyshev on the noisy manufactured problem) and the "
                         "below-saturation serving point")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-iters", type=int, default=4,
                    help="iterations per server step (completion is observed per step)")
    ap.add_argument("--table2", action="store_true",
                    help="instead of the benchmark: the preconditioner comparison of the paper's "
                         "Table 2 on its test problem (255^3 unknowns, mixed faces) on one GPU")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the benchmark: the remaining measurement configurations "
                         "(256^3 solver comparison, 512^3 Block-Jacobi vs Chebyshev to 1e-10, "
                         "mixed vs FP64 at 1e-8 and 1e-10, a below-saturation serving point), one "
                         "JSON line each")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a reference dispatch of known "
                         "size for rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traffic_record(kernel_file, workload):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/hbm_traffic.txt:
    FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the same counter's reading
    for a copy of known size), valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    src = open(os.path.join(ROOT, "paper_2503_08935_amd", "csrc", kernel_file), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    for line in open(path):
        f = line.split()
        if len(f) == 6 and not line.startswith("#") and f[0] == workload and f[2] == sha:
            return float(f[5])
    return None


def host_record():
    """CPU model, sockets, cores and memory of the host the oracle runs on (from /proc)."""
    rec = {"model": None, "sockets": None, "cores": None, "logical_cpus": os.cpu_count(),
           "usable_cpus": len(os.sched_getaffinity(0)), "ram_gib": None}
    try:
        phys, cores = set(), {}
        cur = {}
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and rec["model"] is None:
                rec["model"] = v
            elif k == "physical id":
                cur["pid"] = v
                phys.add(v)
            elif k == "cpu cores":
                cores[cur.get("pid")] = int(v)
        rec["sockets"] = len(phys) or None
        rec["cores"] = sum(cores.values()) or None
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                rec["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    return rec


def oracle_iteration_s(n, h, degree, seed, reps):
    """Seconds of one oracle iteration of the n^3 FP64 Chebyshev solve: the median over
    reps of time(maxit=2) - time(maxit=1), which cancels the setup."""
    import oracle
    from paper_2503_08935_amd import workloads
    b = workloads.uniform_grid(seed, (n, n, n))
    diffs, raw = [], []
    for _ in range(reps):
        ts = []
        for it in (1, 2):
            t0 = time.perf_counter()
            oracle.bicgstab(b, h, pc=oracle.PC_CHEBYSHEV, degree=degree, tol=1e-8, maxit=it)
            ts.append(time.perf_counter() - t0)
        diffs.append(max(ts[1] - ts[0], 1e-9))
        raw.append([round(t, 3) for t in ts])
    diffs.sort()
    return diffs[len(diffs) // 2], raw


def cpu_baseline(n, h, degree, seed):
    """The CPU oracle (oracle.c: -O3 -ffp-contract=off, OpenMP over z-planes, exact dots)
    on a bounded sample of the benchmark solve: one iteration at n^3 with every thread
    of this host (median of 3), and one iteration at 128^3 on one thread (median of 3),
    with the oracle's GB/s under the byte model of one Chebyshev step per pass (the
    oracle's own pass structure)."""
    import oracle
    from paper_2503_08935_amd import workloads
    threads = oracle.get_threads()
    per_it, raw = oracle_iteration_s(n, h, degree, seed, 3)
    log(f"cpu oracle {n}^3, {threads} threads: {per_it:.2f} s per iteration {raw}")
    model_b = 632.0 if degree == 8 else None
    oracle.set_threads(1)
    n1 = 128
    try:
        per_it1, raw1 = oracle_iteration_s(n1, workloads.spacing(n1), degree, seed, 3)
    finally:
        oracle.set_threads(threads)
    log(f"cpu oracle {n1}^3, 1 thread: {per_it1:.3f} s per iteration {raw1}")
    rec = {"value": 1.0 / per_it, "unit": "iter/s", "cores": threads, "kind": "oracle",
           "sample": f"one Bi-CGSTAB iteration of the {n}^3 FP64 Chebyshev-{degree} solve "
                     f"(seed {seed}): median over 3 of time(maxit=2) - time(maxit=1), setup "
                     f"excluded, {threads} OpenMP threads",
           "seconds_per_iteration": round(per_it, 4), "seconds_maxit_1_2": raw,
           "one_thread": {"grid": n1, "seconds_per_iteration": round(per_it1, 4),
                          "seconds_maxit_1_2": raw1,
                          "unknown_iterations_per_s": round(n1 ** 3 / per_it1, 1)},
           "unknown_iterations_per_s": round(n ** 3 / per_it, 1),
           "host": host_record()}
    if model_b:
        rec["model_bytes_per_unknown"] = model_b
        rec["oracle_gbps"] = round(model_b * n ** 3 / per_it / 1e9, 2)
        rec["oracle_gbps_one_thread"] = round(model_b * n1 ** 3 / per_it1 / 1e9, 3)
    return rec


def median(v):
    v = sorted(v)
    return v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])


def golden_x_sha256(name):
    """sha256 of the oracle's x stored by tests/golden/make_golden.py (None if absent)."""
    path = os.path.join(ROOT, "tests", "golden", name + ".txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("x_sha256 "):
            return line.split()[1]
    return None


def sha256_of(t):
    return hashlib.sha256(t.cpu().numpy().tobytes()).hexdigest()


def extra_configs(P, workloads, b, stream, degree):
    """The other 512^3 configurations: f ~ U[-1,1) seed 4 to 1e-10 in FP64 and mixed
    (median of 3 time-to-tolerance each), and the noisy manufactured problem (seed 3)
    with Block-Jacobi(CI) on 64^3 blocks vs Chebyshev, both degree 8, to 1e-10."""
    import torch
    n = 512
    shape = (n, n, n)
    h = workloads.spacing(n)

    def timed(rhs, pc, tol, precision, reps=3):
        x = torch.zeros_like(rhs)
        with P.Solver(shape, h, stream=stream, precision=precision) as s:
            tts = []
            for _ in range(reps):
                with torch.cuda.stream(stream):
                    x.zero_()
                st = s.solve(rhs, x, pc, degree, tol, 5000)
                d = s.stats()
                tts.append(d["solve_ms"] / 1e3)
        torch.cuda.synchronize()
        return x, {"status": st, "iterations": d["iterations"], "tts_s": round(median(tts), 4),
                   "runs": reps, "relres_true": d["relres_true"],
                   "hbm_gbps": round(d["model_gbps"], 1)}

    out = {}
    x64, r64 = timed(b, P.PC_CHEBYSHEV, 1e-10, P.FP64)
    xm, rm = timed(b, P.PC_CHEBYSHEV, 1e-10, P.MIXED)
    rel = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
    out["tol_1e-10"] = {"fp64": r64, "mixed": rm,
                        "mixed_speedup": round(r64["tts_s"] / rm["tts_s"], 3),
                        "mixed_vs_fp64_rel_diff": rel}
    ref = golden_x_sha256(f"full_512_cheb{degree}_fp64_tol1e-10")
    if ref is not None:
        out["tol_1e-10"]["fp64_x_is_oracle_x"] = sha256_of(x64) == ref
    log(f"1e-10: FP64 {r64['iterations']} it {r64['tts_s']} s, mixed {rm['iterations']} it "
        f"{rm['tts_s']} s, rel diff {rel:.2e}")
    del x64, xm
    # mixed vs FP64 over right-hand sides: the FP32 preconditioner's rounding slows
    # Bi-CGSTAB's convergence below about 1e-3 on some of them
    bs = torch.empty_like(b)
    seeds = {}
    for seed in (3, 5, 6, 7, 8):
        P.fill_uniform(bs, seed, stream)
        stream.synchronize()
        _, a64 = timed(bs, P.PC_CHEBYSHEV, 1e-8, P.FP64, reps=1)
        _, am = timed(bs, P.PC_CHEBYSHEV, 1e-8, P.MIXED, reps=1)
        seeds[seed] = {"fp64_iterations": a64["iterations"], "fp64_s": a64["tts_s"],
                       "mixed_iterations": am["iterations"], "mixed_s": am["tts_s"],
                       "speedup": round(a64["tts_s"] / am["tts_s"], 3)}
        log(f"seed {seed}: FP64 {a64['iterations']} it {a64['tts_s']} s, mixed "
            f"{am['iterations']} it {am['tts_s']} s")
    del bs
    out["mixed_over_seeds_tol_1e-8"] = {
        "seeds": seeds,
        "median_speedup_with_seed_4": None,
        "median_speedup": round(median([v["speedup"] for v in seeds.values()]), 3)}
    # 256^3, f ~ U[-1,1) seed 2: the solver comparison, each x against the oracle's
    n2 = 256
    b2 = torch.empty(n2 ** 3, dtype=torch.float64, device=b.device)
    P.fill_uniform(b2, 2, stream)
    stream.synchronize()
    cmp256 = {}
    for name, pc, m in (("none", P.PC_NONE, 0), ("jacobi", P.PC_JACOBI, 0),
                        ("bj64x8", P.PC_BLOCK_JACOBI, 8), ("cheb4", P.PC_CHEBYSHEV, 4),
                        ("cheb8", P.PC_CHEBYSHEV, 8)):
        x2 = torch.zeros_like(b2)
        with P.Solver((n2, n2, n2), workloads.spacing(n2), stream=stream) as s2:
            tts = []
            for _ in range(3):
                with torch.cuda.stream(stream):
                    x2.zero_()
                st = s2.solve(b2, x2, pc, m, 1e-8, 5000)
                d = s2.stats()
                tts.append(d["solve_ms"] / 1e3)
        torch.cuda.synchronize()
        r = {"status": st, "iterations": d["iterations"], "tts_s": round(median(tts), 4),
             "relres_true": d["relres_true"], "hbm_gbps": round(d["model_gbps"], 1)}
        ref = golden_x_sha256(f"full_256_{name}")
        if ref is not None:
            r["x_is_oracle_x"] = sha256_of(x2) == ref
        cmp256[name] = r
        log(f"256^3 {name}: {r['iterations']} it {r['tts_s']} s")
        del x2
    del b2
    out["solvers_256_tol_1e-8"] = cmp256
    f = torch.from_numpy(workloads.manufactured_noisy(shape, 3).ravel()).to(b.device)
    noisy = {}
    for name, pc in (("block_jacobi_64", P.PC_BLOCK_JACOBI), ("chebyshev", P.PC_CHEBYSHEV)):
        x, r = timed(f, pc, 1e-10, P.FP64)
        noisy[name] = r
        log(f"noisy 1e-10 {name}: {r['iterations']} it {r['tts_s']} s")
        del x
    del f
    torch.cuda.empty_cache()
    out["noisy_manufactured_tol_1e-10"] = noisy
    return out


def table2():
    """The solver comparison of the paper's Table 2 (Results section) on its test
    problem, one GPU: BiCGS, BJ(CI), G(CI) and GNoComm(CI) with 24 Chebyshev
    iterations per apply, the G/GNoComm interval rescaled by 100 and (1 - 1e-4)
    (Experimental Setup), 64^3 blocks, tolerance 1e-10, FP64."""
    import torch

    import paper_2503_08935_amd as P
    from paper_2503_08935_amd import workloads
    f, shape, h, bc = workloads.paper_problem()
    b = torch.from_numpy(f.ravel()).to("cuda:0")
    x = torch.zeros_like(b)
    rows = []
    cases = [("BiCGS", P.PC_NONE, 0, {}),
             ("BiCGS-BJ(CI)", P.PC_BLOCK_JACOBI, 24, {}),
             ("BiCGS-G(CI)", P.PC_CHEBYSHEV, 24, dict(lmin_scale=100.0, lmax_scale=1 - 1e-4)),
             ("BiCGS-GNoComm(CI)", P.PC_BLOCK_JACOBI, 24,
              dict(bj_global_interval=1, lmin_scale=100.0, lmax_scale=1 - 1e-4)),
             ("BiCGS-G(CI), analytic interval", P.PC_CHEBYSHEV, 24, {}),
             ("BiCGS-G(CI) degree 8", P.PC_CHEBYSHEV, 8, {})]
    for name, pc, m, opts in cases:
        with P.Solver(shape, h, bc=bc, **opts) as s:
            best = None
            for rep in range(2):
                x.zero_()
                st = s.solve(b, x, pc, m, 1e-10, 20000)
                d = s.stats()
                best = d if best is None or d["solve_ms"] < best["solve_ms"] else best
            rows.append({"solver": name, "status": st, "outer_iterations": best["iterations"],
                         "precond_iterations_per_outer": 2 * m,
                         "tts_s": round(best["solve_ms"] / 1e3, 4),
                         "relres_true": best["relres_true"],
                         "hbm_gbps": round(best["model_gbps"], 1)})
            log(json.dumps(rows[-1]))
    print(json.dumps({"table2_one_gpu": rows, "grid": shape, "h": h, "bc_neumann_mask": bc}))


def suite():
    """One JSON line per configuration; every solve is timed by the library (solve_ms
    from entry to return, on the device stream) and its true residual reported."""
    import torch

    import paper_2503_08935_amd as P
    from paper_2503_08935_amd import workloads
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()

    def run(shape, h, b, pc, m, tol, reps=3, **opts):
        x = torch.zeros_like(b)
        with P.Solver(shape, h, stream=stream, **opts) as s:
            ts = []
            for _ in range(reps):
                with torch.cuda.stream(stream):
                    x.zero_()
                st = s.solve(b, x, pc, m, tol, 20000)
                d = s.stats()
                ts.append(d["solve_ms"])
        ts.sort()
        return x, {"status": st, "iterations": d["iterations"], "half_step": d["half_step_exit"],
                   "tts_median_s": round(ts[len(ts) // 2] / 1e3, 4),
                   "relres_true": d["relres_true"], "hbm_gbps": round(d["model_gbps"], 1)}

    names = {P.PC_NONE: "none", P.PC_JACOBI: "jacobi", P.PC_CHEBYSHEV: "chebyshev",
             P.PC_BLOCK_JACOBI: "block_jacobi_64"}
    # 256^3, f ~ U[-1,1) seed 2, FP64, tol 1e-8
    n = 256
    h = workloads.spacing(n)
    b = torch.empty(n ** 3, dtype=torch.float64, device=dev)
    P.fill_uniform(b, 2, stream)
    stream.synchronize()
    for pc, m in ((P.PC_NONE, 0), (P.PC_JACOBI, 0), (P.PC_BLOCK_JACOBI, 8), (P.PC_CHEBYSHEV, 4),
                  (P.PC_CHEBYSHEV, 8)):
        _, r = run((n, n, n), h, b, pc, m, 1e-8)
        r.update({"config": "256^3 U[-1,1) seed 2, FP64, tol 1e-8", "precond": names[pc],
                  "degree": m})
        print(json.dumps(r), flush=True)
    del b
    # 512^3 noisy manufactured (seed 3), Block-Jacobi 64^3 vs Chebyshev-8, tol 1e-10
    n = 512
    h = workloads.spacing(n)
    f = torch.from_numpy(workloads.manufactured_noisy((n, n, n), 3).ravel()).to(dev)
    for pc in (P.PC_BLOCK_JACOBI, P.PC_CHEBYSHEV):
        _, r = run((n, n, n), h, f, pc, 8, 1e-10)
        r.update({"config": "512^3 3pi^2 sin sin sin + 1e-3 N(0,1) seed 3, FP64, tol 1e-10",
                  "precond": names[pc], "degree": 8})
        print(json.dumps(r), flush=True)
    del f
    # 512^3 f ~ U[-1,1) seed 4: mixed vs FP64 Chebyshev-8 at 1e-8 and 1e-10
    b = torch.empty(n ** 3, dtype=torch.float64, device=dev)
    P.fill_uniform(b, 4, stream)
    stream.synchronize()
    for tol in (1e-8, 1e-10):
        x64, r64 = run((n, n, n), h, b, P.PC_CHEBYSHEV, 8, tol, precision=P.FP64)
        xm, rm = run((n, n, n), h, b, P.PC_CHEBYSHEV, 8, tol, precision=P.MIXED)
        rel = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
        print(json.dumps({"config": f"512^3 U[-1,1) seed 4, Chebyshev-8, tol {tol}",
                          "fp64": r64, "mixed": rm,
                          "mixed_speedup": round(r64["tts_median_s"] / rm["tts_median_s"], 3),
                          "mixed_vs_fp64_rel_diff": rel}), flush=True)
        del x64, xm
    del b
    torch.cuda.empty_cache()
    # serving below saturation: 400 requests at 10/s
    from paper_2503_08935_amd import serving
    sv = serving.run_stream(n_requests=400, rate=10.0, progress=log)
    print(json.dumps({"config": "serving, 400 requests at 10/s (below saturation)",
                      **{k: (float(f"{v:.6g}") if isinstance(v, float) else v)
                         for k, v in sv.items()}}), flush=True)


def main():
    a = parse()
    if a.table2:
        return table2()
    if a.suite:
        return suite()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {a.gpus}); the solver has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2503_08935_amd as P
    from paper_2503_08935_amd import workloads

    dev = torch.device("cuda:0")
    n = a.n
    shape = (n, n, n)
    N = n ** 3
    h = workloads.spacing(n)
    stream = torch.cuda.Stream()  # default priority
    if a.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
    log(f"grid {n}^3, FP64 Chebyshev-{a.degree}, tol {a.tol}")
    with torch.cuda.stream(stream):
        b = torch.empty(N, dtype=torch.float64, device=dev)
        x = torch.zeros(N, dtype=torch.float64, device=dev)
        P.fill_uniform(b, a.seed, stream)
    stream.synchronize()

    s64 = P.Solver(shape, h, stream=stream, precision=P.FP64)

    def solve64():
        with torch.cuda.stream(stream):
            x.zero_()
            st = s64.solve(b, x, P.PC_CHEBYSHEV, a.degree, a.tol, 5000)
        if st != P.OK:
            raise RuntimeError(f"FP64 solve status {st}")
        return s64.stats()

    for w in range(a.warmup):
        st = solve64()
        log(f"warmup {w}: {st['iterations']} iterations, {st['solve_ms']:.1f} ms")
    torch.cuda.synchronize()
    iters = 0
    loop_ms = 0.0
    model_bytes = 0.0
    stats = []
    t0 = time.perf_counter()
    for k in range(a.steps):
        st = solve64()
        iters += st["iterations"]
        loop_ms += st["loop_ms"]
        model_bytes += st["model_bytes"]
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    last = stats[-1]
    log(f"timed: {a.steps} solves, {iters} iterations in {wall:.3f} s, true relres "
        f"{last['relres_true']:.3e}")
    x64 = x.clone()

    # kernels timed with HIP events on the solver's stream: the dominant one
    # (below), the fused pair and the single interior step for reference
    reps = a.kernel_reps

    def kernel_time(kernel, batches=5):
        # the median over batches of back-to-back launches, so that one slow
        # batch does not stand for the kernel
        s64.kernel_bench(kernel, P.FP64, 2)  # warm
        per = []
        for _ in range(batches):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s64.kernel_bench(kernel, P.FP64, reps)
            e1.record(stream)
            e1.synchronize()
            per.append(e0.elapsed_time(e1) / reps)
        ms = sorted(per)[len(per) // 2]
        nbytes = s64.kernel_bytes(kernel, P.FP64)
        return ms, nbytes, nbytes / (ms * 1e6)

    # the dominant kernel of the default plan: three fused Chebyshev steps per
    # pass (two per pass where three are not available)
    try:
        k_ms, k_bytes, k_gbps = kernel_time(P.KERNEL_CHEB_TRIPLE)
        dom, dom_name, dom_work = "triple", "k_cheb_triple_lds<double,double,false,false,1,4,8,false,true,0>", "cheb_triple"
    except P.PoissonError:
        k_ms, k_bytes, k_gbps = kernel_time(P.KERNEL_CHEB_PAIR)
        dom, dom_name, dom_work = "pair", "k_cheb_pair_lds<double,double,false,false,2,8,4,false,true,0>", "cheb_pair"
    p_ms, p_bytes, p_gbps = kernel_time(P.KERNEL_CHEB_PAIR)
    s_ms, s_bytes, s_gbps = kernel_time(P.KERNEL_CHEB_STEP)
    log(f"cheb {dom} FP64: {k_ms * 1e3:.1f} us/launch, {k_gbps:.0f} GB/s algorithmic; pair "
        f"{p_ms * 1e3:.1f} us, {p_gbps:.0f} GB/s; single step {s_ms * 1e3:.1f} us, {s_gbps:.0f} GB/s")
    workload = f"{dom_work}_fp64_{n}^3"
    roofline = {"bound": "hbm", "achieved": round(k_gbps, 1), "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": round(k_gbps / PEAK_HBM_GBPS, 4),
                "traffic": traffic_record("device.hip", workload),
                "kernel": dom_name, "kernel_us": round(k_ms * 1e3, 2),
                "bytes_per_launch": k_bytes,
                "pair": {"kernel": "k_cheb_pair_lds<double,double,false,false,2,8,4,false,true,0>",
                         "kernel_us": round(p_ms * 1e3, 2), "bytes_per_launch": p_bytes,
                         "achieved": round(p_gbps, 1), "frac": round(p_gbps / PEAK_HBM_GBPS, 4),
                         "traffic": traffic_record("device.hip", f"cheb_pair_fp64_{n}^3")},
                "single_step": {"kernel": "k_stencil<S_CHEBK,double,double,false>",
                                "kernel_us": round(s_ms * 1e3, 2), "bytes_per_launch": s_bytes,
                                "achieved": round(s_gbps, 1)}}
    others = {}
    if not a.no_unfused:
        for fuse, key in ((4, "fp64_four_steps_per_pass"), (1, "fp64_two_steps_per_pass"),
                          (0, "fp64_one_step_per_pass")):
            s64.set_option("fuse", fuse)
            st = solve64()
            others[key] = {"iterations": st["iterations"], "solve_s": round(st["solve_ms"] / 1e3, 4),
                           "hbm_gbps": round(st["model_gbps"], 1)}
            log(f"FP64 with fuse={fuse}: {st['iterations']} iterations, {st['solve_ms']:.1f} ms")
    s64.close()

    out = {"metric": METRIC, "value": round(iters / wall, 3), "unit": "iter/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(wall * 1e3 / a.steps, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{n}^3 unit-cube Poisson, zero Dirichlet, f~U[-1,1) seed "
                                  f"{a.seed}, FP64 Bi-CGSTAB + Chebyshev degree {a.degree}, "
                                  f"analytic interval, tol {a.tol}, x0=0; one step = one solve",
                      "grid": n, "unknowns": N, "precond": "chebyshev", "degree": a.degree,
                      "tol": a.tol},
           "iterations_per_solve": last["iterations"],
           "loop_iter_per_s": round(iters / (loop_ms / 1e3), 3),
           "outside_loop_ms_per_solve": round((wall * 1e3 - loop_ms) / a.steps, 2),
           "hbm_gbps": round(model_bytes / (loop_ms * 1e6), 1),
           "hbm_frac": round(model_bytes / (loop_ms * 1e6) / PEAK_HBM_GBPS, 4),
           "tts_fp64_s": round(median([st["solve_ms"] for st in stats]) / 1e3, 4),
           "tts_fp64_runs": len(stats),
           "relres_true_fp64": last["relres_true"]}
    out.update(others)

    fp64_oracle = golden_x_sha256(f"full_{n}_cheb{a.degree}_fp64") if a.seed == 4 else None
    if fp64_oracle is not None and a.tol == 1e-8:
        out["fp64_x_is_oracle_x"] = sha256_of(x64) == fp64_oracle
    if not a.no_mixed:
        sm = P.Solver(shape, h, stream=stream, precision=P.MIXED)
        xm = torch.zeros_like(x)
        tts = []
        for rep in range(5):
            with torch.cuda.stream(stream):
                xm.zero_()
                st = sm.solve(b, xm, P.PC_CHEBYSHEV, a.degree, a.tol, 5000)
            if st != P.OK:
                raise RuntimeError(f"mixed solve status {st}")
            ms = sm.stats()
            tts.append(ms["solve_ms"] / 1e3)
        torch.cuda.synchronize()
        rel = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
        out.update({"tts_mixed_s": round(median(tts), 4), "tts_mixed_runs": len(tts),
                    "iterations_mixed": ms["iterations"],
                    "mixed_speedup": round(out["tts_fp64_s"] / median(tts), 3),
                    "relres_true_mixed": ms["relres_true"],
                    "mixed_vs_fp64_rel_diff": rel,
                    "hbm_gbps_mixed": round(ms["model_gbps"], 1)})
        log(f"mixed: {ms['iterations']} iterations, {median(tts):.3f} s, rel diff vs FP64 {rel:.2e}")
        sm.close()
        del xm
    if not a.no_extra and n == 512:
        out.update(extra_configs(P, workloads, b, stream, a.degree))
        if "mixed_speedup" in out:
            ms = out["mixed_over_seeds_tol_1e-8"]
            ms["median_speedup_with_seed_4"] = round(median(
                [v["speedup"] for v in ms["seeds"].values()] + [out["mixed_speedup"]]), 3)
    out["roofline"] = roofline
    del b, x, x64
    torch.cuda.empty_cache()
    if not a.no_serve:
        from paper_2503_08935_amd import serving
        log(f"serving stream: {a.serve_requests} requests at {a.serve_rate}/s ...")
        sv = serving.run_stream(n_requests=a.serve_requests, rate=a.serve_rate, iters=a.serve_iters,
                                progress=log)
        log(f"serving: p50 {sv['p50_ms']:.0f} ms, p99 {sv['p99_ms']:.0f} ms, "
            f"{sv['solves_per_s']:.1f} solves/s, utilization {sv['utilization']:.2f}")
        out["p99_solve_ms"] = round(sv["p99_ms"], 1)
        out["serving"] = {k: (float(f"{v:.6g}") if isinstance(v, float) else v)
                          for k, v in sv.items()}
        torch.cuda.empty_cache()
        if not a.no_extra:
            log("serving below saturation: 400 requests at 10/s ...")
            sv = serving.run_stream(n_requests=400, rate=10.0, iters=a.serve_iters, progress=log)
            log(f"serving at 10/s: p50 {sv['p50_ms']:.0f} ms, p99 {sv['p99_ms']:.0f} ms, "
                f"utilization {sv['utilization']:.2f}")
            out["serving_below_saturation"] = {
                k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in sv.items()}
            torch.cuda.empty_cache()
    if not a.no_cpu:
        log("cpu oracle baseline (bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(n, h, a.degree, a.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
