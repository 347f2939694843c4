"""Benchmark of the patchy SL solver on one MI355X.

One step = the whole hot path on one synthetic problem, inputs resident in
HBM: Step 1 coarse solve (hjb_coarse_solve, FP64), Steps 2 and 3.1
(hjb_build_patches, FP64 feedback and colour transport), Steps 3.2 and 4
(hjb_solve_patches, FP32 values, FP64 stopping residual).

Workload: the 2D variable-speed patchy problem, 1025^2 fine / 65^2 coarse
grid on [-1,1]^2, c = 1 + 0.5 sin(2 pi k1 x) sin(2 pi k2 y), 32 controls,
target ball r = 0.1 at a seeded centre split into 16 equal-angle parts,
stopping tolerance 1e-5 (seed 0).

Prints one JSON line (rank 0).  `value` = node-control updates of the value
iteration executed per second over the timed steps (the patch sweeps and the
Step 1 coarse solve; the Step 2 feedback evaluations are listed apart);
beside it the solve time per step, the plain global GPU solve of the same
problem, the roofline of the dominant kernel (the FP32 tiled sweep), the
other seeds, the 3D workload (257^3), a serving run with p50/p99 latency and
the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations of one node-control update (foot point,
# cell and weights, bilinear / trilinear interpolation, Kruzkov map, min).
VALU_OPS_PER_UPDATE = {2: 13, 3: 25}
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes/clk x clock = 39.3e12 /s
PEAK_HBM = 8.0e12


# Sources of the tiled sweep kernel; HBM counters recorded for it count only
# while these files are unchanged.
SWEEP_SOURCES = ("paper_1109_3577_amd/csrc/sweep.hip", "paper_1109_3577_amd/csrc/device_math.h",
                 "paper_1109_3577_amd/csrc/hjb_internal.h")
PMC_SUMMARIES = ("profiles/k_sweep_f32_2d_1025_pmc.md", "profiles/k_sweep_f32_3d_257_pmc.md")


def sweep_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary:
    (FETCH_SIZE x fetch factor + WRITE_SIZE x write factor), the factors being
    what the same counters read for a copy of known size.  None when there is
    no record for this kernel or its sources changed since it was taken."""
    for name in PMC_SUMMARIES:
        path = os.path.join(ROOT, name)
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            for line in fh:
                if line.startswith("pmc: "):
                    rec = json.loads(line[5:])
                    if rec.get("kernel") == kernel and rec.get("source_hash") == sweep_source_hash():
                        return (rec["fetch_kib_per_dispatch"] * 1024.0 * rec["fetch_factor"]
                                + rec["write_kib_per_dispatch"] * 1024.0 * rec["write_factor"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1025)
    ap.add_argument("--ncoarse", type=int, default=65)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-global", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=100)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--no-addons", action="store_true",
                    help="skip the side measurement of the add-ons (dbc data, AO3 cones)")
    ap.add_argument("--ao3-r", type=float, default=4.0, help="AO3 reduction factor r")
    ap.add_argument("--mode", choices=("solve", "solve3d", "batch", "serve", "copy", "paper"),
                    default="solve",
                    help="solve: the 1025^2 patchy problem (default, the headline line); "
                         "solve3d: the 257^3 patchy problem (98 controls, 64 parts); "
                         "batch: many uneven problems in shared rounds; serve: Poisson "
                         "request stream through the continuous-batching server")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the 257^3 block of the default line")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving block of the default line")
    ap.add_argument("--no-seeds", action="store_true",
                    help="skip the other seeds of the 2D workload")
    ap.add_argument("--serve-count", type=int, default=300,
                    help="requests of the serving block of the default line")
    ap.add_argument("--count", type=int, default=0, help="problems (batch) / requests (serve)")
    ap.add_argument("--load", type=float, default=0.7, help="serve: arrival rate / capacity")
    return ap.parse_args()


def bench_copy(args):
    """A plain device-to-device copy of known size, for calibrating the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) of the profiler."""
    import torch
    nbytes = args.count or (256 << 20)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "copies": 3}))


def bench_paper(args):
    """The paper's own tables replayed on the GPU with its dynamics, domains
    and step rule: patchy error E1 (E_inf) against the global solve for
    Eikonal, Fan and Zermelo in 2D (R = 16, N_c = 32, coarse 51^2 and
    101^2), the 3D tests with the add-ons on, and the add-ons table
    (R = 8).  Errors are reported in the Kruzkov variable and in the time
    variable T = -ln(1 - v) where both solutions are finite; the 2D tables
    also from FP64 solves (`fp64`), since FP32 storage of v limits T to
    about 1e-7 e^T where T is large (Zermelo upstream of the target)."""
    import numpy as np
    import torch

    from paper_1109_3577_amd import hjb, problems

    def solve(fine, coarse, opts=None, tol=0.0, fp64=False):
        P, Cp = hjb.Problem(fine, device=True), hjb.Problem(coarse, device=True)
        ch = hjb.hjb_coarse_solve(Cp)
        ph = hjb.hjb_build_patches(P, ch)
        prec, dt = (hjb.HJB_F64, torch.float64) if fp64 else (hjb.HJB_F32, torch.float32)
        v = torch.empty(P.N, dtype=dt, device="cuda")
        st = hjb.hjb_solve_patches(P, ph, prec, v, tol, 0,
                                   opts if opts is not None else hjb.make_opts(time_kernels=True))
        g = torch.empty(P.N, dtype=dt, device="cuda")
        hjb.hjb_solve_global(P, prec, g, tol, 0, None)
        torch.cuda.synchronize()
        return v.double().cpu().numpy(), g.double().cpu().numpy(), st, ph.stats

    def errors(vp, vg):
        e = np.abs(vp - vg)
        fin = (vp < 1.0) & (vg < 1.0)
        et = np.abs(np.log1p(-vp[fin]) - np.log1p(-vg[fin])) if fin.any() else np.zeros(1)
        return {"E1": float(e.mean()), "Einf": float(e.max()),
                "E1_T": float(et.mean()), "Einf_T": float(et.max())}

    gens = {"eikonal": lambda n, fp32: problems.eikonal_paper_2d(n, 32, 16, fp32),
            "fan": lambda n, fp32: problems.fan_2d(n, 32, 16, fp32),
            "zermelo": lambda n, fp32: problems.zermelo_paper_2d(n, 32, 16, fp32)}
    sides = [101, 201, 401, 801]
    out = {"mode": "paper", "tables": {}}
    for name, gen in gens.items():
        tab = {}
        for nc in (51, 101):
            coarse = gen(nc, False)
            for n in sides:
                if n < nc:
                    continue
                vp, vg, st, bst = solve(gen(n, True), coarse)
                wp, wg, _, _ = solve(gen(n, False), coarse, fp64=True)
                tab[f"{nc}->{n}"] = {**errors(vp, vg), "fp64": errors(wp, wg),
                                     "solve_ms": st["ms_wall"], "build_ms": bst["ms_wall"]}
                print(f"[paper] {name} {nc}->{n} {tab[f'{nc}->{n}']}", file=sys.stderr, flush=True)
        out["tables"][f"patchy_error_{name}"] = tab

    # add-ons table: R = 8, N_c = 32, controls reduced by factor 4 (r = 4)
    gens8 = {"eikonal": lambda n, fp32: problems.eikonal_paper_2d(n, 32, 8, fp32),
             "fan": lambda n, fp32: problems.fan_2d(n, 32, 8, fp32),
             "zermelo": lambda n, fp32: problems.zermelo_paper_2d(n, 32, 8, fp32)}
    addons = {}
    for name, gen in gens8.items():
        coarse = gen(101, False)
        for n in (201, 401, 801):
            P, Cp = hjb.Problem(gen(n, True), device=True), hjb.Problem(coarse, device=True)
            ch = hjb.hjb_coarse_solve(Cp)
            ph = hjb.hjb_build_patches(P, ch)
            v = torch.empty(P.N, dtype=torch.float32, device="cuda")
            row = {}
            tabulated = name == "zermelo"
            variants = {"basic": {}, "AO1": {"start_u0": 1}, "AO2": {"order_window": 6.0}}
            if not tabulated:
                variants["AO3"] = {"control_cone": 4.0}
            variants["all"] = {**variants["AO1"], **variants["AO2"],
                               **({} if tabulated else variants["AO3"]),
                               "patch_bc": hjb.HJB_BC_DIRICHLET}
            for vname, kw in variants.items():
                o = hjb.make_opts(time_kernels=True, **kw)
                runs = [hjb.hjb_solve_patches(P, ph, hjb.HJB_F32, v, 1e-6, 0, o) for _ in range(3)]
                row[vname] = min(r["ms_kernel"] for r in runs)
            addons[f"101->{n}"] = addons.get(f"101->{n}", {})
            addons[f"101->{n}"][name] = row
            print(f"[paper] add-ons {name} 101->{n} {row}", file=sys.stderr, flush=True)
    out["tables"]["addons_kernel_ms"] = addons

    # 3D tests with the add-ons on (Eikonal and Fan: cones r = 4; Brockett:
    # no cones), R = 8
    gens3 = {"eikonal3d": lambda n, fp32: problems.eikonal_paper_3d(n, 189, 8, fp32),
             "fan3d": lambda n, fp32: problems.fan_3d(n, 189, 8, fp32),
             "brockett3d": lambda n, fp32: problems.brockett_3d(n, 8, fp32)}
    t3 = {}
    for name, gen in gens3.items():
        coarse = gen(51, False)
        for n in (101,) + ((201,) if args.count >= 201 else ()):
            kw = {"patch_bc": hjb.HJB_BC_DIRICHLET, "order_window": 2.5, "inner_sweeps": 4}
            if name != "brockett3d":
                kw["control_cone"] = 4.0
            vp, vg, st, bst = solve(gen(n, True), coarse, hjb.make_opts(time_kernels=True, **kw),
                                    1e-6)
            t3[f"51->{n}"] = t3.get(f"51->{n}", {})
            t3[f"51->{n}"][name] = {**errors(vp, vg), "solve_ms": st["ms_wall"],
                                    "build_ms": bst["ms_wall"], "kernel_ms": st["ms_kernel"]}
            print(f"[paper] 3D {name} 51->{n} {t3[f'51->{n}'][name]}", file=sys.stderr, flush=True)
    out["tables"]["3d"] = t3
    print(json.dumps(out))


def bench_batch(args):
    """Uneven 2D problems (grid side 65..769, 16..64 controls, 4..32 parts,
    seeded-sign drift) solved together, against the same problems solved one
    after the other with the plain global GPU solve."""
    import numpy as np
    import torch

    from paper_1109_3577_amd import autotune, hjb, problems

    count = args.count or 512
    t = time.perf_counter()
    probs = problems.config4(count)
    print(f"[bench] generated {count} problems in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    fines = [hjb.Problem(f, device=True) for f, _ in probs]
    coarses = [hjb.Problem(c, device=True) for _, c in probs]
    # a sample large enough that its rounds are throughput-bound like the
    # full batch's (small samples favour small tiles)
    choice, _ = autotune.tune_batch(fines, coarses, hjb.HJB_F32, args.tol, sample=64)
    opts = autotune.opts_from(choice)
    # the first preparation also fills the library's device allocation pool
    # (hipMalloc of the colour fields); the second is the steady state
    t = time.perf_counter()
    b = hjb.hjb_batch_create(fines, coarses, hjb.HJB_F32, args.tol, 0, opts)
    torch.cuda.synchronize()
    t_prep_cold = time.perf_counter() - t
    b.free()
    t = time.perf_counter()
    b = hjb.hjb_batch_create(fines, coarses, hjb.HJB_F32, args.tol, 0, opts)
    torch.cuda.synchronize()
    t_prep = time.perf_counter() - t
    t = time.perf_counter()
    st = b.run()
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t
    nodes = sum(p.N for p in fines)
    # the same batch in the other launch forms: rounds replayed as a
    # hipGraph, and one persistent launch per dimension draining a device
    # queue of items
    forms = {}
    fs = torch.cuda.Stream()  # graph capture needs a stream other than the null stream
    for name, kw in (("graph", {"use_graph": True}), ("async", {"schedule": hjb.HJB_SCHED_ASYNC})):
        o = autotune.opts_from(choice, **kw)
        bf = hjb.hjb_batch_create(fines, coarses, hjb.HJB_F32, args.tol, 0, o, stream=fs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sf = bf.run()
        torch.cuda.synchronize()
        forms[name] = {"sweep_s": time.perf_counter() - t, "updates": sf["updates"],
                       "rounds": sf["rounds"]}
        bf.free()
        print(f"[bench] batch {name}: {forms[name]['sweep_s']:.3f} s", file=sys.stderr, flush=True)
    # a few problems solved alone: at tol > 0 the stopping point depends on
    # the schedule, so the batch may differ from them within the tolerance
    sampled = []
    for i in (0, count // 3, (2 * count) // 3, count - 1):
        got, _ = hjb.hjb_batch_result(b, i)
        ch = hjb.hjb_coarse_solve(coarses[i])
        ph = hjb.hjb_build_patches(fines[i], ch)
        v = torch.empty(fines[i].N, dtype=torch.float32, device="cuda")
        hjb.hjb_solve_patches(fines[i], ph, hjb.HJB_F32, v, args.tol, 0, opts)
        sampled.append(float(np.abs(got.astype(np.float64) - v.cpu().double().numpy()).max()))
        ph.free()
        ch.free()
    # baseline: the plain global solve of every problem, one after the other
    t = time.perf_counter()
    gupd = 0
    for f in fines:
        v = torch.empty(f.N, dtype=torch.float32, device="cuda")
        g = hjb.hjb_solve_global(f, hjb.HJB_F32, v, args.tol, 0,
                                 hjb.make_opts(schedule=hjb.HJB_SCHED_JACOBI, rounds_per_poll=8))
        gupd += g["updates"]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    print(json.dumps({
        "metric": "batched patchy solve: node-control updates/s and wall time vs sequential "
                  "plain solves", "mode": "batch", "problems": count, "nodes": nodes,
        "autotuned": choice, "prepare_s": t_prep, "prepare_first_call_s": t_prep_cold,
        "sweep_s": t_run,
        "batch_total_s": t_prep + t_run, "sampled_max_diff_vs_alone": max(sampled),
        "sweep_forms": {"rounds": {"sweep_s": t_run, "updates": st["updates"],
                                   "rounds": st["rounds"]}, **forms},
        "updates": st["updates"],
        "updates_per_s": st["updates"] / t_run, "items": st["items"], "rounds": st["rounds"],
        "sequential_plain_global_s": t_seq, "sequential_plain_updates": gupd,
        "speedup_vs_sequential_plain": t_seq / (t_prep + t_run)}))


def pooled_requests(specs, pool, window=96):
    """Builds the requests of `specs` on a process pool, in order, at most
    `window` of them ahead of the consumer."""
    from collections import deque

    from paper_1109_3577_amd import problems
    q = deque()
    for spec in specs:
        q.append(pool.submit(problems.serving_request, spec))
        if len(q) >= window:
            yield q.popleft().result()
    while q:
        yield q.popleft().result()


def bench_serve_stream(args, pool):
    """The serving workload at its stated length (e.g. 10,000 requests):
    the closed-loop capacity is measured on the first 300 requests, then the
    whole Poisson stream at load x capacity is served with the requests
    built on the fly by a pool of host processes (the arrays of 10,000
    requests would not fit host memory at once)."""
    import torch

    from paper_1109_3577_amd import problems, serve
    torch.cuda.set_device(0)
    budget = int(0.8 * torch.cuda.mem_get_info()[0])
    sample = list(pooled_requests(problems.serving_specs(300, 1.0, seed=0), pool))
    cap = serve.run(sample, budget, tol=args.tol, closed_loop=True)
    del sample
    rate = args.load * cap["requests_per_s"]
    print(f"[bench] capacity {cap['requests_per_s']:.1f} requests/s; serving {args.count} requests "
          f"at {rate:.1f}/s", file=sys.stderr, flush=True)
    specs = list(problems.serving_specs(args.count, rate, seed=0))
    n3 = sum(1 for s in specs if s[2] == 3)
    res = serve.run_stream(pooled_requests(specs, pool), budget, tol=args.tol,
                           progress_every=500)
    print(json.dumps({
        "metric": "serving: p50/p99 latency and node-control updates/s at a fixed Poisson rate",
        "mode": "serve", "requests": args.count, "requests_3d": n3,
        "capacity_requests_per_s": cap["requests_per_s"], "capacity_sample": 300,
        "load": args.load, "arrival_rate_per_s": rate, **res}))


def bench_serve(args):
    """Poisson stream of solve requests through the continuous-batching
    server: 80% 2D (side 129..1025; half eikonal with 16 parts, half the
    batched generator), 20% 3D (side 65..193, the 3D generator)."""
    import numpy as np
    import torch

    from paper_1109_3577_amd import problems, serve

    count = args.count or 300
    t = time.perf_counter()
    reqs = []
    for r in problems.serving_stream(count, 1.0, seed=0):
        reqs.append(r)
        if len(reqs) % 25 == 0:
            print(f"[bench] generated {len(reqs)}/{count} requests", file=sys.stderr, flush=True)
    print(f"[bench] generated {count} requests in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    budget = int(0.8 * torch.cuda.mem_get_info()[0])
    # capacity: every request submitted at t = 0 (closed loop)
    cap = serve.run(reqs, budget, tol=args.tol, closed_loop=True, verbose=True)
    print(f"[bench] capacity {cap['requests_per_s']:.2f} requests/s", file=sys.stderr, flush=True)
    n3 = sum(1 for r in reqs if r.fine.dim == 3)
    loads = sorted({0.3, 0.5, float(args.load)})
    runs = []
    for load in loads:
        rate = load * cap["requests_per_s"]
        # re-time the same requests on a Poisson clock at this rate
        rng = np.random.default_rng(1)
        tt = 0.0
        for r in reqs:
            tt += float(rng.exponential(1.0 / rate))
            r.arrival_s = tt
        res = serve.run(reqs, budget, tol=args.tol, verbose=True)
        runs.append({"load": load, "arrival_rate_per_s": rate, "p50_ms": res["p50_ms"],
                     "p99_ms": res["p99_ms"], "mean_ms": res["mean_ms"],
                     "requests_per_s": res["requests_per_s"],
                     "updates_per_s": res["updates_per_s"], "wall_s": res["wall_s"]})
        print(f"[bench] load {load:.2f}: p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    main_run = [r for r in runs if r["load"] == float(args.load)][0]
    print(json.dumps({
        "metric": "serving: p50/p99 latency and node-control updates/s at a fixed Poisson rate",
        "mode": "serve", "requests": count, "requests_3d": n3,
        "capacity_requests_per_s": cap["requests_per_s"],
        "capacity_updates_per_s": cap["updates_per_s"], **main_run, "loads": runs}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; the patches would be "
                          "sharded across GPUs with no exchange during the solve, which is "
                          "not implemented here", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.mode == "serve" and args.count > 1000:
        # the request builders run in processes started before this one
        # touches the GPU
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        workers = max(2, min(14, len(os.sched_getaffinity(0)) - 2))
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as pool:
            return bench_serve_stream(args, pool)
    import numpy as np
    import torch

    from paper_1109_3577_amd import hjb, problems

    torch.cuda.set_device(0)
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "serve":
        return bench_serve(args)
    if args.mode == "copy":
        return bench_copy(args)
    if args.mode == "paper":
        return bench_paper(args)
    stream = torch.cuda.Stream()
    dim = 3 if args.mode == "solve3d" else 2
    if dim == 2:
        fine_src, coarse_src = problems.config2(args.seed, args.n, args.ncoarse)
        label = (f"2D variable-speed patchy solve {args.n}^2 / {args.ncoarse}^2, 32 controls, "
                 f"16 parts, seed {args.seed}, tol {args.tol:g}")
        cfg = {"n": args.n, "n_coarse": args.ncoarse, "controls": 32, "parts": 16}
    else:
        fine_src, coarse_src = problems.config3(args.seed)
        label = (f"3D variable-speed patchy solve 257^3 / 33^3, 98 controls, 64 parts, "
                 f"seed {args.seed}, tol {args.tol:g}")
        cfg = {"n": 257, "n_coarse": 33, "controls": 98, "parts": 64}
    print(f"[bench] workload {label}", file=sys.stderr, flush=True)
    r = run_patchy(hjb, fine_src, coarse_src, args.steps, args.warmup, args.tol, stream,
                   graph=bool(args.graph))
    out = {
        "metric": "node-control updates/s and solve time, patchy vs global at ||dv||inf<=1e-5; p99",
        "value": r["value"],
        "unit": "node-control updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (values), f64 (coarse solve, feedback, colours, residual)",
        "data": "synthetic (seeded generator)",
        "config": {"workload": label, **cfg, "tol": args.tol},
        "value_counts": "node-control updates of the value iteration: patch sweeps (FP32) and "
                        "the Step 1 coarse solve (FP64); the Step 2 feedback evaluations are "
                        "listed in updates_per_step and not counted",
        "step_ms": r["step_ms"],
        "updates_per_step": r["updates_per_step"],
        "build": r["build"],
    }
    if "roofline" in r:
        out["roofline"] = r["roofline"]
    fine, coarse, v = r["fine"], r["coarse"], r["v"]
    N = fine.N

    # Plain global GPU solve of the same fine problem (full-grid Jacobi,
    # FP32, same tolerance) and the tiled global schedule.
    vt = None
    if not args.no_global:
        g = run_global(hjb, fine, args.tol, stream)
        vt = g.pop("v_tiled")
        vg = g.pop("v_jacobi")
        out["global"] = {**g, "speedup_patchy_step_vs_jacobi": g["jacobi_ms"] / r["ms_per_step"],
                         "speedup_patch_solve_vs_jacobi": g["jacobi_ms"] / r["step_ms"]["solve_patches"],
                         "speedup_patchy_step_vs_tiled": g["tiled_ms"] / r["ms_per_step"],
                         **patchy_errors(v, vg)}
        print(f"[bench] global Jacobi {g['jacobi_ms']:.1f} ms, tiled {g['tiled_ms']:.1f} ms; "
              f"patchy E_inf {out['global']['patchy_error_Einf']:.3g}, cut-off nodes "
              f"{out['global']['cutoff_nodes']}", file=sys.stderr, flush=True)

    # The paper's add-ons beside the basic patch solve, on the same patches:
    # the Dirichlet patch data U^(0) (eq. dbc), AO3 (control cones of
    # half-angle pi/r around the Step 2 feedback) and both; kernel time of
    # each and its error against the global solution (when measured).
    if not args.no_addons:
        out["addons"] = run_addons(hjb, fine, coarse, dim, args, stream, vt)

    # The other seeds of the 2D workload (same shapes, other speed fields
    # and target centres).
    if dim == 2 and not args.no_seeds and args.n == 1025:
        seeds = {}
        for sd in (1, 2):
            f2, c2 = problems.config2(sd, args.n, args.ncoarse)
            rs = run_patchy(hjb, f2, c2, 3, 1, args.tol, stream)
            seeds[str(sd)] = {"ms_per_step": rs["ms_per_step"], "value": rs["value"],
                              "step_ms": rs["step_ms"],
                              "roofline_frac": rs.get("roofline", {}).get("frac")}
            print(f"[bench] seed {sd}: {rs['ms_per_step']:.2f} ms per step", file=sys.stderr,
                  flush=True)
        out["seeds"] = seeds

    # The 3D workload: 257^3 / 33^3, 98 controls, 64 parts.
    if dim == 2 and not args.no_c3:
        f3, c3 = problems.config3(args.seed)
        r3 = run_patchy(hjb, f3, c3, 2, 1, args.tol, stream)
        g3 = run_global(hjb, r3["fine"], args.tol, stream)
        e3 = patchy_errors(r3["v"], g3.pop("v_jacobi"))
        g3.pop("v_tiled")
        out["c3"] = {"workload": "3D variable-speed patchy solve 257^3 / 33^3, 98 controls, "
                                 f"64 parts, seed {args.seed}, tol {args.tol:g}",
                     "value": r3["value"], "ms_per_step": r3["ms_per_step"],
                     "step_ms": r3["step_ms"], "updates_per_step": r3["updates_per_step"],
                     "roofline": r3.get("roofline"), "global": g3,
                     "speedup_patchy_step_vs_jacobi": g3["jacobi_ms"] / r3["ms_per_step"],
                     "speedup_patch_solve_vs_jacobi":
                         g3["jacobi_ms"] / r3["step_ms"]["solve_patches"],
                     "speedup_patchy_step_vs_tiled": g3["tiled_ms"] / r3["ms_per_step"], **e3}
        print(f"[bench] 3D: {r3['ms_per_step']:.1f} ms per step, Jacobi {g3['jacobi_ms']:.1f} ms, "
              f"tiled {g3['tiled_ms']:.1f} ms", file=sys.stderr, flush=True)
        del r3, f3, c3

    # Serving: a Poisson stream at a fixed rate, 0.7 x the closed-loop
    # capacity measured on the same requests in the same run.
    if dim == 2 and not args.no_serve:
        out["serve"] = run_serve(args.serve_count, args.tol, args.load)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(hjb, args, stream)
    print(json.dumps(out))


def run_patchy(hjb, fine_src, coarse_src, steps, warmup, tol, stream, graph=False):
    """Timed patchy steps (coarse solve, build, patch solve) of one problem;
    node-control updates counted as in the header of this file."""
    import numpy as np
    import torch
    fine = hjb.Problem(fine_src, device=True)
    coarse = hjb.Problem(coarse_src, device=True)
    dim = fine_src.dim
    v = torch.empty(fine.N, dtype=torch.float32, device="cuda")
    opts = hjb.make_opts(time_kernels=not graph, use_graph=graph)

    def step():
        ch = hjb.hjb_coarse_solve(coarse, 0.0, 0, stream)
        ph = hjb.hjb_build_patches(fine, ch, stream)
        ch.free()
        st = hjb.hjb_solve_patches(fine, ph, hjb.HJB_F32, v, tol, 0, opts, stream)
        ph_stats = ph.stats
        ph.free()
        return st, ph_stats

    with torch.cuda.stream(stream):
        for i in range(warmup):
            step()
            print(f"[bench] warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = [step() for _ in range(steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    elapsed = t1 - t0
    print(f"[bench] {steps} timed steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    solve_upd = sum(s[0]["updates"] for s in sts)
    feedback_upd = sum(s[1]["updates"] for s in sts)
    kernel_ms = sum(s[0]["ms_kernel"] for s in sts)
    launches = sum(s[0]["kernel_launches"] for s in sts)
    solve_ms = float(np.mean([s[0]["ms_wall"] for s in sts]))
    build_ms = float(np.mean([s[1]["ms_wall"] for s in sts]))
    trace_ms = float(np.mean([s[1]["ms_trace"] for s in sts]))
    # coarse solve work: the same FP64 solve once more, with statistics
    with torch.cuda.stream(stream):
        vc = torch.empty(coarse.N, dtype=torch.float64, device="cuda")
        cst = hjb.hjb_solve_global(coarse, hjb.HJB_F64, vc, 0.0, 0, None, stream)
    coarse_upd = cst["updates"] * steps
    ms_per_step = elapsed / steps * 1e3
    out = {"fine": fine, "coarse": coarse, "v": v,
           "value": (solve_upd + coarse_upd) / elapsed, "ms_per_step": ms_per_step,
           "step_ms": {"solve_patches": solve_ms, "build_patches": build_ms, "trace": trace_ms,
                       "coarse_and_other": ms_per_step - solve_ms - build_ms},
           "updates_per_step": {"patch_sweeps": solve_upd // steps,
                                "coarse": coarse_upd // steps,
                                "feedback_evaluations": feedback_upd // steps},
           "build": {"unreached": sts[0][1]["unreached"], "detached": sts[0][1]["detached"],
                     "trace_rounds": sts[0][1]["rounds"]}}
    # Dominant kernel: the FP32 tiled sweep, HIP events around every block of
    # launches on the solve's stream.
    if launches:
        ops = VALU_OPS_PER_UPDATE[dim] * solve_upd
        achieved = ops / (kernel_ms * 1e-3)
        s0 = sts[0][0]
        kernel = "k_sweep<float, %d, %d, %d, %d, %d>" % (dim, *s0["tile"], s0["threads"])
        avg_s = kernel_ms * 1e-3 / launches
        traffic = recorded_traffic(kernel)
        out["roofline"] = {
            "bound": "alu", "kernel": kernel,
            "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
            "unit": "TOP/s (VALU lane-ops)", "frac": achieved / PEAK_VALU_LANE_OPS,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch",
            "hbm_gbps": None if traffic is None else traffic / avg_s / 1e9,
            "avg_launch_us": avg_s * 1e6, "launches": launches,
            "ops_per_update": VALU_OPS_PER_UPDATE[dim],
            "updates_per_launch": solve_upd / launches,
            "inner_sweeps": s0["inner_sweeps"],
        }
    return out


def run_global(hjb, fine, tol, stream):
    """The plain global GPU solve (full-grid Jacobi, FP32) and the tiled
    global schedule of the same problem."""
    import torch
    N = fine.N
    with torch.cuda.stream(stream):
        vg = torch.empty(N, dtype=torch.float32, device="cuda")
        gj = hjb.hjb_solve_global(fine, hjb.HJB_F32, vg, tol, 0,
                                  hjb.make_opts(schedule=hjb.HJB_SCHED_JACOBI, rounds_per_poll=8),
                                  stream)
        vt = torch.empty(N, dtype=torch.float32, device="cuda")
        gt = hjb.hjb_solve_global(fine, hjb.HJB_F32, vt, tol, 0, None, stream)
        torch.cuda.synchronize()
    return {"jacobi_ms": gj["ms_wall"], "jacobi_sweeps": gj["sweeps"],
            "jacobi_updates": gj["updates"], "tiled_ms": gt["ms_wall"],
            "tiled_updates": gt["updates"], "v_jacobi": vg, "v_tiled": vt}


def patchy_errors(v, vg):
    """Patchy error against the global solve in the Kruzkov variable, and
    the nodes the patchy solve leaves at v = 1 (T = +inf) where the global
    solve reaches the target."""
    E = (v.double() - vg.double()).abs()
    cut = int(((v == 1.0) & (vg < 1.0)).sum().item())
    return {"patchy_error_E1": float(E.mean()), "patchy_error_Einf": float(E.max()),
            "cutoff_nodes": cut}


def run_addons(hjb, fine, coarse, dim, args, stream, vt):
    import torch
    N = fine.N
    # AO2 window (time steps per round) and in-tile sweeps that suit it
    ao2 = {"order_window": 6.0} if dim == 2 else {"order_window": 2.5, "inner_sweeps": 4}
    dbc = {"patch_bc": hjb.HJB_BC_DIRICHLET}
    ao3 = {"control_cone": args.ao3_r}
    variants = {"basic": {}, "dbc": dbc, "ao2": ao2, "ao3": ao3,
                "dbc_ao2_ao3": {**dbc, **ao2, **ao3}}
    if args.tol >= 1e-7:  # AO1 iterates v <- F(v) and needs a tolerance
        variants["ao1"] = {"start_u0": 1}
    res = {}
    with torch.cuda.stream(stream):
        ch = hjb.hjb_coarse_solve(coarse, 0.0, 0, stream)
        ph = hjb.hjb_build_patches(fine, ch, stream)
        va = torch.empty(N, dtype=torch.float32, device="cuda")
        for name, kw in variants.items():
            o = hjb.make_opts(time_kernels=True, **kw)
            runs = [hjb.hjb_solve_patches(fine, ph, hjb.HJB_F32, va, args.tol, 0, o, stream)
                    for _ in range(3)]
            torch.cuda.synchronize()
            r = {"opts": {k: float(v) for k, v in kw.items()},
                 "kernel_ms": min(x["ms_kernel"] for x in runs),
                 "wall_ms": min(x["ms_wall"] for x in runs),
                 "updates": runs[0]["updates"], "node_updates": runs[0]["node_updates"],
                 "rounds": runs[0]["rounds"],
                 "controls_per_node_update": runs[0]["updates"] / max(1, runs[0]["node_updates"]),
                 "inner_sweeps": runs[0]["inner_sweeps"]}
            if vt is not None:
                e = patchy_errors(va, vt)
                r["E1_vs_global"] = e["patchy_error_E1"]
                r["Einf_vs_global"] = e["patchy_error_Einf"]
                r["cutoff_nodes"] = e["cutoff_nodes"]
            res[name] = r
        ph.free()
        ch.free()
    for name in [k for k in res if k != "basic"]:
        res[name]["speedup_kernel_vs_basic"] = res["basic"]["kernel_ms"] / res[name]["kernel_ms"]
    print(f"[bench] add-ons (kernel ms): " + ", ".join(
        f"{k} {v['kernel_ms']:.2f}" for k, v in res.items()), file=sys.stderr, flush=True)
    return {"r": args.ao3_r, **res}


def run_serve(count, tol, load):
    """The serving block of the default line: `count` requests of the
    serving mix, the closed-loop capacity, then one Poisson run at
    load x capacity."""
    import numpy as np
    import torch

    from paper_1109_3577_amd import problems, serve
    t = time.perf_counter()
    reqs = []
    for r in problems.serving_stream(count, 1.0, seed=0):
        reqs.append(r)
        if len(reqs) % 50 == 0:
            print(f"[bench] serve: generated {len(reqs)}/{count} requests", file=sys.stderr,
                  flush=True)
    gen_s = time.perf_counter() - t
    budget = int(0.8 * torch.cuda.mem_get_info()[0])
    cap = serve.run(reqs, budget, tol=tol, closed_loop=True)
    rate = load * cap["requests_per_s"]
    rng = np.random.default_rng(1)
    tt = 0.0
    for r in reqs:
        tt += float(rng.exponential(1.0 / rate))
        r.arrival_s = tt
    res = serve.run(reqs, budget, tol=tol)
    print(f"[bench] serve: capacity {cap['requests_per_s']:.1f} requests/s; load {load}: "
          f"p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    return {"requests": count, "requests_3d": sum(1 for r in reqs if r.fine.dim == 3),
            "generate_s": gen_s, "capacity_requests_per_s": cap["requests_per_s"],
            "load": load, "arrival_rate_per_s": rate, "p50_ms": res["p50_ms"],
            "p99_ms": res["p99_ms"], "mean_ms": res["mean_ms"],
            "requests_per_s": res["requests_per_s"], "updates_per_s": res["updates_per_s"],
            "wall_s": res["wall_s"]}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(hjb, args, stream):
    """The CPU oracle on a bounded sample of the same workload: the whole
    patchy pipeline (Step 1 coarse solve, Steps 2-3.1 build, Steps 3.2-4
    patch solves, same tolerance) of the 2D variable-speed generator at
    257^2 / 17^2, timed per step on all host cores and on one core; the GPU
    pipeline on the same sample beside it."""
    import torch

    from oracle import oracle as O
    from paper_1109_3577_amd import problems
    O.build(force=False)
    n = 257
    f, c = problems.config2(args.seed, n, problems.coarse_size_2d(n))

    def oracle_pipeline():
        t0 = time.perf_counter()
        vc, cst = O.solve_global(c)
        t1 = time.perf_counter()
        u0 = O.prolong(c, vc, f)
        fb = O.feedback(f, u0)
        lab = O.labels(f, fb)
        t2 = time.perf_counter()
        _, st = O.solve_patches(f, lab, args.tol)
        t3 = time.perf_counter()
        upd = cst["updates"] + st["updates"]
        return {"coarse_ms": (t1 - t0) * 1e3, "build_ms": (t2 - t1) * 1e3,
                "solve_ms": (t3 - t2) * 1e3, "total_ms": (t3 - t0) * 1e3,
                "updates": upd, "updates_per_s": upd / (t3 - t0)}

    threads = O.num_threads()
    allc = oracle_pipeline()
    O.set_threads(1)
    one = oracle_pipeline()
    O.set_threads(threads)
    g = run_patchy(hjb, f, c, 5, 2, args.tol, stream)
    return {"value": allc["updates_per_s"], "unit": "node-control updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the oracle's patchy pipeline (coarse solve, build, patch solves, tol "
                      f"{args.tol:g}) on the 2D variable-speed generator at {n}^2 / 17^2, seed "
                      f"{args.seed}: {allc['updates']:.3g} updates in "
                      f"{allc['total_ms'] / 1e3:.1f} s on {threads} threads",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "per_step_all_cores_ms": allc, "per_step_1_core_ms": one,
            "gpu_same_sample": {"ms_per_step": g["ms_per_step"], "step_ms": g["step_ms"],
                                "value": g["value"]}}


if __name__ == "__main__":
    main()
