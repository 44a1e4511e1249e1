#!/usr/bin/env python3
"""Benchmark: time to a 1e-8 relative residual of the asynchronous vs the
synchronous restricted additive Schwarz solver on one MI355X.

Default workload (one step = one full solve, setup excluded as in the paper's
timings): 2-D 5-point Poisson on a 1024 x 1024 grid (1,048,576 unknowns),
b ~ U[0,1] (seed 1), regular 8 x 8 boxes (64 subdomains), overlap 4, local
solve = 10 CG iterations in float64, tolerance 1e-8.  The timed steps run the
asynchronous (barrier-free persistent) solver; the synchronous variant is
timed the same way beside it.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 residual async vs sync RAS; sweep HBM GB/s vs peak; solves/s + p99"
HBM_PEAK_GBPS = 8000.0
# workloads whose working set fits the 256 MB Infinity Cache (MALL)
MALL_RESIDENT = {"poisson2d_1024_8x8", "laplace3d_128_rcb256", "poisson2d_64_strips4"}

WORKLOADS = {
    # name: (ras_inputs config, local kind, storage, cg iters, partition spec)
    "poisson2d_1024_8x8": ("poisson2d_1024_8x8", "cg", "fp64", 10),
    "laplace3d_128_rcb256": ("laplace3d_128_rcb256", "cg", "fp32", 8),
    "diffusion2d_2048_16x16_fp64": ("diffusion2d_2048_16x16", "chol", "fp64", 0),
    "diffusion2d_2048_16x16_fp32": ("diffusion2d_2048_16x16", "chol", "fp32", 0),
    "diffusion2d_2048_16x16_fp16": ("diffusion2d_2048_16x16", "chol", "fp16", 0),
    "diffusion2d_2048_16x16_sparse_fp64": ("diffusion2d_2048_16x16", "chol_sparse", "fp64", 0),
    "diffusion2d_2048_16x16_sparse_fp32": ("diffusion2d_2048_16x16", "chol_sparse", "fp32", 0),
    "poisson2d_512_strips64_sparse_fp64": ("poisson2d_512_strips64", "chol_sparse", "fp64", 0),
    "poisson2d_512_strips64_fp64": ("poisson2d_512_strips64", "chol", "fp64", 0),
    "poisson2d_64_strips4": ("poisson2d_64_strips4", "chol", "fp64", 0),
    "serving": (None, None, None, 0),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson2d_1024_8x8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sync", action="store_true", help="skip the synchronous comparison (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 2 GiB device copy (hardware-counter calibration)")
    ap.add_argument("--sweeps", type=int, default=0,
                    help="fixed-sweep throughput mode: time N sweeps (synchronous) and N local solves per "
                         "subdomain (asynchronous) instead of solving to the tolerance; value = sweep GB/s")
    ap.add_argument("--no-slab-legs", action="store_true",
                    help="skip the fixed-sweep legs of the 2048^2 diffusion workload in the default run")
    ap.add_argument("--serve-count", type=int, default=200, help="systems in the serving stream")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-local2d", default="chol_sparse", choices=("chol", "chol_sparse"),
                    help="exact local solver of the stream's 2-D systems (3-D systems use CG-8)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2003_05361_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def subdomain_shapes(A, part_kind, part_arg, gamma, kind="cg"):
    """(n_p, owned_p, K_p, w_p[, nnz(L_p)]) per subdomain from the library's own host setup."""
    import paper_2003_05361_amd as ras
    from paper_2003_05361_amd.perfmodel import subdomain_shapes as shapes_of

    sparse = kind == "chol_sparse"
    loc = ras.local("chol_sparse", "fp64") if sparse else ras.local("cg", "fp64", 1)
    plan = ras.Plan(A, part_spec(ras, A, part_kind, part_arg), gamma, loc)
    shapes = shapes_of(plan, A.indptr, sparse)
    plan.close()
    return shapes


def part_spec(ras, A, kind, arg):
    if kind == "rcb":
        P, seed, jit = arg
        return ras.partition("rcb", P, grid=A.grid, seed=seed, jitter=jit)
    return ras.partition(kind, arg, grid=A.grid)


def host_cpu() -> dict:
    """Host CPU model and core count (lscpu, os.cpu_count)."""
    import subprocess

    model = None
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "os_cpu_count": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(A, b, part_kind, part_arg, gamma, kind, storage, k, gpu_sync_sweeps, budget=10.0):
    """The oracle (plain FP64 CPU synchronous RAS), timed on a bounded sample of
    sweeps on this host -- single-threaded, then with the local solves of each sweep
    on a thread pool over all usable cores (inner BLAS threads 1) -- and extrapolated
    to the GPU's synchronous sweep count."""
    import concurrent.futures as cf

    from threadpoolctl import threadpool_limits

    from oracle import partition as opart
    from oracle import schwarz

    if part_kind == "regular_1d":
        owner = opart.regular_1d(A.n, part_arg)
    elif part_kind == "rcb":
        owner = opart.rcb(A.coords(), *part_arg)
    else:
        owner = opart.regular_grid(A.grid, part_arg)
    cpu = host_cpu()
    # at most 16 workers: the host share of one GPU on the measurement machines
    workers = max(1, min(16, cpu["affinity"] or os.cpu_count() or 1))
    legs = {}
    with threadpool_limits(1):
        # the sparse factor solves the same local systems exactly: the oracle's exact local solve
        orc = schwarz.RAS(A, owner, gamma, "chol" if kind == "chol_sparse" else kind, storage, k)
        for label, nw in (("single_core", 1), ("all_cores", workers)):
            pool = cf.ThreadPoolExecutor(nw) if nw > 1 else None
            # calibrate on two sweeps (the first one of a pool also starts its threads)
            t0 = time.perf_counter()
            orc.sync(b, 0.0, 2, pool=pool)
            t1 = (time.perf_counter() - t0) / 2
            sweeps = max(1, min(int(budget / max(t1, 1e-6)), 2000))
            t0 = time.perf_counter()
            orc.sync(b, 0.0, sweeps, pool=pool)
            dt = time.perf_counter() - t0
            if pool is not None:
                pool.shutdown()
            legs[label] = {"threads": nw, "sweeps": sweeps, "seconds": dt, "ms_per_sweep": 1e3 * dt / sweeps,
                           "extrapolated_s": dt / sweeps * gpu_sync_sweeps}
    best = min(legs.values(), key=lambda v: v["ms_per_sweep"])
    return {
        "value": best["extrapolated_s"],
        "unit": "s (extrapolated time-to-tolerance)",
        "cores": best["threads"],
        "kind": "oracle",
        "sample": f"{best['sweeps']} synchronous FP64 sweeps of the same workload in {best['seconds']:.2f} s on "
                  f"{best['threads']} host threads ({best['ms_per_sweep']:.1f} ms/sweep; local solves of a sweep "
                  f"on a thread pool, BLAS threads 1), scaled by the GPU synchronous sweep count {gpu_sync_sweeps}",
        "legs": legs,
        "host_cpu": cpu,
    }


def traffic_from_profiles(workload: str, algo_bytes_per_launch: float):
    """HBM bytes per launch derived from the committed hardware-counter summary
    (copy-calibrated FETCH_SIZE + WRITE_SIZE over the streaming-model bytes of the
    profiled dispatch, times this run's model bytes), if it was taken on the current
    kernel source; else None.  Returns (bytes, source description)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_source_hash():
        return None, None
    ratio = t["counter_bytes_per_dispatch"] / t["algorithmic_bytes_per_dispatch"]
    return ratio * algo_bytes_per_launch, f"derived_from_profile profiles/traffic_{workload}.json (counter/model {ratio:.3f})"


def occupancy_summary(occ, budget):
    """Admitted systems and held device memory over the stream: time-weighted means,
    maxima, and a coarse timeline (ten equal time bins, mean active systems)."""
    import numpy as np

    if occ.shape[0] < 2:
        return None
    t = occ[:, 0]
    dt = np.diff(t, append=t[-1])
    w = dt / max(dt.sum(), 1e-12)
    bins = np.linspace(t[0], t[-1], 11)
    idx = np.clip(np.searchsorted(bins, t, side="right") - 1, 0, 9)
    timeline = [float(occ[idx == k, 1].mean()) if np.any(idx == k) else None for k in range(10)]
    return {"samples": int(occ.shape[0]), "active_mean": float(np.dot(w, occ[:, 1])),
            "active_max": int(occ[:, 1].max()), "queued_mean": float(np.dot(w, occ[:, 2])),
            "queued_max": int(occ[:, 2].max()), "in_use_frac_of_budget_mean": float(np.dot(w, occ[:, 3])) / budget,
            "in_use_frac_of_budget_max": float(occ[:, 3].max()) / budget, "active_timeline_10_bins": timeline}


def serving_bench(args):
    """Continuous-batching service: a stream of independent SPD systems (half 2-D
    five-point, half 3-D seven-point finite volumes, log-normal coefficients,
    log-uniform sizes, 1-8 right-hand sides) with Poisson arrivals, admitted by
    device-memory budget.  A closed-loop pass over the first systems measures the
    saturated rate; the timed open-loop pass arrives at 0.7 x that rate."""
    import numpy as np

    import paper_2003_05361_amd as ras
    import ras_inputs as R

    specs = list(R.serving_stream(count=args.serve_count, rate=1.0))
    systems = []
    for sp in specs:
        A, B, parts = R.serving_system(sp)
        if sp["dims"] == 2:
            part, loc = ras.partition("regular_2d", parts, grid=A.grid), ras.local(args.serve_local2d, "fp32")
        else:
            part, loc = ras.partition("regular_3d", parts, grid=A.grid), ras.local("cg", "fp32", 8)
        systems.append((A, part, loc, B))
    budget = int(args.serve_budget_gib * (1 << 30))

    def run(subset, arrivals):
        import threading

        srv = ras.Server(budget, slice_seconds=0.02)
        t0 = time.perf_counter()
        # admitted-slot occupancy over time: (seconds, active systems, queued systems, device bytes held)
        occ, stop = [], threading.Event()

        def sample():
            while not stop.is_set():
                q = srv.stats()
                occ.append((time.perf_counter() - t0, q["active"], q["queued"], q["in_use_bytes"]))
                stop.wait(0.05)

        sampler = threading.Thread(target=sample, daemon=True)
        sampler.start()
        tickets = []
        for (A, part, loc, B), ta in zip(subset, arrivals):
            delay = ta - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(A, part, 2, loc, B, 1e-8))
            if len(tickets) % 200 == 0:
                print(f"serving: {len(tickets)} submitted, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        lat, rhs, bad = [], 0, 0
        for k, ((A, part, loc, B), tk) in enumerate(zip(subset, tickets)):
            srv.wait(tk, 600.0)
            done, x, infos, l = srv.poll(tk, A.n, B.shape[0])
            lat.append(l)
            rhs += B.shape[0]
            bad += sum(1 for i in infos if not i["converged"])
            if (k + 1) % 100 == 0:
                q = srv.stats()
                print(f"serving: {k + 1} of {len(subset)} retired, {time.perf_counter() - t0:.1f} s, "
                      f"active {q['active']}, queued {q['queued']}, in use {q['in_use_bytes'] / 2**30:.2f} GiB",
                      file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        stop.set()
        sampler.join()
        st = srv.stats()
        srv.close()
        run.occupancy = np.array(occ) if occ else np.zeros((0, 4))
        return wall, np.array(lat), rhs, bad, st

    warm = systems[: min(40, len(systems))]
    wall0, _, _, _, _ = run(warm, [0.0] * len(warm))
    sat_rate = len(warm) / wall0
    rate = 0.7 * sat_rate
    arr = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, len(systems)))
    arr -= arr[0]
    wall, lat, rhs, bad, st = run(systems, list(arr))
    line = {
        "metric": METRIC,
        "value": rhs / wall,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 local",
        "data": "synthetic",
        "config": {"workload": "serving", "systems": len(systems), "rhs": int(rhs),
                   "arrival_rate_per_s": rate, "saturated_rate_per_s": sat_rate,
                   "budget_bytes": budget, "tol": 1e-8,
                   "local": {"2d": f"{args.serve_local2d}-fp32", "3d": "cg8-fp32"}},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "occupancy": occupancy_summary(run.occupancy, budget),
        "unconverged_rhs": int(bad),
        "server": st,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)

def fixed_sweep_leg(h, bt, bps, N, reps, warmup, label_workload, kind, storage, k, with_sync=True):
    """Fixed work on one handle: N local solves per subdomain of the asynchronous
    kernel (tolerance 0, so nothing stops early), `reps` times, and N synchronous
    sweeps.  Kernel time = HIP events the library records on the solve stream around
    each persistent launch; bandwidth = algorithmic bytes of the local solves done
    (streaming model) / kernel time."""
    import numpy as np

    for _ in range(warmup):  # the same launch as the timed ones (one profile average for all)
        h.solve(bt, tol=0.0, mode="async", max_sweeps=N)
    t0 = time.perf_counter()
    ar = []
    for _ in range(reps):
        _, info = h.solve(bt, tol=0.0, mode="async", max_sweeps=N)
        ar.append((info[0], h.local_solve_counts()))
    wall = time.perf_counter() - t0
    a_bytes = [float(np.dot(c, bps)) for _, c in ar]
    a_ks = [i["kernel_seconds"] for i, _ in ar]
    a_gbps = float(np.mean([bb / ks for bb, ks in zip(a_bytes, a_ks)])) / 1e9
    leg = {"workload": label_workload, "local": f"{kind}{k if kind == 'cg' else ''}-{storage}", "sweeps": N,
           "wall_s": wall,
           "async": {"GBps": a_gbps, "kernel_seconds": float(np.mean(a_ks)),
                     "local_solves_total": int(ar[-1][0]["total_local_solves"]),
                     "ms_per_sweep_equivalent": 1e3 * float(np.mean(a_ks)) * len(bps)
                     / max(1, int(ar[-1][0]["total_local_solves"]))},
           "algorithmic_bytes_per_launch": float(np.mean(a_bytes))}
    if with_sync:
        _, info = h.solve(bt, tol=0.0, mode="sync", max_sweeps=N)
        i = info[0]
        # the synchronous kernel computes one speculative update after the last sweep
        sb = float((i["sweeps"] + 1) * bps.sum())
        leg["sync"] = {"GBps": sb / i["kernel_seconds"] / 1e9, "kernel_seconds": i["kernel_seconds"],
                       "ms_per_sweep": 1e3 * i["kernel_seconds"] / (i["sweeps"] + 1)}
    traffic, src = traffic_from_profiles(f"{label_workload}_sweeps{N}", leg["algorithmic_bytes_per_launch"])
    leg["roofline"] = {"bound": "hbm", "achieved": round(a_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(a_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic, "traffic_source": src,
                       "kernel": f"persistent async {kind}{'-' + str(k) if kind == 'cg' else ''} {storage}",
                       "workload": f"{label_workload}, {N} local solves per subdomain",
                       "algorithmic_bytes_per_launch": leg["algorithmic_bytes_per_launch"],
                       "kernel_seconds_per_launch": float(np.mean(a_ks))}
    if label_workload in MALL_RESIDENT:
        resident_roofline(leg["roofline"], None if traffic is None else traffic / float(np.mean(a_ks)) / 1e9)
    return leg


def resident_roofline(roof: dict, counter_gbps):
    """For a working set resident in the 256 MB Infinity Cache the streaming model
    counts re-reads the cache serves: the HBM figure is the counter-derived rate
    (null without a counter profile of this kernel source), the model rate moves to
    model_GBps."""
    roof["model_GBps"] = roof["achieved"]
    roof["counter_GBps"] = None if counter_gbps is None else round(counter_gbps, 1)
    roof["achieved"] = roof["counter_GBps"]
    roof["frac"] = None if counter_gbps is None else round(counter_gbps / HBM_PEAK_GBPS, 4)
    roof["note"] = ("working set resident in the 256 MB Infinity Cache: achieved and frac are the counter-derived "
                    "fabric rate (null without a counter profile of this kernel source); model_GBps is the "
                    "streaming-model rate, which counts re-reads the cache serves")


def slab_legs(locals_, N=200, reps=3):
    """The 2048^2 log-normal diffusion workload (16 x 16 boxes, overlap 4, exact
    local solves: banded Cholesky, or sparse Cholesky with suffix _sparse):
    factors of 1.3-5.1 GB (band) or 2.9 GB (sparse FP64) per triangular pass, far
    beyond the 256 MB Infinity Cache, so the sweep streams from HBM -- the honest
    roofline test.  locals_: (kind, storage) pairs."""
    import numpy as np
    import torch

    import paper_2003_05361_amd as ras
    import ras_inputs as R
    from paper_2003_05361_amd.perfmodel import bytes_per_local_solve

    A, b, cfg = R.config_problem("diffusion2d_2048_16x16")
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    legs = []
    for kind, st in locals_:
        shapes = subdomain_shapes(A, "regular_2d", (16, 16), 4, kind)
        t0 = time.perf_counter()
        h = ras.setup(A, ras.partition("regular_2d", (16, 16), grid=A.grid), 4, ras.local(kind, st))
        setup_s = time.perf_counter() - t0
        bps = np.array(bytes_per_local_solve(shapes, kind, st, 0), dtype=np.float64)
        name = f"diffusion2d_2048_16x16_{'sparse_' if kind == 'chol_sparse' else ''}{st}"
        leg = fixed_sweep_leg(h, bt, bps, N, reps, 1, name, kind, st, 0)
        leg["setup_s"] = setup_s
        h.close()
        torch.cuda.empty_cache()
        print(f"leg {name}: {leg['async']['GBps']:.0f} GB/s async, {leg['sync']['GBps']:.0f} GB/s sync",
              file=sys.stderr, flush=True)
        legs.append(leg)
    return legs


def sweep_bench(args, A, b, h, bt, bps, st, kind, storage, k, gamma, part_kind, part_arg, setup_s):
    """--sweeps N: fixed-work throughput of the named workload; value = sweep GB/s."""
    leg = fixed_sweep_leg(h, bt, bps, args.sweeps, args.steps, args.warmup, args.workload, kind, storage, k,
                          with_sync=not args.no_sync)
    N = args.sweeps
    line = {
        "metric": METRIC,
        "value": leg["async"]["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * leg["wall_s"] / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if storage == "fp64" else f"f64 outer / {storage} local",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": int(A.n), "subdomains": int(st["parts"]), "overlap": gamma,
                   "local": leg["local"], "mode": "fixed sweeps", "sweeps": N},
        "async": leg["async"],
        "sync": leg.get("sync"),
        "setup_s": setup_s,
        "roofline": leg["roofline"],
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(A, b, part_kind, part_arg, gamma, kind, storage, k, N)
        cb["unit"] = f"s for {N} synchronous sweeps (extrapolated)"
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (every subdomain of a system "
              "lives on one device). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = (2 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 2 * n * 8, "kernel": "torch copy", "launches": 3}))
        return

    if args.workload == "serving":
        serving_bench(args)
        return

    import paper_2003_05361_amd as ras
    import ras_inputs as R
    from paper_2003_05361_amd.perfmodel import bytes_per_local_solve

    cfg_name, kind, storage, k = WORKLOADS[args.workload]
    A, b, cfg = R.config_problem(cfg_name)
    part_kind, *part_rest = cfg["partition"]
    part_arg = part_rest[0] if len(part_rest) == 1 else tuple(part_rest)
    gamma = cfg["overlap"]
    tol = cfg["tol"]
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    h = ras.setup(A, part_spec(ras, A, part_kind, part_arg), gamma, ras.local(kind, storage, k), stream=stream)
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    tuned = h.autotune(bt, 20) if kind == "cg" else (1, None)  # part of setup, outside the timed steps
    setup_s = time.perf_counter() - t0
    st = h.stats()
    shapes = subdomain_shapes(A, part_kind, part_arg, gamma, kind)
    bps = bytes_per_local_solve(shapes, kind, storage, k)
    bps = np.array(bps, dtype=np.float64)

    def solve(mode):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        x, info = h.solve(bt, tol=tol, mode=mode, max_sweeps=5_000_000, max_seconds=300)
        e1.record(stream)
        torch.cuda.synchronize()
        counts = h.local_solve_counts()
        return x, info[0], e0.elapsed_time(e1) * 1e-3, counts

    if args.sweeps > 0:
        sweep_bench(args, A, b, h, bt, bps, st, kind, storage, k, gamma, part_kind, part_arg, setup_s)
        h.close()
        return

    for _ in range(args.warmup):
        solve("async")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for i in range(args.steps):
        runs.append(solve("async"))
        print(f"async run {i}: {runs[-1][2]:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    a_times = [r[2] for r in runs]
    a_kernel = [r[1]["kernel_seconds"] for r in runs]

    def dist(v):
        v = np.asarray(v, dtype=np.float64)
        return {"mean": float(v.mean()), "median": float(np.median(v)), "min": float(v.min()), "max": float(v.max())}

    # local-solve spread of every asynchronous run (min / median / max over subdomains)
    a_spread = [{"min": int(c.min()), "median": float(np.median(c)), "max": int(c.max())} for c in (r[3] for r in runs)]
    a_info = runs[-1][1]
    a_bytes = [float(np.dot(r[3], bps)) for r in runs]
    x_async = runs[-1][0]

    sync_res = None
    if not args.no_sync:
        sruns = []
        for i in range(max(1, args.steps)):
            sruns.append(solve("sync"))
            print(f"sync run {i}: {sruns[-1][2]:.3f} s, {sruns[-1][1]['sweeps']} sweeps", file=sys.stderr, flush=True)
        s_info = sruns[-1][1]
        # the synchronous kernel also computes one speculative update after the last sweep
        s_bytes = [float((r[1]["sweeps"] + 1) * bps.sum()) for r in sruns]
        sync_res = dict(seconds=float(np.mean([r[2] for r in sruns])), sweeps=int(s_info["sweeps"]),
                        seconds_stats=dist([r[2] for r in sruns]), sweeps_per_run=[int(r[1]["sweeps"]) for r in sruns],
                        kernel_seconds=float(np.mean([r[1]["kernel_seconds"] for r in sruns])),
                        rel_residual=s_info["rel_residual"],
                        model_GBps=float(np.mean([bb / r[1]["kernel_seconds"] for bb, r in zip(s_bytes, sruns)]) / 1e9))

    # verification on the host copy: exact residual and error against the direct solve
    xa = x_async.cpu().numpy()
    relres = float(np.linalg.norm(b - A.matvec(xa)) / np.linalg.norm(b))
    achieved = float(np.mean([bb / ks for bb, ks in zip(a_bytes, a_kernel)])) / 1e9
    algo_per_launch = float(np.mean(a_bytes))
    traffic, traffic_src = traffic_from_profiles(args.workload, algo_per_launch)
    ks_mean = float(np.mean(a_kernel))
    own_roof = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": traffic,
        "traffic_source": traffic_src,
        "counter_GBps": None if traffic is None else round(traffic / ks_mean / 1e9, 1),
        "kernel": f"persistent async {kind}{'-' + str(k) if kind == 'cg' else ''} {storage}",
        "workload": f"{args.workload}, solve to tolerance",
        "algorithmic_bytes_per_launch": algo_per_launch,
        "kernel_seconds_per_launch": ks_mean,
    }
    if args.workload in MALL_RESIDENT:
        resident_roofline(own_roof, own_roof["counter_GBps"])
    legs = []
    if args.workload == "poisson2d_1024_8x8" and not args.no_slab_legs:
        legs = slab_legs((("chol", "fp64"), ("chol", "fp16"), ("chol_sparse", "fp64")))
    # the roofline row: the streamed (beyond-cache) sweep of the 2048^2 diffusion
    # workload when it ran, else this workload's own kernel
    roof = dict(legs[0]["roofline"]) if legs else own_roof
    line = {
        "metric": METRIC,
        "value": float(np.mean(a_times)),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(1, args.steps),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if storage == "fp64" else f"f64 outer / {storage} local",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": int(A.n), "subdomains": int(st["parts"]), "overlap": gamma,
                   "local": f"{kind}{k if kind == 'cg' else ''}-{storage}", "tol": tol, "mode": "async",
                   "team": int(tuned[0])},
        "async": {"seconds": float(np.mean(a_times)), "seconds_stats": dist(a_times), "runs": len(runs),
                  "local_solve_spread": a_spread,
                  "local_solves_total": int(a_info["total_local_solves"]),
                  "local_solves_min": int(a_info["min_local_solves"]), "local_solves_max": int(a_info["max_local_solves"]),
                  "rel_residual": relres, "launches": int(a_info["launches"])},
        "sync": sync_res,
        "async_speedup_vs_sync": None if sync_res is None else sync_res["seconds"] / float(np.mean(a_times)),
        "setup_s": setup_s,
        "roofline": roof,
        "rooflines": [own_roof] + [leg["roofline"] for leg in legs],
        "sweep_legs": legs,
    }
    if not args.no_cpu_baseline and sync_res is not None:
        line["cpu_baseline"] = cpu_baseline(A, b, part_kind, part_arg, gamma, kind, storage, k, sync_res["sweeps"])
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    h.close()


if __name__ == "__main__":
    main()
