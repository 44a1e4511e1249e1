"""One-GPU parameter studies: partitioning scheme and overlap (Sec. 3.2.1 Fig. 2, Secs. 4.2-4.3 Figs. 3-4),
and time to tolerance by local solver, storage, mode and detector (Secs. 4.5-4.6).

Every case builds the host plan, records its shape (local rows, band width,
band entries as the fill of the local factors, communication volume between
subdomains as in Fig. 2), sets it up on the device and solves the same system
synchronously and asynchronously to the tolerance, both through the library's
device kernels.  The per-sweep breakdown is the algorithmic byte model of the
three steps of one update (restriction and residual, local solve, restricted
prolongation) with the values read from other subdomains' points singled out:
the fused kernels do not expose a per-step clock, so the split is modelled and
only the sweep time is measured.

    python -m paper_2003_05361_amd.studies partitioners [--parts 4,16,36,64] [--overlap 4]
    python -m paper_2003_05361_amd.studies overlap [--sizes 128,256] [--overlaps 0,1,2,4,8,12,16]
    python -m paper_2003_05361_amd.studies time_to_tolerance [--config diffusion2d_2048_16x16] [--local chol]

Each case prints one JSON line; --markdown writes a summary with the tables and
the communication-volume matrices.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

PARTITIONERS = ("regular_1d", "regular_2d", "rcb")


def _square_split(P: int) -> tuple[int, int]:
    a = int(math.isqrt(P))
    while P % a:
        a -= 1
    return (P // a, a)


def partition_spec(ras, A, kind: str, P: int) -> dict:
    """Fig. 2's three schemes; recursive coordinate bisection stands in for the
    graph partitioner (balanced parts with short boundaries)."""
    if kind == "regular_1d":
        return ras.partition("regular_1d", P, grid=A.grid)
    if kind == "regular_2d":
        return ras.partition("regular_2d", _square_split(P), grid=A.grid)
    if kind == "rcb":
        return ras.partition("rcb", P, grid=A.grid, seed=0, jitter=0.0)
    raise ValueError(kind)


def comm_summary(vol: np.ndarray) -> dict:
    nb = np.count_nonzero(vol, axis=1)
    recv = vol.sum(axis=1)
    return {"total_values": int(vol.sum()), "max_recv": int(recv.max()), "mean_recv": float(recv.mean()),
            "max_neighbours": int(nb.max()), "mean_neighbours": float(nb.mean())}


def run_case(A, b, spec: dict, gamma: int, loc: dict, tol: float, max_seconds: float, stream, label: dict) -> dict:
    import torch

    import paper_2003_05361_amd as ras
    from paper_2003_05361_amd.perfmodel import local_solve_parts, subdomain_shapes

    t0 = time.perf_counter()
    plan = ras.Plan(A, spec, gamma, loc)
    st = plan.stats()
    vol = plan.comm_volume()
    shapes = subdomain_shapes(plan, A.indptr, loc["kind"] == "chol_sparse")
    h = plan.setup(stream=stream)
    setup_s = time.perf_counter() - t0
    plan.close()
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    h.solve(bt, tol=0.0, mode="sync", max_sweeps=2)  # first launch outside the timings

    def timed(mode, pace=None):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        x, info = h.solve(bt, tol=tol, mode=mode, max_sweeps=1_000_000, max_seconds=max_seconds, pace=pace)
        e1.record(stream)
        torch.cuda.synchronize()
        return info[0], e0.elapsed_time(e1) * 1e-3, h.local_solve_counts()

    def async_result(info, sec, counts):
        return {"converged": bool(info["converged"]), "seconds": sec, "rel_residual": info["rel_residual"],
                "local_solves_min": int(counts.min()), "local_solves_median": float(np.median(counts)),
                "local_solves_max": int(counts.max())}

    def shares():
        # measured device time per phase, summed over subdomains (Figs. 3a, 4a, 7a)
        ph = h.phase_seconds().sum(axis=0)
        tot = float(ph.sum())
        return {k: float(v) / tot if tot > 0 else 0.0 for k, v in zip(h.PHASES, ph)}, tot

    s_info, s_sec, _ = timed("sync")
    s_share, s_phase_total = shares()
    a_info, a_sec, a_counts = timed("async")  # the library's pace for this local solver
    a_share, _ = shares()
    f_info, f_sec, f_counts = timed("async", 0.0)  # free running: reads never wait
    h.close()

    kind, storage, k = loc["kind"], loc.get("storage", "fp64"), loc.get("cg_iters", 0)
    parts = np.array([local_solve_parts(sh, kind, storage, k) for sh in shapes]).sum(axis=0)
    exchange = 8.0 * float(vol.sum())
    sweep_bytes = float(parts.sum())
    sweeps = int(s_info["sweeps"])
    res = dict(label)
    res.update({
        "n": int(A.n), "parts": int(st["parts"]), "overlap": gamma, "local": f"{kind}-{storage}",
        "local_rows_mean": st["sum_local_rows"] / st["parts"], "local_rows_max": int(st["max_local_rows"]),
        "max_band": int(st["max_band"]), "band_entries": int(st["band_entries"]),
        "comm": comm_summary(vol),
        "setup_s": setup_s,
        "sync": {"converged": bool(s_info["converged"]), "sweeps": sweeps, "seconds": s_sec,
                 "ms_per_sweep": 1e3 * s_sec / max(1, sweeps), "rel_residual": s_info["rel_residual"]},
        "async": async_result(a_info, a_sec, a_counts),
        "async_free": async_result(f_info, f_sec, f_counts),
        "async_speedup": s_sec / a_sec if a_sec > 0 else None,
        "async_free_speedup": s_sec / f_sec if f_sec > 0 else None,
        "measured_share_sync": s_share,
        "measured_share_async": a_share,
        "measured_phase_seconds_sync": s_phase_total,
        "model_bytes_per_sweep": {"restrict_residual": float(parts[0]), "local_solve": float(parts[1]),
                                  "prolong": float(parts[2]), "exchange_of_residual": exchange},
        "model_share": {"restrict_residual": float(parts[0]) / sweep_bytes, "local_solve": float(parts[1]) / sweep_bytes,
                        "prolong": float(parts[2]) / sweep_bytes, "exchange": exchange / sweep_bytes},
        "model_GBps_sync": sweep_bytes * (sweeps + 1) / s_info["kernel_seconds"] / 1e9
        if s_info["kernel_seconds"] > 0 else None,
    })
    return res, vol


def _progress(msg):
    print(msg, file=sys.stderr, flush=True)


def partitioners(args, stream) -> tuple[list, dict]:
    """Fig. 3 analog: fixed local size (per_part unknowns), P grown, three schemes."""
    import paper_2003_05361_amd as ras
    import ras_inputs as R

    rows, heat = [], {}
    for P in args.parts:
        N = int(round(math.sqrt(P * args.per_part)))
        A = R.laplace2d(N)
        b = R.uniform_rhs(A.n, 1)
        for kind in PARTITIONERS:
            _progress(f"partitioners: P={P} N={N} {kind}")
            r, vol = run_case(A, b, partition_spec(ras, A, kind, P), args.overlap, ras.local(args.local, "fp64", args.cg_iters),
                              args.tol, args.max_seconds, stream,
                              {"study": "partitioners", "grid": N, "partitioner": kind})
            print(json.dumps(r), flush=True)
            rows.append(r)
            if P == args.heatmap_parts:
                heat[kind] = vol
    base = {r["parts"]: r["sync"]["seconds"] for r in rows if r["partitioner"] == "regular_1d"}
    for r in rows:
        r["sync_speedup_vs_1d"] = base[r["parts"]] / r["sync"]["seconds"]
    return rows, heat


def overlaps(args, stream) -> tuple[list, dict]:
    """Fig. 4 analog: one partition (bisection, args.nparts parts), overlap varied,
    at each grid size."""
    import paper_2003_05361_amd as ras
    import ras_inputs as R

    rows, heat = [], {}
    for N in args.sizes:
        A = R.laplace2d(N)
        b = R.uniform_rhs(A.n, 1)
        for gamma in args.overlaps:
            _progress(f"overlap: N={N} gamma={gamma}")
            r, vol = run_case(A, b, partition_spec(ras, A, "rcb", args.nparts), gamma, ras.local(args.local, "fp64", args.cg_iters),
                              args.tol, args.max_seconds, stream, {"study": "overlap", "grid": N, "partitioner": "rcb"})
            print(json.dumps(r), flush=True)
            rows.append(r)
            if N == args.sizes[0]:
                heat[f"overlap {gamma}"] = vol
    return rows, heat


def time_to_tolerance(args, stream) -> tuple[list, dict]:
    """Solve a named workload to its tolerance, synchronously and asynchronously,
    for each requested storage of the local solver, in chunks of at most
    args.chunk seconds (x carried from chunk to chunk, which continues the same
    iteration), printing one progress line per chunk; the time is the sum of the
    chunks' HIP-event times on the solve stream.  With fp64 among the storages,
    every solution's relative difference from the fp64 one of the same mode is
    reported."""
    import torch

    import paper_2003_05361_amd as ras
    import ras_inputs as R

    A, b, cfg = R.config_problem(args.config, args.grid)
    kind, arg = cfg["partition"][0], cfg["partition"][1:]
    arg = arg[0] if len(arg) == 1 else tuple(arg)
    spec = (ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2]) if kind == "rcb"
            else ras.partition(kind, arg, grid=A.grid))
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    storages = args.storages.split(",") if args.storages else [args.storage]
    rows, sols = [], {}
    for storage in storages:
        t0 = time.perf_counter()
        h = ras.setup(A, spec, cfg["overlap"], ras.local(args.local, storage, args.cg_iters), stream=stream)
        if args.local == "cg":
            h.autotune(bt, 20)  # team size, as the bench sets it up
        setup_s = time.perf_counter() - t0
        h.solve(bt, tol=0.0, mode="sync", max_sweeps=2)
        for mode_name in args.modes.split(","):
            # "async-decentral": the asynchronous solver with decentralized detection
            mode, _, detect = mode_name.partition("-")
            detect = detect or "central"
            x = torch.zeros_like(bt)
            total, counts, sweeps, info = 0.0, None, 0, None
            while total < args.budget:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                x, infos = h.solve(bt, x0=x, tol=cfg["tol"], mode=mode, max_sweeps=1 << 40,
                                   max_seconds=min(args.chunk, args.budget - total), detect=detect,
                                   pace=args.pace)
                e1.record(stream)
                torch.cuda.synchronize()
                total += e0.elapsed_time(e1) * 1e-3
                info = infos[0]
                c = h.local_solve_counts()
                counts = c if counts is None else counts + c
                sweeps += int(info["sweeps"])
                _progress(json.dumps({"storage": storage, "mode": mode_name, "seconds": total, "sweeps": sweeps,
                                      "rel_residual": info["rel_residual"], "converged": bool(info["converged"])}))
                if info["converged"]:
                    break
            xh = x.cpu().numpy()
            relres_dev = h.relative_residual(bt, x)
            sols[(storage, mode_name)] = xh
            if args.save_x:
                np.save(f"{args.save_x}_{mode_name}_{args.local}_{storage}.npy", xh)
            r = {"study": "time_to_tolerance", "config": args.config, "n": int(A.n),
                 "local": f"{args.local}-{storage}",
                 "mode": mode_name if args.pace is None or mode == "sync" else f"{mode_name} pace {args.pace:g}",
                 "converged": bool(info["converged"]),
                 "seconds": total, "tol": cfg["tol"],
                 "rel_residual": relres_dev,
                 "rel_residual_host_plain": float(np.linalg.norm(b - A.matvec(xh)) / np.linalg.norm(b)),
                 "local_solves_min": int(counts.min()), "local_solves_median": float(np.median(counts)),
                 "local_solves_max": int(counts.max()), "setup_s": setup_s}
            if mode == "sync":
                r["sweeps"] = sweeps
                r["ms_per_sweep"] = 1e3 * total / max(1, sweeps)
            rows.append(r)
        h.close()
    for r in rows:
        ref = sols.get(("fp64", r["mode"]))
        if ref is not None:
            xs = sols[(r["local"].split("-")[-1], r["mode"])]
            r["rel_diff_vs_fp64"] = float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))
        print(json.dumps(r), flush=True)
    return rows, {}


def oras(args, stream) -> tuple[list, dict]:
    """Optimized RAS (Robin transmission, the paper's future work) against RAS on a
    named workload with a direct local solver: synchronous sweeps and seconds to the
    tolerance, and the asynchronous (library pace) seconds, for each Robin weight q
    (q = 1 is RAS)."""
    import torch

    import paper_2003_05361_amd as ras
    import ras_inputs as R

    A, b, cfg = R.config_problem(args.config, args.grid)
    kind, arg = cfg["partition"][0], cfg["partition"][1:]
    arg = arg[0] if len(arg) == 1 else tuple(arg)
    spec = (ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2]) if kind == "rcb"
            else ras.partition(kind, arg, grid=A.grid))
    bt = torch.tensor(b, dtype=torch.float64, device="cuda")
    rows = []
    for q in args.robin_q:
        h = ras.setup(A, spec, cfg["overlap"], ras.local(args.local, args.storage, robin_q=None if q >= 1.0 else q),
                      stream=stream)
        h.solve(bt, tol=0.0, mode="sync", max_sweeps=2)
        res = {"study": "oras", "config": args.config, "n": int(A.n), "local": f"{args.local}-{args.storage}",
               "robin_q": q, "tol": args.tol}
        for mode in ("sync", "async"):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            x, infos = h.solve(bt, tol=args.tol, mode=mode, max_sweeps=1_000_000, max_seconds=args.max_seconds)
            e1.record(stream)
            torch.cuda.synchronize()
            i = infos[0]
            c = h.local_solve_counts()
            res[mode] = {"converged": bool(i["converged"]), "seconds": e0.elapsed_time(e1) * 1e-3,
                         "sweeps": int(i["sweeps"]), "local_solves_median": float(np.median(c)),
                         "rel_residual": i["rel_residual"]}
        h.close()
        _progress(json.dumps(res))
        rows.append(res)
    return rows, {}


def markdown_oras(rows: list, cmd: str) -> str:
    L = [f"# Optimized RAS (Robin transmission) vs RAS: {rows[0]['config']} (n = {rows[0]['n']})", "",
         "Command (one MI355X):", "", f"    {cmd}", "",
         "Local matrices A[Omega_p, Omega_p] with the diagonal lowered by (1 - q) times each row's coupling "
         "to points outside the subdomain (q = 1: RAS). Same kernels; times are HIP events around one solve, "
         f"setup excluded; local solver {rows[0]['local']}, tolerance {rows[0]['tol']:g}.", "",
         "| q | sync sweeps | sync s | async s (median local solves) | sweeps vs RAS |", "|---|---|---|---|---|"]
    base = next((r["sync"]["sweeps"] for r in rows if r["robin_q"] >= 1.0), None)
    for r in rows:
        s, a = r["sync"], r["async"]
        nc = "" if s["converged"] else " (not conv.)"
        anc = "" if a["converged"] else " not conv."
        ratio = f"{base / s['sweeps']:.2f}x fewer" if base and s["sweeps"] and s["converged"] else "-"
        L.append(f"| {r['robin_q']:g} | {s['sweeps']}{nc} | {s['seconds']:.3f} | {a['seconds']:.3f} "
                 f"({a['local_solves_median']:.0f}{anc}) | {ratio} |")
    return "\n".join(L) + "\n"


def batching(args, stream) -> tuple[list, dict]:
    """Many independent systems: the 2-D systems of the serving stream (log-normal
    finite volumes, regular boxes of about 4,096 unknowns, overlap 2, banded
    Cholesky FP32, every right-hand side), solved to 1e-8 one launch per system
    and all in one batched persistent launch, in both modes."""
    import torch

    import paper_2003_05361_amd as ras
    import ras_inputs as R

    specs = [sp for sp in R.serving_stream(count=4 * args.systems) if sp["dims"] == 2][: args.systems]
    hs, bs = [], []
    for sp in specs:
        A, B, parts = R.serving_system(sp)
        hs.append(ras.setup(A, ras.partition("regular_2d", parts, grid=A.grid), 2, ras.local("chol", "fp32"),
                            stream=stream))
        bs.append(torch.tensor(B, dtype=torch.float64, device="cuda"))
    rows = []
    for mode in ("sync", "async"):
        ras.batch_solve(hs, bs, tol=1e-8, mode=mode, max_seconds=60)  # first launch outside the timings
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for h, b in zip(hs, bs):
            h.solve(b, tol=1e-8, mode=mode, max_seconds=60)
        e1.record(stream)
        torch.cuda.synchronize()
        t_seq = e0.elapsed_time(e1) * 1e-3
        e0.record(stream)
        _, infos = ras.batch_solve(hs, bs, tol=1e-8, mode=mode, max_seconds=60)
        e1.record(stream)
        torch.cuda.synchronize()
        t_bat = e0.elapsed_time(e1) * 1e-3
        conv = all(i["converged"] for inf in infos for i in inf)
        nrhs = sum(int(b.shape[0]) for b in bs)
        r = {"study": "batching", "systems": len(hs), "rhs": nrhs, "unknowns": int(sum(h.n for h in hs)),
             "mode": mode, "one_launch_per_system_s": t_seq, "one_batched_launch_s": t_bat,
             "speedup": t_seq / t_bat, "all_converged": conv}
        print(json.dumps(r), flush=True)
        rows.append(r)
    return rows, {}


def markdown_batching(rows: list, cmd: str) -> str:
    L = ["# Batching: independent systems in one persistent launch", "", "Command (one MI355X):", "", f"    {cmd}", "",
         "The 2-D systems of the seeded serving stream (log-normal finite volumes, regular boxes of about 4,096 "
         "unknowns, overlap 2, banded Cholesky FP32, all right-hand sides), solved to 1e-8 from x = 0: once as "
         "one launch per system (the same handles, back to back on one stream), once as one batched launch. "
         "HIP-event times, a first batched launch of each mode untimed.", "",
         "| mode | systems | right-hand sides | unknowns | one launch per system (s) | one batched launch (s) | speedup | all converged |",
         "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        L.append(f"| {r['mode']} | {r['systems']} | {r['rhs']} | {r['unknowns']} | {r['one_launch_per_system_s']:.3f} | "
                 f"{r['one_batched_launch_s']:.3f} | {r['speedup']:.2f} | {r['all_converged']} |")
    return "\n".join(L) + "\n"


def _fmt_matrix(vol: np.ndarray) -> list:
    P = vol.shape[0]
    out = ["| p \\ q | " + " | ".join(str(q) for q in range(P)) + " |", "|---" * (P + 1) + "|"]
    for p in range(P):
        out.append(f"| {p} | " + " | ".join(str(int(v)) if v else "." for v in vol[p]) + " |")
    return out


def markdown_ttt(rows: list, cmd: str) -> str:
    L = [f"# Time to tolerance: {rows[0]['config']} (n = {rows[0]['n']})", "", "Command (one MI355X):", "",
         f"    {cmd}", "",
         "x0 = 0; the solve runs in chunks (x carried over, which continues the same iteration) so that "
         "the run reports progress; seconds = the sum of the chunks' HIP-event times on the solve stream, "
         "setup excluded. The relative residual is the library's compensated float64 recomputation "
         "from the returned x; the plain float64 host value is beside it.", "",
         "| local | mode | converged | seconds | sweeps (sync) | ms per sweep | local solves min / median / max | "
         "rel. residual | plain float64 host | rel. difference from FP64 |",
         "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        sw = f"{r['sweeps']} | {r['ms_per_sweep']:.3f}" if "ms_per_sweep" in r else "- | -"
        dv = f"{r['rel_diff_vs_fp64']:.2e}" if "rel_diff_vs_fp64" in r else "-"
        L.append(f"| {r['local']} | {r['mode']} | {r['converged']} | {r['seconds']:.1f} | {sw} | "
                 f"{r['local_solves_min']} / {r['local_solves_median']:.0f} / {r['local_solves_max']} | "
                 f"{r['rel_residual']:.3e} | {r['rel_residual_host_plain']:.3e} | {dv} |")
    if len(rows) == 2 and rows[0]["local"] == rows[1]["local"]:
        L += ["", f"Asynchronous speedup over synchronous: {rows[0]['seconds'] / rows[1]['seconds']:.3f}."]
    return "\n".join(L) + "\n"


def markdown(study: str, rows: list, heat: dict, cmd: str) -> str:
    L = [f"# Parameter study: {study}", "", "Command (one MI355X):", "", f"    {cmd}", ""]
    L += [f"Local solves: {'nested-dissection sparse' if rows and rows[0].get('local', '').startswith('chol_sparse') else 'banded'} "
          "Cholesky, float64; tolerance on the relative residual as given per row. "
          "Times are HIP events around one solve call, setup excluded. Sweep time is the measured "
          "synchronous time over its sweep count. The shares are measured: device wall-clock time "
          "per phase summed over subdomains (residual = restriction and residual, with the read "
          "snapshot when asynchronous; solve = local solve; prolong = restricted prolongation and "
          "publication; other = waiting at the sweep barrier and the convergence check when "
          "synchronous, paced waits and detection when asynchronous).", ""]
    L += ["Async runs twice: with paced reads (the library's choice for the banded solver: a subdomain "
          "waits up to a quarter of its previous update's time for neighbours that are behind) and free "
          "running (reads never wait). Updates = median local solves per subdomain.", ""]
    L += ["| grid | P | scheme | overlap | max band | factor entries | comm values | max nbrs | sync sweeps | "
          "sync s | ms/sweep | async s (updates) | free async s (updates) | async speedup | free speedup | "
          "sync speedup vs 1-D | sync: residual / solve / prolong / other | async: residual / solve / prolong / other |",
          "|---" * 18 + "|"]
    for r in rows:
        ss, sa = r["measured_share_sync"], r["measured_share_async"]
        conv = "" if r["sync"]["converged"] else " (not conv.)"
        def amode(a):
            c = "" if a["converged"] else " not conv."
            return f"{a['seconds']:.4f} ({a['local_solves_median']:.0f}{c})"

        vs1d = f"{r['sync_speedup_vs_1d']:.2f}" if "sync_speedup_vs_1d" in r else "-"
        L.append(f"| {r['grid']}^2 | {r['parts']} | {r['partitioner']} | {r['overlap']} | {r['max_band']} | "
                 f"{r['band_entries']} | {r['comm']['total_values']} | {r['comm']['max_neighbours']} | "
                 f"{r['sync']['sweeps']}{conv} | {r['sync']['seconds']:.4f} | {r['sync']['ms_per_sweep']:.3f} | "
                 f"{amode(r['async'])} | {amode(r['async_free'])} | {r['async_speedup']:.2f} | "
                 f"{r['async_free_speedup']:.2f} | {vs1d} | "
                 f"{ss['residual']:.2f} / {ss['local_solve']:.2f} / {ss['prolong']:.2f} / {ss['other']:.2f} | "
                 f"{sa['residual']:.2f} / {sa['local_solve']:.2f} / {sa['prolong']:.2f} / {sa['other']:.2f} |")
    for name, vol in heat.items():
        L += ["", f"Communication volume, {name} (row p receives from column q; values per local solve):", ""]
        L += _fmt_matrix(vol)
    return "\n".join(L) + "\n"


def _ints(s: str) -> list:
    return [int(v) for v in s.split(",") if v]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("study", choices=("partitioners", "overlap", "time_to_tolerance", "batching", "oras"))
    ap.add_argument("--robin-q", type=lambda v: [float(t) for t in v.split(",") if t],
                    default=[1.0, 0.7, 0.5, 0.3, 0.2, 0.1], help="oras: Robin weights (1 = RAS)")
    ap.add_argument("--systems", type=int, default=64, help="batching: number of systems")
    ap.add_argument("--config", default="diffusion2d_2048_16x16", help="time_to_tolerance: ras_inputs workload")
    ap.add_argument("--storage", default="fp64")
    ap.add_argument("--storages", default=None, help="time_to_tolerance: comma-separated storages (overrides --storage)")
    ap.add_argument("--grid", type=int, default=None, help="time_to_tolerance: grid side override of the workload")
    ap.add_argument("--cg-iters", type=int, default=0)
    ap.add_argument("--modes", default="sync,async",
                    help="time_to_tolerance: any of sync, async, async-decentral (decentralized detection)")
    ap.add_argument("--chunk", type=float, default=50.0)
    ap.add_argument("--pace", type=float, default=None,
                    help="time_to_tolerance: asynchronous read pacing (default: the library's choice)")
    ap.add_argument("--budget", type=float, default=1000.0, help="time_to_tolerance: seconds per mode at most")
    ap.add_argument("--save-x", default=None, help="time_to_tolerance: save each solution as <prefix>_<mode>_<local>_<storage>.npy")
    ap.add_argument("--parts", type=_ints, default=[4, 16, 36, 64])
    ap.add_argument("--per-part", type=int, default=4096)
    ap.add_argument("--overlap", type=int, default=4)
    ap.add_argument("--heatmap-parts", type=int, default=16)
    ap.add_argument("--sizes", type=_ints, default=[128, 256])
    ap.add_argument("--overlaps", type=_ints, default=[0, 1, 2, 4, 8, 12, 16])
    ap.add_argument("--nparts", type=int, default=6)
    ap.add_argument("--local", default="chol", choices=("chol", "chol_sparse", "cg"),
                    help="local solver: banded or nested-dissection sparse Cholesky, or CG (--cg-iters steps)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-seconds", type=float, default=30.0)
    ap.add_argument("--markdown", default=None)
    args = ap.parse_args(argv)

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("the studies run the device solver: no GPU visible")
    stream = torch.cuda.current_stream()
    run = {"partitioners": partitioners, "overlap": overlaps, "time_to_tolerance": time_to_tolerance,
           "batching": batching, "oras": oras}[args.study]
    rows, heat = run(args, stream)
    if args.markdown:
        cmd = "python -m paper_2003_05361_amd.studies " + " ".join(sys.argv[1:] if argv is None else argv)
        with open(args.markdown, "w") as f:
            if args.study == "time_to_tolerance":
                f.write(markdown_ttt(rows, cmd))
            elif args.study == "batching":
                f.write(markdown_batching(rows, cmd))
            elif args.study == "oras":
                f.write(markdown_oras(rows, cmd))
            else:
                f.write(markdown(args.study, rows, heat, cmd))
    return rows


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
