#!/usr/bin/env python
"""Benchmark of the FSI Newton-step linear solve on one MI355X.

One step = the whole hot path for one Newton Jacobian of the 2D 128x32
four-level system (79,108 unknowns, Q2-P1disc, 4x4-element Schwarz blocks):
extraction and Gauss-Jordan inversion of every Schwarz block and of the
coarsest operator from the device-resident operators, then FGMRES(30) with
the multigrid V-cycle to rtol 1e-10 in FP64.  Inputs are resident in HBM when
the timed region starts.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "V-cycle ms & FGMRES solves/s, FP64 vs mixed; served solves/s + p50/p99 latency"
WORKLOAD = "c1_2d_128x32"


def ras_bytes(info, wbytes, vbytes):
    """Algorithmic bytes of one finest-level Schwarz launch: the owned rows of
    every block inverse once, the gathered residual entries (index + value),
    and the owned corrections (index, read, write)."""
    return wbytes * info["sum_om"] + (4 + vbytes) * info["sum_m"] + (4 + 2 * vbytes) * info["n_owned"]


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ras_finest_c1_2d_128x32_fp64_traffic.md")


def ras_kernel_digest():
    """Digest of the device code of the Schwarz kernel (helpers and kernel
    body, not the host launchers): counter readings apply only to this code."""
    src = open(os.path.join(ROOT, "paper_1709_05660_amd", "csrc", "fsi_kernels.hip")).read()
    a = src.index("__device__ inline float w16val")
    b = src.index("// ev0/ev1 (optional, finest level)")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per finest-level Schwarz launch from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None
    when the summary was taken on other kernel code."""
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    b = re.search(r"traffic_bytes_per_launch:\s*(\d+)", txt)
    d = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", txt)
    if not b or not d or d.group(1) != ras_kernel_digest():
        return None
    return int(b.group(1))


_TUNING_DB = None


def tuning_db():
    """The autotuner's database: FSI_TUNING_DB when set (to reuse the choices
    of an earlier run, e.g. one made without a profiler), else a fresh file
    for this run, so that no earlier run's timings decide."""
    global _TUNING_DB
    if os.environ.get("FSI_TUNING_DB"):
        return os.environ["FSI_TUNING_DB"]
    if _TUNING_DB is None:
        import atexit
        import tempfile
        fd, _TUNING_DB = tempfile.mkstemp(prefix="fsi_tuning_", suffix=".db")
        os.close(fd)
        atexit.register(lambda: os.path.exists(_TUNING_DB) and os.remove(_TUNING_DB))
    return _TUNING_DB


def tuning_choices(db):
    """The batched inversion's variant and grid as the autotuner left them in
    its database (keys gj3:... and gjg:...)."""
    names = {1: "NB16 x 256", 2: "NB16 x 512", 3: "NB32 x 512 (LDS panel)", 4: "wide panel from the block",
             5: "NB24 x 512 (LDS panel)"}
    out = {}
    try:
        for line in open(db):
            k, v = line.split()
            if k.startswith("gj3:"):
                out.setdefault("gj_variant", {})[k] = names.get(int(v), v)
            elif k.startswith("gjg:"):
                out.setdefault("gj_grid", {})[k] = int(v)
    except OSError:
        pass
    return out


def vcycle_times(mg, n, stream, reps=50, warm=5):
    """Median V-cycle time over reps applications after warm ones, each cycle
    between its own events (warm: the operators may stay in the 256 MB
    last-level cache between cycles)."""
    import torch
    r = torch.randn(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    for _ in range(warm):
        mg.vcycle(r, z)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record(stream)
        mg.vcycle(r, z)
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))


def vcycle_cold_ms(mg, n, stream, reps=20):
    """Median V-cycle time with the caches flushed first: a 512 MiB fill (twice
    the last-level cache) runs before each timed cycle, outside its events."""
    import torch
    r = torch.randn(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    flush = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    mg.vcycle(r, z)
    ts = []
    for i in range(reps):
        flush.fill_(float(i))
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        mg.vcycle(r, z)
        ev1.record(stream)
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    del flush
    return float(np.median(ts))


def three_d_leg(args):
    """The 3D 32x8x8 three-level system (120,902 unknowns, 2x2x2-element
    Schwarz blocks of 416-782 dofs) in FP64 and in the mixed form, both to the
    workload's rtol 1e-8: steps/s, V-cycle (warm and cold), refactor split."""
    import torch

    from paper_1709_05660_amd import MG, Problem
    from synth import config, fourier_coefficients

    spec = config("c3_3d_32x8x8")
    p = Problem(spec, fourier_coefficients(spec.dim, spec.seed))
    stream = torch.cuda.Stream()
    res = {"unknowns": p.n, "rtol": spec.rtol}
    tune_db = tuning_db()
    with torch.cuda.stream(stream):
        b = torch.as_tensor(p.b).to("cuda")
        x = torch.zeros_like(b)
        for prec in ("fp64", args.mixed):
            mg = MG(p, precision=prec, use_graph=True)
            mg.autotune(tune_db)
            if prec == "fp64":
                gf = 0.0
                for l in range(1, p.nlevels):
                    m = np.diff(mg.export_patches(l)[0]).astype(np.float64)
                    gf += 2.0 * float((m ** 3).sum()) / 1e9
                res["block_inversion_gflop"] = round(gf, 2)
            infos = []
            torch.cuda.synchronize()
            for k in range(args.warmup + args.steps_3d):
                if k == args.warmup:
                    torch.cuda.synchronize()
                    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    ev0.record(stream)
                mg.refactor()
                _, info = mg.fgmres(b, x, restart=spec.restart, rtol=spec.rtol, maxit=spec.maxit)
                infos.append(info)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.steps_3d
            res[prec] = {"ms_per_step": round(ms, 3), "solves_per_s": round(1e3 / ms, 2),
                         "iters": infos[-1]["iters"], "true_relres": float(f"{infos[-1]['true_relres']:.4g}"),
                         "converged": all(i["converged"] == 1 for i in infos),
                         "refactor_ms": round(infos[-1]["setup_ms"], 3),
                         "solve_ms": round(infos[-1]["solve_ms"], 3),
                         "vcycle_ms": round(vcycle_times(mg, p.n, stream, 20), 4),
                         "vcycle_ms_cold": round(vcycle_cold_ms(mg, p.n, stream, 10), 4)}
            mg.close()
    return res


def small_leg(args):
    """The 16x4 two-level system (1,380 unknowns): V-cycle and solve in FP64,
    where launch latency, not bandwidth, sets the time."""
    import torch

    from paper_1709_05660_amd import MG, Problem
    from synth import config, fourier_coefficients

    spec = config("c0_2d_16x4")
    p = Problem(spec, fourier_coefficients(spec.dim, spec.seed))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = torch.as_tensor(p.b).to("cuda")
        x = torch.zeros_like(b)
        mg = MG(p, precision="fp64", use_graph=True)
        for _ in range(args.warmup):
            mg.refactor()
            mg.fgmres(b, x, restart=spec.restart, rtol=spec.rtol, maxit=spec.maxit)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            mg.refactor()
            _, info = mg.fgmres(b, x, restart=spec.restart, rtol=spec.rtol, maxit=spec.maxit)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        res = {"unknowns": p.n, "vcycle_us": round(1e3 * vcycle_times(mg, p.n, stream), 2),
               "ms_per_step": round(ms, 3), "solves_per_s": round(1e3 / ms, 1),
               "iters": info["iters"], "true_relres": float(f"{info['true_relres']:.4g}")}
        mg.close()
    return res


def gpu_leg(args):
    import torch

    from paper_1709_05660_amd import MG, Problem, stream_read_gbps
    from synth import config, fourier_coefficients

    spec = config(WORKLOAD)
    t = time.time()
    p = Problem(spec, fourier_coefficients(spec.dim, spec.seed))
    build_s = time.time() - t
    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        b = torch.as_tensor(p.b).to("cuda")
        x = torch.zeros_like(b)

        def timed_steps(mg, k, rtol):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record(stream)
            infos = []
            for _ in range(k):
                mg.refactor()
                _, info = mg.fgmres(b, x, restart=spec.restart, rtol=rtol, maxit=spec.maxit)
                infos.append(info)
            ev1.record(stream)
            torch.cuda.synchronize()
            return ev0.elapsed_time(ev1), infos

        def vcycle_ms(mg, reps=50):
            return vcycle_times(mg, p.n, stream, reps)

        # ---- FP64 (the workload's precision): value
        t = time.time()
        mg = MG(p, precision="fp64", use_graph=True)
        setup_upload_ms = (time.time() - t) * 1e3
        tune_db = tuning_db()
        t = time.time()
        out["autotune_new_measurements"] = mg.autotune(tune_db)
        out["autotune_s"] = round(time.time() - t, 3)
        out["autotune_choices"] = tuning_choices(tune_db)
        _, warm = timed_steps(mg, args.warmup, spec.rtol)
        total_ms, infos = timed_steps(mg, args.steps, spec.rtol)
        out["ms_per_step"] = total_ms / args.steps
        out["iters"] = infos[-1]["iters"]
        out["true_relres"] = infos[-1]["true_relres"]
        out["converged"] = all(i["converged"] == 1 for i in infos)
        x64 = x.clone()
        out["vcycle_ms_fp64"] = vcycle_ms(mg)
        out["vcycle_ms_fp64_cold"] = vcycle_cold_ms(mg, p.n, stream)
        out["refactor_ms_fp64"] = infos[-1]["setup_ms"]
        out["solve_ms_fp64"] = infos[-1]["solve_ms"]
        out["setup_with_upload_ms"] = setup_upload_ms
        out["build_s"] = build_s
        # ---- dominant kernel: finest-level Schwarz GEMV, event-timed on its stream
        fine = mg.level_info(p.nlevels - 1)
        ptr, dof, owned, _ = mg.export_patches(p.nlevels - 1)
        fine["n_owned"] = int(owned.sum())
        mg.profile_start()
        for _ in range(args.prof_steps):
            mg.fgmres(b, x, restart=spec.restart, rtol=spec.rtol, maxit=spec.maxit)
        kms, cnt, _, _ = mg.profile_stop()
        avg_ms = kms / max(cnt, 1)
        bytes_per_launch = ras_bytes(fine, 8, 8)
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if cnt else 0.0
        out["roofline"] = {"bound": "hbm", "kernel": "k_ras<double> (finest level)",
                           "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                           "frac": round(achieved / 8000.0, 4), "traffic": measured_traffic(),
                           "avg_launch_us": round(avg_ms * 1e3, 2), "launches": cnt,
                           "bytes_per_launch": int(bytes_per_launch)}
        # what a plain streaming read of the same byte count achieves on this
        # device (a library reduction over a float64 tensor), for context
        ceil = stream_read_gbps(int(bytes_per_launch))
        out["roofline"]["read_ceiling"] = {
            "kernel": "fsi_stream_read: plain 16-byte streaming read of the same byte count",
            "achieved": round(ceil, 1), "unit": "GB/s",
            "frac_of_ceiling": round(achieved / ceil, 4) if ceil else None}
        if args.traffic_probe:
            # plain copy of known size (512 MiB read + 512 MiB written), to
            # calibrate the FETCH_SIZE / WRITE_SIZE counters of a profiler run
            src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
        mg.close()
        # ---- mixed precision forms (FP32 V-cycle, 16-bit block inverses, FP64 Krylov)
        if not args.no_mixed:
            precs = [args.mixed] + [q for q in ("bf16", "fp16") if q != args.mixed]
            for q in precs:
                mgm = MG(p, precision=q, use_graph=True)
                mgm.autotune(tune_db)
                timed_steps(mgm, args.warmup, 1e-8)
                tm, im = timed_steps(mgm, args.steps, 1e-8)
                err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
                out["mixed" if q == args.mixed else "mixed_" + q] = {
                    "precision": q, "rtol": 1e-8, "ms_per_step": tm / args.steps,
                    "solves_per_s": args.steps / (tm * 1e-3), "iters": im[-1]["iters"],
                    "true_relres": im[-1]["true_relres"], "err_vs_fp64": err,
                    "vcycle_ms": vcycle_ms(mgm)}
                mgm.close()
    out["n"] = p.n
    return out


def serve_leg(args):
    """Served solves/s and latency percentiles for the stream of independent 2D
    systems (mesh, solid stiffness and inflow drawn per request), mixed
    precision, admission by device-memory budget, continuous batching."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    from paper_1709_05660_amd import Problem, Server
    from synth import config, fourier_coefficients, serving_stream

    reqs = serving_stream(args.serve_n)
    base = config("c2_2d_128x32_mixed")

    def make(r):
        s = base.with_(nx=r.nx, ny=r.ny, levels=r.levels, mu_s=r.mu_s, u_peak=r.u_peak, seed=r.seed)
        return Problem(s, fourier_coefficients(2, r.seed))

    t = time.time()
    with ThreadPoolExecutor(4) as ex:
        probs = list(ex.map(make, reqs))
    build_s = time.time() - t
    budget, slots = args.serve_budget_gb << 30, args.serve_slots

    def run(arrivals):
        srv = Server(hbm_budget_bytes=budget, max_slots=slots)
        done_at = {}
        sub_at = {}
        tickets = [None] * len(probs)
        t0 = time.perf_counter()

        def producer():
            for i, p in enumerate(probs):
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                sub_at[i] = time.perf_counter()
                tickets[i] = srv.submit(p, precision=args.mixed, rtol=1e-8)

        th = threading.Thread(target=producer)
        th.start()
        bad = 0
        iters = []
        while len(done_at) < len(probs):
            for i, tk in enumerate(tickets):
                if tk is None or i in done_at:
                    continue
                st, x, info = srv.poll(tk)
                if st != 2:
                    done_at[i] = time.perf_counter()
                    bad += st != 0
                    if info and "iters" in info:
                        iters.append(info["iters"])
            time.sleep(0.0002)
        th.join()
        stats = srv.stats()
        srv.close()
        lat = np.array([done_at[i] - sub_at[i] for i in range(len(probs))]) * 1e3
        span = max(done_at.values()) - min(sub_at.values())
        return {"solves_per_s": round(len(probs) / span, 2), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2), "failed": int(bad),
                "mean_iters": round(float(np.mean(iters)), 2) if iters else None,
                "max_coresident": stats["max_coresident"], "peak_bytes": stats["peak_bytes"]}

    closed = run([0.0] * len(probs))
    out = {"systems": len(probs), "precision": args.mixed, "rtol": 1e-8,
           "budget_bytes": budget, "max_slots": slots, "host_build_s": round(build_s, 1),
           "closed_loop": closed}
    # the same Poisson stream scaled to 0.7 (the headline), 0.5 and 1.0 of
    # the measured closed-loop rate
    stream_rate = len(reqs) / reqs[-1].arrival_s
    for frac in (0.7, 0.5, 1.0):
        rate = frac * closed["solves_per_s"]
        arrivals = [r.arrival_s * stream_rate / rate for r in reqs]
        out[f"poisson_{frac}x_saturation"] = dict(run(arrivals), rate_per_s=round(rate, 2))
    return out


def cpu_leg(args):
    """The checker as it stands, on a bounded sample: the same step (block and
    coarse factorisation + FGMRES solve) of the same system."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import problem as oprob
    from oracle import solver as osolver
    from synth import config, fourier_coefficients

    spec = config(WORKLOAD)
    h = oprob.build(spec, fourier_coefficients(spec.dim, spec.seed), factor=False)

    def timed(steps):
        t = time.time()
        for _ in range(steps):
            osolver.setup_factors(h.levels)
            oprob.solve(h)
        return time.time() - t

    timed(1)                                   # untimed warm-up (first-touch, library set-up)
    steps = args.cpu_steps
    dt_all = timed(steps)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):          # the same steps on one thread
        dt1 = timed(steps)
    # host memory bandwidth: a STREAM-like triad a = b + 3 c over 128 MB
    # arrays, in two numpy passes (c read, a written; a and b read, a written)
    b_, c_ = np.ones(16 << 20), np.full(16 << 20, 2.0)
    a_ = np.empty_like(b_)
    best = 1e30
    for _ in range(5):
        t = time.perf_counter()
        np.multiply(c_, 3.0, out=a_)
        np.add(a_, b_, out=a_)
        best = min(best, time.perf_counter() - t)
    triad_gbs = 5 * a_.nbytes / best / 1e9
    host = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                host = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # the faster of the two runs is the baseline; both are reported
    best_dt, best_cores = (dt_all, int(threads)) if dt_all <= dt1 else (dt1, 1)
    return {"value": round(steps / best_dt, 4), "unit": "solves/s", "cores": best_cores, "kind": "oracle",
            "sample": f"{steps} full steps (block LU + coarse LU + FGMRES to 1e-10) of {WORKLOAD} after one "
                      f"untimed step, {best_dt:.1f} s",
            "all_threads_value": round(steps / dt_all, 4), "all_threads": int(threads),
            "one_thread_value": round(steps / dt1, 4),
            "host_cpu": host, "host_logical_cpus": os.cpu_count(), "host_triad_gb_s": round(triad_gbs, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prof-steps", type=int, default=2)
    ap.add_argument("--mixed", default="bf16")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--steps-3d", type=int, default=5)
    ap.add_argument("--only-3d", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true")
    ap.add_argument("--serve-n", type=int, default=256)
    ap.add_argument("--serve-budget-gb", type=int, default=4)
    ap.add_argument("--serve-slots", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    if args.only_3d:
        # profiling aid: the 3D leg alone, its own JSON line
        print(json.dumps({"three_d": three_d_leg(args)}), flush=True)
        return
    g = gpu_leg(args)
    value = args.steps / (g["ms_per_step"] * args.steps * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(g["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D steady FSI 128x32 Q2-P1disc, 4 MG levels, 4x4 Schwarz blocks, "
                               "FGMRES(30) rtol 1e-10, FP64 (one Newton step: block inversion + solve)",
                   "unknowns": g["n"]},
        "roofline": g["roofline"],
        "fgmres_iters": g["iters"], "true_relres": g["true_relres"], "converged": g["converged"],
        "vcycle_ms_fp64": round(g["vcycle_ms_fp64"], 4),
        "vcycle_ms_fp64_cold": round(g["vcycle_ms_fp64_cold"], 4),
        "refactor_ms_fp64": round(g["refactor_ms_fp64"], 3), "solve_ms_fp64": round(g["solve_ms_fp64"], 3),
        "dof_per_s": round(value * g["n"], 1),
        "autotune": {"new_measurements": g["autotune_new_measurements"], "seconds": g["autotune_s"],
                     "choices": g["autotune_choices"]},
        "setup_with_upload_ms": round(g["setup_with_upload_ms"], 1),
    }
    if "mixed" in g:
        line["mixed"] = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in g["mixed"].items()}
    for key in sorted(k for k in g if k.startswith("mixed_")):
        line[key] = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in g[key].items()}
    if not args.no_small:
        line["small_c0"] = small_leg(args)
    if not args.no_3d:
        line["three_d"] = three_d_leg(args)
    if not args.no_serve:
        line["served"] = serve_leg(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_leg(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
