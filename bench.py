"""Benchmark: SPDE field samples/s at 128^3 on one MI355X.

A step is one call of the whole sampling path on one batch: noise -> RT0/P0
mixed solve by block-preconditioned MINRES with a multigrid V-cycle -> L2
projection onto the 2,431,344-tet mesh.  Inputs are resident in HBM before
the timed region.  The headline value is the batched mixed-precision rate
(64 right-hand sides per launch, float32 V-cycle inside float64 MINRES); the
plain float64 rates (batch 64 and batch 1) are reported beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources and the compiler flags they are built with:
    the counter-measured traffic in profiles/ holds only for that build."""
    h = hashlib.sha256()
    for f in ("spde_kernels.hip", "spde_vcycle.inc", "spde_launch.inc", "spde_internal.h"):
        with open(os.path.join(ROOT, "paper_1712_06758_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    from paper_1712_06758_amd.build import FLAGS
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()[:16]


def time_steps(torch, box, xi, steps, warmup, timing=0):
    """timing: 0 none; 1 every kernel class (plain launches); 2 the operator pass
    only, its events recorded inside the iteration graphs."""
    if timing:
        box.timing(timing)       # graphs are captured (with their event nodes) in the warm-up
    for _ in range(warmup):
        box.sample(xi)
    torch.cuda.synchronize()
    if timing:
        box.timing(-1)           # clear the totals; the mode and the graphs stay
    iters = []
    t0 = time.perf_counter()
    for _ in range(steps):
        out = box.sample(xi)
        iters.append(out["iters"].copy())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = None
    if timing:
        box.timing(0)
        rep = box.timing_report()
    return (t1 - t0) / steps, np.concatenate(iters), rep


def roofline_from(rep, traffic):
    # dominant kernel by total time inside the timed region
    name, r = max(rep.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = r["total_ms"] / r["launches"]
    achieved = r["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
    tr = None
    if traffic and traffic.get("kernel") == name:
        tr = traffic.get("bytes_per_launch")
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": tr,
            "avg_ms": round(avg_ms, 4), "bytes_per_launch": r["bytes_per_launch"]}


def vcycle_gbs(rep):
    ms = sum(rep[k]["total_ms"] for k in rep if k.startswith("mg_"))
    by = sum(rep[k]["bytes_per_launch"] * rep[k]["launches"] for k in rep if k.startswith("mg_"))
    return round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None


def cpu_baseline(n, kappa, g, xi_np):
    """The oracle on the host's cores: its block-preconditioned MINRES route
    (the method, with the exact DCT Schur preconditioner, to the same relative
    tolerance as the float64 GPU path) on one noise vector of the workload, and
    its closed-form spectral solve on all of them."""
    import oracle
    from oracle import discretize, minres
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    ops = discretize.assemble(n)
    F = discretize.rhs(ops, g, xi_np[0])
    t0 = time.perf_counter()
    _, _, it = minres.solve(ops, kappa, F, tol=3e-11)
    t_minres = time.perf_counter() - t0
    t0 = time.perf_counter()
    for b in range(xi_np.shape[0]):
        oracle.sample_box(n, kappa, g, xi_np[b])
    t_spec = time.perf_counter() - t0
    return {"value": round(1.0 / t_minres, 5), "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"1 of the {xi_np.shape[0]} noise vectors of the {n}^3 workload through the oracle's preconditioned "
                      f"MINRES (SciPy sparse operator, exact DCT Schur preconditioner, rtol 3e-11, {it} "
                      f"iterations): {t_minres:.1f} s; transfer apply not included",
            "spectral_exact_samples_per_s": round(xi_np.shape[0] / t_spec, 3),
            "spectral_note": f"closed-form DCT solve (valid only for this constant-coefficient box), "
                             f"{xi_np.shape[0]} vectors in {t_spec:.1f} s"}


def serving_run(seconds, scale):
    """MLMC serving load: levels 32/64/128/256 with Poisson arrivals in the
    1000:250:60:15 per-second mix (times `scale`), continuous batching, mixed precision."""
    import torch
    from paper_1712_06758_amd.serve import build_gpu_server
    from workloads import SERVE_LEVELS, SERVE_CORR_LEN, poisson_arrivals
    levels = sorted(SERVE_LEVELS)
    srv = build_gpu_server(levels, SERVE_CORR_LEN, "mixed")
    srv.run([(0.0, n, 10 ** 6 + i) for i, n in enumerate(levels)])   # warm-up, not reported
    srv.done.clear()
    srv.queue_depth.clear()
    rates = {n: SERVE_LEVELS[n] * scale for n in levels}
    arrivals = poisson_arrivals(rates, seconds, seed=2)
    rep = srv.run(arrivals, time_limit=seconds * 4 + 30, progress_every=2.0)
    rep["rates_per_s"] = rates
    rep["arrival_window_s"] = seconds
    del srv
    torch.cuda.empty_cache()
    return rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["box16", "box64", "box128", "box256"], default="box128",
                    help="named workload (the 16^3 x 1, 64^3 x 32 and 256^3 x 8 configurations beside the default)")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-mesh", action="store_true", help="skip the tet transfer (solve only)")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="length of the serving load run reported beside the throughput (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=0.5, help="request-rate multiplier of the serving run")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this sampler runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1712_06758_amd as P
    from workloads import WORKLOADS, Workload, coefficient_field

    w = WORKLOADS[args.workload]
    if args.workload == "box128" and (args.n != 128 or args.batch != 64):
        w = Workload(f"box{args.n}", args.n, w.corr_len, args.batch, w.mesh_lo, w.mesh_hi,
                     max(2, round(w.mesh_m * args.n / 128)), 0.0)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mib} MiB done")
        del src, dst
    log(f"workload {w.name}: n={w.n} batch={w.batch} kappa={w.kappa} g={w.g:.4f}")
    t0 = time.perf_counter()
    xi_np = w.noise()
    xi = torch.tensor(xi_np, device=dev)
    log(f"noise generated in {time.perf_counter() - t0:.1f} s")

    mesh = None if args.no_mesh else w.mesh()
    results = {}
    setup = {}
    for prec in ((args.only,) if args.only else ("mixed", "fp64")):
        box = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=w.batch, device=dev)
        if mesh is not None:
            t0 = time.perf_counter()
            nt, nnz = box.set_mesh(*mesh)
            setup["transfer_build_s"] = round(time.perf_counter() - t0, 2)
            setup["n_tet"], setup["nnz"] = int(nt), int(nnz)
            if "transfer_build_device_s" not in setup:
                # the same matrix built by the device clipper (mesh upload included;
                # the first call also loads the kernels)
                P.build_transfer_device(w.n, *mesh, device=dev)
                torch.cuda.synchronize(dev)
                t0 = time.perf_counter()
                rp_d, _, _ = P.build_transfer_device(w.n, *mesh, device=dev)
                torch.cuda.synchronize(dev)
                setup["transfer_build_device_s"] = round(time.perf_counter() - t0, 4)
                setup["transfer_device_nnz"] = int(rp_d[-1].item())
                del rp_d
        log(f"{prec}: timing batch {w.batch}")
        # the timed region runs as in production (iteration graphs), with the
        # operator pass bracketed by event pairs recorded inside the graphs
        dt, iters, rep = time_steps(torch, box, xi, args.steps, args.warmup, timing=2)
        results[prec] = {"s_per_step": dt, "samples_per_s": w.batch / dt, "iters_mean": float(iters.mean()),
                         "iters_max": int(iters.max()), "report": rep}
        log(f"{prec}: {w.batch / dt:.1f} samples/s, {dt * 1e3:.1f} ms/step, iters {iters.mean():.1f}, "
            f"operator avg {rep['operator']['total_ms'] / rep['operator']['launches']:.4f} ms, info {box.info()}")
        # per-kernel breakdown outside the timed region: plain launches with an
        # event pair around every kernel
        rep_all = rep if args.only else time_steps(torch, box, xi, 2, 1, timing=1)[2]
        results[prec]["report_all"] = rep_all
        for k, v in sorted(rep_all.items(), key=lambda kv: -kv[1]["total_ms"]):
            avg = v["total_ms"] / v["launches"]
            gbs = v["bytes_per_launch"] / (avg * 1e-3) / 1e9 if v["bytes_per_launch"] else 0.0
            log(f"   {k:14s} {v['total_ms'] / 2:9.2f} ms/step  {v['launches']:6d} launches  "
                f"avg {avg:8.4f} ms  {gbs:8.1f} GB/s")
        if args.only:
            results[prec]["batch1_samples_per_s"] = float("nan")
            del box
            continue
        # the same batch with the noise drawn inside the initialisation kernel
        # (counter-based generator) instead of read from memory
        sd_steps = max(3, args.steps // 2)
        box.sample_seeded(2024, 0, w.batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(sd_steps):
            box.sample_seeded(2024, k * w.batch, w.batch)
        torch.cuda.synchronize()
        results[prec]["seeded_samples_per_s"] = w.batch * sd_steps / (time.perf_counter() - t0)
        log(f"{prec}: generated noise: {results[prec]['seeded_samples_per_s']:.1f} samples/s")
        # space-dependent correlation length: kappa(x) spanning [kappa/2, 2 kappa] with
        # g(x) for unit marginal variance, the preconditioner at the geometric-mean kappa
        kf = coefficient_field(w.n, w.kappa / 2, 2 * w.kappa, 5)
        box.set_coefficients(kf, np.sqrt(8 * np.pi * kf))
        out = box.sample(xi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(sd_steps):
            out = box.sample(xi)
        torch.cuda.synchronize()
        results[prec]["variable"] = {"samples_per_s": round(w.batch * sd_steps / (time.perf_counter() - t0), 2),
                                     "iterations": float(out["iters"].mean()),
                                     "kappa_range": [float(kf.min()), float(kf.max())],
                                     "kappa_ref": round(box.kappa_ref, 4)}
        box.set_coefficients()
        log(f"{prec}: cell-wise kappa: {results[prec]['variable']}")
        # true residual of the plain solve, and for the mixed path float64
        # iterative refinement to a true residual of 1e-11 (float64 accuracy):
        # correction solves on F - A U with the float32 multigrid
        out = box.sample(xi, relres=True)
        results[prec]["relres_max"] = float(out["relres"].max())
        if prec == "mixed":
            box.set_refinement(1e-11, 3)
            out = box.sample(xi, relres=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(sd_steps):
                out = box.sample(xi, relres=True)
            torch.cuda.synchronize()
            results[prec]["refined"] = {
                "samples_per_s": round(w.batch * sd_steps / (time.perf_counter() - t0), 2),
                "iterations": float(out["iters"].mean()), "relres_max": float(out["relres"].max()),
                "target": 1e-11}
            box.set_refinement(0.0, 0)
            log(f"{prec}: refined to 1e-11: {results[prec]['refined']}")
        info = box.info()
        results[prec]["info"] = info
        del box
        torch.cuda.empty_cache()
        # one sample per call on a single-sample sampler (its own tiles), same path
        box1 = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=1, device=dev)
        if mesh is not None:
            box1.set_mesh(*mesh)
        x1 = xi[:1].contiguous()
        b1_steps = max(3, args.steps // 2)
        dt1, it1, _ = time_steps(torch, box1, x1, b1_steps, 1)
        results[prec]["batch1_samples_per_s"] = 1.0 / dt1
        log(f"{prec}: batch 1: {1.0 / dt1:.1f} samples/s, tiles {box1.info()['tiles']}")
        del box1
        torch.cuda.empty_cache()

    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            t = json.load(fh)
        # the counters were taken on the 128^3 x 64 workload
        if t.get("source_hash") == kernel_source_hash() and w.name == "box128" and w.batch == 64:
            traffic = t

    if args.only:
        r = results[args.only]
        print(json.dumps({"mode": "profile", "precision": args.only, "samples_per_s": r["samples_per_s"]}))
        return
    mx = results["mixed"]
    fp = results["fp64"]
    roof = roofline_from(mx["report"], traffic.get("mixed") if traffic else None)
    line = {
        "metric": f"field samples/s at {w.n}^3 (batched mixed precision, whole path: solve + projection)",
        "value": round(mx["samples_per_s"], 2),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["s_per_step"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 MINRES + f32 multigrid",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n}^3 box on [0,1]^3, lambda={w.corr_len}, kappa={w.kappa}, "
                               f"batch {w.batch} seeded N(0,1) noise vectors, transfer to "
                               f"{setup.get('n_tet', 0)}-tet jittered Kuhn mesh of [0.1,0.9]^3",
                   "n": w.n, "batch": w.batch, "rtol_mixed": 1e-8, "rtol_fp64": 3e-11},
        "fp64_samples_per_s": round(fp["samples_per_s"], 2),
        "fp64_batch1_samples_per_s": round(fp["batch1_samples_per_s"], 2),
        "mixed_batch1_samples_per_s": round(mx["batch1_samples_per_s"], 2),
        "device_noise_samples_per_s": {"mixed": round(mx["seeded_samples_per_s"], 2),
                                       "fp64": round(fp["seeded_samples_per_s"], 2)},
        "cellwise_kappa": {"mixed": mx["variable"], "fp64": fp["variable"]},
        "true_relres_max": {"mixed": mx["relres_max"], "fp64": fp["relres_max"]},
        "mixed_refined_to_1e-11": mx["refined"],
        "mixed_over_fp64": round(mx["samples_per_s"] / fp["samples_per_s"], 3),
        "batched_mixed_over_plain_fp64_batch1": round(mx["samples_per_s"] / fp["batch1_samples_per_s"], 3),
        "iterations": {"mixed": mx["iters_mean"], "fp64": fp["iters_mean"]},
        "vcycle_hbm_gbs": {"mixed": vcycle_gbs(mx["report_all"]), "fp64": vcycle_gbs(fp["report_all"])},
        "roofline": roof,
        "roofline_fp64": roofline_from(fp["report"], traffic.get("fp64") if traffic else None),
        "kernels": {p: {k: {"avg_ms": round(v["total_ms"] / v["launches"], 4),
                            "gbs": round(v["bytes_per_launch"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e9, 1)
                            if v["bytes_per_launch"] else None}
                        for k, v in results[p]["report_all"].items()} for p in results},
        "setup": setup,
    }
    if args.serve_seconds > 0:
        log(f"serving run: {args.serve_seconds} s at {args.serve_scale} x the request mix")
        line["serving"] = serving_run(args.serve_seconds, args.serve_scale)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(w.n, w.kappa, w.g, xi_np)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
