"""Benchmark: SPDE field samples/s at 128^3 on one MI355X.

A step is one call of the whole sampling path on one batch: noise -> RT0/P0
mixed solve by block-preconditioned MINRES with a multigrid V-cycle -> L2
projection onto the 2,431,344-tet mesh.  Inputs are resident in HBM before
the timed region.  The headline value is the batched mixed-precision rate
(64 right-hand sides per launch, float32 V-cycle inside float64 MINRES); the
plain float64 rates (batch 64 and batch 1) are reported beside it, with the
same measurements on the 64^3 x 32 and 256^3 x 8 workloads, a serving run,
and the CPU oracle (its timing and the error of every result against it).

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
# the kernel sources and build flags that the counter traffic in profiles/ was taken with
HASHED_SOURCES = ("spde_kernels.hip", "spde_operator.hip", "spde_mg_f32.hip", "spde_mg_f64.hip", "spde_common.inc",
                  "spde_mg.inc", "spde_mg_launch.inc", "spde_vcycle.inc", "spde_launch.inc", "spde_internal.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources and the compiler flags they are built with:
    the counter-measured traffic in profiles/ holds only for that build."""
    h = hashlib.sha256()
    for f in HASHED_SOURCES:
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


def roofline_from(rep, traffic, kernel=None):
    # the dominant kernel by total time inside the timed region (or the one named)
    name, r = (kernel, rep[kernel]) if kernel else max(rep.items(), key=lambda kv: kv[1]["total_ms"])
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


def vcycle_counter_gbs(rep, traffic):
    """(FETCH + WRITE bytes) / time aggregated over the V-cycle kernels, with the
    counter bytes per dispatch of profiles/traffic.json and this run's times."""
    mg = (traffic or {}).get("vcycle")
    if not mg:
        return None
    ms = sum(rep[k]["total_ms"] for k in mg if k in rep)
    by = sum(mg[k] * rep[k]["launches"] for k in mg if k in rep)
    return round(by / (ms * 1e-3) / 1e9, 1) if ms > 0 else None


def copy_bandwidth(torch, dev, mib=1024):
    """A plain device copy of `mib` MiB (read + write), the achievable streaming rate."""
    nb = mib << 20
    src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del src, dst
    return round(2 * nb / (ms * 1e-3) / 1e9, 1)


def kernel_table(rep):
    return {k: {"avg_ms": round(v["total_ms"] / v["launches"], 4), "launches": v["launches"],
                "gbs": round(v["bytes_per_launch"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e9, 1)
                if v["bytes_per_launch"] else None}
            for k, v in rep.items()}


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return model, cores


def oracle_leg(main_w, xi_np, fields, mesh, cpu_rows):
    """The oracle on the host's cores: its timing (the method's preconditioned
    MINRES route on one noise vector of the workload, its closed-form spectral
    solve on all of them, the overlap rows of a sample of tets and their
    product), and the error of every GPU result against it."""
    import oracle
    from oracle import discretize, minres, transfer
    model, cores = cpu_info()
    n, kappa, g = main_w.n, main_w.kappa, main_w.g
    ops = discretize.assemble(n)
    F = discretize.rhs(ops, g, xi_np[0])
    t0 = time.perf_counter()
    _, _, it = minres.solve(ops, kappa, F, tol=3e-11)
    t_minres = time.perf_counter() - t0
    t0 = time.perf_counter()
    u_ref = oracle.sample_box(n, kappa, g, xi_np)
    t_spec = time.perf_counter() - t0
    # transfer: exact overlap rows of a sample of tets, and their product
    xyz, tets = mesh
    rows = np.sort(np.random.default_rng(7).choice(tets.shape[0], cpu_rows, replace=False))
    t0 = time.perf_counter()
    Pi = transfer.build_pi(xyz, tets, n, rows=rows)
    t_build = time.perf_counter() - t0
    ut_ref = transfer.apply(Pi, u_ref)
    vol = np.array([transfer.tet_volume(xyz[tets[r]]) for r in rows])
    # the product at the mesh's size: a matrix of its row count made of the
    # sampled rows repeated (same entries per row), applied to one field
    import scipy.sparse as sp
    reps = -(-tets.shape[0] // rows.size)
    Pi_full = sp.vstack([Pi] * reps, format="csr")[:tets.shape[0]]
    transfer.apply(Pi_full, u_ref[0])
    t0 = time.perf_counter()
    for _ in range(3):
        transfer.apply(Pi_full, u_ref[0])
    apply_per_sample = (time.perf_counter() - t0) / 3
    del Pi_full
    errors = {}
    for key, (u_box, u_tet) in fields.items():
        e_box = [float(np.linalg.norm(u_box[b] - u_ref[b]) / np.linalg.norm(u_ref[b])) for b in range(u_ref.shape[0])]
        e_tet = [float(np.sqrt(np.sum(vol * (u_tet[b][rows] - ut_ref[b]) ** 2) / np.sum(vol * ut_ref[b] ** 2)))
                 for b in range(u_ref.shape[0])]
        errors[key] = {"box_rel_l2_max": max(e_box), "tet_vol_rel_l2_max": max(e_tet),
                       "bar": 1e-10 if key == "fp64" else 1e-7}
    per_sample = t_minres + apply_per_sample
    return {
        "value": round(1.0 / per_sample, 5), "unit": "samples/s", "cores": cores, "kind": "oracle",
        "sample": f"1 of the {xi_np.shape[0]} noise vectors of the {n}^3 workload through the oracle's preconditioned "
                  f"MINRES (SciPy sparse operator, exact DCT Schur preconditioner, rtol 3e-11, {it} iterations): "
                  f"{t_minres:.1f} s; plus the product with a transfer matrix of the mesh's {tets.shape[0]} rows "
                  f"(the oracle's exact rows of {rows.size} sampled tets, repeated): "
                  f"{apply_per_sample * 1e3:.1f} ms per sample",
        "cpu_model": model, "omp_num_threads": os.environ.get("OMP_NUM_THREADS", "unset"),
        "fft_workers": "all cores (scipy.fft workers=-1)",
        "sparse_note": "SciPy sparse matrix-vector products run on one thread",
        "spectral_exact_samples_per_s": round(xi_np.shape[0] / t_spec, 3),
        "spectral_note": f"closed-form DCT solve (valid only for this constant-coefficient box), "
                         f"{xi_np.shape[0]} vectors in {t_spec:.1f} s",
        "transfer_rows_build_ms_per_row": round(t_build / rows.size * 1e3, 3),
        "transfer_apply_ms_per_sample": round(apply_per_sample * 1e3, 3),
        "err_vs_oracle": errors,
        "err_note": f"every sample of the batch: box relative L2 against the exact spectral solve; tets: volume-weighted "
                    f"relative L2 over the {rows.size} sampled rows of the oracle's exact overlap matrix",
    }


def field_errors(w, fields, mesh, nrows):
    """Error of every result of a workload against the oracle: box relative L2
    (exact spectral solve) and, with a mesh, the volume-weighted relative L2
    over nrows sampled tets of the oracle's exact overlap matrix."""
    import oracle
    from oracle import transfer
    u_ref = oracle.sample_box(w.n, w.kappa, w.g, w.noise())
    rows = Pi = vol = None
    if mesh is not None:
        xyz, tets = mesh
        rows = np.sort(np.random.default_rng(7).choice(tets.shape[0], nrows, replace=False))
        Pi = transfer.build_pi(xyz, tets, w.n, rows=rows)
        vol = np.array([transfer.tet_volume(xyz[tets[r]]) for r in rows])
        ut_ref = transfer.apply(Pi, u_ref)
    out = {}
    for p, (u_box, u_tet) in fields.items():
        e = {"box_rel_l2_max": max(float(np.linalg.norm(u_box[b] - u_ref[b]) / np.linalg.norm(u_ref[b]))
                                   for b in range(u_ref.shape[0])),
             "bar": 1e-10 if p == "fp64" else 1e-7}
        if rows is not None and u_tet is not None:
            e["tet_vol_rel_l2_max"] = max(
                float(np.sqrt(np.sum(vol * (u_tet[b][rows] - ut_ref[b]) ** 2) / np.sum(vol * ut_ref[b] ** 2)))
                for b in range(u_ref.shape[0]))
            e["tet_rows"] = int(rows.size)
        out[p] = e
    return out


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
    rep = srv.run(arrivals, time_limit=seconds * 3 + 30, progress_every=5.0)
    rep["rates_per_s"] = rates
    rep["rate_scale"] = scale
    rep["arrival_window_s"] = seconds
    rep["offered_requests"] = len(arrivals)
    del srv
    torch.cuda.empty_cache()
    return rep


def run_workload(torch, P, w, dev, steps, warmup, mesh, detail, only=None):
    """Time the batched path on one workload in both precisions (timed mode 2:
    graphs with the operator pass sampled by event pairs).  detail: also the
    per-kernel breakdown, the generated-noise, cell-wise kappa, refined and
    batch-1 variants.  Returns per precision a dict (u fields of one call kept
    for the oracle check)."""
    from workloads import coefficient_field
    xi = torch.tensor(w.noise(), device=dev)
    res = {}
    setup = {}
    csr = None
    if mesh is not None:
        t0 = time.perf_counter()
        csr = P.build_transfer_host(w.n, *mesh)
        setup["transfer_build_s"] = round(time.perf_counter() - t0, 2)
        setup["n_tet"], setup["nnz"] = int(csr[0].size - 1), int(csr[1].size)
        if detail:
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
    for prec in ((only,) if only else ("mixed", "fp64")):
        box = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=w.batch, device=dev)
        if csr is not None:
            box.set_transfer(*csr)
        log(f"{w.name} {prec}: timing batch {w.batch}")
        dt, iters, rep = time_steps(torch, box, xi, steps, warmup, timing=2)
        r = {"s_per_step": dt, "samples_per_s": w.batch / dt, "iters_mean": float(iters.mean()),
             "iters_max": int(iters.max()), "report": rep, "tiles": box.info()["tiles"]}
        res[prec] = r
        log(f"{w.name} {prec}: {w.batch / dt:.1f} samples/s, {dt * 1e3:.1f} ms/step, iters {iters.mean():.1f}, "
            f"operator avg {rep['operator']['total_ms'] / rep['operator']['launches']:.4f} ms, tiles {r['tiles']}")
        # one call's fields for the oracle check
        out = box.sample(xi, u_box=True, relres=True)
        r["relres_max"] = float(out["relres"].max())
        r["u_box"] = out["u_box"].cpu().numpy()
        r["u_tet"] = out["u_tet"].cpu().numpy() if "u_tet" in out else None
        del out
        if only or not detail:
            del box
            torch.cuda.empty_cache()
            continue
        # per-kernel breakdown outside the timed region: plain launches with an
        # event pair around every kernel
        rep_all = time_steps(torch, box, xi, 2, 1, timing=1)[2]
        r["report_all"] = rep_all
        for k, v in sorted(rep_all.items(), key=lambda kv: -kv[1]["total_ms"]):
            avg = v["total_ms"] / v["launches"]
            gbs = v["bytes_per_launch"] / (avg * 1e-3) / 1e9 if v["bytes_per_launch"] else 0.0
            log(f"   {k:14s} {v['total_ms'] / 2:9.2f} ms/step  {v['launches']:6d} launches  "
                f"avg {avg:8.4f} ms  {gbs:8.1f} GB/s")
        sd_steps = max(3, steps // 2)
        # the same batch with the noise drawn inside the initialisation kernel
        box.sample_seeded(2024, 0, w.batch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(sd_steps):
            box.sample_seeded(2024, k * w.batch, w.batch)
        torch.cuda.synchronize()
        r["seeded_samples_per_s"] = w.batch * sd_steps / (time.perf_counter() - t0)
        # space-dependent correlation length: kappa(x) spanning [kappa/2, 2 kappa]
        # with g(x) for unit marginal variance; the multigrid takes the cell-wise
        # kappa (Galerkin coarse kappa^2)
        kf = coefficient_field(w.n, w.kappa / 2, 2 * w.kappa, 5)
        variable = {}
        for mg, kref in (("cellwise_multigrid", 0.0), ("constant_multigrid", float(np.sqrt(kf.min() * kf.max())))):
            box.set_coefficients(kf, np.sqrt(8 * np.pi * kf), kappa_ref=kref)
            out = box.sample(xi)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(sd_steps):
                out = box.sample(xi)
            torch.cuda.synchronize()
            variable[mg] = {"samples_per_s": round(w.batch * sd_steps / (time.perf_counter() - t0), 2),
                            "iterations": float(out["iters"].mean())}
        variable["kappa_range"] = [float(kf.min()), float(kf.max())]
        r["variable"] = variable
        box.set_coefficients()
        log(f"{w.name} {prec}: cell-wise kappa: {variable}")
        if prec == "mixed":
            # float64 iterative refinement to a true residual of 1e-11
            box.set_refinement(1e-11, 3)
            out = box.sample(xi, relres=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(sd_steps):
                out = box.sample(xi, relres=True)
            torch.cuda.synchronize()
            r["refined"] = {"samples_per_s": round(w.batch * sd_steps / (time.perf_counter() - t0), 2),
                            "iterations": float(out["iters"].mean()), "relres_max": float(out["relres"].max()),
                            "target": 1e-11}
            box.set_refinement(0.0, 0)
        else:
            # plain float64 solved to the same true-residual target, for the
            # comparison with the refined mixed path above
            boxr = P.Box(w.n, w.kappa, w.g, precision=prec, rtol=1e-11, max_batch=w.batch, device=dev)
            if csr is not None:
                boxr.set_transfer(*csr)
            out = boxr.sample(xi, relres=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(sd_steps):
                out = boxr.sample(xi, relres=True)
            torch.cuda.synchronize()
            r["to_1e-11"] = {"samples_per_s": round(w.batch * sd_steps / (time.perf_counter() - t0), 2),
                             "iterations": float(out["iters"].mean()), "relres_max": float(out["relres"].max()),
                             "rtol": 1e-11}
            del boxr
        del box
        torch.cuda.empty_cache()
        # one sample per call on a single-sample sampler (its own tiles), same path
        box1 = P.Box(w.n, w.kappa, w.g, precision=prec, max_batch=1, device=dev)
        if csr is not None:
            box1.set_transfer(*csr)
        x1 = xi[:1].contiguous()
        dt1, _, _ = time_steps(torch, box1, x1, max(3, steps // 2), 1)
        r["batch1_samples_per_s"] = 1.0 / dt1
        log(f"{w.name} {prec}: batch 1: {1.0 / dt1:.1f} samples/s")
        del box1
        torch.cuda.empty_cache()
    return res, setup


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["box16", "box64", "box128", "box256"], default="box128",
                    help="named workload of the headline line (the other sizes are reported in 'workloads')")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-mesh", action="store_true", help="skip the tet transfer (solve only)")
    ap.add_argument("--no-other", action="store_true", help="skip the 64^3 x 32 and 256^3 x 8 workloads")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one precision of the headline workload only (profiling runs)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="arrival window of the serving load run reported beside the throughput (0: skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0, help="request-rate multiplier of the serving run")
    ap.add_argument("--cpu-rows", type=int, default=600, help="tet rows of the oracle's transfer sample")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this sampler runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1712_06758_amd as P
    from workloads import WORKLOADS

    w = WORKLOADS[args.workload]
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
    copy_gbs = copy_bandwidth(torch, dev)
    log(f"device copy (read + write): {copy_gbs} GB/s")
    log(f"workload {w.name}: n={w.n} batch={w.batch} kappa={w.kappa} g={w.g:.4f}")
    mesh = None if args.no_mesh else w.mesh()
    results, setup = run_workload(torch, P, w, dev, args.steps, args.warmup, mesh, detail=True, only=args.only)

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
        "fp64_to_1e-11": fp.get("to_1e-11"),
        "mixed_over_fp64": round(mx["samples_per_s"] / fp["samples_per_s"], 3),
        "batched_mixed_over_plain_fp64_batch1": round(mx["samples_per_s"] / fp["batch1_samples_per_s"], 3),
        "iterations": {"mixed": mx["iters_mean"], "fp64": fp["iters_mean"]},
        "tiles": {"mixed": mx["tiles"], "fp64": fp["tiles"]},
        "copy_kernel_gbs": copy_gbs,
        "vcycle_hbm_gbs": {"mixed": vcycle_gbs(mx["report_all"]), "fp64": vcycle_gbs(fp["report_all"])},
        "vcycle_counter_gbs": {"mixed": vcycle_counter_gbs(mx["report_all"], traffic.get("mixed") if traffic else None),
                               "fp64": vcycle_counter_gbs(fp["report_all"], traffic.get("fp64") if traffic else None)},
        "roofline": roof,
        "roofline_fp64": roofline_from(fp["report"], traffic.get("fp64") if traffic else None),
        "kernels": {p: kernel_table(results[p]["report_all"]) for p in results},
        "setup": setup,
    }
    fields = {f"{w.name}:{p}": (results[p]["u_box"], results[p]["u_tet"]) for p in results}
    if not args.no_other:
        others = {}
        for name in ("box64", "box256"):
            ow = WORKLOADS[name]
            log(f"workload {name}: n={ow.n} batch={ow.batch} kappa={ow.kappa}")
            res, st = run_workload(torch, P, ow, dev, max(3, args.steps // 2), 1, None if args.no_mesh else ow.mesh(),
                                   detail=False)
            others[name] = {
                "config": f"{ow.n}^3 box, lambda={ow.corr_len}, batch {ow.batch}, transfer to {st.get('n_tet', 0)} tets",
                "setup": st}
            for p, r in res.items():
                rf = roofline_from(r["report"], None, kernel="operator")
                others[name][p] = {"samples_per_s": round(r["samples_per_s"], 2), "iterations": r["iters_mean"],
                                   "ms_per_step": round(r["s_per_step"] * 1e3, 3), "relres_max": r["relres_max"],
                                   "operator_frac": rf["frac"], "operator_gbs": rf["achieved"]}
                fields[f"{name}:{p}"] = (r["u_box"], r["u_tet"])
        line["workloads"] = others
    if args.serve_seconds > 0:
        log(f"serving run: {args.serve_seconds} s at {args.serve_scale} x the request mix")
        line["serving"] = serving_run(args.serve_seconds, args.serve_scale)
    if not args.no_cpu:
        log("oracle leg (CPU)")
        by_w = {}
        for key, fu in fields.items():
            by_w.setdefault(key.split(":")[0], {})[key.split(":")[1]] = fu
        cb = None
        errs = {}
        for name, fs in by_w.items():
            ow = WORKLOADS[name]
            if name == w.name:
                cb = oracle_leg(ow, ow.noise(), fs, mesh if mesh is not None else ow.mesh(), args.cpu_rows)
                errs[name] = cb.pop("err_vs_oracle")
            else:
                errs[name] = field_errors(ow, fs, None if args.no_mesh else ow.mesh(), max(100, args.cpu_rows // 3))
            log(f"errors against the oracle, {name}: {errs[name]}")
        line["cpu_baseline"] = cb
        line["err_vs_oracle"] = errs
        line["err_vs_oracle_max"] = {p: max(errs[name][p]["box_rel_l2_max"] for name in errs if p in errs[name])
                                     for p in ("mixed", "fp64")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
