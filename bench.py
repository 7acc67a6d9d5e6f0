"""Benchmark: time and iterations of a gPLMM-preconditioned Newton-FGMRES
solve to 1e-8 relative residual on a 128^3 steady Navier-Stokes sphere
packing, plus the HBM bandwidth of the preconditioner's dominant kernel.

One step = one gplmm_newton_solve from x = 0: preconditioner builds (local
factorisations, shape vectors, coarse operator), every Newton iteration and
every FGMRES iteration.  The geometry setup (decomposition, uploads) happens
once before the warm-up and is reported separately.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time & iters to 1e-8 rel. residual, 128³ steady NS; precond-apply HBM GB/s"
HBM_PEAK_GBS = 8000.0


def _cpu_baseline(workload, crop):
    """The FP64 oracle, untuned, on a bounded sample: the full Newton-FGMRES-
    gPLMM solve of a crop^3 corner of the same packing, one thread, scaled to
    the full image by its number of unknowns (linear scaling, which favours
    the CPU)."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle.mac import MacGrid, Operators, Phys
    from oracle.decomp import decompose, largest_component
    from oracle import newton

    m = workload["mask"][:crop, :crop, :crop].copy()
    lab = workload["labels"][:crop, :crop, :crop].copy()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        g = MacGrid(largest_component(m))
        ops = Operators(g)
        dc = decompose(g, lab)
        ph = Phys(workload["rho"], workload["mu"], workload["body"], None, dc.pin)
        x, st = newton.solve(ops, dc, ph, tol=1e-8, lin_tol=1e-9)
        el = time.perf_counter() - t0
    full = MacGrid(largest_component(workload["mask"]))
    scale = full.N / g.N
    return dict(value=el * scale, unit="s", cores=1, kind="oracle",
                sample="full oracle solve (setup + Newton-FGMRES-gPLMM to 1e-8) of the %d^3 corner "
                       "crop (N=%d, %d Newton / %d FGMRES its, %.1f s), scaled by N ratio %.1f to "
                       "N=%d" % (crop, g.N, st.newton_its, sum(st.lin_its), el, scale, full.N),
                converged=bool(st.converged))


def _measured_traffic(workload, precision):
    """HBM bytes per launch of the skyline-solve kernel from the committed PMC summary, if
    it was taken on this workload and precision with the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "trsv_sub_kernel_traffic_%s_%s.txt" % (workload, precision))
    src = os.path.join(ROOT, "paper_2510_22077_amd", "csrc", "lu.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha:
        return None
    return float(kv["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spheres3d_128")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--restart", type=int, default=256)
    ap.add_argument("--cpu-crop", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true",
                    help="skip the comparison solve with the plain FP64 preconditioner")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-cal", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, five times (the reference "
                         "point for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.copy_cal:
        import torch
        n = args.copy_cal // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path (it would shard "
              "by subdomain: whole pores per GPU, one halo exchange per stencil application)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from synth import make_workload
    from paper_2510_22077_amd import Solver

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    w = make_workload(args.workload, args.seed)
    log("workload %s generated in %.1f s" % (args.workload, time.perf_counter() - t0))
    t0 = time.perf_counter()
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"],
               precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = s.info()
    log("setup %.1f s: %s" % (setup_s, json.dumps(info)))
    tuning = None
    if not args.no_autotune:
        s.build()
        tuning = s.autotune()
        log("autotune: %s" % json.dumps(tuning))

    for k in range(args.warmup):
        x, st = s.newton_solve()
        torch.cuda.synchronize()
        log("warmup %d: %s" % (k, json.dumps({a: st[a] for a in ("newton_its", "lin_its", "t_total_ms")})))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        x, st = s.newton_solve()
        stats.append(st)
        log("step %d: %s" % (k, json.dumps({a: st[a] for a in ("newton_its", "lin_its", "t_build_ms",
                                                                "t_solve_ms", "t_total_ms")})))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = stats[-1]
    sec = el / args.steps
    # one more solve with per-launch event timers (kernel by kernel, no graph replay) for
    # the kernel-level figures; not part of the timed steps
    s.reset_timers()
    s.set_timing(True)
    xt, stt = s.newton_solve()
    torch.cuda.synchronize()
    s.set_timing(False)
    log("timed solve: %s" % json.dumps({a: stt[a] for a in ("newton_its", "lin_its", "t_total_ms")}))

    # achieved Reynolds number Re = rho U l / mu, U = U_D / phi, l = V_s / A_w
    nrec = info["nrec"]
    xr = x.view(-1, nrec)
    mask = w["mask"].astype(bool)
    nvox = mask.size
    ud = float(xr[:, 0].sum().item()) / nvox
    phi = mask.mean()
    from synth.workloads import _surface_area
    aw = _surface_area(mask)
    l = (nvox - mask.sum()) / aw
    re = w["rho"] * (ud / phi) * l / w["mu"]

    kt = {k: s.kernel_time(k) for k in ("trsv_p", "trsv_d", "precond_apply", "jv", "arnoldi")}
    tr = kt["trsv_p"]   # trsv_sub_kernel: the primary grids' solves, the dominant launch
    achieved = tr["bytes"] / (tr["avg_ms"] * 1e-3) / 1e9 if tr["avg_ms"] > 0 else 0.0
    ap_ = kt["precond_apply"]
    apply_gbs = ap_["bytes"] / (ap_["avg_ms"] * 1e-3) / 1e9 if ap_["avg_ms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 preconditioner, f64 Newton/FGMRES/coarse" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: 128^3 lognormal sphere packing (mean r 8, sigma 0.3), porosity %.3f, "
                               "seed %d, body force for Re~1, periodic x, steady NS" % (args.workload, phi, args.seed),
                   "unknowns": info["N"], "pores": info["Np"], "interfaces": info["Nc"],
                   "precision": args.precision, "restart": args.restart},
        "newton_its": st["newton_its"],
        "fgmres_its": st["lin_its"],
        "fgmres_its_total": st["lin_its_total"],
        "gs_reorth_steps": st["gs_reorth"],
        "newton_res_hist": st["res_hist"],
        "final_rel_residual": st["res_hist"][-1],
        "t_build_ms": st["t_build_ms"],
        "t_solve_ms": st["t_solve_ms"],
        "setup_s": setup_s,
        "reynolds": re,
        "precond_apply_ms": ap_["avg_ms"],
        "precond_apply_GBps": apply_gbs,
        "roofline": {"bound": "hbm", "kernel": "trsv_sub_kernel (batched skyline triangular solves of the primary grids)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(args.workload, args.precision),
                     "avg_launch_ms": tr["avg_ms"], "algorithmic_bytes_per_launch": tr["bytes"],
                     "launches": tr["samples"]},
        "kernel_times": kt,
    }
    out["autotune"] = tuning
    if not args.no_fp64_plain:
        log("plain FP64 preconditioner on the same workload ...")
        del s
        torch.cuda.empty_cache()
        s64 = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"],
                     precision="fp64", newton_tol=1e-8, lin_tol=1e-9, restart=args.restart)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x64, st64 = s64.newton_solve()
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        out["fp64_plain"] = {"s": t64, "newton_its": st64["newton_its"], "fgmres_its_total": st64["lin_its_total"],
                             "t_build_ms": st64["t_build_ms"],
                             "rel_diff_vs_fp32_solution": float(torch.linalg.norm(x64 - x) / torch.linalg.norm(x64))}
        del s64
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a %d^3 crop) ..." % args.cpu_crop)
        out["cpu_baseline"] = _cpu_baseline(w, args.cpu_crop)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
