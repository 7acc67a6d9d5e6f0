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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor()


def _cpu_baseline(workload, crop, its_full):
    """The FP64 oracle, untuned, on a bounded sample: the full Newton-FGMRES-gPLMM solve
    (restart 256, the bench's tolerances) of the crop^3 corner of the same packing on one
    thread (SuperLU and the Python loops are single-threaded; BLAS is held to one thread),
    extrapolated to the full image by the law
        T = (T_MG + T_ML) * N_full / N_crop + (T_sol / its_crop) * (N_full / N_crop) * its_full,
    i.e. build work linear in the unknowns and FGMRES time linear in the unknowns per
    iteration, with its_full the FGMRES iterations the same algorithm needs on the full
    image (measured by the plain FP64 GPU solve of this run)."""
    from threadpoolctl import threadpool_limits
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
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, st = newton.solve(ops, dc, ph, tol=1e-8, lin_tol=1e-9, restart=256, lin_maxit=3000)
        el = time.perf_counter() - t0
    full = MacGrid(largest_component(workload["mask"]))
    ratio = full.N / g.N
    its_crop = sum(st.lin_its)
    est = (st.t_mg + st.t_ml) * ratio + (st.t_sol / max(its_crop, 1)) * ratio * its_full
    return dict(value=est, unit="s", cores=1, kind="oracle", nproc=os.cpu_count(), cpu_model=_cpu_model(),
                blas_threads=1,
                sample="oracle Newton-FGMRES(256)-gPLMM to 1e-8 on the %d^3 corner crop (N=%d, %d Newton / %d "
                       "FGMRES its, T_MG %.1f s, T_ML %.1f s, T_sol %.1f s, total %.1f s, setup %.1f s), "
                       "extrapolated to N=%d with T = (T_MG+T_ML)*r + T_sol/its_crop*r*its_full, r = %.2f, "
                       "its_full = %d" % (crop, g.N, st.newton_its, its_crop, st.t_mg, st.t_ml, st.t_sol, el,
                                          t_setup, full.N, ratio, its_full),
                crop_measured_s=el, t_mg_s=st.t_mg, t_ml_s=st.t_ml, t_sol_s=st.t_sol, newton_its=st.newton_its,
                fgmres_its=list(st.lin_its), converged=bool(st.converged))


def _oracle_full_record():
    """The oracle's own full-size solve, recorded when the stored 128^3 solution was
    written (tests/golden, another machine: the one stated): time until the Newton
    residual first met 1e-8, and the run to 1e-12."""
    import json as _json
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "spheres3d_128_s0_full.npz")
    if not os.path.exists(path):
        return None
    meta = _json.loads(str(np.load(path, allow_pickle=False)["meta"]))
    t8 = None
    for r, t in zip(meta.get("res_hist", []), meta.get("t_hist", [])):
        if r <= 1e-8:
            t8 = t
            break
    return dict(s_to_1e8=t8, s_to_1e12=meta["wall_s"], newton_its=meta["newton_its"], fgmres_its=meta["fgmres_its"],
                t_mg_s=meta["t_mg_s"], t_ml_s=meta["t_ml_s"], t_sol_s=meta["t_sol_s"], nproc=meta["nproc"],
                cpu_model=meta["cpu_model"], blas=meta["blas"], restart=meta["restart"],
                note="measured once by tests/golden/make_oracle_solutions.py (not on the GPU host)")


def _paper_e2(solver, mask, xa, xt, nrec):
    """E_2 of the paper's coarse-solver tests (root mean square over the fluid cells of
    |xi_t - xi_a| / sup |xi_t|, percent) for xi = mean-free pressure and the velocity
    magnitude at the cell centres (each component the mean of the cell's two faces)."""
    import numpy as np
    m = solver.maps()
    cv = m["cell_voxel"]
    nz, ny, nx = mask.shape
    nd = nrec - 1
    vox2cell = np.full(mask.size, -1, dtype=np.int64)
    vox2cell[cv] = np.arange(cv.size)
    k, j, i = np.unravel_index(cv, mask.shape)
    up = []
    for a, (kk, jj, ii) in enumerate([(k, j, (i + 1) % nx), (k, j + 1, i), (k + 1, j, i)][:nd]):
        ok = (jj < ny) & (kk < nz)
        c = np.full(cv.size, -1, dtype=np.int64)
        c[ok] = vox2cell[(kk[ok] * ny + jj[ok]) * nx + ii[ok]]
        up.append(c)

    def fields(x):
        X = x.reshape(-1, nrec)
        sp2 = np.zeros(X.shape[0])
        for a in range(nd):
            upper = np.where(up[a] >= 0, X[np.maximum(up[a], 0), a], 0.0)
            sp2 += (0.5 * (X[:, a] + upper)) ** 2
        p = X[:, nd] - X[:, nd].mean()
        return np.sqrt(sp2), p

    sa, pa = fields(xa)
    st_, pt = fields(xt)
    e_u = 100.0 * float(np.sqrt(np.mean(((st_ - sa) / np.abs(st_).max()) ** 2)))
    e_p = 100.0 * float(np.sqrt(np.mean(((pt - pa) / np.abs(pt).max()) ** 2)))
    return e_p, e_u


def _train_mlp(m, feats, targets, epochs=60, seed=0):
    """Train the coarse model with the library's BF16 kernels and Adam on standardised
    features; the standardisation is folded into the first layer afterwards."""
    import numpy as np
    X = np.concatenate(feats)
    T = np.concatenate(targets)[:, None].astype(np.float32)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(X))
    X, T = X[perm], T[perm]
    mu, sd = X.mean(0), X.std(0)
    const = sd < 1e-6
    sd[const], mu[const] = 1.0, 0.0
    nin, nh = X.shape[1], 128
    flat = []
    fan = [nin, nh, nh, nh, 1]
    for a, b in zip(fan[:-1], fan[1:]):   # Glorot-uniform weights, zero biases
        lim = np.sqrt(6.0 / (a + b))
        flat += [rng.uniform(-lim, lim, size=a * b), np.zeros(b)]
    m.set_params(np.concatenate(flat).astype(np.float32))
    loss = m.train(((X - mu) / sd).astype(np.float32), T, epochs=epochs, batch=1024, lr=1e-3)
    p = m.get_params()
    W1 = p[:nin * nh].reshape(nin, nh)
    b1 = p[nin * nh:nin * nh + nh]
    b1 -= (mu / sd) @ W1
    W1 /= sd[:, None]
    m.set_params(p)
    return float(loss), float(np.var(T))


def _measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of the skyline-solve kernel from the committed PMC summary, if
    it was taken on this workload and precision with the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_traffic_%s_%s.txt" % (kernel, workload, precision))
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


def _sensitivity(args):
    """FGMRES iterations of the steady solve of the 64^3 corner of the packing against the
    dual-grid dilations (0, 1, 2; tag layers 1) and the tag layers (0, 1, 2; no dilation),
    at Re 1, 10 and 20 (FP32 preconditioner, restart 256, at most 600 FGMRES iterations per
    Newton step and 12 Newton steps).  One JSON line."""
    import torch
    from synth import make_workload
    from paper_2510_22077_amd import Solver
    rows = []
    for re in (1.0, 10.0, 20.0):
        w = make_workload(args.workload, args.seed, re=re)
        m, lab = w["mask"][:64, :64, :64].copy(), w["labels"][:64, :64, :64].copy()
        for dd, tl in ((0, 0), (0, 1), (0, 2), (1, 1), (2, 1)):
            s = Solver(m, lab, rho=w["rho"], mu=w["mu"], body=w["body"], precision="fp32", restart=256,
                       dual_dilations=dd, tag_layers=tl, newton_tol=1e-8, lin_tol=1e-9, lin_maxit=600,
                       newton_maxit=12)
            s.set_progress(lambda k, its, r: print("  newton %d: %d its, rel %.2e" % (k, its, r), file=sys.stderr,
                                                   flush=True) if r >= 0 else None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = s.newton_solve()
            torch.cuda.synchronize()
            row = {"re": re, "dual_dilations": dd, "tag_layers": tl, "converged": bool(st["converged"]),
                   "newton_its": st["newton_its"], "fgmres_its": st["lin_its"], "fgmres_total": st["lin_its_total"],
                   "s": time.perf_counter() - t0}
            print(json.dumps(row), file=sys.stderr, flush=True)
            rows.append(row)
            s.close()
    print(json.dumps({"sensitivity": rows, "workload": "%s seed %d, 64^3 corner" % (args.workload, args.seed)}))


def _batch(args):
    """The many-sample configuration: args.batch independent samples (each axis 48..96
    voxels, porosity 0.3..0.6, target Re log-uniform in 0.1..20, seed args.seed) in one
    context, every subdomain of every sample in the same launches, one Newton-FGMRES over
    the batch with per-sample Krylov coefficients (FP32 preconditioner, restart
    args.batch_restart, at most args.batch_maxit FGMRES iterations per Newton step, 12
    Newton steps).  One JSON
    line: wall time, per-sample relative residuals and convergence."""
    import numpy as np
    import torch
    from synth import make_batch
    from paper_2510_22077_amd import BatchSolver
    t0 = time.perf_counter()
    ws = make_batch(args.batch, args.seed, progress=lambda k, w: print(
        "sample %d: %s, Re target %.2f" % (k, "x".join(str(v) for v in w["mask"].shape), w["re_target"]),
        file=sys.stderr, flush=True))
    tg = time.perf_counter() - t0
    print("batch of %d generated in %.1f s" % (len(ws), tg), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    B = BatchSolver([w["mask"] for w in ws], [w["labels"] for w in ws], rho=[w["rho"] for w in ws],
                    mu=[w["mu"] for w in ws], bodies=[w["body"] for w in ws], precision=args.precision,
                    restart=args.batch_restart, newton_tol=1e-8, lin_tol=1e-9, lin_maxit=args.batch_maxit,
                    newton_maxit=12)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = B.info()
    print("setup %.1f s: N %d, pores %d, interfaces %d" % (setup_s, info["N"], info["Np"], info["Nc"]),
          file=sys.stderr, flush=True)
    B.set_progress(lambda k, its, r: print("  newton %d: %d its%s" % (k, its, ", rel %.2e" % r if r >= 0 else ""),
                                           file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = B.newton_solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rs = B.sample_residuals(x)
    out = {"metric": "batch solve wall time", "value": el, "unit": "s", "samples": len(ws), "unknowns": info["N"],
           "pores": info["Np"], "interfaces": info["Nc"], "setup_s": setup_s, "precision": args.precision,
           "restart": args.batch_restart, "lin_maxit": args.batch_maxit, "newton_its": st["newton_its"], "fgmres_its": st["lin_its"],
           "fgmres_its_total": st["lin_its_total"], "converged": bool(st["converged"]),
           "samples_converged": int((rs <= 1e-8).sum()), "sample_rel_residual": [float(v) for v in rs],
           "sample_re_target": [w["re_target"] for w in ws], "sample_shape": [list(w["mask"].shape) for w in ws],
           "t_build_ms": st["t_build_ms"], "t_solve_ms": st["t_solve_ms"]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spheres3d_128")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--restart", type=int, default=256)
    ap.add_argument("--cpu-crop", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-plain", action="store_true",
                    help="skip the comparison solve with the plain FP64 preconditioner")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--split-tiles", type=int, default=0,
                    help="primaries spanning more tiles are solved by nested dissection (0, the library "
                         "default, and -1: never)")
    ap.add_argument("--mg-form", type=int, default=0, choices=[0, 1, 2],
                    help="coarse correction: 0 the compact form of Remark 1 (default), 1 Eq. iMG with the "
                         "back-substitution of Eq. xf, 2 the compact form with that back-substitution")
    ap.add_argument("--no-coarse", action="store_true", help="skip the coarse-scale solver leg")
    ap.add_argument("--no-aplmm", action="store_true", help="skip the aPLMM_S / aPLMM_NS comparison solves")
    ap.add_argument("--no-pnm", action="store_true", help="skip the gPNM (pore-network decomposition) solve")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned coarse operator leg")
    ap.add_argument("--learned-seeds", type=int, default=5, help="packings (seeds 1..n) the coarse model is trained on")
    ap.add_argument("--coarse-increments", type=int, default=3,
                    help="body-force steps of the coarse-scale solver (one step from rest stalls at "
                         "128^3, as Algorithm 1 warns for starts far from the solution)")
    ap.add_argument("--sensitivity", action="store_true",
                    help="only run the decomposition sensitivity study on the 64^3 corner of the packing: "
                         "FGMRES iterations against dual dilations and tag layers at Re 1, 10 and 20")
    ap.add_argument("--no-continuation", action="store_true",
                    help="skip the Re 10 solves (direct, and continuation through half the force)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the extra solve on the finer pore split (about 1.5k pores)")
    ap.add_argument("--copy-cal", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, five times (the reference "
                         "point for scaling hardware byte counters)")
    ap.add_argument("--batch", type=int, default=0, metavar="SAMPLES",
                    help="only run the many-sample configuration with this many samples (64: each axis "
                         "48..96, porosity 0.3..0.6, Re 0.1..20)")
    ap.add_argument("--batch-maxit", type=int, default=2000, help="FGMRES iterations per Newton step (--batch)")
    ap.add_argument("--batch-restart", type=int, default=128, help="FGMRES restart length (--batch)")
    args = ap.parse_args()
    if args.batch:
        _batch(args)
        return
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
    if args.sensitivity:
        _sensitivity(args)
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
               precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart,
               split_tiles=args.split_tiles, mg_form=args.mg_form)
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

    kt = {k: s.kernel_time(k) for k in ("trsv_p", "trsv_p_fwd", "trsv_sep", "trsv_p_bwd", "trsv_d", "trsv_f",
                                         "precond_apply", "jv", "arnoldi", "lu",
                                         "build_closure_dual_lu", "build_shape", "build_primary_lu",
                                         "build_coarse")}
    for k, v in kt.items():
        if k not in ("lu", "build_closure_dual_lu", "build_primary_lu") and v["avg_ms"] > 0 and v["bytes"] > 0:
            v["GBps"] = v["bytes"] / (v["avg_ms"] * 1e-3) / 1e9
    lu = kt["lu"]
    lu_tflops = lu["bytes"] / (lu["avg_ms"] * 1e-3) / 1e12 if lu["avg_ms"] > 0 else 0.0
    nb = stt["builds"]
    ph = {k: kt[k]["avg_ms"] * kt[k]["samples"] / max(nb, 1) for k in
          ("build_closure_dual_lu", "build_shape", "build_primary_lu", "build_coarse")}
    tr = kt["trsv_p"]   # the primary grids' solves, the dominant launch
    # the variant that ran: four-group 16-byte loads (2, the default) or one element per thread
    trsv_mode = tuning["trsv_mode"] if tuning else 2
    # (FP64 factors of a primary over 255 tiles exceed the LDS bound: one-element variant)
    trsv_kernel = "trsv_quad_kernel" if trsv_mode == 2 and args.precision == "fp32" else "trsv_sub_kernel"
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
                   "split_pores": info["nsplit"], "separator_unknowns": info["sep_unknowns"],
                   "precision": args.precision, "restart": args.restart, "mg_form": args.mg_form,
                   "f_blocks": info.get("nfblock", 0)},
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
        "roofline": {"bound": "hbm", "kernel": "%s (batched skyline triangular solves of the primary grids)" % trsv_kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(trsv_kernel, args.workload, args.precision),
                     "avg_launch_ms": tr["avg_ms"], "algorithmic_bytes_per_launch": tr["bytes"],
                     "launches": tr["samples"]},
        "kernel_times": kt,
        "lu_mfma": {"kernel": "lu_diag_kernel + lu_row_kernel (tile LU: FP32 panels and trailing updates on "
                              "v_mfma_f32_32x32x2f32, FP64 diagonal tiles)" if args.precision == "fp32" else
                              "lu_diag_kernel + lu_row_kernel (FP64)",
                    "flops_per_schedule_avg": lu["bytes"], "avg_ms": lu["avg_ms"], "achieved_TFLOPs": lu_tflops,
                    "peak_TFLOPs": 157.3 if args.precision == "fp32" else 78.6,
                    "frac": lu_tflops / (157.3 if args.precision == "fp32" else 78.6),
                    "lu_flops_per_build": info["lu_flops"]},
        "time_split_ms_per_solve": {
            "T_MG": ph["build_closure_dual_lu"] + ph["build_shape"] + ph["build_coarse"],
            "T_ML": ph["build_primary_lu"],
            "T_sol": stt["t_solve_ms"],
            "note": "event-timed solve; T_MG = closure LU (shared launches with the dual LU) + shape vectors + "
                    "coarse operator, T_ML = primary-block LU; the dual-block LU is inside T_MG",
            "phases_ms": ph, "builds": nb},
    }
    out["autotune"] = tuning
    # coarse-scale solver (Algorithm 1) on the same context: time, coarse Newton
    # iterations, and the paper's E2 errors against the fine solution x just computed
    if not args.no_coarse:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xc, stc = s.coarse_solve(increments=args.coarse_increments)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        e_p, e_u = _paper_e2(s, w["mask"], xc.cpu().numpy(), x.cpu().numpy(), nrec)
        out["coarse_solver"] = {"s": tc, "increments": stc["increments"], "coarse_newton_its": stc["newton_its"],
                                "rc_rel": stc["rc_rel"], "converged": stc["converged"],
                                "fine_rel_residual": stc["fine_rel_residual"], "t_build_ms": stc["t_build_ms"],
                                "E2_p_percent": e_p, "E2_speed_percent": e_u,
                                "speedup_vs_fine_solve": sec / tc}
    # Reynolds-number continuation (Section 8's protocol) at Re ~ 10 on the same packing:
    # one direct Newton solve against raising the force in two steps (half, then full)
    if not args.no_continuation:
        log("Re 10: direct solve and continuation ...")
        wr = make_workload(args.workload, args.seed, re=10.0)
        sr = Solver(wr["mask"], wr["labels"], rho=wr["rho"], mu=wr["mu"], body=wr["body"],
                    precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart,
                    lin_maxit=4000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sd = sr.newton_solve()
        torch.cuda.synchronize()
        td = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, sc_, rcc = sr.continuation([0.5, 1.0])
        torch.cuda.synchronize()
        tcn = time.perf_counter() - t0
        out["re10_continuation"] = {
            "body_x": wr["body"][0], "re_target": 10.0,
            "direct": {"s": td, "newton_its": sd["newton_its"], "fgmres_its_total": sd["lin_its_total"],
                       "converged": sd["converged"]},
            "continuation_half_full": {"s": tcn, "newton_its": [q["newton_its"] for q in sc_],
                                       "fgmres_its_total": [q["lin_its_total"] for q in sc_],
                                       "converged": rcc == 0}}
        sr.close()
        del sr
        torch.cuda.empty_cache()
        # the direct Re 10 solve with the Eq. xf step in the coarse correction (mg_form 2)
        sr = Solver(wr["mask"], wr["labels"], rho=wr["rho"], mu=wr["mu"], body=wr["body"],
                    precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart,
                    lin_maxit=4000, mg_form=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, sx2 = sr.newton_solve()
        torch.cuda.synchronize()
        out["re10_continuation"]["direct_eq_xf"] = {"s": time.perf_counter() - t0, "newton_its": sx2["newton_its"],
                                                    "fgmres_its_total": sx2["lin_its_total"],
                                                    "converged": sx2["converged"]}
        log("Re 10 with Eq. xf: %s" % json.dumps(out["re10_continuation"]["direct_eq_xf"]))
        sr.close()
        del sr
        torch.cuda.empty_cache()
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
    if not args.no_aplmm:
        # the paper's comparison preconditioners on the same workload (Section 8):
        # aPLMM_S = gPLMM_S (built once from the Stokes matrix) and aPLMM_NS (built from the
        # Newton Jacobian, rebuilt once at the first Newton iterate as gPLMM is)
        for key, kw in (("aplmm_s", dict(wind="zero")), ("aplmm_ns", dict(build_matrix="jacobian"))):
            log("%s preconditioner on the same workload ..." % key)
            sa = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=args.precision,
                        newton_tol=1e-8, lin_tol=1e-9, restart=args.restart, **kw)
            sa.newton_solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xa, sta = sa.newton_solve()
            torch.cuda.synchronize()
            out[key] = {"s": time.perf_counter() - t0, "newton_its": sta["newton_its"], "fgmres_its": sta["lin_its"],
                        "fgmres_its_total": sta["lin_its_total"], "t_build_ms": sta["t_build_ms"],
                        "builds": sta["builds"], "converged": sta["converged"]}
            del sa
            torch.cuda.empty_cache()
    if not args.no_learned:
        # FP32 + learned coarse operator (the structured model: predicted entries, interface
        # diagonals and correction rows set by conservation), trained on the exact coarse
        # entries of other seeds of the same packing law, evaluated on this one
        from synth import make_workload as _mk
        from paper_2510_22077_amd import Mlp
        import numpy as np
        log("learned coarse operator: training on seeds %s ..." % list(range(1, 1 + args.learned_seeds)))
        t0 = time.perf_counter()
        feats, targets = [], []
        nthroats = 0
        for sd_ in range(1, 1 + args.learned_seeds):
            wt = _mk(args.workload, sd_)
            st_ = Solver(wt["mask"], wt["labels"], rho=wt["rho"], mu=wt["mu"], body=wt["body"],
                         precision=args.precision, restart=args.restart)
            st_.build()
            e_ = st_.coarse_entries(exact=True)
            feats.append(e_["feat"])
            targets.append(np.arcsinh(e_["exact"] / e_["scale"]))
            nthroats += st_.info()["Nc"]
            del st_
        mlp = Mlp(16, 128, 3, 1, max_batch=4096)
        loss, var = _train_mlp(mlp, feats, targets)
        t_train = time.perf_counter() - t0
        sl = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=args.precision,
                    newton_tol=1e-8, lin_tol=1e-9, restart=args.restart)
        sl.set_coarse_model(mlp)
        sl.newton_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xl, stl = sl.newton_solve()
        torch.cuda.synchronize()
        out["learned_coarse"] = {"s": time.perf_counter() - t0, "newton_its": stl["newton_its"],
                                 "fgmres_its": stl["lin_its"], "fgmres_its_total": stl["lin_its_total"],
                                 "learned_builds": stl["learned_builds"], "fallbacks": stl["coarse_fallbacks"],
                                 "t_coarse_ms": stl["t_coarse_ms"], "t_build_ms": stl["t_build_ms"],
                                 "rel_diff_vs_exact_solution": float(torch.linalg.norm(xl - x) / torch.linalg.norm(x)),
                                 "train": {"seeds": args.learned_seeds, "entries": int(sum(len(f) for f in feats)),
                                           "throats": nthroats, "loss": loss, "target_var": var,
                                           "s": t_train}}
        sl.set_coarse_model(None)
        del sl
        mlp.close()
        torch.cuda.empty_cache()
    if not args.no_pnm:
        # the pore-network decomposition (Section 3.3): throat regions as primary grids,
        # one interface per pore body; same preconditioner machinery (gPNM)
        from synth import throat_labels
        log("gPNM (pore-network decomposition) on the same workload ...")
        th = throat_labels(w["mask"], w["labels"])
        sp_ = Solver(w["mask"], th, rho=w["rho"], mu=w["mu"], body=w["body"], groups=w["labels"],
                     precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart, lin_maxit=4000)
        sp_.newton_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xp_, stp = sp_.newton_solve()
        torch.cuda.synchronize()
        out["gpnm"] = {"s": time.perf_counter() - t0, "primaries_throats": sp_.info()["Np"],
                       "interfaces_pores": sp_.info()["Nc"], "newton_its": stp["newton_its"],
                       "fgmres_its": stp["lin_its"], "fgmres_its_total": stp["lin_its_total"],
                       "t_build_ms": stp["t_build_ms"], "converged": stp["converged"]}
        del sp_
        torch.cuda.empty_cache()
    if not args.no_variants:
        from synth import make_workload as _mk
        log("finer pore split (pores > 1000 voxels split) ...")
        wv = _mk(args.workload, args.seed, max_size=1000)
        sv = Solver(wv["mask"], wv["labels"], rho=wv["rho"], mu=wv["mu"], body=wv["body"],
                    precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart)
        if not args.no_autotune:
            sv.build()
            sv.autotune()
        sv.newton_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xv_, stv = sv.newton_solve()
        torch.cuda.synchronize()
        out["variant_pores_split_1000"] = {"s": time.perf_counter() - t0, "pores": sv.info()["Np"],
                                           "interfaces": sv.info()["Nc"], "newton_its": stv["newton_its"],
                                           "fgmres_its_total": stv["lin_its_total"], "t_build_ms": stv["t_build_ms"]}
        del sv
        torch.cuda.empty_cache()
    if not args.no_variants and args.mg_form == 0:
        # the same solve with the f-faces' unknowns of the coarse correction recovered by the
        # back-substitution of Eq. xf (mg_form 2) instead of left at zero
        log("coarse correction with the Eq. xf back-substitution ...")
        sx = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"],
                    precision=args.precision, newton_tol=1e-8, lin_tol=1e-9, restart=args.restart, mg_form=2)
        if not args.no_autotune:
            sx.build()
            sx.autotune()
        for k in range(args.warmup):
            sx.newton_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            xx_, stx = sx.newton_solve()
        torch.cuda.synchronize()
        tx = (time.perf_counter() - t0) / args.steps
        dx = float((xx_ - x).norm().item() / x.norm().item())
        out["variant_eq_xf_back_substitution"] = {
            "s": tx, "speedup_vs_value": sec / tx, "mg_form": 2, "f_blocks": sx.info()["nfblock"],
            "f_unknowns": sx.info()["f_unknowns"], "newton_its": stx["newton_its"], "fgmres_its": stx["lin_its"],
            "fgmres_its_total": stx["lin_its_total"], "t_build_ms": stx["t_build_ms"],
            "final_rel_residual": stx["res_hist"][-1], "rel_diff_to_value_solution": dx}
        log("Eq. xf variant: %s" % json.dumps(out["variant_eq_xf_back_substitution"]))
        del sx
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a %d^3 crop) ..." % args.cpu_crop)
        its_full = out["fp64_plain"]["fgmres_its_total"] if "fp64_plain" in out else st["lin_its_total"]
        out["cpu_baseline"] = _cpu_baseline(w, args.cpu_crop, its_full)
        out["oracle_full_128_recorded"] = _oracle_full_record()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
