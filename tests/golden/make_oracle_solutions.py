"""Write the oracle's converged solutions of the 128^3 sphere-packing benchmark
(spheres3d_128, seed 0) and of its 64^3 corner crop, for the element-wise GPU
parity tests.

Calls only ``oracle`` and ``synth``: the stored values are the FP64 CPU oracle's
Newton-FGMRES-gPLMM solution (Section 1 Newton, Section 8 right-preconditioned
GMRES, Sections 3.2 and 4 gPLMM) solved to ||r(x)|| <= 1e-12 ||r(0)||.

    python tests/golden/make_oracle_solutions.py crop64
    python tests/golden/make_oracle_solutions.py full

Each run writes tests/golden/<name>.npz holding the velocity unknowns ``u`` (the
oracle's [u; v; w] order: x-, y-, z-faces, each in raster (k, j, i) order of the
face), the pressures ``p`` (raster order of the fluid cells, gauge p = 0 at the
oracle's pin) and ``meta`` (a JSON string: wall time, host cores and CPU model,
BLAS threads, Newton and FGMRES iteration counts, the T_MG / T_ML / T_sol split,
the relative residual reached).  The mantissas are rounded to 36 bits (relative
rounding 1.5e-11, far below the 1e-8 and 1e-10 parity tolerances) so that the
archive compresses.
"""
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.mac import MacGrid, Operators, Phys, residual   # noqa: E402
from oracle.decomp import decompose, largest_component      # noqa: E402
from oracle import newton                                    # noqa: E402
from synth import make_workload                              # noqa: E402

CASES = {"crop64": 64, "full": 128}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def round_mantissa(a, bits=36):
    """Round float64 values to `bits` explicit mantissa bits (round half away from zero
    on the bit pattern), keeping sign and exponent."""
    b = np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)
    drop = np.uint64(52 - bits)
    half = np.uint64(1) << (drop - np.uint64(1))
    r = ((b + half) >> drop) << drop
    return r.view(np.float64)


def solve(name, restart=256, tol=1e-12):
    n = CASES[name]
    w = make_workload("spheres3d_128", 0)
    mask = w["mask"][:n, :n, :n].copy()
    labels = w["labels"][:n, :n, :n].copy()
    t0 = time.perf_counter()
    g = MacGrid(largest_component(mask))
    ops = Operators(g)
    dc = decompose(g, labels)
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    t_setup = time.perf_counter() - t0

    def progress(msg):
        print(msg, flush=True)

    st = newton.NewtonStats()
    t0 = time.perf_counter()
    x, st = newton.solve(ops, dc, ph, tol=tol, lin_tol=0.1 * tol, restart=restart, lin_maxit=5000,
                         stats=st)
    wall = time.perf_counter() - t0
    r = residual(ops, x, ph)
    r0 = residual(ops, np.zeros(g.N), ph)
    rel = float(np.linalg.norm(r) / np.linalg.norm(r0))
    try:
        from threadpoolctl import threadpool_info
        blas = [dict(api=i.get("internal_api"), threads=i.get("num_threads")) for i in threadpool_info()]
    except Exception:   # pragma: no cover
        blas = []
    meta = dict(workload="spheres3d_128", seed=0, crop=n, N=int(g.N), nu=int(g.nu), ncell=int(g.nc),
                Np=int(dc.Np), Nc=int(dc.Nc), pin=int(dc.pin), body=list(w["body"]), tol=tol,
                lin_tol=0.1 * tol, restart=restart, newton_its=st.newton_its, fgmres_its=list(st.lin_its),
                step_length=list(st.step_length), res_hist=list(st.res_hist), t_hist=list(st.t_hist),
                rel_residual=rel,
                converged=bool(st.converged), wall_s=wall, setup_s=t_setup, t_mg_s=st.t_mg,
                t_ml_s=st.t_ml, t_sol_s=st.t_sol, nproc=os.cpu_count(), cpu_model=cpu_model(), blas=blas,
                python=platform.python_version(), numpy=np.__version__)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres3d_128_s0_%s.npz" % name)
    np.savez_compressed(out, u=round_mantissa(x[:g.nu]), p=round_mantissa(x[g.nu:]),
                        meta=np.array(json.dumps(meta)))
    progress(json.dumps(meta))
    return out


if __name__ == "__main__":
    for name in sys.argv[1:] or ["crop64"]:
        solve(name)
