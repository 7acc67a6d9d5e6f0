"""GPU parity of the nested-dissection solves of large primary blocks (options.split_tiles):
the halves' stopped eliminations, the separators' Schur complements and their inverses,
and the three-phase application, against the FP64 oracle's preconditioner (which solves
every primary block directly) and against the library with splitting off.

Bars: FP64 application 1e-11 relative (as the unsplit path: the block solve in the order
[A, B, S] is exact up to rounding); FP32 application 5e-3 from the FP64 oracle (the bar of
the unsplit FP32 path); one pore with no interface (no coarse space, no duals) is the
exact inverse of X to 1e-12; Newton solutions with split primaries converge with full
steps and match the oracle to 1e-10 (FP64).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import gplmm as G
from oracle import newton
from oracle.mac import build_matrix, origin_rhs
from tests.helpers import oracle_case, record_index, rel, to_record, workload


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(name, seed):
    if name == "crop48":
        w = workload("spheres3d_128", 0)
        return dict(w, mask=w["mask"][:48, :48, :48].copy(), labels=w["labels"][:48, :48, :48].copy())
    return workload(name, seed)


@pytest.mark.parametrize("name,seed,thr", [("spheres3d_24", 0, 2), ("disks2d_64", 1, 2), ("crop48", 0, 16)])
def test_split_preconditioner_parity_fp64(name, seed, thr):
    torch = _torch()
    from paper_2510_22077_amd import Solver
    w = _case(name, seed)
    _say("case split fp64", name, seed, thr)
    kw = dict(rho=w["rho"], mu=w["mu"], body=w["body"])
    s = Solver(w["mask"], w["labels"], split_tiles=thr, **kw)
    assert s.layout.nsplit >= 1
    ref = Solver(w["mask"], w["labels"], split_tiles=-1, **kw)
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    rng = np.random.default_rng(30 + seed)
    wind = rng.standard_normal(g.N)
    wd = torch.tensor(to_record(wind, rec, s.N), dtype=torch.float64, device="cuda")
    s.build(wd)
    ref.build(wd)
    M = G.build(build_matrix(ops, ph, wind=wind, tags=dc.tags), dc, origin_rhs(ops, ph))
    for trial in range(2):
        v = rng.standard_normal(g.N)
        vr = torch.tensor(to_record(v, rec, s.N), dtype=torch.float64, device="cuda")
        z = s.precond_apply(vr).cpu().numpy()
        zr = ref.precond_apply(vr).cpu().numpy()
        err, err_ref = rel(z[rec], G.apply(M, v)), rel(z[rec], zr[rec])
        _say("split %d: apply vs oracle %.2e, vs unsplit %.2e" % (s.layout.nsplit, err, err_ref))
        assert err <= 1e-11 and err_ref <= 1e-11
    s.close()
    ref.close()


def test_split_preconditioner_fp32_crop48():
    torch = _torch()
    from paper_2510_22077_amd import Solver
    w = _case("crop48", 0)
    _say("case split fp32 crop48")
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision="fp32", split_tiles=16)
    assert s.layout.nsplit >= 1
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    rng = np.random.default_rng(41)
    wind = 0.05 * rng.standard_normal(g.N)
    s.build(torch.tensor(to_record(wind, rec, s.N), dtype=torch.float64, device="cuda"))
    M = G.build(build_matrix(ops, ph, wind=wind, tags=dc.tags), dc, origin_rhs(ops, ph))
    v = rng.standard_normal(g.N)
    z = s.precond_apply(torch.tensor(to_record(v, rec, s.N), dtype=torch.float64, device="cuda")).cpu().numpy()
    err = rel(z[rec], G.apply(M, v))
    _say("split fp32 apply rel err", err)
    assert err <= 5e-3
    s.close()


def test_split_single_pore_is_exact_inverse():
    torch = _torch()
    from paper_2510_22077_amd import Solver
    m = np.ones((16, 10, 12), np.uint8)   # longest along z (not periodic), cut there
    m[6:9, 4:6, 4:7] = 0
    lab = np.ones_like(m, dtype=np.int32)
    _say("case split single pore")
    s = Solver(m, lab, body=(1.0, 0.0, 0.0), split_tiles=2)
    assert s.info()["Nc"] == 0 and s.layout.nsplit == 1
    s.build()
    g, ops, dc, ph = oracle_case(m, lab)
    rec = record_index(g, s.maps()["cell_voxel"])
    v = np.zeros(s.N)
    v[rec] = np.random.default_rng(5).standard_normal(len(rec))
    vd = torch.tensor(v, dtype=torch.float64, device="cuda")
    back = s.build_matvec(s.precond_apply(vd)).cpu().numpy()
    assert rel(back, v) <= 1e-12
    s.close()


def test_split_newton_solution_parity():
    torch = _torch()
    from paper_2510_22077_amd import Solver
    w = workload("spheres3d_24", 0, re=1.0)
    _say("case split newton spheres3d_24")
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], split_tiles=2,
               newton_tol=1e-13, lin_tol=1e-14)
    assert s.layout.nsplit >= 1
    x, st = s.newton_solve()
    assert st["converged"] and st["step_length"] == [1.0] * st["newton_its"]
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    xo, _ = newton.solve(ops, dc, ph, tol=1e-14, precond="exact")
    xg = x.cpu().numpy()[rec]
    assert rel(xg[:g.nu], xo[:g.nu]) <= 1e-10
    p = g.p_slice
    assert rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean()) <= 1e-10
    s.close()
