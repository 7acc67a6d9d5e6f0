"""GPU parity of the pore-network variant (Section 3.3: throat regions as primary grids,
one contact interface per pore body) through gplmm_setup_pnm: the preconditioner
application against the oracle built on the same decomposition (FP64 1e-11, FP32 5e-3)
and the converged Newton solution (FP64 1e-10, FP32 1e-8, full steps)."""
import sys

import numpy as np
import pytest

from oracle import gplmm as G
from oracle import newton
from oracle.mac import MacGrid, Operators, Phys, build_matrix, origin_rhs
from oracle.decomp import decompose, largest_component
from synth import throat_labels
from tests.helpers import record_index, rel, to_record, workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(name, seed, re=None, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22077_amd import Solver
    w = workload(name, seed, re=re)
    th = throat_labels(w["mask"], w["labels"])
    _say("case pnm", name, seed, kw)
    s = Solver(w["mask"], th, rho=w["rho"], mu=w["mu"], body=w["body"], groups=w["labels"], **kw)
    g = MacGrid(largest_component(w["mask"]))
    ops = Operators(g)
    dc = decompose(g, th, groups=w["labels"])
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    rec = record_index(g, s.maps()["cell_voxel"])
    return torch, s, g, ops, dc, ph, rec


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 5e-3)])
@pytest.mark.parametrize("name,seed", [("disks2d_64", 0), ("spheres3d_24", 0)])
def test_pnm_preconditioner_matches_the_oracle(name, seed, precision, tol):
    torch, s, g, ops, dc, ph, rec = _case(name, seed, precision=precision)
    rng = np.random.default_rng(40 + seed)
    wind = 0.1 * rng.standard_normal(g.N)
    s.build(torch.tensor(to_record(wind, rec, s.N), dtype=torch.float64, device="cuda"))
    M = G.build(build_matrix(ops, ph, wind=wind, tags=dc.tags), dc, origin_rhs(ops, ph))
    # the coarse operator: FP64 probing of FP64 (or FP32-rounded) shape vectors
    atol = (1e-9 if precision == "fp64" else 1e-5) * np.abs(M.Ao).max()
    assert np.allclose(s.coarse_operator(), M.Ao, rtol=0, atol=atol)
    v = rng.standard_normal(g.N)
    z = s.precond_apply(torch.tensor(to_record(v, rec, s.N), dtype=torch.float64, device="cuda")).cpu().numpy()
    err = rel(z[rec], G.apply(M, v))
    _say("gPNM apply rel err", precision, err)
    assert err <= tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
def test_pnm_newton_solution(precision, tol):
    torch, s, g, ops, dc, ph, rec = _case("spheres3d_24", 0, re=5.0, precision=precision, newton_tol=1e-12,
                                          lin_tol=1e-13, restart=60)
    x, st = s.newton_solve()
    assert st["converged"] and st["step_length"] == [1.0] * st["newton_its"]
    xo, _ = newton.solve(ops, dc, ph, tol=1e-14, precond="exact")
    xg = x.cpu().numpy()[rec]
    u, p = slice(0, g.nu), g.p_slice
    eu, ep = rel(xg[u], xo[u]), rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean())
    _say("gPNM newton %s: its %s, u err %.2e p err %.2e" % (precision, st["lin_its"], eu, ep))
    assert eu <= tol and ep <= tol
