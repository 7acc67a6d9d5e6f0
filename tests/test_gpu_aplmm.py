"""GPU parity of the algebraic variants (Sections 3 and 8): the preconditioner built from
the Newton Jacobian J(w) at a state w (build_matrix = "jacobian", untagged) instead of the
gPLMM matrix X = J~_w, through the C ABI, against the oracle built from the same matrix.

* J(w) v from the tabulated rows (with the transverse couplings of the advecting
  velocity) against the oracle's Jacobian, 1e-13;
* the preconditioner application, FP64 to 1e-11 and FP32 to 5e-3 (the bars of the gPLMM
  application tests);
* aPLMM_S = gPLMM with w = 0 (Section 8): both library builds at zero wind equal the
  oracle built from the Stokes matrix, 1e-11;
* aPLMM_NS Newton solves (rebuilt from J at the first iterate): FP64 solution within
  1e-10 and FP32 within 1e-8 of the oracle's exact Newton solution, full steps, and
  FP64 FGMRES counts within 2 per Newton step of the oracle's aPLMM_NS run.
"""
import sys

import numpy as np
import pytest

from oracle import gplmm as G
from oracle import newton
from oracle.mac import build_matrix as build_matrix_of, jacobian, origin_rhs
from tests.helpers import oracle_case, record_index, rel, to_record, workload

pytestmark = pytest.mark.gpu


def build_matrix_stokes(ops, ph):
    return build_matrix_of(ops, ph, wind=None, tags=None)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(torch, a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def _setup(name, seed, re=None, **kw):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22077_amd import Solver
    w = workload(name, seed, re=re)
    _say("case aplmm", name, seed, kw)
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], **kw)
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    return torch, s, g, ops, dc, ph, rec


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 5e-3)])
@pytest.mark.parametrize("name,seed", [("disks2d_32", 0), ("disks2d_64", 1), ("spheres3d_24", 0)])
def test_jacobian_built_preconditioner_matches_the_oracle(name, seed, precision, tol):
    torch, s, g, ops, dc, ph, rec = _setup(name, seed, precision=precision, build_matrix="jacobian")
    rng = np.random.default_rng(30 + seed)
    state = rng.standard_normal(g.N)
    s.build(_dev(torch, to_record(state, rec, s.N)))
    J = jacobian(ops, state, ph)
    v = rng.standard_normal(g.N)
    vr = _dev(torch, to_record(v, rec, s.N))
    if precision == "fp64":
        y = s.build_matvec(vr).cpu().numpy()
        assert rel(y[rec], J @ v) <= 1e-13
    M = G.build(J, dc, origin_rhs(ops, ph))
    z = s.precond_apply(vr).cpu().numpy()
    err = rel(z[rec], G.apply(M, v))
    _say("aPLMM apply rel err", err)
    assert err <= tol


@pytest.mark.parametrize("build_matrix", ["geometric", "jacobian"])
def test_aplmm_s_equals_zero_wind_build(build_matrix):
    """Both library builds at zero wind against the oracle built from the Stokes matrix."""
    torch, s, g, ops, dc, ph, rec = _setup("spheres3d_24", 1, build_matrix=build_matrix)
    s.build(None)
    M = G.build(build_matrix_stokes(ops, ph), dc, origin_rhs(ops, ph))
    v = np.random.default_rng(5).standard_normal(g.N)
    z = s.precond_apply(_dev(torch, to_record(v, rec, s.N))).cpu().numpy()
    err = rel(z[rec], G.apply(M, v))
    _say("aPLMM_S apply rel err", build_matrix, err)
    assert err <= 1e-11


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
@pytest.mark.parametrize("name,seed,re", [("disks2d_32", 1, 10.0), ("spheres3d_24", 0, 10.0)])
def test_aplmm_ns_newton_solution(name, seed, re, precision, tol):
    torch, s, g, ops, dc, ph, rec = _setup(name, seed, re=re, precision=precision, build_matrix="jacobian",
                                           newton_tol=1e-12, lin_tol=1e-13)
    x, st = s.newton_solve()
    assert st["converged"] and st["step_length"] == [1.0] * st["newton_its"]
    xo, _ = newton.solve(ops, dc, ph, tol=1e-14, precond="exact")
    xg = x.cpu().numpy()[rec]
    u, p = slice(0, g.nu), g.p_slice
    eu, ep = rel(xg[u], xo[u]), rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean())
    xa, sa = newton.solve(ops, dc, ph, tol=1e-12, lin_tol=1e-13, build="jacobian")
    _say("aPLMM_NS %s: gpu its %s oracle its %s, u err %.2e p err %.2e" % (precision, st["lin_its"], sa.lin_its, eu, ep))
    assert eu <= tol and ep <= tol
    if precision == "fp64":
        assert st["newton_its"] == sa.newton_its
        assert all(abs(a - b) <= 2 for a, b in zip(st["lin_its"], sa.lin_its))
