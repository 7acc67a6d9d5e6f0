"""GPU parity of the coarse-scale solver (Section 5, Algorithm 1) through the C ABI.

The library's gplmm_coarse_solve against the oracle's coarse_solver.solve on the same
inputs.  Both stop a body-force step when the coarse residual falls below tol of its
start; run at tol = 1e-10 the approximate solution is the fixed point of the coarse
iteration, which FP64 reaches to rounding (compared to 1e-9; the coarse Jacobian is
assembled by probing and inverted explicitly) and the FP32-prolongation mode to the
rounding of its FP32 shape vectors (1e-4).  The slab channel gives plane Poiseuille flow
exactly at Re > 1 (closed form, 1e-12).
"""
import sys

import numpy as np
import pytest

from oracle import coarse_solver as CS
from oracle.mac import MacGrid, Operators, Phys
from oracle.decomp import decompose
from synth import channel
from tests.helpers import oracle_case, record_index, rel, workload

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
@pytest.mark.parametrize("name,seed,re,inc", [("disks2d_64", 1, 1.0, 1), ("disks2d_64", 1, 10.0, 4),
                                              ("spheres3d_24", 0, 1.0, 1), ("spheres3d_24", 0, 5.0, 2)])
def test_coarse_solver_matches_the_oracle(name, seed, re, inc, precision, tol):
    _torch()
    from paper_2510_22077_amd import Solver
    w = workload(name, seed, re=re)
    _say("case coarse solve", name, seed, re, inc, precision)
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=precision)
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    x, st = s.coarse_solve(increments=inc, tol=1e-10)
    xo, sto, _ = CS.solve(ops, dc, ph, increments=inc, tol=1e-10)
    xg = x.cpu().numpy()[rec]
    u, p = slice(0, g.nu), g.p_slice
    eu = rel(xg[u], xo[u])
    ep = rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean())
    _say("  gpu its", st["newton_its"], "oracle its", sto.newton_its, "u err %.2e p err %.2e" % (eu, ep),
         "fine residual %.2e" % st["fine_rel_residual"])
    assert st["converged"] and sto.converged
    assert eu <= tol and ep <= tol
    # the default stopping rule (1e-6) holds on the GPU as well
    x6, st6 = s.coarse_solve(increments=inc)
    assert st6["converged"] and all(r < 1e-6 for r in st6["rc_rel"])
    s.close()


def test_coarse_solver_slab_channel_is_poiseuille():
    _torch()
    from paper_2510_22077_amd import Solver
    from tests.test_oracle_mac import poiseuille_profile
    nz, ny, nx = 6, 8, 24
    m = channel(nx, ny, nz)
    lab = np.zeros_like(m, dtype=np.int32)
    for k in range(4):
        lab[:, :, 6 * k:6 * (k + 1)] = k + 1
    rho, mu, b = 1.0, 0.05, 0.4
    s = Solver(m, lab, rho=rho, mu=mu, body=(b, 0.0, 0.0), periodic=(1, 0, 1))
    x, st = s.coarse_solve(increments=2)
    assert st["converged"]
    xr = x.cpu().numpy().reshape(-1, 4)
    ref = np.tile(poiseuille_profile(ny, rho, b, mu, 1.0)[None, :, None], (nz, 1, nx))
    assert np.max(np.abs(xr[:, 0].reshape(nz, ny, nx) - ref)) <= 1e-12 * ref.max()
    assert np.max(np.abs(xr[:, 1:])) <= 1e-12 * ref.max()
    assert st["fine_rel_residual"] <= 1e-11   # the residual of the closed form in FP64 rounding
    s.close()


def test_coarse_solver_rejects_what_it_does_not_cover():
    _torch()
    from paper_2510_22077_amd import Solver, binding
    w = workload("disks2d_32", 0)
    s = Solver(w["mask"], w["labels"], body=w["body"], tag_layers=0)
    with pytest.raises(binding.GplmmError):
        s.coarse_solve()
    s.close()
    s = Solver(w["mask"], w["labels"], body=w["body"], dt=0.1)
    with pytest.raises(binding.GplmmError):
        s.coarse_solve()
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_coarse_solver_on_a_crop_of_the_benchmark_packing(precision, tol):
    """The 48^3 corner of the 128^3 packing (about 110 pores, 400 interfaces): many
    columns per probing colour."""
    _torch()
    from paper_2510_22077_amd import Solver
    w = workload("spheres3d_128", 0)
    m, lab = w["mask"][:48, :48, :48].copy(), w["labels"][:48, :48, :48].copy()
    _say("case coarse solve crop 48", precision)
    s = Solver(m, lab, rho=w["rho"], mu=w["mu"], body=w["body"], precision=precision)
    g, ops, dc, ph = oracle_case(m, lab, w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    x, st = s.coarse_solve(increments=1, tol=1e-10)
    xo, sto, _ = CS.solve(ops, dc, ph, increments=1, tol=1e-10)
    xg = x.cpu().numpy()[rec]
    u, p = slice(0, g.nu), g.p_slice
    eu = rel(xg[u], xo[u])
    ep = rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean())
    _say("  gpu its", st["newton_its"], st["rc_rel"], "oracle its", sto.newton_its, "u err %.2e p err %.2e" % (eu, ep))
    assert st["converged"] and sto.converged
    assert eu <= tol and ep <= tol
    s.close()
