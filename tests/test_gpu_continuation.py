"""Reynolds-number continuation on the GPU (gplmm_continuation; the protocol of Section 8:
the driving force raised in steps, Newton warm-started from the previous step, each
step's preconditioner built from the previous velocity).

The steady solution at the full force is unique, so the continuation must end where a
direct FP64 oracle solve ends: u and the mean-free p to 1e-10 relative (FP64 mode, Newton
to 1e-13, every step a full step).  Bad scale lists are refused.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import newton
from tests.helpers import oracle_case, record_index, rel, workload


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("name,seed,re", [("disks2d_32", 2, 10.0), ("spheres3d_24", 0, 20.0)])
def test_continuation_ends_at_the_oracle_solution(name, seed, re):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22077_amd import Solver
    w = workload(name, seed, re=re)
    _say("case continuation", name, seed, re)
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], newton_tol=1e-13, lin_tol=1e-14)
    x, steps, rc = s.continuation([0.25, 0.5, 1.0])
    assert rc == 0
    assert len(steps) == 3 and all(st["converged"] for st in steps)
    for st in steps:
        assert st["step_length"] == [1.0] * st["newton_its"]
    assert steps[1]["builds"] == 1 and steps[2]["builds"] == 1
    _say("continuation newton its", [st["newton_its"] for st in steps],
         "fgmres", [st["lin_its_total"] for st in steps])
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec = record_index(g, s.maps()["cell_voxel"])
    xo, _ = newton.solve(ops, dc, ph, tol=1e-14, precond="exact")
    xg = x.cpu().numpy()[rec]
    assert rel(xg[:g.nu], xo[:g.nu]) <= 1e-10
    p = g.p_slice
    assert rel(xg[p] - xg[p].mean(), xo[p] - xo[p].mean()) <= 1e-10
    # the context keeps its full force: a direct solve from the result is already converged
    x2, st2 = s.newton_solve(x0=x)
    assert st2["converged"] and st2["newton_its"] == 0
    s.close()


def test_continuation_rejects_bad_scales():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_22077_amd import Solver
    from paper_2510_22077_amd.binding import GplmmError
    w = workload("disks2d_32", 0)
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"])
    for bad in ([0.5, 0.5, 1.0], [0.5, 0.8], [0.0, 1.0], [0.5, 1.2], [1.0, 0.5, 1.0]):
        with pytest.raises(GplmmError):
            s.continuation(bad)
    s.close()
