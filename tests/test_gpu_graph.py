"""The preconditioner application replayed from a HIP graph gives bitwise the
result of the same kernels launched one by one: several replays with other eager
work and synchronisations in between, after a rebuild with a new wind, after new
launch parameters (recapture), and inside a whole Newton solve."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(name, precision, use_graph):
    from paper_2510_22077_amd import Solver
    from synth import make_workload
    w = make_workload(name, 0)
    return Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=precision,
                  use_graph=use_graph)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replays_match_eager_launches(precision):
    torch = _torch()
    s = _solver("spheres3d_24", precision, True)
    s.build()
    g = torch.Generator(device="cuda").manual_seed(3)
    for rep in range(4):
        v = s.residual(torch.randn(s.N, dtype=torch.float64, device="cuda", generator=g))
        zg = s.precond_apply(v).clone()          # graph replay
        _ = torch.linalg.norm(v) * 2.0           # unrelated eager work in between
        torch.cuda.synchronize()
        s.set_timing(True)                       # timed runs launch kernel by kernel
        ze = s.precond_apply(v).clone()
        s.set_timing(False)
        assert torch.equal(zg, ze), rep
    # new wind: same buffers, new contents
    wind = s.residual(torch.randn(s.N, dtype=torch.float64, device="cuda", generator=g)) * 1e-2
    s.build(wind)
    v = s.residual(torch.randn(s.N, dtype=torch.float64, device="cuda", generator=g))
    zg = s.precond_apply(v).clone()
    s.set_timing(True)
    ze = s.precond_apply(v).clone()
    s.set_timing(False)
    assert torch.equal(zg, ze)
    # new launch parameters: the graph is captured again
    s.set_tuning(red_blocks=512, stencil_block=128, trsv_mode=1)
    zg = s.precond_apply(v).clone()
    s.set_timing(True)
    ze = s.precond_apply(v).clone()
    s.set_timing(False)
    assert torch.equal(zg, ze)
    s.close()


def test_newton_solve_with_and_without_graph():
    torch = _torch()
    a = _solver("disks2d_64", "fp32", True)
    b = _solver("disks2d_64", "fp32", False)
    xa, sa = a.newton_solve()
    xb, sb = b.newton_solve()
    assert sa["converged"] and sb["converged"]
    assert sa["lin_its"] == sb["lin_its"]
    assert torch.equal(xa, xb)
    a.close()
    b.close()
