"""Autotuner of the launch parameters: the measured choice, the cache file, and that
every variant computes the same preconditioner (identical arithmetic, so bitwise) and
the same Newton solution (the reduction block count only reorders FP64 sums)."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(precision):
    from paper_2510_22077_amd import Solver
    from synth import make_workload
    w = make_workload("spheres3d_24", 0)
    return Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=precision,
                  newton_tol=1e-12, lin_tol=1e-13)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_variant_gives_the_same_preconditioner(precision):
    torch = _torch()
    s = _solver(precision)
    s.build()
    v = s.residual(torch.randn(s.N, dtype=torch.float64, device="cuda"))
    s.set_tuning(red_blocks=1024, stencil_block=256, trsv_mode=0)   # the reference: variant 0
    ref = s.precond_apply(v).clone()
    # variants 0 and 1 run the same arithmetic in the same order (bit-identical); variant 2
    # sums each row's tiles in four interleaved groups, a different rounding order: its
    # difference is bounded by a few units of rounding of the local solves' precision
    tol = 1e-11 if precision == "fp64" else 1e-4
    for rb in (256, 2048):
        for sb in (128, 512):
            for tm in (0, 1, 2):
                s.set_tuning(red_blocks=rb, stencil_block=sb, trsv_mode=tm)
                z = s.precond_apply(v)
                if tm < 2:
                    assert torch.equal(z, ref), (rb, sb, tm)
                else:
                    d = float(torch.linalg.norm(z - ref) / torch.linalg.norm(ref))
                    print("variant 2 rel diff", precision, d)
                    assert d <= tol, (rb, sb, tm, d)
    s.close()


def test_autotune_choice_cache_and_solution(tmp_path):
    torch = _torch()
    s = _solver("fp64")
    x0, st0 = s.newton_solve()
    cache = str(tmp_path / "tune.txt")
    t = s.autotune(cache)
    print("tuning", t)
    assert t["from_cache"] == 0
    assert t["red_blocks"] in (256, 512, 1024, 2048)
    assert t["stencil_block"] in (128, 256, 512) and t["trsv_mode"] in (0, 1, 2)
    assert t["t_trsv_ms"] > 0 and t["t_reduction_ms"] > 0 and t["t_stencil_ms"] > 0
    assert os.path.getsize(cache) > 0
    x1, st1 = s.newton_solve()
    assert st1["converged"]
    assert float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0)) <= 1e-10
    t2 = s.autotune(cache)
    assert t2["from_cache"] == 1
    assert (t2["red_blocks"], t2["stencil_block"], t2["trsv_mode"]) == (t["red_blocks"], t["stencil_block"],
                                                                         t["trsv_mode"])
    s.close()
