"""The allocation-free residual-norm entry point against gplmm_sample_residuals.

gplmm_sample_residuals_noalloc keeps its partial sums in a static device array shared by
every call on the GPU.  Two calls in a row, the second on a smaller context, must both
give the norms of gplmm_sample_residuals (same arithmetic, another summation order: to
1e-12 relative), and a further call must leave the device's free memory unchanged.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _random_state(s, seed):
    """A random vector on the context's unknowns (void slots zero)."""
    g = torch.Generator().manual_seed(seed)
    info = s.info()
    x = torch.randn(info["N"], generator=g, dtype=torch.float64)
    void = torch.from_numpy(s.maps()["face_owner"] == -2)
    x[void] = 0.0
    return x.cuda()


def _check(s, seed, x_prev=None):
    x = _random_state(s, seed)
    ref = s.sample_residuals(x, x_prev)
    out = torch.full((len(ref),), float("nan"), dtype=torch.float64, device="cuda")
    s.sample_residuals_noalloc(x, out, x_prev)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref) / np.abs(ref)) <= 1e-12, (got, ref)
    return x


def test_noalloc_residual_norms_match_two_calls_second_smaller():
    from paper_2510_22077_amd import Solver, BatchSolver
    from synth import make_workload
    ws = [make_workload("disks2d_32", k) for k in range(3)] + [make_workload("spheres3d_24", 0)]
    ws = ws[:3]
    big = BatchSolver([w["mask"] for w in ws], [w["labels"] for w in ws], bodies=[w["body"] for w in ws],
                      dt=[0.05, 0.0, 0.02])
    xb = _check(big, 1)
    _check(big, 2, x_prev=xb * 0.5)
    w = make_workload("disks2d_32", 4)
    small = Solver(w["mask"], w["labels"], body=w["body"])
    assert small.info()["N"] < big.info()["N"]
    _check(small, 3)
    # a repeated call allocates nothing on the device
    x = _random_state(small, 5)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    small.sample_residuals_noalloc(x, out)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        small.sample_residuals_noalloc(x, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    small.close()
    big.close()


def test_noalloc_3d_single_image():
    from paper_2510_22077_amd import Solver
    from synth import make_workload
    w = make_workload("spheres3d_24", 0)
    s = Solver(w["mask"], w["labels"], body=w["body"])
    _check(s, 7)
    s.close()
