"""Parity at the full sizes of the benchmark configurations, where the oracle
cannot solve the whole problem: the GPU Newton-FGMRES-gPLMM solve is run exactly
as bench.py times it, and

* the residual the library computes is checked unknown by unknown, on a random
  sample of faces and cells, against the oracle's residual evaluated on a small
  window of the image around each sampled unknown (every term of a row lives
  within two cells of it; a window of radius 3 holds the whole stencil);
* those oracle residuals of the converged solution are below the tolerance the
  solve claims (||r|| <= 1e-8 ||r(0)||, with ||r(0)|| = rho |b| sqrt(#active
  faces along b) counted from the image);
* the discrete divergence of the converged velocity, formed with numpy from the
  face values, is within the same bound on every kept cell but the pinned one.
"""
import numpy as np
import pytest

from oracle.decomp import largest_component
from oracle.mac import MacGrid, Operators, Phys, residual

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _window_residuals(fluid, periodic, x_rec, nrec, vox2cell, samples, rho, mu, body, pin_cell, R=3):
    """Oracle residual at each sampled unknown (kind, k, j, i), from a (2R+1)^ndim window."""
    nz, ny, nx = fluid.shape
    nd = 2 if nz == 1 else 3
    out = []
    for kind, k, j, i in samples:
        ks = [k] if nd == 2 else list(range(k - R, k + R + 1))
        js, is_ = list(range(j - R, j + R + 1)), list(range(i - R, i + R + 1))

        def idx(vals, n, per):
            v = np.array(vals)
            ok = (v >= 0) & (v < n)
            if per:
                return v % n, np.ones_like(ok)
            return np.clip(v, 0, n - 1), ok

        kk, okk = idx(ks, nz, nd == 3 and periodic[2])
        jj, okj = idx(js, ny, periodic[1])
        ii, oki = idx(is_, nx, periodic[0])
        win = fluid[np.ix_(kk, jj, ii)] & okk[:, None, None] & okj[None, :, None] & oki[None, None, :]
        g = MacGrid(win, periodic=(False, False, False))
        ops = Operators(g)
        co = g.unknown_coords()
        gk, gj, gi = kk[co[:, 1]], jj[co[:, 2]], ii[co[:, 3]]
        cell = vox2cell[(gk * ny + gj) * nx + gi]
        assert np.all(cell >= 0)
        comp = np.where(co[:, 0] == 3, nd, co[:, 0])
        xw = x_rec[nrec * cell + comp]
        ck = 0 if nd == 2 else R
        center = np.flatnonzero((co[:, 0] == kind) & (co[:, 1] == ck) & (co[:, 2] == R) & (co[:, 3] == R))
        assert center.size == 1
        # pin: a window cell that is not the centre (the pinned row is p = 0 and is never sampled)
        wcells = np.flatnonzero(co[:, 0] == 3)
        wpin = int([c for c in range(wcells.size) if wcells[c] != center[0]][0])
        r = residual(ops, xw, Phys(rho, mu, tuple(body), None, wpin))
        out.append(r[center[0]])
    return np.array(out)


def _full_size_case(name, precision, restart, n_samples, seed=0):
    torch = _torch()
    from paper_2510_22077_amd import Solver
    from synth import make_workload
    w = make_workload(name, seed)
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], precision=precision,
               restart=restart, newton_tol=1e-8, lin_tol=1e-9, lin_maxit=3000)
    x, st = s.newton_solve()
    assert st["converged"], st
    m = s.maps()
    info = s.info()
    nrec, nd = info["nrec"], info["ndim"]
    mask = w["mask"] if w["mask"].ndim == 3 else w["mask"][None]
    periodic = (True, False, False)
    fluid = largest_component(mask.astype(bool), periodic)
    assert np.array_equal(np.flatnonzero(fluid), m["cell_voxel"])
    vox2cell = np.full(fluid.size, -1, dtype=np.int64)
    vox2cell[m["cell_voxel"]] = np.arange(m["cell_voxel"].size)
    xr = x.cpu().numpy()
    r_gpu = s.residual(x).cpu().numpy()
    # ||r(0)||: rho |b_a| on every active a-face, zero on cells
    gfull = MacGrid(fluid, periodic=periodic)
    body = np.array(w["body"] + (0.0,) * (3 - len(w["body"])))[:nd]
    r0 = w["rho"] * np.sqrt(sum((body[a] ** 2) * gfull.ncomp[a] for a in range(nd)))
    assert np.linalg.norm(r_gpu) <= 1e-8 * r0 * 1.0001
    # random sample of faces and cells (not the pinned cell)
    rng = np.random.default_rng(7)
    co = gfull.unknown_coords()
    pin_cell = info["pin"]
    pin_vox = m["cell_voxel"][pin_cell]
    pick = rng.choice(gfull.N, size=n_samples, replace=False)
    samples = []
    for t in pick:
        kind, k, j, i = co[t]
        if kind == 3 and (k * gfull.ny + j) * gfull.nx + i == pin_vox:
            continue
        samples.append((int(kind), int(k), int(j), int(i)))
    ro = _window_residuals(fluid, periodic, xr, nrec, vox2cell, samples, w["rho"], w["mu"], body, pin_cell)
    recs = np.array([nrec * vox2cell[(k * gfull.ny + j) * gfull.nx + i] + (nd if kind == 3 else kind)
                     for kind, k, j, i in samples])
    err = np.max(np.abs(r_gpu[recs] - ro))
    print("%s: %d sampled rows, max |r_gpu - r_oracle| = %.3e (||r(0)|| = %.3e), max |r_oracle| = %.3e"
          % (name, len(samples), err, r0, np.max(np.abs(ro))))
    assert err <= 1e-12 * r0
    assert np.max(np.abs(ro)) <= 1e-8 * r0
    # divergence of the converged velocity on every cell but the pin
    X = xr.reshape(-1, nrec)
    div = np.zeros(X.shape[0])
    for a in range(nd):
        lower = X[:, a]
        up_cell = np.full(fluid.shape, -1, dtype=np.int64)
        up_cell.ravel()[m["cell_voxel"]] = np.arange(X.shape[0])
        shifted = gfull.shift(up_cell, a, 1, -1)           # cell + e_a (wrapping on periodic x)
        upper_idx = shifted.ravel()[m["cell_voxel"]]
        upper = np.where(upper_idx >= 0, X[np.maximum(upper_idx, 0), a], 0.0)
        div += upper - lower
    div[pin_cell] = 0.0
    umax = np.max(np.abs(X[:, :nd]))
    print("max |div u| = %.3e (max |u| = %.3e)" % (np.max(np.abs(div)), umax))
    assert np.max(np.abs(div)) <= 1e-8 * r0 * 1.0   # each mass row is div/h, h = 1, within ||r||
    s.close()


def test_benchmark_packing_128_fp32_at_full_size():
    _full_size_case("spheres3d_128", "fp32", 128, 1500)


def test_disk_packing_1024_fp64_at_full_size():
    _full_size_case("disks2d_1024", "fp64", 1024, 1500)
