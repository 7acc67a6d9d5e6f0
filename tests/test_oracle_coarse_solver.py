"""Pins of the oracle's coarse-scale Navier-Stokes solver (Section 5, Algorithm 1; CPU).

* the tagged Jacobian (the derivative of the residual whose tagged faces carry no
  inertia) against central finite differences of that residual;
* Remark 2: for the Stokes equations the coarse Newton iteration stops after one
  step, at Phat (Rhat A Phat)^-1 Rhat b, i.e. the Remark-1 M_G^-1 applied to b;
* a channel cut into slabs: the coarse solution is plane Poiseuille flow exactly, at
  any Reynolds number and with any number of increments (the closure problems of the
  slabs hold fully developed flow, whose inertia vanishes on the MAC grid);
* on a disk packing the coarse residual falls below 1e-6 of its start at every
  increment (the stopping rule of Algorithm 1), and the approximate solution is
  reported against the fine Newton solution.
"""
import numpy as np
import pytest

from oracle.mac import MacGrid, Operators, Phys, residual, jacobian, build_matrix, origin_rhs
from oracle.decomp import decompose, largest_component
from oracle import gplmm as G
from oracle import coarse_solver as CS
from oracle import newton
from synth import make_workload, channel
from tests.test_oracle_mac import poiseuille_profile


def _case(name, seed, re):
    w = make_workload(name, seed, re=re)
    g = MacGrid(largest_component(w["mask"]))
    ops = Operators(g)
    dc = decompose(g, w["labels"])
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    return g, ops, dc, ph


def test_tagged_jacobian_matches_finite_differences():
    g, ops, dc, ph = _case("disks2d_32", 0, 10.0)
    rng = np.random.default_rng(3)
    x = 0.5 + rng.random(g.N)      # positive velocities: no upwind branch changes under the probe
    v = rng.standard_normal(g.N)
    J = jacobian(ops, x, ph, tags=dc.tags)
    eps = 1e-6
    fd = (residual(ops, x + eps * v, ph, tags=dc.tags) - residual(ops, x - eps * v, ph, tags=dc.tags)) / (2 * eps)
    assert np.linalg.norm(J @ v - fd) <= 1e-8 * np.linalg.norm(fd)
    # and it differs from the untagged Jacobian exactly on the tagged rows
    J0 = jacobian(ops, x, ph)
    diff = np.abs((J - J0) @ v)[:g.nu] > 0
    tagged = np.concatenate(dc.tags)
    assert np.all(tagged[diff])


def test_stokes_coarse_solve_is_one_step_of_remark1_mg():
    g, ops, dc, ph = _case("disks2d_64", 0, 1.0)
    x, st, M = CS.solve(ops, dc, ph, increments=1, stokes=True)
    assert st.newton_its == [1] and st.converged
    b = origin_rhs(ops, ph)
    Xs = build_matrix(ops, ph, tags=dc.tags)
    Ms = G.build(Xs, dc, b)
    ref = G.apply_MG(Ms, b)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert st.rc_rel[0] <= 1e-12


@pytest.mark.parametrize("dims,increments", [((1, 8, 24), 1), ((1, 8, 24), 3), ((6, 8, 24), 2)])
def test_slab_channel_coarse_solution_is_poiseuille(dims, increments):
    nz, ny, nx = dims
    m = channel(nx, ny, nz)
    lab = np.zeros_like(m, dtype=np.int32)
    for s in range(4):
        lab[:, :, s * 6:(s + 1) * 6] = s + 1
    per = (True, False, True) if nz > 1 else (True, False, False)
    g = MacGrid(m, periodic=per)
    ops = Operators(g)
    dc = decompose(g, lab)
    rho, mu, b = 1.0, 0.05, 0.4            # Re well above 1 on this channel
    ph = Phys(rho, mu, (b, 0.0, 0.0), None, dc.pin)
    x, st, _ = CS.solve(ops, dc, ph, increments=increments)
    assert st.converged
    u = x[g.comp_slice(0)]
    ref = np.tile(poiseuille_profile(ny, rho, b, mu, 1.0)[None, :, None], (nz, 1, nx))[g.act[0]]
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(ref)
    assert np.max(np.abs(x[g.nu:])) <= 1e-12 * np.max(ref)


@pytest.mark.parametrize("re,increments", [(1.0, 1), (10.0, 4)])
def test_coarse_solver_converges_on_a_disk_packing(re, increments):
    """The increments keep each step of Re small (2.5 here), as the outer loop of
    Algorithm 1 intends: a coarse Newton iteration started far from the solution may
    not converge (measured: a single step to Re 5 from rest stalls at 0.34)."""
    g, ops, dc, ph = _case("disks2d_64", 1, re)
    x, st, _ = CS.solve(ops, dc, ph, increments=increments)
    assert st.converged and all(r < 1e-6 for r in st.rc_rel)
    xf, sf = newton.solve(ops, dc, ph, tol=1e-12, precond="exact")
    e_p, e_u = CS.paper_errors(g, x, xf)
    rf = np.linalg.norm(residual(ops, x, ph)) / np.linalg.norm(residual(ops, np.zeros(g.N), ph))
    print("Re %.0f: coarse Newton %s, E2^p %.1f%%, E2^|u| %.1f%%, fine residual %.2e"
          % (re, st.newton_its, e_p, e_u, rf))
    # accuracy is reported, not pinned: the paper's bounds (E2^p < 3 %, E2^|u| < 6 % in 2D)
    # are for its own images and pressure-driven flow; here a loose sanity bound
    assert e_p < 20.0 and e_u < 50.0
