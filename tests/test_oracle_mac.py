"""Pins of the oracle's MAC discretisation and Newton driver (CPU only).

Closed forms and invariants: plane Poiseuille flow (exact on the MAC grid),
discrete divergence at convergence, the Jacobian against finite differences,
quadratic Newton convergence, symmetry of the Stokes matrix (the paper states
the Stokes block is symmetric, Section 2), and every Newton correction against
a direct sparse solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.mac import MacGrid, Operators, Phys, residual, jacobian, build_matrix, origin_rhs
from oracle.decomp import decompose, largest_component
from oracle import newton
from synth import make_workload, channel


def poiseuille_profile(n, rho, b, mu, h):
    """Discrete plane Poiseuille velocity of an n-cell channel with the wall
    half a cell beyond the last face row: (rho b h^2 / 2 mu) ((n^2+1)/4 - (j-(n-1)/2)^2).
    It equals the continuous profile rho b y (H - y) / (2 mu) plus rho b h^2 / (8 mu)."""
    j = np.arange(n)
    return (rho * b * h * h / (2 * mu)) * ((n * n + 1) / 4.0 - (j - (n - 1) / 2.0) ** 2)


@pytest.mark.parametrize("dims,h", [((1, 7, 10), 1.0), ((1, 12, 6), 0.5), ((5, 9, 6), 1.0)])
def test_plane_poiseuille_exact(dims, h):
    nz, ny, nx = dims
    mask = channel(nx, ny, nz)
    per = (True, False, True)
    g = MacGrid(mask, h=h, periodic=per)
    ops = Operators(g)
    rho, mu, b = 1.3, 0.7, 0.9
    labels = np.ones_like(mask, dtype=np.int32)
    dc = decompose(g, labels)
    ph = Phys(rho, mu, (b, 0.0, 0.0), None, dc.pin)
    x, st = newton.solve(ops, dc, ph, tol=1e-13, lin_tol=1e-14, wind="zero")
    assert st.converged and st.newton_its == 1
    u = x[g.comp_slice(0)]
    ref = np.tile(poiseuille_profile(ny, rho, b, mu, h)[None, :, None], (nz, 1, nx))
    ref = ref[g.act[0]]
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
    for c in g.comps[1:]:
        assert np.max(np.abs(x[g.comp_slice(c)])) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(x[g.p_slice])) <= 1e-12 * np.max(np.abs(ref))
    # the residual vanishes at the closed form itself
    xc = np.zeros(g.N)
    xc[g.comp_slice(0)] = ref
    r = residual(ops, xc, ph)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(origin_rhs(ops, ph))


def _small_case(name="disks2d_32", seed=0, re=None):
    w = make_workload(name, seed, re=re)
    mask = largest_component(w["mask"])
    g = MacGrid(mask)
    ops = Operators(g)
    dc = decompose(g, w["labels"])
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    return g, ops, dc, ph


def divergence(g, x):
    div = np.zeros(g.fluid.shape)
    for c in g.comps:
        uf = np.zeros(g.fluid.shape)
        uf[g.act[c]] = x[g.comp_slice(c)]
        div += (g.shift(uf, c, +1, 0.0) - uf) / g.h
    return div[g.fluid]


@pytest.mark.parametrize("re", [1.0, 10.0])
def test_divergence_free_at_convergence(re):
    g, ops, dc, ph = _small_case(re=re)
    x, st = newton.solve(ops, dc, ph, tol=1e-12, lin_tol=1e-13)
    assert st.converged
    u = x[:g.nu]
    d = divergence(g, x)
    assert np.max(np.abs(d)) * g.h / np.max(np.abs(u)) <= 1e-12


@pytest.mark.parametrize("name", ["disks2d_32", "spheres3d_24"])
def test_jacobian_matches_finite_differences(name):
    g, ops, dc, ph = _small_case(name)
    ph = Phys(ph.rho, ph.mu, (0.5, 0.2, 0.1), 0.3, ph.pin)
    rng = np.random.default_rng(1)
    # velocities bounded away from zero keep every upwind branch fixed under
    # the perturbation (the Jacobian freezes the branch)
    x = rng.standard_normal(g.N)
    x[:g.nu] = 1.0 + 0.2 * rng.random(g.nu)
    xo = rng.standard_normal(g.N)
    v = rng.standard_normal(g.N)
    J = jacobian(ops, x, ph)
    errs = []
    for eps in (1e-3, 1e-4):
        d = residual(ops, x + eps * v, ph, x_old=xo) - residual(ops, x, ph, x_old=xo) - eps * (J @ v)
        errs.append(np.linalg.norm(d))
    # second order: a tenfold smaller step gives about a hundredfold smaller error
    assert errs[1] < errs[0] / 50.0


def test_newton_converges_quadratically():
    g, ops, dc, ph = _small_case(re=10.0)
    x, st = newton.solve(ops, dc, ph, tol=1e-14, precond="exact")
    r = np.array(st.res_hist)
    assert st.converged
    # once in the asymptotic regime: log r_{k+1} / log r_k >= 1.8
    rates = [np.log(r[k + 1]) / np.log(r[k]) for k in range(len(r) - 1)
             if 1e-12 < r[k] < 1e-2 and r[k + 1] > 1e-15]
    assert rates and min(rates) >= 1.8


def test_stokes_matrix_symmetric_except_pin():
    g, ops, dc, ph = _small_case("spheres3d_24")
    X = build_matrix(ops, ph, tags=dc.tags).toarray()
    pin = g.nu + ph.pin
    D = X - X.T
    D[pin, :] = 0.0
    D[:, pin] = 0.0
    assert np.max(np.abs(D)) == 0.0


def test_wind_zero_build_matrix_is_stokes_jacobian():
    g, ops, dc, ph = _small_case()
    X0 = build_matrix(ops, ph, wind=None, tags=dc.tags)
    J0 = jacobian(ops, np.zeros(g.N), ph)
    Xs = build_matrix(ops, ph, wind=None, tags=None)
    assert abs(X0 - J0).max() == 0.0 and abs(X0 - Xs).max() == 0.0


def test_oseen_residual_is_affine_in_x():
    g, ops, dc, ph = _small_case("spheres3d_24")
    rng = np.random.default_rng(2)
    w = rng.standard_normal(g.N)
    v = rng.standard_normal(g.N)
    X = build_matrix(ops, ph, wind=w, tags=dc.tags)
    d = residual(ops, v, ph, wind=w, tags=dc.tags) - residual(ops, np.zeros(g.N), ph, wind=w, tags=dc.tags)
    assert np.linalg.norm(d - X @ v) <= 1e-13 * np.linalg.norm(d)


def test_newton_corrections_match_direct_solve():
    g, ops, dc, ph = _small_case(re=3.0)
    from oracle import gplmm as G
    from oracle.krylov import fgmres
    M = newton.build_precond(ops, dc, ph, None)
    x = np.zeros(g.N)
    for _ in range(3):
        r = residual(ops, x, ph)
        J = jacobian(ops, x, ph)
        d, its, ok = fgmres(lambda v: J @ v, -r, lambda v: G.apply(M, v),
                            1e-14 * np.linalg.norm(r), m=30, maxit=400)
        ds = spla.spsolve(J.tocsc(), -r)
        assert ok
        assert np.linalg.norm(d - ds) <= 1e-10 * np.linalg.norm(ds)
        x = x + ds


def test_dense_newton_matches_sparse_newton():
    w = make_workload("disks2d_32", 3, re=5.0)
    mask = largest_component(w["mask"])[:, 4:12, 6:20].copy()
    mask = largest_component(mask)
    g = MacGrid(mask)
    ops = Operators(g)
    labels = np.ones_like(mask, dtype=np.int32)
    dc = decompose(g, labels)
    ph = Phys(1.0, 1.0, (2.0, 0.3, 0.0), None, dc.pin)
    x = np.zeros(g.N)
    for _ in range(8):
        r = residual(ops, x, ph)
        J = jacobian(ops, x, ph).toarray()
        x = x + np.linalg.solve(J, -r)
    xs, st = newton.solve(ops, dc, ph, tol=1e-14, precond="exact", maxit=8)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
