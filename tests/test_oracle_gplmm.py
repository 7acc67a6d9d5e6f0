"""Pins of the oracle's decomposition, gPLMM preconditioner and FGMRES (CPU).

* the sparse preconditioner against a literal dense transcription of the
  paper's matrices W, Q, P, R, csum and the Schwarz sums (brute force, tiny
  grids);
* special cases with exact answers: one pore (M^-1 = X^-1), a channel cut into
  slabs (M_G^-1 reproduces Poiseuille flow exactly), the Remark-1 coarse
  operator as an oblique projection, sign invariance in b_B, partition of
  unity of the shape vectors, zero row sums of the coarse operator;
* FGMRES with a fixed preconditioner against textbook right-preconditioned
  GMRES (same residual history);
* decomposition invariants (carving separates primaries, p/c/f partition).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.mac import MacGrid, Operators, Phys, build_matrix, origin_rhs, residual
from oracle.decomp import decompose, largest_component
from oracle import gplmm as G
from oracle.literal import literal_preconditioner
from oracle.krylov import fgmres, gmres_right_history
from synth import make_workload, channel
from synth.packing import boolean_packing
from synth.watershed import watershed_labels


def _case(mask, labels, body=(1.0, 0.0, 0.0), periodic=(True, False, False), wind_seed=None,
          dt=None):
    mask = largest_component(mask, periodic)
    g = MacGrid(mask, periodic=periodic)
    ops = Operators(g)
    dc = decompose(g, labels)
    ph = Phys(1.0, 1.0, body, dt, dc.pin)
    wind = None
    if wind_seed is not None:
        wind = np.random.default_rng(wind_seed).standard_normal(g.N)
    X = build_matrix(ops, ph, wind=wind, tags=dc.tags)
    bB = origin_rhs(ops, ph)
    return g, ops, dc, ph, X, bB


def _tiny_2d(seed=0):
    w = make_workload("disks2d_32", seed)
    m = w["mask"][:, 2:14, 3:21].copy()
    lab = watershed_labels(m, footprint=5, min_size=6)
    return m, lab


def _tiny_3d(seed=1):
    m = boolean_packing((6, 8, 9), 2.2, 0.3, 0.5, seed)
    lab = watershed_labels(m, footprint=3, min_size=6)
    return m, lab


@pytest.mark.parametrize("mg_form", [0, 1, 2])
@pytest.mark.parametrize("maker,wind_seed,dt", [(_tiny_2d, None, None), (_tiny_2d, 5, None),
                                                (_tiny_3d, None, None), (_tiny_3d, 7, 0.5)])
def test_sparse_gplmm_matches_literal_matrices(maker, wind_seed, dt, mg_form):
    m, lab = maker()
    g, ops, dc, ph, X, bB = _case(m, lab, body=(1.0, 0.2, 0.1), wind_seed=wind_seed, dt=dt)
    assert dc.Np >= 2 and dc.Nc >= 1
    if mg_form >= 1:
        assert dc.f_faces.size >= 1      # the back-substitution of Eq. xf has work to do
    M = G.build(X, dc, bB, mg_form=mg_form)
    Mlit, MGlit = literal_preconditioner(X.toarray(), dc, bB, mg_form=mg_form)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(g.N)
        z = G.apply(M, v)
        zl = Mlit @ v
        assert np.linalg.norm(z - zl) <= 1e-11 * np.linalg.norm(zl)
        zg = G.apply_MG(M, v)
        assert np.linalg.norm(zg - MGlit @ v) <= 1e-11 * np.linalg.norm(MGlit @ v)


def test_single_pore_preconditioner_is_exact_inverse():
    m = np.ones((5, 7, 8), np.uint8)
    m[1:3, 3, 3:5] = 0
    g, ops, dc, ph, X, bB = _case(m, np.ones_like(m, dtype=np.int32))
    assert dc.Nc == 0 and dc.Np == 1
    M = G.build(X, dc, bB)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(g.N)
    z = G.apply(M, v)
    assert np.linalg.norm(X @ z - v) <= 1e-12 * np.linalg.norm(v)
    x, its, ok = fgmres(lambda a: X @ a, bB, lambda a: G.apply(M, a), 1e-12 * np.linalg.norm(bB))
    assert ok and its == 1


@pytest.mark.parametrize("dims,per", [((1, 8, 24), (True, False, False)),
                                      ((6, 8, 24), (True, False, False)),
                                      ((6, 8, 24), (True, False, True))])
@pytest.mark.parametrize("mg_form", [0, 1, 2])
def test_slab_channel_coarse_solve_is_poiseuille(dims, per, mg_form):
    nz, ny, nx = dims
    m = channel(nx, ny, nz)
    lab = np.zeros_like(m, dtype=np.int32)
    for s in range(4):
        lab[:, :, s * 6:(s + 1) * 6] = s + 1
    g, ops, dc, ph, X, bB = _case(m, lab, periodic=per)
    assert dc.Np == 4 and dc.Nc == 4
    M = G.build(X, dc, bB, mg_form=mg_form)
    xg = G.apply_MG(M, bB)
    xs = spla.spsolve(X.tocsc(), bB)
    assert np.linalg.norm(xg - xs) <= 1e-12 * np.linalg.norm(xs)
    x, its, ok = fgmres(lambda a: X @ a, bB, lambda a: G.apply(M, a), 1e-12 * np.linalg.norm(bB))
    assert ok and its == 1


def test_remark1_coarse_operator_is_a_projection():
    m, lab = _tiny_3d()
    g, ops, dc, ph, X, bB = _case(m, lab, wind_seed=3)
    M = G.build(X, dc, bB)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(g.N)
    a = G.apply_MG(M, X @ v)
    b = G.apply_MG(M, X @ a)
    assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(a)


def test_column_summed_form_is_not_a_projection():
    """Proposition 1: with the column-summed operator of Eq. iMG, M_G^-1 A is not a
    projection (it is one in the Remark-1 form, previous test); the x^f of Eq. xf makes
    A z_G and the right-hand side agree on the f rows."""
    m, lab = _tiny_3d()
    g, ops, dc, ph, X, bB = _case(m, lab, wind_seed=3)
    M = G.build(X, dc, bB, mg_form=1)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(g.N)
    a = G.apply_MG(M, X @ v)
    b = G.apply_MG(M, X @ a)
    assert np.linalg.norm(a - b) >= 1e-6 * np.linalg.norm(a)
    F = dc.f_faces
    assert F.size >= 1
    w = rng.standard_normal(g.N)
    z = G.apply_MG(M, w)
    assert np.linalg.norm((X @ z - w)[F]) <= 1e-11 * np.linalg.norm(w)


def test_correction_sign_does_not_change_coarse_operator():
    m, lab = _tiny_2d()
    g, ops, dc, ph, X, bB = _case(m, lab)
    M1 = G.build(X, dc, bB)
    M2 = G.build(X, dc, -bB)
    v = np.random.default_rng(5).standard_normal(g.N)
    a, b = G.apply_MG(M1, v), G.apply_MG(M2, v)
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


def test_shape_vectors_partition_of_unity():
    m, lab = _tiny_3d()
    g, ops, dc, ph, X, bB = _case(m, lab, wind_seed=9)
    M = G.build(X, dc, bB)
    pin_prim = dc.prim[dc.pin]
    for i in range(dc.Np):
        if i == pin_prim or dc.Cp[i].size == 0:
            continue
        s = M.phi[i].sum(1)
        S = dc.S[i]
        want = (S >= g.nu).astype(float)       # u = 0, p = 1
        assert np.max(np.abs(s - want)) <= 1e-11


def test_coarse_interface_columns_sum_to_zero_away_from_pin():
    m, lab = _tiny_2d(1)
    g, ops, dc, ph, X, bB = _case(m, lab)
    M = G.build(X, dc, bB)
    rows = M.Ao[:, :dc.Nc].sum(1)
    # rows whose restriction stencil never reaches the pin's primary
    pin_prim = dc.prim[dc.pin]
    Spin = set(dc.S[pin_prim].tolist())
    far = []
    Xc = X.tocsr()
    for q in range(M.Ao.shape[0]):
        rowset = dc.icells[q] if q < dc.Nc else dc.S[M.ycols[q - dc.Nc]]
        cols = set(np.unique(Xc[rowset].indices).tolist())
        if not (cols & Spin) and not (set(rowset.tolist()) & Spin):
            far.append(q)
    assert far
    scale = np.abs(M.Ao).max()
    assert np.max(np.abs(rows[far])) <= 1e-11 * scale


def test_fgmres_fixed_preconditioner_equals_right_gmres():
    m, lab = _tiny_2d(2)
    g, ops, dc, ph, X, bB = _case(m, lab, wind_seed=1)
    M = G.build(X, dc, bB)
    Xd = X.toarray()
    Minv = np.stack([G.apply(M, e) for e in np.eye(g.N)], 1)
    b = np.random.default_rng(3).standard_normal(g.N)
    ref = gmres_right_history(Xd, Minv, b, 12)
    hist = []
    fgmres(lambda a: Xd @ a, b, lambda a: Minv @ a, 0.0, m=12, maxit=12, history=hist)
    hist = np.array(hist[:13])
    # the same minimal-residual iterates: histories agree to rounding
    assert np.max(np.abs(hist - ref)) <= 1e-12 * ref[0]
    ok = ref > 1e-6 * ref[0]
    assert np.max(np.abs(hist[ok] - ref[ok]) / ref[ok]) <= 1e-10


@pytest.mark.parametrize("name,seed", [("disks2d_64", 0), ("spheres3d_24", 0), ("spheres3d_24", 2)])
def test_decomposition_invariants(name, seed):
    w = make_workload(name, seed)
    mask = largest_component(w["mask"])
    g = MacGrid(mask)
    dc = decompose(g, w["labels"])
    # p (primaries' unknowns), c (interface cells), f (faces between interface cells) partition
    allp = np.concatenate(dc.S)
    allc = np.concatenate(dc.icells)
    parts = np.concatenate([allp, allc, dc.f_faces])
    assert np.array_equal(np.sort(parts), np.arange(g.N))
    # an f-face has two interface cells; a primary face at least one primary cell
    from oracle.decomp import cell_faces
    fc = cell_faces(g)
    for d in g.comps:
        for t in (0, 1):
            f = fc[:, 2 * d + t]
            ok = f >= 0
            own = dc.owner[f[ok]]
            pr = dc.prim[ok]
            assert np.all((pr < 0) | (own == pr))
    # every interface touches a primary, every primary's closure is nonsingular
    X = build_matrix(Operators(g), Phys(1, 1, (1, 0, 0), None, dc.pin), tags=dc.tags)
    M = G.build(X, dc, origin_rhs(Operators(g), Phys(1, 1, (1, 0, 0), None, dc.pin)))
    for i, Ab in enumerate(M.Abar):
        if Ab.shape[0] <= 1500:
            s = np.linalg.svd(Ab.toarray(), compute_uv=False)
            assert s[-1] > 1e-10 * s[0]
    touched = np.zeros(dc.Nc, dtype=bool)
    for i in range(dc.Np):
        touched[dc.Cp[i]] = True
    assert touched.all()
    # the pin is a primary cell; each dual grid contains its interface
    assert dc.iface[dc.pin] < 0
    for j in range(dc.Nc):
        assert np.all(np.isin(dc.icells[j] - g.nu, dc.dual_cells[j]))


def test_slab_carving_puts_interfaces_on_the_higher_label_side():
    m = channel(24, 5, 1)
    lab = np.zeros_like(m, dtype=np.int32)
    for s in range(4):
        lab[:, :, s * 6:(s + 1) * 6] = s + 1
    g = MacGrid(m)
    dc = decompose(g, lab)
    iface = np.full(m.shape, -1)
    iface[g.fluid] = dc.iface
    # label 2 starts at column 6, label 3 at 12, label 4 at 18; label 4 also
    # touches label 1 across the periodic wrap (column 23)
    assert set(np.unique(np.nonzero(iface[0] >= 0)[1]).tolist()) == {6, 12, 18, 23}
    assert [tuple(p) for p in dc.pairs] == [(1, 2), (1, 4), (2, 3), (3, 4)]


def test_fragment_pocket_interface_is_merged_and_coarse_operator_regular():
    """Carving can cut a fragment off a pore; a one-cell interface whose only primary
    neighbour is such a fragment is a dead-end pocket (reached otherwise only through
    faces between interface cells, which the coarse space leaves at zero), so it is
    merged, and Rhat X Phat (Section 3.2.2, Remark 1) is invertible.  Fixture: a 12^3
    window of a seeded batch sample (tests/golden/make_fragment_fixture.py)."""
    from tests.helpers import fragment_pocket, oracle_case
    w = fragment_pocket()
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    assert dc.Nc == 11 and dc.Np == 8
    X = build_matrix(ops, ph, wind=None, tags=dc.tags)
    M = G.build(X, dc, origin_rhs(ops, ph))
    sv = np.linalg.svd(M.Ao, compute_uv=False)
    assert sv[-1] / sv[0] > 1e-8


def test_aplmm_s_is_gplmm_with_zero_wind():
    """Section 8: gPLMM_S = aPLMM_S.  With w = 0 the build matrix X = J~_0 is the Stokes
    matrix whatever the tags (no inertia is left to remove), and so is the Newton Jacobian
    at rest, so the three preconditioners are the same operator."""
    from oracle.mac import jacobian
    m, lab = _tiny_3d()
    g, ops, dc, ph, X, bB = _case(m, lab, dt=None)
    Xg = build_matrix(ops, ph, wind=None, tags=dc.tags)
    Xs = build_matrix(ops, ph, wind=None, tags=None, )
    Js = jacobian(ops, np.zeros(g.N), ph)
    assert abs(Xg - Xs).max() == 0.0 and abs(Js - Xs).max() == 0.0
    v = np.random.default_rng(2).standard_normal(g.N)
    za = G.apply(G.build(Xg, dc, bB), v)
    zb = G.apply(G.build(Js, dc, bB), v)
    assert np.array_equal(za, zb)


def test_aplmm_ns_from_the_newton_jacobian_converges():
    """aPLMM_NS (the preconditioner rebuilt from the Newton Jacobian at the first
    iterate) drives FGMRES to the same Newton solution as gPLMM and as exact solves."""
    from oracle import newton
    w = make_workload("disks2d_32", 1, re=10.0)
    g = MacGrid(largest_component(w["mask"]))
    ops = Operators(g)
    dc = decompose(g, w["labels"])
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    xg, sg = newton.solve(ops, dc, ph, tol=1e-12, lin_tol=1e-13)
    xa, sa = newton.solve(ops, dc, ph, tol=1e-12, lin_tol=1e-13, build="jacobian")
    xe, se = newton.solve(ops, dc, ph, tol=1e-13, precond="exact")
    assert sg.converged and sa.converged
    assert np.linalg.norm(xa - xe) <= 1e-9 * np.linalg.norm(xe)
    assert np.linalg.norm(xg - xe) <= 1e-9 * np.linalg.norm(xe)
    print("FGMRES its gPLMM %s, aPLMM_NS %s" % (sg.lin_its, sa.lin_its))


def test_remark1_form_with_back_substitution():
    """mg_form 2: the Remark-1 coarse correction with the f entries from Eq. xf.  On the
    p and c unknowns it is the Remark-1 correction itself; on the f rows A z_G equals the
    right-hand side; and it differs from the Remark-1 correction (which leaves x^f = 0)."""
    m, lab = _tiny_3d()
    g, ops, dc, ph, X, bB = _case(m, lab, wind_seed=3)
    M0 = G.build(X, dc, bB, mg_form=0)
    M2 = G.build(X, dc, bB, mg_form=2)
    F = dc.f_faces
    assert F.size >= 1
    notf = np.setdiff1d(np.arange(g.N), F)
    rng = np.random.default_rng(6)
    w = rng.standard_normal(g.N)
    z0, z2 = G.apply_MG(M0, w), G.apply_MG(M2, w)
    assert np.array_equal(z0[notf], z2[notf])
    assert np.all(z0[F] == 0.0)
    assert np.linalg.norm(z2[F]) >= 1e-3 * np.linalg.norm(z2)
    assert np.linalg.norm((X @ z2 - w)[F]) <= 1e-11 * np.linalg.norm(w)


def test_column_summed_form_newton_converges_to_the_same_solution():
    """Newton-FGMRES with the Eq. iMG coarse correction ends at the solution the
    Remark-1 form reaches (the preconditioner changes the iterations, not the answer)."""
    from oracle import newton
    w = make_workload("disks2d_32", 2, re=10.0)
    m = largest_component(w["mask"], (True, False, False))
    g = MacGrid(m, periodic=(True, False, False))
    ops = Operators(g)
    dc = decompose(g, w["labels"])
    ph = Phys(w["rho"], w["mu"], tuple(w["body"]), None, dc.pin)
    x0, s0 = newton.solve(ops, dc, ph, tol=1e-11)
    for mg_form in (1, 2):
        x1, s1 = newton.solve(ops, dc, ph, tol=1e-11, mg_form=mg_form)
        assert s0.res_hist[-1] <= 1e-11 and s1.res_hist[-1] <= 1e-11
        assert np.linalg.norm(x1 - x0) <= 1e-8 * np.linalg.norm(x0)
