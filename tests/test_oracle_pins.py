"""Pins of the oracle's open readings against facts fixed outside the oracle (CPU only).

* Convective term (Section 1, rho u . grad u; its upwind MAC form is this project's
  reading): on a smooth, fully periodic velocity field the oracle's inertia term must
  converge to the analytic (u . grad) u, and its first-order error must be the upwind
  scheme's known leading term -(h/2) sum_d |a_d| d^2u/dx_d^2 (numerical diffusion of
  the backward difference taken on the upwind side).  The remainder after that term is
  second order.  A downwind branch (the sign of the leading term flips) or a transverse
  advecting velocity averaged over the wrong pair of cells (an O(h) error in a_d) keeps
  a first-order remainder; both mutations are planted below in copies of the oracle's
  functions and must fail the same check.
* Tags (Section 4: inertia removed on faces within a few layers of a contact
  interface) and dual grids (Section 3.2.1: successive dilations of each interface):
  expected sets written out by hand for a 2D 6x5 and a 3D 4^3 image with a corner
  pore, for tag_layers 0/1/2 and dual_dilations 0/1/2, checked against the oracle and
  against the library's host decomposition.
* Newton (Section 1: x^{k+1} = x^k + delta^k): full steps by default.
"""
import numpy as np
import pytest

from oracle import mac
from oracle.mac import MacGrid, Operators, Phys, residual
from oracle.decomp import decompose
from oracle import newton


# ---------------------------------------------------------------------------
# Convective term against the analytic (u . grad) u on a periodic field
# ---------------------------------------------------------------------------

# Each velocity component is m + sum of plane waves c sin(2 pi k.x + phase) on the unit
# cube (period 1 on every axis); the mean m is small against the amplitudes, so every
# advecting velocity changes sign and both upwind branches are exercised.
_FIELDS = {
    2: [(0.2, [(1.0, (1, 1, 0), 0.3), (0.5, (2, -1, 0), 1.1)]),
        (-0.1, [(0.9, (1, -2, 0), 0.7), (0.4, (0, 1, 0), 2.0)])],
    3: [(0.2, [(1.0, (1, 1, 0), 0.3), (0.5, (0, 1, 1), 1.1)]),
        (-0.1, [(0.9, (1, 0, -1), 0.7), (0.4, (1, 1, 1), 2.0)]),
        (0.15, [(0.8, (0, 1, -1), 0.2), (0.6, (1, 0, 1), 1.5)])],
}


def _wave(comp, pts, deriv=()):
    """Value (deriv = ()), first derivative (deriv = (d,)) or second derivative
    (deriv = (d, d)) of one field component at points pts (n x 3, x y z)."""
    m, waves = comp
    out = np.full(pts.shape[0], m if not deriv else 0.0)
    for c, k, ph in waves:
        arg = 2 * np.pi * (pts @ np.array(k, float)) + ph
        if not deriv:
            out += c * np.sin(arg)
        elif len(deriv) == 1:
            out += c * 2 * np.pi * k[deriv[0]] * np.cos(arg)
        else:
            out -= c * (2 * np.pi) ** 2 * k[deriv[0]] * k[deriv[1]] * np.sin(arg)
    return out


def _face_points(g, c):
    """Physical positions (x, y, z) of the active c-faces: the c coordinate on the
    cell boundary, the others at cell centres."""
    co = g.unknown_coords()[g.comp_slice(c)]
    ijk = np.stack([co[:, 3], co[:, 2], co[:, 1]], 1).astype(float) + 0.5
    ijk[:, c] -= 0.5
    if g.ndim == 2:
        ijk[:, 2] = 0.0
    return ijk * g.h


def _convection_error(n, ndim):
    """Max over faces of |e - lead| and |lead|, e = oracle inertia - exact (u.grad)u,
    lead = -(h/2) sum_d |U_d| d^2 U_c / dx_d^2, on an all-fluid periodic n^ndim grid."""
    shape = (n, n) if ndim == 2 else (n, n, n)
    g = MacGrid(np.ones(shape, np.uint8), h=1.0 / n, periodic=(True, True, True))
    ops = Operators(g)
    field = _FIELDS[ndim]
    x = np.zeros(g.N)
    for c in g.comps:
        x[g.comp_slice(c)] = _wave(field[c], _face_points(g, c))
    ph = Phys(1.0, 1.0, (0.0, 0.0, 0.0), None, 0)
    conv = residual(ops, x, ph) - residual(ops, x, ph, inertia=False)
    err_rem, lead_max = 0.0, 0.0
    for c in g.comps:
        pts = _face_points(g, c)
        exact = sum(_wave(field[d], pts) * _wave(field[c], pts, (d,)) for d in g.comps)
        lead = -0.5 * g.h * sum(np.abs(_wave(field[d], pts)) * _wave(field[c], pts, (d, d)) for d in g.comps)
        e = conv[g.comp_slice(c)] - exact
        err_rem = max(err_rem, float(np.max(np.abs(e - lead))))
        lead_max = max(lead_max, float(np.max(np.abs(lead))))
    return err_rem, lead_max


def _convection_pin_holds(ndim, sizes):
    """The remainder after the leading upwind term is small against that term and
    falls at second order (ratio of remainders >= 3 per halving of h)."""
    rem = [_convection_error(n, ndim) for n in sizes]
    rel = [r / l for r, l in rem]
    ratios = [rem[k][0] / rem[k + 1][0] for k in range(len(rem) - 1)]
    return rel[-1] < 0.1 and all(q >= 3.0 for q in ratios), rel, ratios


_SIZES = {2: (16, 32, 64), 3: (8, 16, 32)}


@pytest.mark.parametrize("ndim", [2, 3])
def test_convective_term_matches_upwind_modified_equation(ndim):
    ok, rel, ratios = _convection_pin_holds(ndim, _SIZES[ndim])
    assert ok, (rel, ratios)


def _downwind(ops, c, d, a, u):
    """Mutated copy of the oracle's upwind difference: the branch is flipped."""
    fwd = a >= 0
    return np.where(fwd, ops.Dm[c, d] @ u, ops.Dp[c, d] @ u), fwd


def _shifted_average(ops, c, d, us):
    """Mutated copy of the oracle's advecting velocity: the transverse average is taken
    over the d-faces of the cells at +0 and +1 along c (one cell too far) instead of
    the face's own two cells."""
    if d == c:
        return us[c]
    return ops.G[c, c, +1] @ (ops.A[c, d] @ us[d])


@pytest.mark.parametrize("mutation", ["downwind", "shifted_average"])
def test_convective_pin_rejects_planted_mistakes(monkeypatch, mutation):
    if mutation == "downwind":
        monkeypatch.setattr(mac, "_upwind", _downwind)
    else:
        monkeypatch.setattr(mac, "advecting", _shifted_average)
    ok, rel, ratios = _convection_pin_holds(2, _SIZES[2])
    assert not ok, (mutation, rel, ratios)


# ---------------------------------------------------------------------------
# Tags and dual grids: hand-written expected sets
# ---------------------------------------------------------------------------

def _grid(rows):
    """Boolean array from rows of 'x' / '.' characters; rows are listed from j = 0
    upwards (first row = lowest j), columns are i = 0, 1, ..."""
    return np.array([[ch == "x" for ch in r.split()] for r in rows], dtype=bool)


# 2D 6x5 image (nx = 6, ny = 5), all void, no periodic axis.  Pore 1 is the 3x3 corner
# block i <= 2, j <= 2; pore 2 is the rest.  The interface cells are the pore-2 cells
# with a pore-1 face neighbour: (j, i) = (0..2, 3) and (3, 0..2).
LABELS_2D = np.array([[1, 1, 1, 2, 2, 2],
                      [1, 1, 1, 2, 2, 2],
                      [1, 1, 1, 2, 2, 2],
                      [2, 2, 2, 2, 2, 2],
                      [2, 2, 2, 2, 2, 2]], dtype=np.int32)

# Tagged x-faces (the x-face (j, i) lies between cells (j, i-1) and (j, i); i = 0 is the
# image edge and never active) and y-faces (between (j-1, i) and (j, i); j = 0 inactive)
# for tag_layers 0, 1, 2: a face is tagged when one of its two cells is within
# Chebyshev distance tag_layers of an interface cell.
TAGS_2D = {
    0: ([". . . x x .",
         ". . . x x .",
         ". . . x x .",
         ". x x x . .",
         ". . . . . ."],
        [". . . . . .",
         ". . . x . .",
         ". . . x . .",
         "x x x x . .",
         "x x x . . ."]),
    1: ([". . x x x x",
         ". . x x x x",
         ". x x x x x",
         ". x x x x x",
         ". x x x x ."],
        [". . . . . .",
         ". . x x x .",
         "x x x x x .",
         "x x x x x .",
         "x x x x x ."]),
    2: ([". x x x x x"] * 5,
        [". . . . . ."] + ["x x x x x x"] * 4),
}

# The one dual grid: the interface cells grown 0, 1, 2 times by face neighbours.
DUAL_2D = {
    0: [". . . x . .",
        ". . . x . .",
        ". . . x . .",
        "x x x . . .",
        ". . . . . ."],
    1: [". . x x x .",
        ". . x x x .",
        "x x x x x .",
        "x x x x . .",
        "x x x . . ."],
    2: [". x x x x x",
        "x x x x x x",
        "x x x x x x",
        "x x x x x .",
        "x x x x . ."],
}

# 3D 4^3 image, all void, no periodic axis.  Pore 1 is the 2x2x2 corner block
# i, j, k <= 1; the 12 interface cells are the pore-2 cells with exactly one coordinate
# equal to 2 and the other two <= 1.  Sets are given per slice k = 0..3 (rows j, columns i).
LABELS_3D = np.full((4, 4, 4), 2, dtype=np.int32)
LABELS_3D[:2, :2, :2] = 1

# Cells within Chebyshev distance tag_layers of an interface cell (faces are tagged when
# one of their cells is such a cell).
NEAR_3D = {
    0: [[". . x .", ". . x .", "x x . .", ". . . ."],
        [". . x .", ". . x .", "x x . .", ". . . ."],
        ["x x . .", "x x . .", ". . . .", ". . . ."],
        [". . . .", ". . . .", ". . . .", ". . . ."]],
    1: [[". x x x", "x x x x", "x x x x", "x x x ."],
        ["x x x x", "x x x x", "x x x x", "x x x ."],
        ["x x x x", "x x x x", "x x x x", "x x x ."],
        ["x x x .", "x x x .", "x x x .", ". . . ."]],
    2: [["x x x x"] * 4] * 4,
}

DUAL_3D = {
    0: NEAR_3D[0],
    1: [[". x x x", "x x x x", "x x x .", "x x . ."],
        ["x x x x", "x x x x", "x x x .", "x x . ."],
        ["x x x .", "x x x .", "x x . .", ". . . ."],
        ["x x . .", "x x . .", ". . . .", ". . . ."]],
    2: [["x x x x", "x x x x", "x x x x", "x x x ."],
        ["x x x x", "x x x x", "x x x x", "x x x ."],
        ["x x x x", "x x x x", "x x x .", "x x . ."],
        ["x x x .", "x x x .", "x x . .", ". . . ."]],
}


def _expected_2d(L):
    xf, yf = TAGS_2D[L]
    return [_grid(xf)[None], _grid(yf)[None]]


def _expected_3d(L):
    """Tagged faces of each axis (as [k, j, i] grids) from the hand-written near-cell sets:
    the a-face at (k, j, i) is tagged when cell (k, j, i) or its lower a-neighbour is near."""
    near = np.array([_grid(s) for s in NEAR_3D[L]])
    out = []
    for a in range(3):
        ax = 2 - a
        lower = np.zeros_like(near)
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax], sl_src[ax] = slice(1, None), slice(0, -1)
        lower[tuple(sl_dst)] = near[tuple(sl_src)]
        out.append(near | lower)
    return out


def _dual_cells_expected(picture3):
    cells = np.array([_grid(s) for s in picture3]) if isinstance(picture3[0], list) else _grid(picture3)[None]
    return np.flatnonzero(cells.ravel())


def _case(ndim):
    if ndim == 2:
        return np.ones((1, 5, 6), np.uint8), LABELS_2D[None]
    return np.ones((4, 4, 4), np.uint8), LABELS_3D


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("layers", [0, 1, 2])
def test_oracle_tags_match_hand_fixture(ndim, layers):
    mask, lab = _case(ndim)
    g = MacGrid(mask, periodic=(False, False, False))
    dc = decompose(g, lab, tag_layers=layers)
    assert dc.Nc == 1 and dc.Np == 2
    exp = _expected_2d(layers) if ndim == 2 else _expected_3d(layers)
    for a in g.comps:
        assert np.array_equal(dc.tags[a], exp[a][g.act[a]]), (a, layers)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("dil", [0, 1, 2])
def test_oracle_dual_grid_matches_hand_fixture(ndim, dil):
    mask, lab = _case(ndim)
    g = MacGrid(mask, periodic=(False, False, False))
    dc = decompose(g, lab, dual_dilations=dil)
    pic = DUAL_2D[dil] if ndim == 2 else DUAL_3D[dil]
    # all-void image: the cell number is the raster index of the voxel
    assert np.array_equal(dc.dual_cells[0], _dual_cells_expected(pic))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("k", [0, 1, 2])
def test_library_host_tags_and_duals_match_hand_fixture(ndim, k):
    import os
    from paper_2510_22077_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgplmm.so not built")
    mask, lab = _case(ndim)
    m = mask if ndim == 3 else mask[0]
    ll = lab if ndim == 3 else lab[0]
    s = binding.Solver(m, ll, body=(1.0, 0.0, 0.0), host_only=True, periodic=(0, 0, 0),
                       tag_layers=k, dual_dilations=k)
    maps = s.maps()
    nrec = ndim + 1
    cv = maps["cell_voxel"]
    assert np.array_equal(cv, np.arange(mask.size))
    exp = _expected_2d(k) if ndim == 2 else _expected_3d(k)
    for a in range(ndim):
        got = (maps["face_tag"][a::nrec] & 1).astype(bool)
        act = (maps["face_owner"][a::nrec] != -2)
        assert np.array_equal(got, exp[a].ravel() & act), (a, k)
    pic = DUAL_2D[k] if ndim == 2 else DUAL_3D[k]
    du = s.duals()
    assert len(du) == 1 and np.array_equal(du[0], _dual_cells_expected(pic))
    s.close()


# ---------------------------------------------------------------------------
# Newton: the paper's full update
# ---------------------------------------------------------------------------

def test_oracle_newton_takes_full_steps_by_default():
    from synth import make_workload
    from oracle.decomp import largest_component
    w = make_workload("disks2d_32", 1, re=10.0)
    g = MacGrid(largest_component(w["mask"]))
    ops = Operators(g)
    dc = decompose(g, w["labels"])
    ph = Phys(w["rho"], w["mu"], w["body"], None, dc.pin)
    x, st = newton.solve(ops, dc, ph, tol=1e-12, lin_tol=1e-13)
    assert st.converged and st.newton_its >= 3
    assert st.step_length == [1.0] * st.newton_its
