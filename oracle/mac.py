"""MAC finite-difference residual, Newton Jacobian and gPLMM build matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: the momentum/mass equations (Section 1, the governing equations), the
Newton system J^k delta^k = -r^k with J = [F G^T; G O] (Section 1), the MAC
staggering of Section 2 (velocities on faces, pressure in cells, no-slip on
grain surfaces) and the modified residual r~_w of Section 4 (inertia
linearised about a wind w, removed on faces near contact interfaces).

The stencil details the paper leaves open are taken as follows (the readings
are listed in the design notes):

* voxels are indexed [k, j, i] with x fastest; the x-face at (k, j, i) lies
  between cells (k, j, i-1) and (k, j, i) (i-1 wraps when x is periodic); a
  face is an unknown ("active") iff both flanking cells are fluid and inside
  the image; image edges that are not periodic act as grains;
* viscous term: -(mu/h^2) * sum over the 2*ndim neighbour faces of
  (g - u_F), where g is the neighbour's velocity if it is active, 0 if the
  neighbour face is inactive but touches a fluid cell (it sits on a grain
  surface, distance h), and -u_F if both its cells are grain or outside (the
  wall is then half a cell away); this keeps the Stokes block symmetric, as
  the paper states it is;
* inertia: first-order upwind in advective form, rho * sum_d a_d * D_d u_F,
  with a_x = u_F and the transverse a_y, a_z the mean of the four transverse
  face velocities of F's two cells (inactive faces count 0); D_d is the
  backward difference when a_d >= 0 and the forward difference otherwise,
  both using the same neighbour value g;
* pressure gradient (p_R - p_L)/h on the face; mass row -div(u) on each fluid
  cell, i.e. the transpose of the gradient, so the Stokes matrix is symmetric;
* backward Euler rho (u - u_old)/dt when dt is given; body force -rho b;
* the gauge: one fluid cell c* (the pin) has its mass row replaced by p = 0.

Vectors are ordered [u (x-faces), v (y-faces), w (z-faces), p (cells)], each
block in lexicographic (k, j, i) order.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
import scipy.sparse as sp


@dataclass
class Phys:
    rho: float = 1.0
    mu: float = 1.0
    body: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    dt: Optional[float] = None       # None: steady
    pin: int = 0                     # cell number (within the p block) of c*


class MacGrid:
    """Fluid mask on a voxel grid and the numbering of the MAC unknowns."""

    def __init__(self, mask, h=1.0, periodic=(True, False, False)):
        m = np.asarray(mask).astype(bool)
        if m.ndim == 2:
            m = m[None]
        self.fluid = m
        self.nz, self.ny, self.nx = m.shape
        self.ndim = 2 if self.nz == 1 else 3
        self.h = float(h)
        self.periodic = tuple(bool(p) for p in periodic)
        if self.ndim == 2:
            self.periodic = (self.periodic[0], self.periodic[1], False)
        self.comps = list(range(self.ndim))
        # face activity and numbering
        self.act, self.touch, self.fid = [], [], []
        off = 0
        self.off = []
        for c in self.comps:
            lo = self.shift(m, c, -1, False)
            act = m & lo
            self.act.append(act)
            self.touch.append(m | lo)
            fid = np.full(m.shape, -1, dtype=np.int64)
            pos = np.flatnonzero(act)
            fid.ravel()[pos] = off + np.arange(pos.size)
            self.fid.append(fid)
            self.off.append(off)
            off += pos.size
        self.nu = off
        self.cid = np.full(m.shape, -1, dtype=np.int64)
        cpos = np.flatnonzero(m)
        self.cid.ravel()[cpos] = off + np.arange(cpos.size)
        self.off.append(off)
        self.nc = cpos.size
        self.N = off + cpos.size
        self.ncomp = [int(self.act[c].sum()) for c in self.comps]

    # ---- index helpers ------------------------------------------------------
    def shift(self, a, d, s, fill):
        """b[pos] = a[pos + s*e_d]; wraps if axis d is periodic, else ``fill``."""
        ax = 2 - d
        if self.periodic[d]:
            return np.roll(a, -s, axis=ax)
        out = np.full_like(a, fill)
        n = a.shape[ax]
        if abs(s) >= n:
            return out
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        if s > 0:
            src[ax], dst[ax] = slice(s, n), slice(0, n - s)
        else:
            src[ax], dst[ax] = slice(0, n + s), slice(-s, n)
        out[tuple(dst)] = a[tuple(src)]
        return out

    def comp_slice(self, c):
        return slice(self.off[c], self.off[c] + self.ncomp[c])

    @property
    def p_slice(self):
        return slice(self.nu, self.N)

    def unknown_coords(self):
        """(kind, k, j, i) of every unknown; kind 0..ndim-1 = face axis, 3 = cell."""
        out = np.zeros((self.N, 4), dtype=np.int64)
        for c in self.comps:
            pos = np.flatnonzero(self.act[c])
            k, j, i = np.unravel_index(pos, self.fluid.shape)
            out[self.comp_slice(c)] = np.stack([np.full_like(k, c), k, j, i], 1)
        pos = np.flatnonzero(self.fluid)
        k, j, i = np.unravel_index(pos, self.fluid.shape)
        out[self.p_slice] = np.stack([np.full_like(k, 3), k, j, i], 1)
        return out


class Operators:
    """Sparse building blocks of the MAC operators (all constant in x)."""

    def __init__(self, g: MacGrid):
        self.g = g
        h = g.h
        self.G = {}        # G[c, d, s]: neighbour value g of c-faces in direction s*e_d
        self.A = {}        # A[c, d]: transverse advecting velocity of c-faces from u_d
        self.Dp = {}       # backward difference (a >= 0)
        self.Dm = {}       # forward difference (a < 0)
        self.visc = {}
        self.grad = {}
        for c in g.comps:
            nc = g.ncomp[c]
            rows_grid = g.fid[c] - g.off[c]
            act = g.act[c]
            r = rows_grid[act]
            I = sp.identity(nc, format="csr")
            vsum = sp.csr_matrix((nc, nc))
            for d in g.comps:
                for s in (-1, +1):
                    nb = g.shift(g.fid[c], d, s, -1)[act]
                    nb_touch = g.shift(g.touch[c], d, s, (d == c and s == +1))[act]
                    has = nb >= 0
                    ghost = (~has) & (~nb_touch)
                    rr = np.concatenate([r[has], r[ghost]])
                    cc = np.concatenate([nb[has] - g.off[c], r[ghost]])
                    vv = np.concatenate([np.ones(has.sum()), -np.ones(ghost.sum())])
                    Gm = sp.csr_matrix((vv, (rr, cc)), shape=(nc, nc))
                    self.G[c, d, s] = Gm
                    vsum = vsum + (Gm - I)
                self.Dp[c, d] = (I - self.G[c, d, -1]) / h
                self.Dm[c, d] = (self.G[c, d, +1] - I) / h
            self.visc[c] = vsum           # times -(mu/h^2) at use
            # transverse advecting velocities
            for d in g.comps:
                if d == c:
                    continue
                nd = g.ncomp[d]
                rr, cc = [], []
                # d-faces of the two cells flanking F: at q - e_c, q - e_c + e_d, q, q + e_d
                low = g.shift(g.fid[d], c, -1, -1)
                for q in (low, g.shift(low, d, +1, -1), g.fid[d], g.shift(g.fid[d], d, +1, -1)):
                    v = q[act]
                    ok = v >= 0
                    rr.append(r[ok])
                    cc.append(v[ok] - g.off[d])
                rr = np.concatenate(rr)
                cc = np.concatenate(cc)
                self.A[c, d] = sp.csr_matrix((np.full(rr.size, 0.25), (rr, cc)), shape=(nc, nd))
            # gradient: +1/h on the cell at the face position (R), -1/h on the one below (L)
            R = g.cid[act] - g.nu
            L = g.shift(g.cid, c, -1, -1)[act] - g.nu
            self.grad[c] = sp.csr_matrix(
                (np.concatenate([np.full(nc, 1.0 / h), np.full(nc, -1.0 / h)]),
                 (np.concatenate([r, r]), np.concatenate([R, L]))), shape=(nc, g.nc))
        self.gradT = sp.vstack([self.grad[c] for c in g.comps]).T.tocsr()


def _split(g, x):
    return [x[g.comp_slice(c)] for c in g.comps], x[g.p_slice]


def _upwind(ops, c, d, a, u):
    """D_d u with the branch of each row chosen by the sign of a (ties: backward)."""
    fwd = a < 0
    return np.where(fwd, ops.Dm[c, d] @ u, ops.Dp[c, d] @ u), fwd


def _upwind_matrix(ops, c, d, fwd):
    f = sp.diags(fwd.astype(float))
    b = sp.diags((~fwd).astype(float))
    return b @ ops.Dp[c, d] + f @ ops.Dm[c, d]


def advecting(ops, c, d, us):
    return us[c] if d == c else ops.A[c, d] @ us[d]


def residual(ops, x, phys: Phys, x_old=None, wind=None, tags=None, inertia=True):
    """r(x).  ``wind`` (a full-length vector whose velocity part is used)
    switches to the linearised inertia w . grad u of the modified residual;
    ``tags`` (list of bool arrays, one per face axis) removes inertia on those
    faces; ``inertia=False`` gives the Stokes residual."""
    g = ops.g
    us, p = _split(g, x)
    ws = _split(g, wind)[0] if wind is not None else us
    rho, mu, h = phys.rho, phys.mu, g.h
    out = np.zeros(g.N)
    for c in g.comps:
        rc = -(mu / h ** 2) * (ops.visc[c] @ us[c]) + ops.grad[c] @ p - rho * phys.body[c]
        if phys.dt is not None:
            uo = np.zeros_like(us[c]) if x_old is None else x_old[g.comp_slice(c)]
            rc = rc + rho * (us[c] - uo) / phys.dt
        if inertia:
            conv = np.zeros(g.ncomp[c])
            for d in g.comps:
                a = advecting(ops, c, d, ws)
                Du, _ = _upwind(ops, c, d, a, us[c])
                conv += a * Du
            if tags is not None:
                conv = np.where(tags[c], 0.0, conv)
            rc = rc + rho * conv
        out[g.comp_slice(c)] = rc
    u_all = x[:g.nu]
    rp = ops.gradT @ u_all
    rp[phys.pin] = p[phys.pin]
    out[g.p_slice] = rp
    return out


def _assemble(g, blocks, pin):
    """blocks[(rc, cc)] -> sparse; rc/cc in comps or 'p'.  Mass rows from gradT."""
    n = len(g.comps) + 1
    keys = list(g.comps) + ["p"]
    grid = [[None] * n for _ in range(n)]
    for a, ka in enumerate(keys):
        for b, kb in enumerate(keys):
            grid[a][b] = blocks.get((ka, kb))
    # sizes for empty blocks
    sizes = [g.ncomp[c] for c in g.comps] + [g.nc]
    for a in range(n):
        for b in range(n):
            if grid[a][b] is None:
                grid[a][b] = sp.csr_matrix((sizes[a], sizes[b]))
    M = sp.bmat(grid, format="csr")
    M = M.tolil()
    M.rows[g.nu + pin] = [g.nu + pin]
    M.data[g.nu + pin] = [1.0]
    return M.tocsr()


def _mass_blocks(ops, phys):
    g = ops.g
    gt = ops.gradT.tolil()
    gt.rows[phys.pin] = []
    gt.data[phys.pin] = []
    gt = gt.tocsr()
    blocks = {}
    for c in g.comps:
        blocks["p", c] = gt[:, g.off[c]:g.off[c] + g.ncomp[c]]
    return blocks


def jacobian(ops, x, phys: Phys, tags=None):
    """Exact derivative of ``residual`` with each upwind branch frozen at the
    state x; ``tags`` (as in ``residual``) differentiates the residual whose
    tagged faces carry no inertia (the modified residual of Section 4 with the
    wind equal to the state itself, used by the coarse-scale solver)."""
    g = ops.g
    us, _ = _split(g, x)
    rho, mu, h = phys.rho, phys.mu, g.h
    blocks = _mass_blocks(ops, phys)
    for c in g.comps:
        nc = g.ncomp[c]
        keep = sp.identity(nc) if tags is None else sp.diags((~tags[c]).astype(float))
        diag = -(mu / h ** 2) * ops.visc[c]
        if phys.dt is not None:
            diag = diag + (rho / phys.dt) * sp.identity(nc)
        conv = sp.csr_matrix((nc, nc))
        for d in g.comps:
            a = advecting(ops, c, d, us)
            Du, fwd = _upwind(ops, c, d, a, us[c])
            Dm = _upwind_matrix(ops, c, d, fwd)
            conv = conv + sp.diags(a) @ Dm
            if d == c:
                conv = conv + sp.diags(Du)
            else:
                blocks[c, d] = rho * (keep @ sp.diags(Du) @ ops.A[c, d])
        blocks[c, c] = diag + rho * (keep @ conv)
        blocks[c, "p"] = ops.grad[c]
    return _assemble(g, blocks, phys.pin)


def build_matrix(ops, phys: Phys, wind=None, tags=None):
    """X = Jacobian of the modified residual with the wind w held fixed
    (Oseen operator); rows of tagged faces carry no inertia.  wind=None means
    w = 0, i.e. the Stokes matrix (plus rho/dt for a transient step)."""
    g = ops.g
    rho, mu, h = phys.rho, phys.mu, g.h
    ws = _split(g, wind)[0] if wind is not None else [np.zeros(n) for n in g.ncomp]
    blocks = _mass_blocks(ops, phys)
    for c in g.comps:
        nc = g.ncomp[c]
        diag = -(mu / h ** 2) * ops.visc[c]
        if phys.dt is not None:
            diag = diag + (rho / phys.dt) * sp.identity(nc)
        conv = sp.csr_matrix((nc, nc))
        for d in g.comps:
            a = advecting(ops, c, d, ws)
            fwd = a < 0
            conv = conv + sp.diags(a) @ _upwind_matrix(ops, c, d, fwd)
        if tags is not None:
            conv = sp.diags((~tags[c]).astype(float)) @ conv
        blocks[c, c] = diag + rho * conv
        blocks[c, "p"] = ops.grad[c]
    return _assemble(g, blocks, phys.pin)


def origin_rhs(ops, phys: Phys):
    """b_B = -r(u = 0, p = 0) of the steady equations (Section 3.2.2,
    correction vectors): only the body force survives."""
    steady = Phys(phys.rho, phys.mu, phys.body, None, phys.pin)
    return -residual(ops, np.zeros(ops.g.N), steady)
