"""Pore decomposition: primary grids, contact interfaces, dual grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Section 3.2.1 (domain decomposition) and the permutation paragraph of
Section 3.2.2: the void space is split into non-overlapping primary grids
(pores); contact interfaces separate adjacent primaries; a face with at least
one flanking cell in a primary belongs to that primary, and a face flanked by
neither belongs to the interface ("f" unknowns); dual grids are successive
dilations of each interface and may overlap.  Section 4 tags the faces near
the interfaces, where the modified residual carries no inertia.

The caller's pore labels stand in for the paper's watershed; the rules that
turn labels into interfaces are this project's reading of the paper (the
paper asks only for a thinnest separating set, which it does not construct):

* gauge / connectivity: only the largest face-connected void component is
  kept (periodic wrap included); the rest is treated as grain;
* carving: a cell is an interface cell iff a face neighbour has a smaller
  positive label; its interface is the pair (smallest such neighbour label,
  own label); interfaces are numbered by sorting the pairs; a primary is the
  set of its label's cells that are not interface cells (empty ones are
  dropped), numbered in label order;
* wall-free face groups: the closure of a primary replaces every coupling to
  an f-face or another primary by a zero normal gradient, so a group of the
  primary's same-axis faces that are linked to each other through the viscous
  stencil, and none of which touches a grain (or the image edge), would leave
  a uniform velocity on that group undetermined (a singular closure matrix).
  The faces of such a group are marked ``free`` and keep their plain rows in
  the closure matrix (no column sums), which keeps it nonsingular;
* an interface is degenerate when no primary cell touches it, or when every
  face-connected piece of a primary touching it touches no other interface (a
  dead-end pocket that reaches the rest of the void only through faces between
  interface cells, which the coarse space leaves at zero, so its coarse pressure
  would be undetermined; carving can cut a fragment off a pore, and a fragment
  reached only through one interface is such a pocket even when the rest of its
  pore touches other interfaces); the lowest-id degenerate interface that shares a face with
  another interface is merged into the one it shares the most faces with
  (lowest id on ties), until none is left; ids are then compacted keeping
  their order;
* the pin c* is the first fluid cell in raster order that is not an interface
  cell;
* tags: a face is tagged iff one of its two cells lies within Chebyshev
  distance ``tag_layers`` of an interface cell;
* dual grid j: the cells of interface j, grown ``dual_dilations`` times by
  face neighbours through the void space (default 1 in 2D, 0 in 3D: a 3D
  interface sheet already covers a large share of the cells, and the default
  keeps the union of the dual grids near the 10-30% of the void space the
  paper reports in its complexity discussion (Section 9.3); wider dual grids overlap more,
  and the additive sum over overlapping duals then over-corrects: two
  dilations in 2D stall FGMRES on large disk packings);
* the unknowns of a cell set: its cells plus every active face with at least
  one flanking cell in the set.
"""
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy import ndimage as ndi

from .mac import MacGrid


def largest_component(mask, periodic=(True, False, False)):
    """Keep the largest face-connected void component (periodic-aware)."""
    m = np.asarray(mask).astype(bool)
    if m.ndim == 2:
        m = m[None]
    two_d = m.shape[0] == 1
    st = ndi.generate_binary_structure(3, 1)
    if two_d:
        st[0] = False
        st[2] = False
    lab, n = ndi.label(m, structure=st)
    if n <= 1:
        return m.astype(np.uint8)
    parent = np.arange(n + 1)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for d, per in enumerate(periodic):
        if not per or (two_d and d == 2):
            continue
        ax = 2 - d
        a = np.take(lab, 0, axis=ax).ravel()
        b = np.take(lab, -1, axis=ax).ravel()
        for x, y in zip(a[(a > 0) & (b > 0)], b[(a > 0) & (b > 0)]):
            rx, ry = find(x), find(y)
            if rx != ry:
                parent[max(rx, ry)] = min(rx, ry)
    root = np.array([find(a) for a in range(n + 1)])
    comp = root[lab]
    sizes = np.bincount(comp.ravel(), minlength=n + 1)
    sizes[0] = 0
    keep = np.argmax(sizes)
    return (comp == keep).astype(np.uint8)


def cell_neighbours(g: MacGrid):
    """nbr[c, 2*d + (s>0)]: cell number across the active face in direction
    s*e_d of fluid cell c, or -1."""
    cid = g.cid - g.nu
    cid[~g.fluid] = -1
    cells = np.flatnonzero(g.fluid)
    nbr = np.full((g.nc, 2 * g.ndim), -1, dtype=np.int64)
    for d in g.comps:
        for t, s in enumerate((-1, +1)):
            nb = g.shift(cid, d, s, -1).ravel()[cells]
            nbr[:, 2 * d + t] = nb
    return nbr


def cell_faces(g: MacGrid):
    """fc[c, 2*d + t]: global unknown of the lower (t=0) / upper (t=1) d-face of
    cell c, or -1 when that face is not active."""
    cells = np.flatnonzero(g.fluid)
    fc = np.full((g.nc, 2 * g.ndim), -1, dtype=np.int64)
    for d in g.comps:
        fc[:, 2 * d] = g.fid[d].ravel()[cells]
        fc[:, 2 * d + 1] = g.shift(g.fid[d], d, +1, -1).ravel()[cells]
    return fc


@dataclass
class Decomp:
    g: MacGrid
    label: np.ndarray           # per cell (p-block numbering), >0
    iface: np.ndarray           # per cell: interface id or -1
    prim: np.ndarray            # per cell: primary id or -1
    Nc: int
    Np: int
    pairs: np.ndarray           # (Nc, 2) label pair of each interface
    pin: int
    owner: np.ndarray           # per velocity unknown (0..nu-1): primary id or -1 (f-face)
    Cp: List[np.ndarray]        # interfaces adjacent to each primary
    tags: List[np.ndarray]      # per face axis: bool per active face
    S: List[np.ndarray]         # unknowns of each primary (sorted global)
    D: List[np.ndarray]         # unknowns of each dual grid (sorted global)
    dual_cells: List[np.ndarray]
    icells: List[np.ndarray]    # global unknowns of each interface's cells
    f_faces: np.ndarray
    free: np.ndarray            # per velocity unknown: in a wall-free face group of its primary


def unknowns_of_cells(g, fc, cells):
    """Cells of the set plus every active face with a flanking cell in it."""
    faces = fc[cells].ravel()
    faces = faces[faces >= 0]
    return np.unique(np.concatenate([faces, g.nu + np.asarray(cells, dtype=np.int64)]))


def walled_faces(g: MacGrid):
    """Per face axis: True for an active face whose viscous stencil reaches a
    position that is not an active face of the same axis (grain, grain surface
    or image edge)."""
    out = []
    for c in g.comps:
        act = g.act[c]
        w = np.zeros(int(act.sum()), dtype=bool)
        for d in g.comps:
            for s in (-1, +1):
                w |= g.shift(g.fid[c], d, s, -1)[act] < 0
        out.append(w)
    return out


def carve(L, nbr):
    nbL = np.where(nbr >= 0, L[np.maximum(nbr, 0)], 0)
    lower = (nbL > 0) & (nbL < L[:, None])
    is_if = lower.any(1)
    minlow = np.where(lower, nbL, np.iinfo(np.int64).max).min(1)
    return is_if, minlow


def free_faces(g, owner, walled):
    """Velocity unknowns whose primary's viscous-connected group of same-axis
    faces contains no walled face."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    out = np.zeros(g.nu, dtype=bool)
    for c in g.comps:
        nc = g.ncomp[c]
        own = owner[g.comp_slice(c)]
        act = g.act[c]
        me = g.fid[c][act] - g.off[c]
        rr, cc = [], []
        for d in g.comps:
            nb = g.shift(g.fid[c], d, +1, -1)[act]
            ok = nb >= 0
            a, b = me[ok], nb[ok] - g.off[c]
            same = (own[a] >= 0) & (own[a] == own[b])
            rr.append(a[same])
            cc.append(b[same])
        rr, cc = np.concatenate(rr), np.concatenate(cc)
        A = csr_matrix((np.ones(rr.size), (rr, cc)), shape=(nc, nc))
        _, grp = connected_components(A, directed=False)
        owned = own >= 0
        has_wall = np.zeros(grp.max() + 1 if grp.size else 0, dtype=bool)
        has_wall[grp[owned & walled[c]]] = True
        out[g.comp_slice(c)] = owned & ~has_wall[grp]
    return out


def decompose(g: MacGrid, labels, tag_layers=1, dual_dilations=None, groups=None):
    """Primary grids, contact interfaces, tags and dual grids from the pore labels.

    ``groups`` (an image of positive labels, the pore decomposition of the same void):
    the pore-network decomposition of Section 3.3, in which ``labels`` are the throat
    regions and every interface cell joins the interface of the pore that contains it
    (one contact interface per pore body, shared by all the throats that meet there),
    instead of one interface per pair of touching labels."""
    if dual_dilations is None:
        dual_dilations = 1 if g.ndim == 2 else 0
    lab_grid = np.asarray(labels)
    if lab_grid.ndim == 2:
        lab_grid = lab_grid[None]
    cells = np.flatnonzero(g.fluid)
    L = lab_grid.ravel()[cells].astype(np.int64)
    if np.any(L <= 0):
        raise ValueError("every fluid cell needs a positive pore label")
    nbr = cell_neighbours(g)
    fc = cell_faces(g)
    nc = g.nc
    # --- carving
    is_if, minlow = carve(L, nbr)
    if groups is None:
        pr = np.stack([minlow[is_if], L[is_if]], 1)
    else:
        grp = np.asarray(groups)
        if grp.ndim == 2:
            grp = grp[None]
        G = grp.ravel()[cells].astype(np.int64)
        if np.any(G[is_if] <= 0):
            raise ValueError("every interface cell needs a positive group label")
        pr = np.stack([G[is_if], np.zeros(int(is_if.sum()), dtype=np.int64)], 1)
    upairs, inv = np.unique(pr, axis=0, return_inverse=True)
    iface = np.full(nc, -1, dtype=np.int64)
    iface[is_if] = inv.ravel()
    # --- merge degenerate interfaces
    # pieces of the primaries: face-connected components of the cells of one label left
    # after carving (interface merges never change which cells are primary cells)
    prim0 = iface < 0
    q_idx = np.repeat(np.arange(nc), nbr.shape[1])
    w_idx = nbr.ravel()
    link = (w_idx >= 0) & prim0[q_idx] & prim0[np.maximum(w_idx, 0)] & (L[q_idx] == L[np.maximum(w_idx, 0)])
    adj = sp.coo_matrix((np.ones(int(link.sum())), (q_idx[link], w_idx[link])), shape=(nc, nc))
    _, piece = connected_components(adj, directed=False)
    while True:
        nif = upairs.shape[0]
        prim_cell = iface < 0
        a_if = iface[:, None].repeat(nbr.shape[1], 1)
        valid = (nbr >= 0) & (a_if >= 0)
        nb_prim = valid & prim_cell[np.maximum(nbr, 0)]
        # (interface, primary piece of the touching primary cell) pairs
        ip = np.unique(np.stack([a_if[nb_prim], piece[np.maximum(nbr, 0)][nb_prim]], 1), axis=0)
        # interfaces touched by each primary label
        lab_ifs = {}
        for j, l in ip:
            lab_ifs.setdefault(int(l), set()).add(int(j))
        touching = {}
        for j, l in ip:
            touching.setdefault(int(j), []).append(int(l))
        nb_if = np.where(valid, iface[np.maximum(nbr, 0)], -1)
        shares = np.zeros(nif, dtype=bool)
        sel = valid & (nb_if >= 0) & (nb_if != a_if)
        shares[a_if[sel]] = True
        bad = []
        for j in range(nif):
            labs = touching.get(j, [])
            dead = all(lab_ifs[l] == {j} for l in labs)
            if dead and shares[j]:
                bad.append(j)
        if not bad:
            break
        j = bad[0]
        sel = (a_if == j) & (nb_if >= 0) & (nb_if != j)
        cnt = np.bincount(nb_if[sel], minlength=nif)
        k = int(np.argmax(cnt))          # argmax returns the lowest id on ties
        iface[iface == j] = k
        keep = np.ones(nif, dtype=bool)
        keep[j] = False
        remap = np.cumsum(keep) - 1
        iface = np.where(iface >= 0, remap[np.maximum(iface, 0)], -1)
        upairs = upairs[keep]
    Nc = upairs.shape[0]
    # --- primaries
    prim_labels = np.unique(L[iface < 0])
    pmap = {int(l): n for n, l in enumerate(prim_labels)}
    prim = np.full(nc, -1, dtype=np.int64)
    pc = iface < 0
    prim[pc] = np.searchsorted(prim_labels, L[pc])
    Np = prim_labels.size
    pin = int(np.flatnonzero(iface < 0)[0])
    # --- face ownership (D3)
    owner = np.full(g.nu, -1, dtype=np.int64)
    for d in g.comps:
        for t in (0, 1):
            f = fc[:, 2 * d + t]
            ok = (f >= 0) & (prim >= 0)
            prev = owner[f[ok]]
            clash = (prev >= 0) & (prev != prim[ok])
            if np.any(clash):
                raise AssertionError("a face lies between two different primaries")
            owner[f[ok]] = prim[ok]
    f_faces = np.flatnonzero(owner < 0)
    free = free_faces(g, owner, walled_faces(g))
    # --- C^{p_i}: interfaces sharing a face with primary i (D4)
    a_pr = prim[:, None].repeat(nbr.shape[1], 1)
    nb_if = np.where(nbr >= 0, iface[np.maximum(nbr, 0)], -1)
    sel = (a_pr >= 0) & (nb_if >= 0)
    pairs_pi = np.unique(np.stack([a_pr[sel], nb_if[sel]], 1), axis=0)
    Cp = [pairs_pi[pairs_pi[:, 0] == i, 1] for i in range(Np)]
    # --- tags (D5)
    ifgrid = np.zeros(g.fluid.shape, dtype=bool)
    ifgrid.ravel()[cells[iface >= 0]] = True
    near = ifgrid.copy()
    for d in g.comps:
        acc = near.copy()
        for s in range(1, tag_layers + 1):
            acc |= g.shift(near, d, s, False) | g.shift(near, d, -s, False)
        near = acc
    tags = []
    for d in g.comps:
        act = g.act[d]
        t = near[act] | g.shift(near, d, -1, False)[act]
        tags.append(t)
    # --- unknown sets
    S = [unknowns_of_cells(g, fc, np.flatnonzero(prim == i)) for i in range(Np)]
    icell_sets = [np.flatnonzero(iface == j) for j in range(Nc)]
    icells = [g.nu + c for c in icell_sets]
    dual_cells, D = [], []
    for j in range(Nc):
        cur = icell_sets[j]
        for _ in range(dual_dilations):
            nb = nbr[cur].ravel()
            cur = np.unique(np.concatenate([cur, nb[nb >= 0]]))
        dual_cells.append(cur)
        D.append(unknowns_of_cells(g, fc, cur))
    return Decomp(g=g, label=L, iface=iface, prim=prim, Nc=Nc, Np=Np, pairs=upairs,
                  pin=pin, owner=owner, Cp=Cp, tags=tags, S=S, D=D,
                  dual_cells=dual_cells, icells=icells, f_faces=f_faces, free=free)
