"""Pore labels from a marker-based watershed of the void-space distance map.

The paper splits the void space into pores (its primary grids) with a modified
watershed from earlier work (Section 3.2.1); that algorithm is not given.  A
plain distance-transform watershed stands in: markers are the local maxima of
the Euclidean distance to the nearest grain, flooded in order of decreasing
distance by a priority queue (Meyer's flooding; ties in arrival order), with
pores under ``min_size`` voxels merged into the neighbour they share the most
faces with.  Labels are 1..Np on void voxels and
0 on grains.
"""
import numpy as np
from scipy import ndimage as ndi


def _periodic_edt(mask, periodic_x=True):
    if not periodic_x:
        return ndi.distance_transform_edt(mask)
    nx = mask.shape[2]
    tiled = np.concatenate([mask, mask, mask], axis=2)
    d = ndi.distance_transform_edt(tiled)
    return d[:, :, nx:2 * nx]


def _face_pairs(lab):
    """Label pairs across every face between two labelled voxels (no wrap)."""
    pairs = []
    for ax in range(3):
        if lab.shape[ax] < 2:
            continue
        a = np.swapaxes(lab, 0, ax)[:-1]
        b = np.swapaxes(lab, 0, ax)[1:]
        m = (a > 0) & (b > 0) & (a != b)
        pairs.append(np.stack([a[m], b[m]], 1))
    if not pairs:
        return np.zeros((0, 2), dtype=lab.dtype)
    return np.concatenate(pairs, 0)


def _merge_small(lab, min_size, max_rounds=50):
    for _ in range(max_rounds):
        sizes = np.bincount(lab.ravel())
        sizes[0] = 0
        small = np.nonzero((sizes > 0) & (sizes < min_size))[0]
        if small.size == 0:
            break
        pairs = _face_pairs(lab)
        if pairs.size == 0:
            break
        both = np.concatenate([pairs, pairs[:, ::-1]], 0)
        key, cnt = np.unique(both, axis=0, return_counts=True)
        target = np.arange(sizes.size)
        is_small = np.zeros(sizes.size, dtype=bool)
        is_small[small] = True
        # each small label moves to its most-shared neighbour (ties: lower label)
        best = {}
        for (a, b), c in zip(key, cnt):
            if not is_small[a]:
                continue
            cur = best.get(a)
            if cur is None or c > cur[1] or (c == cur[1] and b < cur[0]):
                best[a] = (b, c)
        if not best:
            break
        # smallest first; a label that receives a merge this round is not moved itself
        sources, targets = set(), set()
        for a in sorted(best, key=lambda t: (sizes[t], t)):
            b = best[a][0]
            if a in targets or b in sources:
                continue
            target[a] = b
            sources.add(a)
            targets.add(b)
        lab = target[lab]
    return lab


def _lattice_seeds(lab, dist, big, block):
    """One extra marker per (oversized basin, lattice block): the block's
    largest-distance voxel inside that basin."""
    nz, ny, nx = lab.shape
    sel = np.isin(lab, big)
    idx = np.flatnonzero(sel)
    if idx.size == 0:
        return idx
    k, j, i = np.unravel_index(idx, lab.shape)
    bz = k // block if nz > 1 else np.zeros_like(k)
    nby, nbx = -(-ny // block), -(-nx // block)
    bid = (bz * nby + j // block) * nbx + i // block
    key = lab.ravel()[idx].astype(np.int64) * (bid.max() + 1) + bid
    order = np.lexsort((-dist.ravel()[idx], key))
    first = np.ones(order.size, dtype=bool)
    first[1:] = key[order][1:] != key[order][:-1]
    return idx[order[first]]


def _neighbours(mask, periodic_x):
    """Face-neighbour table over the void voxels (compact numbering)."""
    nz, ny, nx = mask.shape
    vox = np.flatnonzero(mask)
    cidx = np.full(mask.size, -1, dtype=np.int64)
    cidx[vox] = np.arange(vox.size)
    cidx = cidx.reshape(mask.shape)
    k, j, i = np.unravel_index(vox, mask.shape)
    nb = []
    for dk, dj, di in ((0, 0, -1), (0, 0, 1), (0, -1, 0), (0, 1, 0), (-1, 0, 0), (1, 0, 0)):
        kk, jj, ii = k + dk, j + dj, i + di
        if periodic_x:
            ii = np.mod(ii, nx)
        ok = (kk >= 0) & (kk < nz) & (jj >= 0) & (jj < ny) & (ii >= 0) & (ii < nx)
        out = np.full(vox.size, -1, dtype=np.int64)
        out[ok] = cidx[kk[ok], jj[ok], ii[ok]]
        nb.append(out)
    return vox, np.stack(nb, 1)


def _flood(dist, markers, mask, periodic_x=True):
    """Meyer flooding from labelled markers, highest distance first."""
    import heapq
    vox, nb = _neighbours(mask, periodic_x)
    d = dist.ravel()[vox]
    lab = markers.ravel()[vox].astype(np.int64)
    nbl = nb.tolist()
    dl = (-d).tolist()
    labl = lab.tolist()
    queued = [l > 0 for l in labl]
    heap = []
    cnt = 0
    for v in np.flatnonzero(lab > 0).tolist():
        for u in nbl[v]:
            if u >= 0 and not queued[u]:
                queued[u] = True
                heap.append((dl[u], cnt, u, labl[v]))
                cnt += 1
    heapq.heapify(heap)
    pop, push = heapq.heappop, heapq.heappush
    while heap:
        _, _, v, l = pop(heap)
        labl[v] = l
        for u in nbl[v]:
            if u >= 0 and not queued[u]:
                queued[u] = True
                push(heap, (dl[u], cnt, u, l))
                cnt += 1
    out = np.zeros(mask.size, dtype=np.int64)
    out[vox] = np.array(labl, dtype=np.int64)
    return out.reshape(mask.shape)


def watershed_labels(mask, footprint=5, h_min=1.0, min_size=0, periodic_x=True,
                     max_size=0, block=0):
    """Label the void voxels of ``mask`` (shape (nz, ny, nx)) into pores.

    ``footprint`` is the edge of the cubic (square in 2D) window in which a
    marker must be a distance-map maximum; ``h_min`` is the smallest distance
    a marker may sit at.  Basins larger than ``max_size`` voxels are re-seeded
    with one marker per ``block``-sized lattice cell and flooded again.
    """
    mask = np.asarray(mask).astype(bool)
    two_d = mask.shape[0] == 1
    dist = _periodic_edt(mask, periodic_x)
    fp = (1, footprint, footprint) if two_d else (footprint,) * 3
    peak = (dist == ndi.maximum_filter(dist, size=fp, mode="wrap")) & mask & (dist >= h_min)
    struct = ndi.generate_binary_structure(3, 3)
    if two_d:
        struct[0] = False
        struct[2] = False
    markers, nm = ndi.label(peak, structure=struct)
    if nm == 0:
        markers = mask.astype(np.int32)
    conn = ndi.generate_binary_structure(3, 1)
    if two_d:
        conn[0] = False
        conn[2] = False
    markers = markers.astype(np.int64)
    lab = _flood(dist, markers, mask, periodic_x)
    for _ in range(3 if (max_size > 0 and block > 0) else 0):
        sizes = np.bincount(lab.ravel())
        sizes[0] = 0
        big = np.nonzero(sizes > max_size)[0]
        if big.size == 0:
            break
        seeds = _lattice_seeds(lab, dist, big, block)
        flat = markers.ravel()
        fresh = seeds[flat[seeds] == 0]
        if fresh.size == 0:
            break
        flat[fresh] = markers.max() + 1 + np.arange(fresh.size)
        markers = flat.reshape(mask.shape)
        lab = _flood(dist, markers, mask, periodic_x)
        block = max(2, block * 3 // 4)
    # void voxels the flood did not reach (separated pockets) get their own labels
    orphan = mask & (lab == 0)
    if orphan.any():
        ol, no = ndi.label(orphan, structure=conn)
        lab = np.where(orphan, ol + lab.max(), lab)
    if min_size > 0:
        lab = _merge_small(lab, min_size)
    # consecutive labels 1..Np in order of first appearance along the raster scan
    u, first = np.unique(lab.ravel(), return_index=True)
    u, first = u[u > 0], first[u > 0]
    order = u[np.argsort(first)]
    remap = np.zeros(int(lab.max()) + 1, dtype=np.int32)
    remap[order] = np.arange(1, order.size + 1, dtype=np.int32)
    return remap[lab].astype(np.int32)


def throat_labels(mask, pore_labels, periodic_x=True):
    """Throat regions for the pore-network decomposition (Section 3.3 of the paper: the
    watershed is seeded at the interface pixels of the pore decomposition, so that its
    regions are the constrictions and their meeting places lie in the pore bodies).

    Seeds: the void voxels with a face neighbour of another pore label, one marker per
    face-connected set of such voxels on the same pair of pores; the markers are grown
    through the void breadth-first (ties in arrival order) until they meet.  Returns
    labels 1..Nt on the void voxels (0 on grains), numbered in raster order of first
    appearance."""
    mask = np.asarray(mask).astype(bool)
    lab = np.asarray(pore_labels).astype(np.int64)
    if mask.ndim == 2:
        mask, lab = mask[None], lab[None]
    vox, nb = _neighbours(mask, periodic_x)
    lv = lab.ravel()[vox]
    nbl = np.where(nb >= 0, lv[np.maximum(nb, 0)], 0)
    other = (nb >= 0) & (nbl != lv[:, None]) & (nbl > 0)
    seed = other.any(1)
    # the pair of pores a seed voxel sits between: its own label and its smallest other
    big = np.iinfo(np.int64).max
    partner = np.where(other, nbl, big).min(1)
    key = np.minimum(lv, partner) * (lab.max() + 1) + np.maximum(lv, partner)
    # components of seed voxels with the same pair
    sidx = np.flatnonzero(seed)
    pos = np.full(vox.size, -1, dtype=np.int64)
    pos[sidx] = np.arange(sidx.size)
    rows, cols = [], []
    for e in range(nb.shape[1]):
        u = nb[sidx, e]
        ok = (u >= 0) & seed[np.maximum(u, 0)]
        ok &= key[np.maximum(u, 0)] == key[sidx]
        rows.append(pos[sidx[ok]])
        cols.append(pos[u[ok]])
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    r, c = np.concatenate(rows), np.concatenate(cols)
    n = sidx.size
    _, comp = connected_components(csr_matrix((np.ones(r.size), (r, c)), shape=(n, n)), directed=False)
    markers = np.zeros(mask.size, dtype=np.int64)
    markers[vox[sidx]] = comp + 1
    out = _flood(np.zeros(mask.shape), markers.reshape(mask.shape), mask, periodic_x)
    orphan = mask & (out == 0)
    if orphan.any():
        conn = ndi.generate_binary_structure(3, 1)
        ol, _ = ndi.label(orphan, structure=conn)
        out = np.where(orphan, ol + out.max(), out)
    u, first = np.unique(out.ravel(), return_index=True)
    u, first = u[u > 0], first[u > 0]
    order = u[np.argsort(first)]
    remap = np.zeros(int(out.max()) + 1, dtype=np.int32)
    remap[order] = np.arange(1, order.size + 1, dtype=np.int32)
    return remap[out].astype(np.int32)
