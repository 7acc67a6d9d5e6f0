"""Seeded grain packings on a voxel grid.

Arrays are indexed [k, j, i] (z, y, x) with x fastest; a 2D image has nz = 1.
``mask`` is uint8 with 1 = void (fluid) and 0 = grain (solid).  A voxel is solid
when its centre lies inside a grain.  Grains wrap around in x (the flow
direction is periodic in x); y and z are bounded by the image edges.
"""
import numpy as np


def channel(nx, ny, nz=1):
    """An empty image: a plane channel between the y walls (and z walls in 3D)."""
    return np.ones((nz, ny, nx), dtype=np.uint8)


def _paint(solid, centres, radii, periodic_x=True):
    nz, ny, nx = solid.shape
    for (cz, cy, cx), r in zip(centres, radii):
        r2 = r * r
        z0, z1 = (0, 1) if nz == 1 else (int(np.floor(cz - r)), int(np.ceil(cz + r)) + 1)
        y0, y1 = int(np.floor(cy - r)), int(np.ceil(cy + r)) + 1
        x0, x1 = int(np.floor(cx - r)), int(np.ceil(cx + r)) + 1
        zs = np.arange(max(z0, 0), min(z1, nz))
        ys = np.arange(max(y0, 0), min(y1, ny))
        xs = np.arange(x0, x1)
        if not periodic_x:
            xs = xs[(xs >= 0) & (xs < nx)]
        if zs.size == 0 or ys.size == 0 or xs.size == 0:
            continue
        dz = (zs + 0.5 - cz) if nz > 1 else np.zeros(1)
        dy = ys + 0.5 - cy
        dx = xs + 0.5 - cx
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        inside = d2 <= r2
        xi = np.mod(xs, nx)
        sub = solid[np.ix_(zs, ys, xi)]
        sub |= inside
        solid[np.ix_(zs, ys, xi)] = sub


def disk_packing_rsa(nx, ny, rmin, rmax, solid_target, seed, max_tries=200000):
    """Random sequential addition of non-overlapping disks (2D).

    Radii are uniform in [rmin, rmax]; centres are uniform in the box; the
    overlap test uses the periodic distance in x.  Disks are added until the
    solid voxel fraction reaches ``solid_target`` (or no more fit).
    """
    rng = np.random.default_rng(seed)
    solid = np.zeros((1, ny, nx), dtype=bool)
    cs, rs = [], []
    tries = 0
    while solid.mean() < solid_target and tries < max_tries:
        tries += 1
        r = rng.uniform(rmin, rmax)
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        ok = True
        for (qy, qx), q in zip(cs, rs):
            dx = abs(cx - qx)
            dx = min(dx, nx - dx)
            if dx * dx + (cy - qy) ** 2 < (r + q) ** 2:
                ok = False
                break
        if not ok:
            continue
        cs.append((cy, cx))
        rs.append(r)
        _paint(solid, [(0.5, cy, cx)], [r])
    return (~solid).astype(np.uint8)


def lognormal_radii(rng, n, mean, sigma, rmin=2.0):
    """Radii r = exp(N(ln m - s^2/2, s^2)) so that E[r] = m; clipped to [rmin, 3m]."""
    mu = np.log(mean) - 0.5 * sigma * sigma
    r = np.exp(rng.normal(mu, sigma, size=n))
    return np.clip(r, rmin, 3.0 * mean)


def boolean_packing(shape, mean_r, sigma, porosity, seed, batch=64):
    """Overlapping (Boolean-model) disks or spheres with lognormal radii.

    ``shape`` is (nz, ny, nx); nz == 1 gives disks.  Grains are added in small
    batches until the void fraction drops to ``porosity`` or below.
    """
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    solid = np.zeros(shape, dtype=bool)
    while 1.0 - solid.mean() > porosity:
        rs = lognormal_radii(rng, batch, mean_r, sigma)
        cz = rng.uniform(0, nz, batch) if nz > 1 else np.full(batch, 0.5)
        cy = rng.uniform(0, ny, batch)
        cx = rng.uniform(0, nx, batch)
        for b in range(batch):
            _paint(solid, [(cz[b], cy[b], cx[b])], [rs[b]])
            if 1.0 - solid.mean() <= porosity:
                break
    return (~solid).astype(np.uint8)
