"""Named synthetic workloads: image, pore labels and physical parameters.

Each workload is a seeded recipe; the same name and seed always give the same
arrays.  The sizes, grain-size laws and porosities follow the paper's sample
types (2D disk packs, 3D grain packs); the paper's own images are not
available, so these stand in for them.

The body force is set from a target Reynolds number Re = rho U l / mu with
U = U_D / phi and l = V_s / A_w (the paper's definitions, Section 6), using a
hydraulic-radius estimate of the Stokes velocity, U ~ rho b R_h^2 / (k mu) with
R_h = V_void / A_w; the achieved Re is measured from the solution afterwards.
"""
import numpy as np

from .packing import disk_packing_rsa, boolean_packing, channel
from .watershed import watershed_labels


def _surface_area(mask):
    """Number of void-solid voxel faces (grains wrap in x; image edges are walls)."""
    m = mask.astype(bool)
    a = 0
    nz, ny, nx = m.shape
    a += np.count_nonzero(m != np.roll(m, 1, axis=2))
    a += np.count_nonzero(m[:, 1:, :] != m[:, :-1, :]) + np.count_nonzero(m[:, 0, :]) + np.count_nonzero(m[:, -1, :])
    if nz > 1:
        a += np.count_nonzero(m[1:] != m[:-1]) + np.count_nonzero(m[0]) + np.count_nonzero(m[-1])
    return a


def body_force_for_re(mask, re, rho=1.0, mu=1.0):
    m = mask.astype(bool)
    aw = max(_surface_area(m), 1)
    v_void = m.sum()
    v_solid = m.size - v_void
    rh = v_void / aw
    l = max(v_solid, 1) / aw
    k = 3.0 if mask.shape[0] == 1 else 2.5
    u_target = re * mu / (rho * l)
    return u_target * k * mu / (rho * rh * rh)


WORKLOADS = {
    # 2D, 64 x 64, non-overlapping disks r ~ U[3, 7], porosity ~0.6, ~20 pores
    "disks2d_64": dict(kind="rsa", nx=64, ny=64, rmin=3.0, rmax=7.0, solid=0.40,
                       footprint=7, min_size=12, re=1.0),
    # 2D, 1024 x 1024, overlapping lognormal disks (mean 10, sigma 0.3), ~3k pores
    "disks2d_1024": dict(kind="boolean", shape=(1, 1024, 1024), mean_r=10.0, sigma=0.3,
                         porosity=0.55, footprint=9, min_size=40, max_size=400, block=14,
                         re=1.0),
    # 3D, 128^3, overlapping lognormal spheres (mean 8, sigma 0.3), porosity ~0.35
    "spheres3d_128": dict(kind="boolean", shape=(128, 128, 128), mean_r=8.0, sigma=0.3,
                          porosity=0.35, footprint=5, min_size=200, max_size=1500, block=8,
                          re=1.0),
    # 3D, 256^3, the same grain law at porosity ~0.35, target Re 10 (backward-Euler runs)
    "spheres3d_256": dict(kind="boolean", shape=(256, 256, 256), mean_r=8.0, sigma=0.3,
                          porosity=0.35, footprint=5, min_size=200, max_size=1500, block=8,
                          re=10.0),
    # 3D, 64^3 crop-sized version of the above (same grain law)
    "spheres3d_64": dict(kind="boolean", shape=(64, 64, 64), mean_r=8.0, sigma=0.3,
                         porosity=0.35, footprint=5, min_size=200, max_size=1500, block=8,
                         re=1.0),
    # 48^3, same grain law as the 128^3 case (mean radius 8)
    "spheres3d_48": dict(kind="boolean", shape=(48, 48, 48), mean_r=8.0, sigma=0.3,
                         porosity=0.35, footprint=5, min_size=200, max_size=1500, block=8,
                         re=1.0),
    # small 3D packing for parity tests
    "spheres3d_24": dict(kind="boolean", shape=(24, 24, 24), mean_r=4.0, sigma=0.3,
                         porosity=0.45, footprint=5, min_size=20, max_size=400, block=6,
                         re=1.0),
    # small 2D packing for parity tests
    "disks2d_32": dict(kind="rsa", nx=32, ny=24, rmin=2.5, rmax=4.5, solid=0.35,
                       footprint=5, min_size=6, re=1.0),
}


def make_workload(name, seed=0, re=None, **over):
    """Return dict(mask, labels, rho, mu, body, name, seed, re_target)."""
    spec = dict(WORKLOADS[name])
    spec.update(over)
    kind = spec["kind"]
    if kind == "rsa":
        mask = disk_packing_rsa(spec["nx"], spec["ny"], spec["rmin"], spec["rmax"],
                                spec["solid"], seed)
    elif kind == "boolean":
        mask = boolean_packing(tuple(spec["shape"]), spec["mean_r"], spec["sigma"],
                               spec["porosity"], seed)
    elif kind == "channel":
        mask = channel(spec["nx"], spec["ny"], spec.get("nz", 1))
    else:
        raise ValueError(kind)
    labels = watershed_labels(mask, footprint=spec["footprint"], min_size=spec["min_size"],
                              max_size=spec.get("max_size", 0), block=spec.get("block", 0))
    rho, mu = 1.0, 1.0
    re_t = spec["re"] if re is None else re
    bx = body_force_for_re(mask, re_t, rho, mu)
    return dict(mask=mask, labels=labels, rho=rho, mu=mu, body=(bx, 0.0, 0.0),
                name=name, seed=seed, re_target=re_t)


def make_batch(nsamples, seed=0, sizes=(48, 96), porosity=(0.3, 0.6), re=(0.1, 20.0), mean_r=8.0,
               sigma=0.3, ndim=3, footprint=5, min_size=200, max_size=1500, block=8, progress=None):
    """A batch of independent samples of uneven size: per sample, each axis drawn
    uniformly from sizes[0]..sizes[1] voxels, the porosity uniformly from ``porosity``
    and the target Re log-uniformly from ``re``; overlapping lognormal grains (Boolean
    model, the grain law of the 3D packings above), labelled by the same watershed.
    Returns a list of workload dicts (as make_workload); progress(k, sample), if given, is
    called after each sample."""
    rng = np.random.default_rng(1000003 + seed)
    out = []
    for k in range(nsamples):
        shp = tuple(int(v) for v in rng.integers(sizes[0], sizes[1] + 1, size=3))
        if ndim == 2:
            shp = (1,) + shp[1:]
        phi = float(rng.uniform(*porosity))
        re_t = float(np.exp(rng.uniform(np.log(re[0]), np.log(re[1]))))
        mask = boolean_packing(shp, mean_r, sigma, phi, int(rng.integers(1 << 30)))
        labels = watershed_labels(mask, footprint=footprint, min_size=min_size, max_size=max_size, block=block)
        bx = body_force_for_re(mask, re_t)
        out.append(dict(mask=mask, labels=labels, rho=1.0, mu=1.0, body=(bx, 0.0, 0.0),
                        name="batch%d_%d" % (seed, k), seed=seed, re_target=re_t, porosity=phi))
        if progress is not None:
            progress(k, out[-1])
    return out
