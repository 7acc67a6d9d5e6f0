"""Shared test helpers: workloads, the oracle <-> cell-record index map."""
import numpy as np

from oracle.mac import MacGrid, Operators, Phys
from oracle.decomp import decompose, largest_component
from synth import make_workload


def oracle_case(mask, labels, rho=1.0, mu=1.0, body=(1.0, 0.0, 0.0), dt=None, periodic=(True, False, False)):
    m = largest_component(mask, periodic)
    g = MacGrid(m, periodic=periodic)
    ops = Operators(g)
    dc = decompose(g, labels)
    ph = Phys(rho, mu, tuple(body), dt, dc.pin)
    return g, ops, dc, ph


def record_index(g, cell_voxel):
    """rec[k] = cell-record slot of oracle unknown k (faces: lower face of the
    upper cell; pressure: last slot of the cell's record)."""
    nrec = g.ndim + 1
    vox2cell = np.full(g.fluid.size, -1, dtype=np.int64)
    vox2cell[cell_voxel] = np.arange(cell_voxel.size)
    co = g.unknown_coords()
    kind, k, j, i = co[:, 0], co[:, 1], co[:, 2], co[:, 3]
    vox = (k * g.ny + j) * g.nx + i
    cell = vox2cell[vox]
    assert np.all(cell >= 0)
    comp = np.where(kind == 3, g.ndim, kind)
    return nrec * cell + comp


def to_record(x_oracle, rec, N):
    out = np.zeros(N)
    out[rec] = x_oracle
    return out


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def workload(name, seed=0, re=None):
    return make_workload(name, seed, re=re)


def fragment_pocket():
    """The 12^3 fragment-pocket window (tests/golden/fragment_pocket.txt)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fragment_pocket.txt")
    head = [l for l in open(path) if l.startswith("#")]
    shape = tuple(int(v) for v in head[1].split()[2:5])
    body = tuple(float(v) for v in head[2].split()[2:5])
    a = np.loadtxt(path, dtype=np.int64)
    return dict(mask=a[:, 0].reshape(shape).astype(np.uint8), labels=a[:, 1].reshape(shape).astype(np.int32),
                body=body, rho=1.0, mu=1.0)
