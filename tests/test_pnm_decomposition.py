"""The pore-network decomposition (Section 3.3: throat regions as primary grids, one
contact interface per pore body) on the CPU: oracle invariants and the library's host
decomposition bit-exact against the oracle."""
import os

import numpy as np
import pytest

from oracle.mac import MacGrid
from oracle.decomp import decompose, largest_component
from synth import make_workload, throat_labels
from tests.helpers import record_index


def _pnm_case(name, seed):
    if name == "crop48":
        w = make_workload("spheres3d_128", 0)
        w = dict(w, mask=w["mask"][:48, :48, :48].copy(), labels=w["labels"][:48, :48, :48].copy())
    else:
        w = make_workload(name, seed)
    th = throat_labels(w["mask"], w["labels"])
    return w, th


@pytest.mark.parametrize("name,seed", [("disks2d_64", 0), ("disks2d_64", 2), ("spheres3d_24", 0), ("crop48", 0)])
def test_pnm_interfaces_are_pore_bodies(name, seed):
    w, th = _pnm_case(name, seed)
    g = MacGrid(largest_component(w["mask"]))
    dc = decompose(g, th, groups=w["labels"])
    pores = (w["labels"] if w["labels"].ndim == 3 else w["labels"][None]).ravel()[np.flatnonzero(g.fluid)]
    # an interface is carved cells of one pore (merged degenerate ones may add a neighbour's)
    for j in range(dc.Nc):
        cells = np.flatnonzero(dc.iface == j)
        assert cells.size > 0
    assert dc.Nc <= np.unique(pores).size
    # a throat region usually touches two pore bodies; most interfaces are shared by >= 2 throats
    nthroats = np.bincount(np.concatenate([c for c in dc.Cp]), minlength=dc.Nc)
    assert np.mean(nthroats >= 2) > 0.5
    # the p/c/f partition still covers every unknown exactly once
    allS = np.concatenate(dc.S)
    assert np.unique(allS).size == allS.size


@pytest.mark.parametrize("name,seed", [("disks2d_64", 0), ("spheres3d_24", 0), ("crop48", 0)])
def test_library_pnm_decomposition_bit_exact(name, seed):
    from paper_2510_22077_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgplmm.so not built")
    w, th = _pnm_case(name, seed)
    s = binding.Solver(w["mask"], th, body=w["body"], groups=w["labels"], host_only=True)
    g = MacGrid(largest_component(w["mask"]))
    dc = decompose(g, th, groups=w["labels"])
    info, m = s.info(), s.maps()
    assert info["Np"] == dc.Np and info["Nc"] == dc.Nc and info["pin"] == dc.pin
    assert np.array_equal(m["cell_iface"], dc.iface)
    assert np.array_equal(m["cell_prim"], dc.prim)
    rec = record_index(g, m["cell_voxel"])
    assert np.array_equal(m["face_owner"][rec[:g.nu]], dc.owner)
    assert np.array_equal(m["face_tag"][rec[:g.nu]] & 1, np.concatenate(dc.tags).astype(np.int8))
    for a, b in zip(s.duals(), dc.dual_cells):
        assert np.array_equal(a, b)
    s.close()
