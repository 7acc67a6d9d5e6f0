"""CPU tests of the C ABI: the library loads, exports every declared entry
point, and its host-side decomposition (carving, admissibility merge, interface
merge, ownership, tags, dual grids, pin) is bit-exact against the oracle's
independent implementation.  No device call is made (host-only contexts)."""
import os
import re

import numpy as np
import pytest

from tests.helpers import oracle_case, record_index, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    from paper_2510_22077_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgplmm.so not built")
    return binding


def test_library_exports_every_declared_symbol():
    binding = _lib_or_skip()
    lib = binding.load()
    hdr = open(os.path.join(ROOT, "include", "gplmm.h")).read()
    declared = set(re.findall(r"\b(gplmm_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(binding.EXPORTS)


_CROPS = {}


def _crop(n):
    """n^3 corner of the 128^3 benchmark packing (generated once per session)."""
    if "w" not in _CROPS:
        _CROPS["w"] = workload("spheres3d_128", 0)
    w = dict(_CROPS["w"])
    w["mask"] = w["mask"][:n, :n, :n].copy()
    w["labels"] = w["labels"][:n, :n, :n].copy()
    return w


@pytest.mark.parametrize("name,seed", [("disks2d_64", 0), ("disks2d_64", 3), ("disks2d_32", 1),
                                       ("spheres3d_24", 0), ("spheres3d_24", 2), ("spheres3d_48", 0),
                                       ("crop", 48), ("crop", 64), ("fragment", 0)])
def test_host_decomposition_bit_exact(name, seed):
    binding = _lib_or_skip()
    if name == "fragment":
        from tests.helpers import fragment_pocket
        w = fragment_pocket()
    else:
        w = _crop(seed) if name == "crop" else workload(name, seed)
    s = binding.Solver(w["mask"], w["labels"], body=w["body"], host_only=True)
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], body=w["body"])
    info = s.info()
    m = s.maps()
    assert info["ncell"] == g.nc and info["nface_active"] == g.nu
    assert info["Np"] == dc.Np and info["Nc"] == dc.Nc and info["pin"] == dc.pin
    assert np.array_equal(m["cell_voxel"], np.flatnonzero(g.fluid))
    assert np.array_equal(m["cell_iface"], dc.iface)
    assert np.array_equal(m["cell_prim"], dc.prim)
    rec = record_index(g, m["cell_voxel"])
    # face ownership and tags on every velocity unknown
    assert np.array_equal(m["face_owner"][rec[:g.nu]], dc.owner)
    tags = np.concatenate([t for t in dc.tags]).astype(np.int8)
    assert np.array_equal(m["face_tag"][rec[:g.nu]] & 1, tags)
    assert np.array_equal((m["face_tag"][rec[:g.nu]] >> 1) & 1, dc.free.astype(np.int8))
    # every other slot is a void slot or a pressure
    other = np.setdiff1d(np.arange(info["N"]), rec[:g.nu])
    assert np.all(np.isin(m["face_owner"][other], [-2, -3]))
    du = s.duals()
    assert len(du) == dc.Nc
    for a, b in zip(du, dc.dual_cells):
        assert np.array_equal(a, b)
    s.close()


def test_host_only_context_refuses_compute_calls():
    binding = _lib_or_skip()
    w = workload("disks2d_32", 0)
    s = binding.Solver(w["mask"], w["labels"], body=w["body"], host_only=True)
    lib = s.lib
    rc = lib.gplmm_build(s.ctx, None)
    assert rc == -5
    assert b"host-only" in lib.gplmm_last_error(s.ctx)
    s.close()


def test_setup_rejects_bad_labels_and_sizes():
    binding = _lib_or_skip()
    w = workload("disks2d_32", 0)
    lab = w["labels"].copy()
    lab[w["mask"] == 1] = 0
    with pytest.raises(binding.GplmmError):
        binding.Solver(w["mask"], lab, host_only=True)
    with pytest.raises(binding.GplmmError):
        binding.Solver(np.zeros((1, 8, 8), np.uint8), np.zeros((1, 8, 8), np.int32), host_only=True)


def test_set_tuning_accepts_the_documented_range_only():
    """gplmm_set_tuning: red_blocks 64..2048, stencil_block 128/256/512, trsv_mode 0..2;
    anything else is GPLMM_E_ARG and leaves the context usable (host-only context)."""
    binding = _lib_or_skip()
    from paper_2510_22077_amd import Solver
    w = workload("disks2d_32", 0)
    s = Solver(w["mask"], w["labels"], body=w["body"], host_only=True)
    for rb, sb, tm in [(64, 128, 0), (2048, 512, 1), (1024, 256, 2)]:
        s.set_tuning(red_blocks=rb, stencil_block=sb, trsv_mode=tm)
    for rb, sb, tm in [(32, 256, 0), (4096, 256, 0), (1024, 100, 0), (1024, 256, 3), (1024, 256, -1)]:
        with pytest.raises(binding.GplmmError):
            s.set_tuning(red_blocks=rb, stencil_block=sb, trsv_mode=tm)
    s.set_tuning(red_blocks=512, stencil_block=128, trsv_mode=0)
    s.close()
