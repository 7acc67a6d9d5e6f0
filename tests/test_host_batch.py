"""CPU tests of the batch set-up (gplmm_setup_batch, host-only contexts): the
decomposition of a batch is the concatenation of the decompositions each sample
gets alone, with cells, primaries, interfaces, voxels and slots shifted by the
sample offsets that gplmm_batch_info reports.  Samples of uneven size, 2D and 3D."""
import os

import numpy as np
import pytest

from synth import make_batch


def _binding():
    from paper_2510_22077_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgplmm.so not built")
    return binding


def _small_batch(ndim, n, seed):
    return make_batch(n, seed, sizes=(16, 26), mean_r=4.0, footprint=5, min_size=20, max_size=400, block=6,
                      ndim=ndim, porosity=(0.4, 0.6))


@pytest.mark.parametrize("ndim,n", [(2, 4), (3, 3)])
def test_batch_decomposition_is_the_concatenation(ndim, n):
    b = _binding()
    ws = _small_batch(ndim, n, seed=ndim)
    if ndim == 2:
        ws = [dict(w, mask=np.ascontiguousarray(w["mask"][:1]), labels=np.ascontiguousarray(w["labels"][:1]))
              for w in ws]
    B = b.BatchSolver([w["mask"] for w in ws], [w["labels"] for w in ws], bodies=[w["body"] for w in ws],
                      host_only=True)
    info = B.batch_info()
    assert info["nsamples"] == n
    mb = B.maps()
    db = B.duals()
    nrec = B.layout.nrec
    for k, w in enumerate(ws):
        S = b.Solver(w["mask"], w["labels"], body=w["body"], host_only=True)
        ms = S.maps()
        c0, c1 = info["cell_off"][k], info["cell_off"][k + 1]
        p0, i0 = info["prim_off"][k], info["iface_off"][k]
        v0 = info["voxel_off"][k]
        assert c1 - c0 == S.layout.ncell
        assert info["prim_off"][k + 1] - p0 == S.layout.Np
        assert info["iface_off"][k + 1] - i0 == S.layout.Nc
        assert info["voxel_off"][k + 1] - v0 == w["mask"].size
        assert np.array_equal(mb["cell_voxel"][c0:c1], ms["cell_voxel"] + v0)
        sh = lambda a, o: np.where(a >= 0, a + o, a)
        assert np.array_equal(mb["cell_iface"][c0:c1], sh(ms["cell_iface"], i0))
        assert np.array_equal(mb["cell_prim"][c0:c1], sh(ms["cell_prim"], p0))
        assert np.array_equal(mb["face_owner"][nrec * c0:nrec * c1], sh(ms["face_owner"], p0))
        assert np.array_equal(mb["face_tag"][nrec * c0:nrec * c1], ms["face_tag"])
        ds = S.duals()
        for j, d in enumerate(ds):
            assert np.array_equal(db[i0 + j], d + c0)
        # local problem sizes of the sample's primaries and duals
        nb_, _ = B.subdomains()
        ns_, _ = S.subdomains()
        Np_b = B.layout.Np
        assert np.array_equal(nb_[p0:p0 + S.layout.Np], ns_[:S.layout.Np])
        assert np.array_equal(nb_[Np_b + i0:Np_b + i0 + S.layout.Nc], ns_[S.layout.Np:])
        S.close()
    B.close()


def test_batch_of_one_equals_the_single_context():
    b = _binding()
    w = _small_batch(3, 1, seed=5)[0]
    B = b.BatchSolver([w["mask"]], [w["labels"]], bodies=[w["body"]], host_only=True)
    S = b.Solver(w["mask"], w["labels"], body=w["body"], host_only=True)
    for key in ("ncell", "N", "Np", "Nc", "Ny", "pin", "factor_bytes", "ncolors"):
        assert getattr(B.layout, key) == getattr(S.layout, key), key
    mb, ms = B.maps(), S.maps()
    for key in mb:
        assert np.array_equal(mb[key], ms[key]), key


def test_batch_rejects_mixed_dimensions():
    b = _binding()
    w2 = _small_batch(2, 1, seed=1)[0]
    w3 = _small_batch(3, 1, seed=1)[0]
    with pytest.raises(b.GplmmError, match="mixed dimension|same dimension"):
        b.BatchSolver([w3["mask"], w2["mask"][:1]], [w3["labels"], w2["labels"][:1]], host_only=True)
