"""Host checks of the f-face blocks behind the back-substitution of Eq. xf
(options.mg_form = 1), against the oracle's decomposition and build matrix X rather than
the library's own structures.

x_f = (A^f_f)^-1 (b - Ahat z)_f is solved block by block, which is exact only if
* the blocks partition exactly the oracle's f-faces (velocity unknowns of no primary);
* X couples no two blocks (the geometric build matrix and the Newton Jacobian with its
  transverse couplings, at a random wind, so every upwind branch is taken somewhere);
and costs least if the blocks are as fine as that allows: for the Stokes matrix (all
couplings of the stencil present) they are exactly the connected components of
X[F, F].  Also: the option's range and its exclusions are enforced at setup.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from oracle.mac import build_matrix, jacobian
from tests.helpers import oracle_case, record_index, workload


def _crop(n):
    w = workload("spheres3d_128", 0)
    return dict(w, mask=w["mask"][:n, :n, :n].copy(), labels=w["labels"][:n, :n, :n].copy())


def _blocks(w, build, g, rec_of):
    from paper_2510_22077_amd import Solver
    s = Solver(w["mask"], w["labels"], rho=w["rho"], mu=w["mu"], body=w["body"], host_only=True, mg_form=1,
               build_matrix=build)
    to_oracle = np.full(s.N, -1, np.int64)
    rec = rec_of(s)
    to_oracle[rec] = np.arange(g.N)
    blocks = [to_oracle[b] for b in s.fblocks()]
    L = s.layout
    assert L.nfblock == len(blocks) >= 1
    assert L.max_fblock == max(b.size for b in blocks)
    s.close()
    return blocks, int(L.f_unknowns)


@pytest.mark.parametrize("name,seed", [("disks2d_64", 1), ("spheres3d_24", 0), ("spheres3d_24", 1), ("crop32", 0)])
def test_fblocks_partition_the_oracle_f_faces(name, seed):
    w = _crop(32) if name == "crop32" else workload(name, seed)
    g, ops, dc, ph = oracle_case(w["mask"], w["labels"], w["rho"], w["mu"], w["body"])
    rec_of = lambda s: record_index(g, s.maps()["cell_voxel"])
    F = np.asarray(dc.f_faces)
    rng = np.random.default_rng(seed)
    wind = rng.standard_normal(g.N)
    for build in ("geometric", "jacobian"):
        blocks, nf = _blocks(w, build, g, rec_of)
        allf = np.concatenate(blocks)
        assert np.all(allf >= 0)
        assert nf == allf.size == F.size
        assert np.array_equal(np.sort(allf), np.sort(F))
        blk = np.full(g.N, -1, np.int64)
        for k, b in enumerate(blocks):
            blk[b] = k
        # X couples no two blocks: the geometric build matrix, or the untagged Newton
        # Jacobian at the state w (whose transverse couplings join more f-faces)
        X = build_matrix(ops, ph, wind=wind, tags=dc.tags) if build == "geometric" else jacobian(ops, wind, ph)
        C = sp.coo_matrix(sp.csr_matrix(X)[F][:, F])
        nz = C.data != 0.0
        assert np.all(blk[F[C.row[nz]]] == blk[F[C.col[nz]]])
        if build == "geometric":
            # the Stokes matrix: the blocks are exactly the connected components of X[F, F]
            C = sp.csr_matrix(build_matrix(ops, ph))[F][:, F]
            C.eliminate_zeros()
            ncomp, lab = connected_components(C, directed=False)
            assert ncomp == len(blocks)
            assert len(set(zip(lab.tolist(), blk[F].tolist()))) == ncomp


def test_mg_form_option_range_and_exclusions():
    from paper_2510_22077_amd import GplmmError, Solver
    w = workload("disks2d_32", 0)
    kw = dict(rho=w["rho"], mu=w["mu"], body=w["body"], host_only=True)
    s = Solver(w["mask"], w["labels"], mg_form=0, **kw)
    assert s.layout.nfblock == 0 and s.fblocks() == []
    s.close()
    s1 = Solver(w["mask"], w["labels"], mg_form=1, **kw)
    s2 = Solver(w["mask"], w["labels"], mg_form=2, **kw)   # same blocks, another coarse operator
    b1, b2 = s1.fblocks(), s2.fblocks()
    assert len(b1) == len(b2) >= 1 and all(np.array_equal(x, y) for x, y in zip(b1, b2))
    s1.close()
    s2.close()
    for bad in (dict(mg_form=3), dict(mg_form=-1), dict(mg_form=1, split_tiles=2), dict(mg_form=2, split_tiles=2)):
        with pytest.raises(GplmmError):
            Solver(w["mask"], w["labels"], **bad, **kw)
