"""gPLMM preconditioner: build and apply, sparse FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper:
* two-level structure M^-1 = M_G^-1 + M_L^-1 (I - A M_G^-1), with one stage of
  the base smoother M_l = M_dp (Section 3.1);
* reduction: the f-face columns and the other primaries' columns of each
  primary row are summed onto its diagonal (Section 3.2.2, the two reduction
  equations), which gives the closure matrices Abar_i; rows of faces in a
  wall-free group (see ``decomp``) are left unsummed so Abar_i stays regular;
* shape vectors  phi_ij = -Abar_i^-1 (A restricted to the rows of primary i
  and summed over the cells of interface j), correction vectors
  chi_i = Abar_i^-1 b_B (Section 3.2.2, prolongation), with b_B the residual
  of the steady equations at the origin;
* restriction: interface rows sum over the interface cells, primary rows sum
  over every row of the primary (the 0/1 pattern of C^T) (Section 3.2.2);
* compact form M_G^-1 = Phat (Rhat A Phat)^-1 Rhat with A in place of the
  column-summed operator (Section 3.2.2, Remark 1); Phat leaves the f-faces
  at zero (``mg_form=0``, the default);
* or the full form of Eq. iMG (``mg_form=1``): the coarse operator
  Rhat Acheck Phat from the column-summed matrix Acheck (the p and c rows after
  both reductions: f columns, and for primary rows the other primaries'
  columns, summed onto the diagonal), and the f unknowns recovered by the
  back-substitution of Eq. xf, x^f = (A^f_f)^-1 (b^f - A^f_p x^p - A^f_c x^c),
  i.e. x^f = (A^f_f)^-1 (b - A x)^f with x^f = 0 in x;
* or (``mg_form=2``) the compact coarse operator of Remark 1 followed by the
  same back-substitution of Eq. xf for the f unknowns;
* dual-primary smoother M_dp^-1 = M_d^-1 + M_p^-1 (I - A M_d^-1), with the
  additive-Schwarz sums over primaries and duals (Section 3.2.3).

For gPLMM the matrix A everywhere above is the build matrix X = J~_w
(Section 4); the Newton right-hand side stays the true residual.
"""
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .decomp import Decomp


@dataclass
class GPLMM:
    X: sp.csr_matrix
    dc: Decomp
    phi: List[np.ndarray]             # per primary: |S_i| x |C^{p_i}| shape vectors
    chi: List[Optional[np.ndarray]]   # per primary: correction vector or None
    ycols: np.ndarray                 # primary ids that carry a y^o unknown
    P: sp.csr_matrix                  # Phat  (N x (Nc + Ny))
    R: sp.csr_matrix                  # Rhat  ((Nc + Ny) x N)
    Ao: np.ndarray                    # Rhat X Phat (dense)
    Ao_lu: object
    lu_p: list
    lu_d: list
    Abar: list
    mg_form: int = 0                  # 0: Remark 1; 1: Eq. iMG with the x^f back-substitution;
                                      # 2: Remark 1 with the x^f back-substitution
    lu_f: object = None               # mg_form 1, 2: LU of A^f_f
    t_mg: float = 0.0                 # seconds spent on M_G (closures, shape vectors, Ao)
    t_ml: float = 0.0                 # seconds spent on the smoother's local factorisations


def closure_matrix(X, S, cols_summed, exempt=None):
    """X[S,S] + diag(row sums of X[S, cols_summed]); rows flagged in ``exempt``
    (faces of wall-free groups) keep their plain row."""
    XS = X[S][:, S].tocsr()
    if cols_summed.size == 0:
        return XS.tocsc()
    extra = np.asarray(X[S][:, cols_summed].sum(axis=1)).ravel()
    if exempt is not None:
        extra = np.where(exempt, 0.0, extra)
    return (XS + sp.diags(extra)).tocsc()


def column_summed(X, dc: Decomp, owner_all):
    """The p and c rows of Acheck (Eq. iMG): row s keeps its columns in its own
    primary and in the interface cells (a primary row) or outside the f-faces (an
    interface-cell row); the columns it drops are summed onto its diagonal (the two
    reductions of Section 3.2.2), except on rows of faces in wall-free groups, which
    drop them.  f rows are zero (Rhat has no f columns)."""
    g = dc.g
    Xc = sp.coo_matrix(X)
    r, c, v = Xc.row, Xc.col, Xc.data
    orow, ocol = owner_all[r], owner_all[c]
    prow = orow >= 0
    crow = orow == -2
    keep = (prow & ((ocol == orow) | (ocol == -2))) | (crow & (ocol != -1))
    move = (prow & ~keep) | (crow & (ocol == -1))
    exempt = np.zeros(g.N, dtype=bool)
    exempt[:g.nu] = dc.free
    move &= ~exempt[r]
    diag = np.bincount(r[move], weights=v[move], minlength=g.N)
    A = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=X.shape)
    return (A + sp.diags(diag)).tocsr()


def build(X, dc: Decomp, bB, mg_form=0):
    import time
    t0 = time.perf_counter()
    X = sp.csr_matrix(X)
    g = dc.g
    N = g.N
    # columns that belong to the "p" or "f" sets of each row's neighbours
    owner_all = np.full(N, -2, dtype=np.int64)         # -2: cell of an interface ("c")
    owner_all[:g.nu] = dc.owner                         # faces: primary id or -1 (f)
    cells = np.arange(g.nc)
    owner_all[g.nu + cells] = np.where(dc.prim >= 0, dc.prim, -2)
    phi, chi, Abar = [], [], []
    Prow, Pcol, Pval = [], [], []
    ycols = []
    for i in range(dc.Np):
        S = dc.S[i]
        # columns outside S that are f-faces or other primaries' unknowns
        XS = X[S]
        nz_cols = np.unique(XS.indices)
        oc = owner_all[nz_cols]
        summed = nz_cols[((oc == -1) | (oc >= 0)) & (oc != i)]
        exempt = np.zeros(S.size, dtype=bool)
        vel = S < g.nu
        exempt[vel] = dc.free[S[vel]]
        Ab = closure_matrix(X, S, summed, exempt)
        lu = spla.splu(Ab)
        Abar.append(Ab)
        cols = []
        for j in dc.Cp[i]:
            gij = -np.asarray(XS[:, dc.icells[j]].sum(axis=1)).ravel()
            cols.append(lu.solve(gij))
        ph = np.stack(cols, 1) if cols else np.zeros((S.size, 0))
        phi.append(ph)
        for n, j in enumerate(dc.Cp[i]):
            Prow.append(S)
            Pcol.append(np.full(S.size, j))
            Pval.append(ph[:, n])
        bS = bB[S]
        if np.any(bS != 0):
            c = lu.solve(bS)
            chi.append(c)
            ycols.append(i)
        else:
            chi.append(None)
    ycols = np.array(ycols, dtype=np.int64)
    nco = dc.Nc + ycols.size
    for j in range(dc.Nc):
        Prow.append(dc.icells[j])
        Pcol.append(np.full(dc.icells[j].size, j))
        Pval.append(np.ones(dc.icells[j].size))
    for n, i in enumerate(ycols):
        Prow.append(dc.S[i])
        Pcol.append(np.full(dc.S[i].size, dc.Nc + n))
        Pval.append(chi[i])
    P = sp.csr_matrix((np.concatenate(Pval), (np.concatenate(Prow), np.concatenate(Pcol))),
                      shape=(N, nco))
    Rr, Rc = [], []
    for j in range(dc.Nc):
        Rr.append(np.full(dc.icells[j].size, j))
        Rc.append(dc.icells[j])
    for n, i in enumerate(ycols):
        Rr.append(np.full(dc.S[i].size, dc.Nc + n))
        Rc.append(dc.S[i])
    R = sp.csr_matrix((np.ones(sum(a.size for a in Rr)), (np.concatenate(Rr), np.concatenate(Rc))),
                      shape=(nco, N))
    lu_f = None
    if mg_form == 1:
        Ao = (R @ column_summed(X, dc, owner_all) @ P).toarray()
    else:
        Ao = (R @ X @ P).toarray()
    if mg_form in (1, 2):
        F = np.asarray(dc.f_faces, dtype=np.int64)
        if F.size:
            lu_f = spla.splu(X[F][:, F].tocsc())
    Ao_lu = _dense_lu(Ao)
    t1 = time.perf_counter()
    lu_p = [spla.splu(X[S][:, S].tocsc()) for S in dc.S]
    lu_d = [spla.splu(X[D][:, D].tocsc()) for D in dc.D]
    t2 = time.perf_counter()
    return GPLMM(X=X, dc=dc, phi=phi, chi=chi, ycols=ycols, P=P, R=R, Ao=Ao, Ao_lu=Ao_lu,
                 lu_p=lu_p, lu_d=lu_d, Abar=Abar, mg_form=mg_form, lu_f=lu_f, t_mg=t1 - t0, t_ml=t2 - t1)


def _dense_lu(A):
    import scipy.linalg as sla
    if A.shape[0] == 0:
        return None
    return sla.lu_factor(A)


def coarse_solve(M: GPLMM, rhs):
    import scipy.linalg as sla
    if M.Ao_lu is None:
        return rhs
    return sla.lu_solve(M.Ao_lu, rhs)


def apply_MG(M: GPLMM, v):
    """z_G = Phat Ao^-1 Rhat v; with mg_form 1 or 2 the f entries then follow from Eq. xf."""
    z = M.P @ coarse_solve(M, M.R @ v)
    if M.mg_form in (1, 2) and M.lu_f is not None:
        F = np.asarray(M.dc.f_faces, dtype=np.int64)
        z[F] = M.lu_f.solve((v - M.X @ z)[F])
    return z


def apply_Md(M: GPLMM, r):
    z = np.zeros_like(r)
    for D, lu in zip(M.dc.D, M.lu_d):
        z[D] += lu.solve(r[D])
    return z


def apply_Mp(M: GPLMM, r):
    z = np.zeros_like(r)
    for S, lu in zip(M.dc.S, M.lu_p):
        z[S] += lu.solve(r[S])
    return z


def apply(M: GPLMM, v):
    """z = M^-1 v: coarse correction, then the dual and primary smoothers."""
    zG = apply_MG(M, v)
    r1 = v - M.X @ zG
    zd = apply_Md(M, r1)
    r2 = r1 - M.X @ zd
    zp = apply_Mp(M, r2)
    return zG + zd + zp
