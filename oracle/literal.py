"""gPLMM written with the paper's explicit dense matrices (tiny grids only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is a second, independent transcription of Section 3.2.2 and 3.2.3 used to
pin the sparse implementation in ``gplmm``: every operator is formed as a
dense matrix exactly as the paper writes it,

* the permutation W with A = W^T A_hat W in [p, c, f] block order;
* reduction 1: A~^p_p = A^p_p + diag(csum(A^p_f)), A~^c_c likewise, f columns
  dropped;
* reduction 2: Abar^{p_i}_{p_i} = A~^{p_i}_{p_i} + diag(sum_{j != i}
  csum(A~^{p_i}_{p_j})), off-diagonal primary blocks dropped;
* both column sums skip the rows of faces in wall-free groups (this
  project's reading, see ``decomp``), which keeps every Abar^{p_i}_{p_i}
  regular;
* the reduction matrix Q = blkdiag(I, Q^o) and A_M = Q^T Abar Q;
* prolongation P = [B C; I O] with shape vectors
  -(Abar^{p_i}_{p_i})^-1 R^{p_i}_p Abar^p_c e^{c_j} and correction vectors
  (Abar^{p_i}_{p_i})^-1 b_B^{p_i};
* restriction R = [O I; Pi(C^T) O], with Pi(C^T) the structural pattern of
  C^T (every row of the primary's block, including rows where a correction
  vector happens to vanish, such as the pinned cell);
* Phat = W Q P (zero rows for the f unknowns), Rhat = R Q^T W^T, and the
  Remark-1 form M_G^-1 = Phat (Rhat A_hat Phat)^-1 Rhat;
* M_p, M_d with 0/1 restriction/extension matrices, M_dp, and the two-level
  M^-1 = M_G^-1 + M_dp^-1 (I - A_hat M_G^-1).
"""
import numpy as np


def csum(B):
    """Sum of all columns of B: one column vector."""
    return B.sum(axis=1) if B.shape[1] else np.zeros(B.shape[0])


def literal_preconditioner(Ahat, dc, bB, mg_form=0):
    """Dense M^-1 (N x N) and M_G^-1 built literally from the paper's matrices.

    mg_form 0: the Remark-1 form Phat (Rhat A_hat Phat)^-1 Rhat.  mg_form 1: Eq. iMG,
    Phat (Rhat Acheck Phat)^-1 Rhat with Acheck = W C(W^T A_hat W) W^T, where C(.) is
    the two reductions (so Rhat Acheck Phat = R Q^T Abar Q P), followed by Eq. xf for
    the f unknowns: x^f = (A^f_f)^-1 (b^f - A^f_p x^p - A^f_c x^c).  mg_form 2: the
    Remark-1 form followed by the same Eq. xf."""
    Ahat = np.asarray(Ahat, dtype=float)
    g = dc.g
    N = g.N
    # --- permutation: p unknowns primary by primary, then c (interface cells), then f
    p_blocks = [np.asarray(S) for S in dc.S]
    c_blocks = [np.asarray(c) for c in dc.icells]
    f_idx = np.asarray(dc.f_faces)
    order = np.concatenate(p_blocks + c_blocks + [f_idx]).astype(np.int64)
    assert np.array_equal(np.sort(order), np.arange(N)), "p, c, f must partition the unknowns"
    W = np.zeros((N, N))
    W[order, np.arange(N)] = 1.0
    A = W.T @ Ahat @ W
    npf = sum(b.size for b in p_blocks)
    ncf = sum(b.size for b in c_blocks)
    P_, C_, F_ = slice(0, npf), slice(npf, npf + ncf), slice(npf + ncf, N)
    # rows of faces in wall-free groups take no column sums (see decomp)
    perm_free = np.zeros(N, dtype=bool)
    vel = order < g.nu
    perm_free[vel] = dc.free[order[vel]]
    keep = (~perm_free).astype(float)
    # --- reduction 1
    Atil = A[:npf + ncf, :npf + ncf].copy()
    Atil[P_, P_] += np.diag(keep[P_] * csum(A[P_, F_]))
    Atil[C_, C_] += np.diag(csum(A[C_, F_]))
    # --- reduction 2: block-diagonalise the primary block
    offs = np.cumsum([0] + [b.size for b in p_blocks])
    Abar = Atil.copy()
    for i in range(dc.Np):
        ri = slice(offs[i], offs[i + 1])
        extra = np.zeros(offs[i + 1] - offs[i])
        for j in range(dc.Np):
            if j == i:
                continue
            rj = slice(offs[j], offs[j + 1])
            extra += csum(Atil[ri, rj])
            Abar[ri, rj] = 0.0
        Abar[ri, ri] += np.diag(keep[ri] * extra)
    # --- reduction matrix Q
    Nc = dc.Nc
    Qo = np.zeros((ncf, Nc))
    co = np.cumsum([0] + [b.size for b in c_blocks])
    for j in range(Nc):
        Qo[co[j]:co[j + 1], j] = 1.0
    Q = np.zeros((npf + ncf, npf + Nc))
    Q[:npf, :npf] = np.eye(npf)
    Q[npf:, npf:] = Qo
    AM = Q.T @ Abar @ Q
    # --- prolongation
    Abar_pc = AM[:npf, npf:]
    bperm = (W.T @ bB)[:npf]
    B = np.zeros((npf, Nc))
    Ccols = []
    Cpat = []
    for i in range(dc.Np):
        ri = slice(offs[i], offs[i + 1])
        Rp = np.zeros((offs[i + 1] - offs[i], npf))
        Rp[:, ri] = np.eye(offs[i + 1] - offs[i])
        Aii = AM[ri, ri]
        for j in range(Nc):
            e = np.zeros(Nc)
            e[j] = 1.0
            B[ri, j] = -np.linalg.solve(Aii, Rp @ Abar_pc @ e)
        bi = Rp @ bperm
        if np.any(bi != 0):
            col = np.zeros(npf)
            col[ri] = np.linalg.solve(Aii, bi)
            Ccols.append(col)
            pat = np.zeros(npf)
            pat[ri] = 1.0          # structural pattern: the whole block of primary i
            Cpat.append(pat)
    Cm = np.stack(Ccols, 1) if Ccols else np.zeros((npf, 0))
    ny = Cm.shape[1]
    P = np.zeros((npf + Nc, Nc + ny))
    P[:npf, :Nc] = B
    P[:npf, Nc:] = Cm
    P[npf:, :Nc] = np.eye(Nc)
    # --- restriction
    R = np.zeros((Nc + ny, npf + Nc))
    R[:Nc, npf:] = np.eye(Nc)
    R[Nc:, :npf] = np.stack(Cpat, 0) if Cpat else np.zeros((0, npf))
    # --- effective operators (f rows of Phat and f columns of Rhat are zero)
    QP = np.zeros((N, Nc + ny))
    QP[:npf + ncf] = Q @ P
    Phat = W @ QP
    RQ = np.zeros((Nc + ny, N))
    RQ[:, :npf + ncf] = R @ Q.T
    Rhat = RQ @ W.T
    if mg_form in (1, 2):
        if mg_form == 1:
            MG = Phat @ np.linalg.solve(R @ AM @ P, Rhat)
        else:
            MG = Phat @ np.linalg.solve(Rhat @ Ahat @ Phat, Rhat)
        if F_.stop > F_.start:
            # x^f from Eq. xf, in the original order: z_f = A_ff^-1 (b - A_hat z)_f
            Ef = W[:, F_]
            Aff = A[F_, F_]
            Sf = Ef @ np.linalg.solve(Aff, Ef.T)
            MG = (np.eye(N) - Sf @ Ahat) @ MG + Sf
    else:
        MG = Phat @ np.linalg.solve(Rhat @ Ahat @ Phat, Rhat)
    # --- additive Schwarz smoothers
    def schwarz(sets):
        out = np.zeros((N, N))
        for S in sets:
            E = np.zeros((N, S.size))
            E[S, np.arange(S.size)] = 1.0
            out += E @ np.linalg.solve(E.T @ Ahat @ E, E.T)
        return out
    Mp = schwarz(dc.S)
    Md = schwarz(dc.D)
    I = np.eye(N)
    Mdp = Md + Mp @ (I - Ahat @ Md)
    M = MG + Mdp @ (I - Ahat @ MG)
    return M, MG
