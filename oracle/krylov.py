"""Flexible GMRES (right preconditioning) and textbook GMRES.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves each Newton system with right-preconditioned GMRES and stops
when ||A x - b|| / ||r(u=0, p=0)|| < 1e-9 (Section 8, first paragraph).  The
restart length is not given; FGMRES(m) with m = 30 is used here, with
classical Gram-Schmidt applied twice and Givens rotations on the Hessenberg
matrix (Saad's flexible variant: the preconditioned vectors z_j are kept, so
the preconditioner may change between applications).
"""
import numpy as np


def fgmres(matvec, b, precond, tol_abs, m=30, maxit=1000, x0=None, history=None):
    """Solve A x = b.  Stops when the (recurrence) residual norm <= tol_abs.

    Returns (x, iterations, converged).  ``history`` (a list) receives the
    residual-norm estimate after every inner iteration, starting with ||r0||.
    """
    n = b.size
    x = np.zeros(n) if x0 is None else x0.copy()
    total = 0
    r = b - matvec(x) if x0 is not None else b.copy()
    beta = np.linalg.norm(r)
    if history is not None:
        history.append(beta)
    if beta <= tol_abs:
        return x, 0, True
    while total < maxit:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gv = np.zeros(m + 1)
        gv[0] = beta
        V[0] = r / beta
        k = 0
        done = False
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            total += 1
            k = j + 1
            if history is not None:
                history.append(abs(gv[j + 1]))
            if abs(gv[j + 1]) <= tol_abs or hn == 0 or total >= maxit:
                done = abs(gv[j + 1]) <= tol_abs or hn == 0
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (gv[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        if done:
            return x, total, True
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= tol_abs:
            return x, total, True
    return x, total, False


def gmres_right_history(A, Minv, b, m):
    """Textbook right-preconditioned GMRES on dense A and Minv without
    restart: at step k the iterate minimises ||b - A Minv y|| over the Krylov
    space K_k(A Minv, b); returns the k = 0..m residual norms, computed by a
    least-squares solve at every step (no Givens, no recurrence)."""
    B = A @ Minv
    n = b.size
    V = np.zeros((n, m + 1))
    V[:, 0] = b / np.linalg.norm(b)
    out = [np.linalg.norm(b)]
    H = np.zeros((m + 1, m))
    for k in range(m):
        w = B @ V[:, k]
        for i in range(k + 1):          # modified Gram-Schmidt, twice
            H[i, k] = V[:, i] @ w
            w = w - H[i, k] * V[:, i]
        for i in range(k + 1):
            c = V[:, i] @ w
            H[i, k] += c
            w = w - c * V[:, i]
        H[k + 1, k] = np.linalg.norm(w)
        V[:, k + 1] = w / H[k + 1, k] if H[k + 1, k] > 0 else 0.0
        e1 = np.zeros(k + 2)
        e1[0] = out[0]
        y = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)[0]
        out.append(np.linalg.norm(b - B @ (V[:, :k + 1] @ y)))
    return np.array(out)
