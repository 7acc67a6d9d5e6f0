"""Newton driver for the MAC Navier-Stokes system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Section 1: x^{k+1} = x^k + delta^k with J^k delta^k = -r^k; each linear
system solved by right-preconditioned Krylov iterations with the tolerance
measured against ||r(u=0, p=0)|| (Section 8).  gPLMM is built from the
modified Jacobian J~_w once and reused for every Newton iteration (Section 4);
with no nearby solution the Stokes velocity serves as the wind.

Readings taken where the paper is silent: full Newton steps (the update of
Section 1), with backtracking on the residual norm as an option (see
``solve``); stop when ||r(x_k)|| <= tol * ||r(0)||; the first step uses w = 0 (the Stokes matrix); with ``wind="stokes"`` the preconditioner is rebuilt once with
w = the velocity after the first Newton step (the Stokes solution) and then
kept.
"""
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import gplmm as G
from .krylov import fgmres
from .mac import Phys, residual, jacobian, build_matrix, origin_rhs


@dataclass
class NewtonStats:
    newton_its: int = 0
    lin_its: list = field(default_factory=list)
    res_hist: list = field(default_factory=list)
    step_length: list = field(default_factory=list)
    t_mg: float = 0.0        # M_G builds: closures, shape/correction vectors, coarse operator
    t_ml: float = 0.0        # smoother builds: LU of every primary and dual block
    t_sol: float = 0.0       # Krylov solves (all Newton steps)
    t_hist: list = field(default_factory=list)   # wall seconds from the start to each res_hist entry
    converged: bool = False


def build_precond(ops, dc, phys, wind, build="geometric", mg_form=0):
    """gPLMM from X = J~_w (Section 4), or, with build="jacobian", the algebraic aPLMM
    from the Newton Jacobian at the state w (no tags; w = None gives the Stokes
    matrix, i.e. aPLMM_S)."""
    t = time.perf_counter()
    if build == "jacobian":
        X = jacobian(ops, np.zeros(ops.g.N) if wind is None else wind, phys)
    else:
        X = build_matrix(ops, phys, wind=wind, tags=dc.tags)
    bB = origin_rhs(ops, phys)
    t_asm = time.perf_counter() - t
    M = G.build(X, dc, bB, mg_form=mg_form)
    M.t_mg += t_asm            # assembling X counts with the M_G build
    return M


def solve(ops, dc, phys: Phys, x0=None, x_old=None, tol=1e-8, lin_tol=None,
          maxit=30, restart=30, lin_maxit=600, wind="stokes", wind_vec=None,
          precond="gplmm", stats=None, line_search=False, build="geometric", mg_form=0):
    """Newton-FGMRES with gPLMM.  ``precond``: "gplmm" or "exact" (spsolve).

    ``build``: "geometric" (gPLMM, Section 4) or "jacobian" (aPLMM from the Newton
    Jacobian at the build state: aPLMM_S at w = 0, aPLMM_NS when rebuilt at the first
    iterate with wind="stokes").

    ``line_search``: False (default) takes the full step x + d of Section 1; True
    backtracks on ||r||, lambda = 1, 1/2, ... down to 1/64, the first lambda with
    ||r(x + lambda d)|| <= (1 - 1e-4 lambda) ||r(x)|| (Armijo's sufficient decrease),
    else the smallest."""
    g = ops.g
    st = stats if stats is not None else NewtonStats()
    t_start = time.perf_counter()
    steady0 = Phys(phys.rho, phys.mu, phys.body, phys.dt, phys.pin)
    r0n = np.linalg.norm(residual(ops, np.zeros(g.N), steady0,
                                  x_old=np.zeros(g.N) if phys.dt is not None else None))
    if lin_tol is None:
        lin_tol = 0.1 * tol
    x = np.zeros(g.N) if x0 is None else x0.copy()
    M = None
    if precond == "gplmm":
        w = wind_vec if wind == "caller" else None
        M = build_precond(ops, dc, phys, w, build, mg_form)
        st.t_mg += M.t_mg
        st.t_ml += M.t_ml
    r = residual(ops, x, phys, x_old=x_old)
    st.res_hist.append(np.linalg.norm(r) / r0n)
    st.t_hist.append(time.perf_counter() - t_start)
    for k in range(maxit):
        if np.linalg.norm(r) <= tol * r0n:
            st.converged = True
            break
        if k == 1 and precond == "gplmm" and wind == "stokes":
            M = build_precond(ops, dc, phys, x, build, mg_form)
            st.t_mg += M.t_mg
            st.t_ml += M.t_ml
        J = jacobian(ops, x, phys)
        t = time.perf_counter()
        if precond == "gplmm":
            d, its, ok = fgmres(lambda v: J @ v, -r, lambda v: G.apply(M, v),
                                lin_tol * r0n, m=restart, maxit=lin_maxit)
        else:
            d, its = spla.spsolve(J.tocsc(), -r), 1
        st.t_sol += time.perf_counter() - t
        st.lin_its.append(its)
        st.newton_its += 1
        rn = np.linalg.norm(r)
        lam = 1.0
        while True:
            xt = x + lam * d
            rt = residual(ops, xt, phys, x_old=x_old)
            if not line_search or np.linalg.norm(rt) <= (1.0 - 1e-4 * lam) * rn or lam <= 1.0 / 64.0:
                break
            lam *= 0.5
        st.step_length.append(lam)
        x, r = xt, rt
        st.res_hist.append(np.linalg.norm(r) / r0n)
        st.t_hist.append(time.perf_counter() - t_start)
    else:
        st.converged = np.linalg.norm(r) <= tol * r0n
    return x, st
