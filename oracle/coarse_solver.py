"""Coarse-scale Navier-Stokes solver: Newton iterations on the coarse unknowns only.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Section 5 (Eqs. approx_formula, coarse_scale_sys, coarse_rJ and
coarse_scale_up; Algorithm 1; Remark 2).  For the steady equations the global
preconditioner of gPLMM serves as a solver on its own:

* an outer loop raises the driving force in equal increments (the paper raises
  the inlet pressure; here the body force, which drives these problems); at each
  increment the wind w is the velocity of the previous increment (zero at the
  first, i.e. the Stokes matrix), and Phat, Rhat are built from X = J~_w with the
  tagged faces free of inertia (Section 4);
* an inner Newton iteration on the coarse unknowns solves
  J_c^k delta_c^k = -r_c^k with r_c^k = Rhat r~(x^k) and J_c^k = Rhat J~^k Phat,
  where r~ is the residual with the inertia removed on tagged faces and J~^k its
  Jacobian at x^k (the wind equal to the state itself), and updates
  x^{k+1} = x^k + Phat delta_c^k;
* an increment ends when ||r_c^{k+1}|| < tol ||r_c^0|| (tol = 1e-6 in the
  paper).

For the Stokes equations (``stokes=True``: no inertia) one Newton step gives
x = Phat (Rhat A Phat)^-1 Rhat b, the Remark-1 form of M_G^-1 applied to b
(Remark 2).
"""
from dataclasses import dataclass, field

import numpy as np

from . import gplmm as G
from .mac import Phys, residual, jacobian, build_matrix, origin_rhs


@dataclass
class CoarseStats:
    newton_its: list = field(default_factory=list)   # coarse Newton iterations per increment
    rc_rel: list = field(default_factory=list)       # final ||r_c|| / ||r_c^0|| per increment
    converged: bool = False


def solve(ops, dc, phys: Phys, increments=1, tol=1e-6, kmax=50, stokes=False, stats=None):
    """Algorithm 1 with ``increments`` equal steps of the body force up to phys.body.
    Returns (x, stats, M) with M the preconditioner of the last increment."""
    g = ops.g
    st = stats if stats is not None else CoarseStats()
    x = np.zeros(g.N)
    wind = None
    M = None
    st.converged = True
    for m in range(1, increments + 1):
        f = m / increments
        ph = Phys(phys.rho, phys.mu, tuple(f * b for b in phys.body), None, phys.pin)
        X = build_matrix(ops, ph, wind=wind, tags=dc.tags)
        M = G.build(X, dc, origin_rhs(ops, ph))
        P, R = M.P, M.R

        def coarse_residual(xx):
            return R @ residual(ops, xx, ph, tags=dc.tags, inertia=not stokes)

        rc = coarse_residual(x)
        rc0 = np.linalg.norm(rc)
        its, rel = 0, 0.0
        for k in range(kmax):
            J = X if stokes else jacobian(ops, x, ph, tags=dc.tags)
            Jc = (R @ J @ P).toarray()
            delta = np.linalg.solve(Jc, -rc)
            x = x + P @ delta
            rc = coarse_residual(x)
            its += 1
            rel = np.linalg.norm(rc) / rc0 if rc0 > 0 else 0.0
            if rel < tol:
                break
        st.newton_its.append(its)
        st.rc_rel.append(rel)
        st.converged = st.converged and rel < tol
        wind = None if stokes else x.copy()
    return x, st, M


def cell_speed(g, x):
    """Velocity magnitude at the fluid cells: each component the mean of the cell's two
    faces on its axis (inactive faces count zero)."""
    comp = []
    for c in g.comps:
        u = np.zeros(g.fluid.shape)
        u[g.act[c]] = x[g.comp_slice(c)]
        upper = g.shift(u, c, +1, 0.0)
        comp.append(0.5 * (u + upper)[g.fluid])
    return np.sqrt(sum(a * a for a in comp))


def paper_errors(g, x_c, x_t):
    """E_2 of Section 7 (Eq. error_L2): root mean square over the fluid cells of the
    pointwise error |xi_t - xi_c| / sup |xi_t|, in percent, for xi = pressure (both
    mean-free, the gauge of these problems being arbitrary) and velocity magnitude."""
    sc, st_ = cell_speed(g, x_c), cell_speed(g, x_t)
    pc = x_c[g.p_slice] - x_c[g.p_slice].mean()
    pt = x_t[g.p_slice] - x_t[g.p_slice].mean()
    e_u = 100.0 * np.sqrt(np.mean(((st_ - sc) / np.max(np.abs(st_))) ** 2))
    e_p = 100.0 * np.sqrt(np.mean(((pt - pc) / np.max(np.abs(pt))) ** 2))
    return e_p, e_u
