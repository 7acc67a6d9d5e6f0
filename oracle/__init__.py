"""Plain FP64 CPU oracle for the gPLMM-preconditioned Newton-Krylov solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library.

It follows Li & Mehmani, "Preconditioning and Reduced-Order Modeling of
Navier-Stokes Equations in Complex Porous Microstructures":

* ``mac``     -- MAC residual r(x), Newton Jacobian J (Section 2, the system
                 J delta = -r) and the gPLMM build matrix X = J~_w
                 (Section 4, the modified residual with wind w and no inertia
                 on tagged faces).
* ``decomp``  -- primary grids, contact interfaces, the p/c/f partition and
                 dual grids (Section 3.2.1 and the permutation paragraph of
                 Section 3.2.2).
* ``gplmm``   -- global preconditioner M_G (reduction, prolongation,
                 restriction, Remark 1) and the dual-primary smoother
                 (Section 3.1 two-level structure; Section 3.2.3).
* ``literal`` -- the same preconditioner written with the paper's explicit
                 matrices W, Q, P, R and csum, dense, for tiny grids only.
* ``krylov``  -- flexible GMRES with right preconditioning (Section 8
                 stopping rule), plus textbook GMRES.
* ``newton``  -- the Newton driver.
* ``mlp``     -- FP64 reference of the coarse-coefficient MLP.

Everything is float64 and uses numpy / scipy only.
"""
