"""FP64 CPU oracle for Sparse Gauss-Newton (SGN) sensitivity analysis.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package; only ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the
GPU library: it reads the same seeded problem data (``sgn_inputs``) and
nothing else.

What it computes is the plain dense definition the paper's method must
reproduce exactly (Sec. 4, Theorem 1 of Appendix A): the sensitivity matrix
S = -(dc/dx)^-1 dc/dp (Sec. 3.1, eq. dxdp), the adjoint gradient (eq.
totalGradient), the reduced Gauss-Newton Hessian H = S^T A S + B S + S^T B^T
+ C (eq. reducedGN) and the Gauss-Newton step H dp = -(df/dp)^T (eq.
newtonStep), together with the forward Newton equilibrium solve with
monotone backtracking (Sec. 5, "Computing Equilibrium States") and the
symbolic structure (pattern, ordering, elimination tree) of the sparse system
(eq. sparseSystemGN).

Modules:
  fem       -- neo-Hookean linear-simplex element: energy and closed-form
               gradient; Hessians by complex-step differentiation.
  dense     -- global assembly, Newton equilibrium, dense S / GN step, dense
               solve of the saddle-point system, objective and gradient; the
               variants of Sec. 4: block Gauss-Newton step (Appendix B) and
               L-BFGS initialised with the Gauss-Newton Hessian.
  newton    -- the Sparse Newton step with inertia control (Sec. 4, eq. totalHessian;
               Appendix A): second derivatives of lam^T c, the Newton saddle-point matrix,
               the reduced Newton Hessian, the inertia test and diagonal regularisation.
  symbolic  -- K_SGN pattern, nested-dissection order, permuted CSR, etree.
  krylov    -- the stabilised saddle-point matrix and BiCGSTAB of the paper's robust fall-back
               solve (Sec. 5).
  precond   -- dense LDL^T with node-group-restricted Bunch-Kaufman pivoting and
               the node-block preconditioner built from it (the library's
               MINRES path; the paper leaves preconditioning to future work).
"""
