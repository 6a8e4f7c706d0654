/*
 * sgn.h -- C ABI of libsgn, the MI355X (gfx950) hot path of Sparse
 * Gauss-Newton sensitivity analysis (Zehnder, Coros, Thomaszewski,
 * "Sparse Gauss-Newton for Accelerated Sensitivity Analysis", ACM TOG 2021).
 *
 * Problem (Sec. 3, eq. optProb): min_{x,p} f(x, p) s.t. c(x, p) = 0 with
 * n_c = n_x and dc/dx of full rank.  Here c is static force balance of a
 * linear-simplex neo-Hookean mesh, c = dPi/dx, Pi = sum_e E_e(x, p) - f_ext^T x,
 * and f is the least-squares objective of eq. leastSquaresObjective plus a
 * Tikhonov term:  f = w/2 sum_{i in T} ((x_i - t_i)/ell)^2 + mu/2 |p - p_ref|^2,
 * so A = (w/ell^2) I_T, B = 0, C = mu I in eq. reducedGN.
 *
 * Each Gauss-Newton iteration solves the sparse symmetric indefinite system
 * of eq. sparseSystemGN,
 *     [ A  B^T  Kx^T ] [dx  ]   [  0 ]
 *     [ B  C    Kp^T ] [dp  ] = [ -g ]      Kx = dc/dx, Kp = dc/dp,
 *     [ Kx Kp   0    ] [dlam]   [  0 ]      g = df/dp^T + Kp^T lam_adj,
 * whose dp equals the dense Gauss-Newton step H dp = -g exactly (Sec. 4,
 * Appendix A Theorem 1).  x(p) comes from a forward Newton solve with
 * monotone backtracking (Sec. 5, "Computing Equilibrium States").
 *
 * Conventions
 *  - Ownership: the library never allocates device memory.  sgn_create does
 *    host work only (it copies the problem and runs the symbolic analysis);
 *    the caller allocates sgn_workspace_size() bytes of device memory and
 *    hands it over with sgn_set_workspace(), which uploads the symbolic
 *    tables.  Every other device buffer is caller-owned and must stay valid
 *    until the call returns (calls that fill an *_info struct or a host
 *    scalar synchronise the context's stream before returning).
 *  - Pointers named d_* are device pointers, h_* host pointers.
 *  - Layouts at the boundary are FP64 whatever the internal precision:
 *      x    [n_x]  free nodes in ascending node id, dim components each;
 *      p    [n_p]  log-modulus: element order; rest positions / nodal
 *                  forces: same layout as x;
 *      sol  [N]    N = 2 n_x + n_p, block order [dx; dp; dlam] (eq.
 *                  sparseSystemGN).
 *  - Errors: every call returns an sgn_status; nothing is thrown across the
 *    ABI and nothing aborts.  A non-OK status is sticky on the context
 *    (later calls return SGN_E_STATE) and sgn_last_error() gives a message.
 *    HIP runtime failures map to SGN_E_HIP.
 *  - Streams: all device work of a context runs on the stream given at
 *    create (a hipStream_t passed as void*; NULL = the null stream).  One
 *    context per stream; distinct contexts are independent.
 */
#ifndef SGN_H
#define SGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgn_ctx_s* sgn_ctx;

typedef enum {
  SGN_OK = 0,
  SGN_E_ARG = 1,        /* invalid argument or problem data */
  SGN_E_STATE = 2,      /* call out of order, or an earlier error is pending */
  SGN_E_NOMEM = 3,      /* host allocation failed, or workspace too small */
  SGN_E_HIP = 4,        /* a HIP runtime call failed */
  SGN_E_NEWTON = 5,     /* equilibrium did not converge in max_newton steps */
  SGN_E_INVERTED = 6,   /* the given state has an inverted element (J <= 0) */
  SGN_E_PIVOT = 7,      /* factorisation met a zero pivot or wrong inertia */
  SGN_E_REFINE = 8,     /* refinement did not reach solve_rtol in max_ir sweeps */
  SGN_E_LINESEARCH = 9  /* outer line search failed after max_halvings */
} sgn_status;

/* parameter kinds */
enum { SGN_P_LOGE = 0, SGN_P_REST_POS = 1, SGN_P_NODAL_FORCE = 2 };
/* internal factor precision of the saddle-point system */
enum { SGN_FP64 = 0, SGN_FP32_IR = 1 };
/* linear solver of the saddle-point system: refined LDL^T; MINRES with the learned preconditioner;
 * BiCGSTAB on K preconditioned by the LDL^T of the stabilised matrix K + diag(eps_x 1, 0, -eps_lambda 1)
 * (Sec. 5, "Solving the saddle point problem"; set eps_x, eps_lambda, e.g. 1e-6 as there); the
 * block solve of Sec. 4 ("Block Solve", Appendix B), which needs no factorisation of K_SGN
 * (see sgn_block_step for its conditions) */
enum { SGN_LDLT = 0, SGN_MINRES_LEARNED = 1, SGN_BICGSTAB = 2, SGN_BLOCK_GN = 3 };
/* right-hand side of the step: [0; -g; 0] (eq. sparseSystemGN) or the KKT
 * form [-df/dx^T; -df/dp^T; 0] (Appendix A), which gives the same dp and a
 * multiplier block shifted by the adjoint multiplier */
enum { SGN_RHS_ADJOINT = 0, SGN_RHS_KKT = 1 };
/* second derivatives in the saddle-point matrix: the Gauss-Newton blocks A = d2f/dx2, B = d2f/dp dx,
 * C = d2f/dp2 (eq. sparseSystemGN; for the least-squares objective with a Tikhonov term this is also
 * the generalised Gauss-Newton form of Sec. 4), or the Newton form of Appendix A: the Hessian of the
 * Lagrangian f + lam^T c at the adjoint multipliers, whose saddle-point solve is the full Newton step
 * (Sec. 4, eq. totalHessian); log-modulus parameters only, one problem, solver SGN_LDLT, rhs_kind
 * SGN_RHS_ADJOINT, eps_x = eps_lambda = 0 (SGN_E_ARG otherwise) */
enum { SGN_HESSIAN_GN = 0, SGN_HESSIAN_NEWTON = 1 };
/* preconditioner of sgn_solve_minres: the node-block preconditioner built on the reference factor
 * (below), or the block-diagonal ablation without a reference factor, M^-1 = S blockdiag_i(|B_i|^-1) S
 * with B_i the diagonal block of S K S over node group i (eigen-absolute value, no corrections) */
enum { SGN_PC_FACTOR = 0, SGN_PC_BLOCK = 1 };
/* which system sgn_get_symbolic / sgn_get_sizes describe */
enum { SGN_SYS_SGN = 0, SGN_SYS_KX = 1 };

/* Problem data (host pointers; copied by sgn_create, caller keeps ownership). */
typedef struct {
  int dim;                      /* 2 (plane strain, unit thickness) or 3 */
  int n_nodes, n_elems;
  const double* rest_pos;       /* [n_nodes*dim] */
  const int32_t* elems;         /* [n_elems*(dim+1)] positively oriented simplices */
  const int32_t* node_grid;     /* [n_nodes*dim] integer grid coordinates (ordering) */
  const uint8_t* fixed;         /* [n_nodes] 1 = Dirichlet on all components */
  const double* f_ext;          /* [n_nodes*dim] dead nodal loads */
  double E0, nu;                /* neo-Hookean: E_e = E0 exp(p_e) for SGN_P_LOGE */
  int param_kind;               /* SGN_P_* */
  int n_targets;
  const int32_t* target_dof;    /* [n_targets] indices into x */
  const double* target_val;     /* [n_targets] (may be NULL until sgn_set_targets) */
  double target_w, length_scale, reg_mu;
  const double* p_ref;          /* [n_p] Tikhonov reference */
  /* Batches of independent problems: n_components > 1 declares the mesh a
   * disjoint union whose component c owns the nodes [component_ptr[c],
   * component_ptr[c+1]) (and only elements among them); node_grid then holds
   * each component's own grid coordinates.  Every component is ordered on its
   * own, so the elimination tree is a forest and each level of the supernodal
   * schedule covers the same level of all components.  0 or 1: one problem. */
  int n_components;
  const int32_t* component_ptr; /* [n_components+1], 0 first, n_nodes last */
} sgn_problem;

typedef struct {
  int precision;                /* SGN_FP64 | SGN_FP32_IR */
  int solver;                   /* SGN_LDLT | SGN_MINRES_LEARNED */
  int rhs_kind;                 /* SGN_RHS_ADJOINT | SGN_RHS_KKT */
  double newton_rtol;           /* |c|_2 <= newton_rtol |f_ext|_2 (+ newton_atol) */
  double newton_atol;
  double solve_rtol;            /* equilibrated residual |S(b - K z)|_2 / |S b|_2 */
  double eps_x, eps_lambda;     /* optional diagonal stabilisation (Sec. 5), default 0 */
  int max_newton, max_ir, max_minres, max_halvings;
  int profile;                  /* 1: time every trailing-update launch with HIP events */
  int max_gmres;                /* restart cycles of the FGMRES(30) escalation of the saddle-point
                                   solves' refinement, 0: none */
  /* Blocking of the factorisation and solve schedules (no effect on the mathematics; chosen per
   * problem family by sgn_autotune, 0 = library default).  Fronts fall in buckets by their order
   * m: m < 1024, 1024 <= m < 4096, m >= 4096. */
  int outer_panels[3];          /* per bucket: trailing update beyond a block of this many 64-column
                                   panels is delayed to the block's end (1..16, default 4) */
  int seq_panels;               /* fronts with at most this many panels are solved by one
                                   workgroup instead of a pipeline of workgroups (-1: none, 0:
                                   default 8, else 1..8) */
  int max_bicgstab;             /* BiCGSTAB iterations of the SGN_BICGSTAB solver (default 50) */
  int lbfgs_m;                  /* curvature pairs kept by sgn_lbfgs_step (default 5, 0..32) */
  int hessian;                  /* SGN_HESSIAN_GN (default) | SGN_HESSIAN_NEWTON, fixed at create
                                   (the Newton form has a larger pattern) */
  int pc_kind;                  /* SGN_PC_FACTOR (default) | SGN_PC_BLOCK, fixed at create */
  int panel_waves;              /* wavefronts per panel's diagonal-block factorisation (no effect on
                                   the results): 1, 2, 4, 8, or 0 = by the launch (panels of at most
                                   32 columns: one when a step has at least 1024 of them; of at most
                                   48 columns: four in a 48-row block from 512 of them; otherwise four
                                   from 512 panels, else eight) */
} sgn_options;

typedef struct { int iters; int halvings; double res_norm; double f_ext_norm; int converged; } sgn_eq_info;
typedef struct {
  int64_t n_pos, n_neg, n_zero; /* inertia counted from D */
  int64_t n_perturbed;          /* tiny pivots replaced */
  double min_abs_pivot;
  double flops;                 /* dense front work executed */
  double ms;                    /* wall time of the call */
} sgn_factor_info;
typedef struct {
  int sweeps;                   /* refinement sweeps or MINRES iterations */
  int fallback;                 /* MINRES fell back to the exact LDL^T */
  double rel_res;               /* equilibrated relative residual (solve_rtol measure) */
  double raw_rel_res;           /* |b - K z|_2 / |b|_2 on the unscaled matrix */
  double ms;
  int gmres_iters;              /* Arnoldi steps of the FGMRES escalation (0: refinement sufficed) */
} sgn_solve_info;
typedef struct {
  double alpha, f0, f1, grad_norm, gtdp;
  int halvings, newton_iters;
  double ms_rhs, ms_assemble, ms_factor, ms_solve, ms_linesearch;
  sgn_solve_info solve;
  double delta;                 /* sgn_newton_step: diagonal regularisation of the accepted factor */
  int inertia_trials;           /* sgn_newton_step: factorisations the inertia test took */
} sgn_step_info;

/* Stage measurements of the last calls (HIP events on the context's stream). */
typedef struct {
  double assemble_ms;           /* element kernel + gathers of the last sgn_assemble */
  double assemble_bytes;        /* algorithmic bytes: x, p, mesh in; K_SGN values out */
  double factor_ms;             /* last sgn_factor: scaling, front assembly, factorisation */
  double factor_flops;          /* dense front flops, sum s^3/3 + s^2 u + s u^2 */
  double update_ms;             /* sum of MFMA trailing-update launch durations (profile = 1) */
  double update_flops;          /* algorithmic flops of those launches, 2 k per updated entry */
  int64_t update_launches;
  double solve_ms;              /* last sgn_solve including refinement */
} sgn_stats;

/* Validate the problem, copy it, run the host symbolic analysis of both the
 * saddle-point system and the Kx system (nested-dissection order, permuted
 * lower CSR, elimination tree, supernodes, slot maps).  No device work. */
sgn_status sgn_create(const sgn_problem* prob, const sgn_options* opt, void* stream, sgn_ctx* out);
/* Fill *opt with the defaults. */
void sgn_default_options(sgn_options* opt);
/* Device bytes the context needs (fronts, CSR values, element buffers, vectors). */
sgn_status sgn_workspace_size(sgn_ctx ctx, size_t* bytes);
/* Hand over caller-owned device memory (256-byte aligned, >= workspace size)
 * and upload the symbolic tables.  Synchronises the stream. */
sgn_status sgn_set_workspace(sgn_ctx ctx, void* d_ws, size_t bytes);
/* Replace target values and the frozen length scale ell (host arrays). */
sgn_status sgn_set_targets(sgn_ctx ctx, const double* h_target_val, double length_scale);
/* Forward simulation x(p): Newton on c(x, p) = 0 with backtracking on Pi and
 * an inversion guard (Sec. 5).  d_x is the initial guess on entry and x(p) on
 * exit.  Leaves a factorisation of Kx(x(p)) for the adjoint right-hand side. */
sgn_status sgn_equilibrium(sgn_ctx ctx, const double* d_p, double* d_x, sgn_eq_info* info);
/* Assemble K_SGN (eq. sparseSystemGN) at (x, p) from per-element blocks and,
 * when d_rhs != NULL, the right-hand side [N] in block order (adjoint form:
 * g from one solve with the Kx factor, eq. totalGradient; KKT form: no solve).
 * d_grad [n_p] (optional) receives g (adjoint form only); h_obj (optional)
 * receives f(x, p).  (x, p) must be an equilibrium for the adjoint form. */
sgn_status sgn_assemble(sgn_ctx ctx, const double* d_x, const double* d_p,
                        double* d_rhs, double* d_grad, double* h_obj);
/* Supernodal LDL^T of the assembled K_SGN (Bunch-Kaufman pivots restricted
 * to each mesh node's variable group).  Checks the inertia (n_x+n_p, n_x, 0).
 * Part of the trailing updates runs on a second stream that the context creates
 * (default priority) and owns; it is forked from and joined back into the
 * context's stream with events, so the caller sees only its own stream's order. */
sgn_status sgn_factor(sgn_ctx ctx, sgn_factor_info* info);
/* Solve K_SGN sol = rhs with the current factor plus FP64 iterative
 * refinement to solve_rtol (both device arrays, [N], block order).  When a
 * refinement sweep shrinks the equilibrated residual by less than half, or
 * max_ir sweeps did not reach solve_rtol, the solve continues with restarted
 * flexible GMRES(30) in FP64 on the equilibrated system, right-preconditioned
 * by the factor (at most max_gmres cycles).  SGN_E_REFINE if solve_rtol is
 * still not met. */
sgn_status sgn_solve(sgn_ctx ctx, const double* d_rhs, double* d_sol, sgn_solve_info* info);
/* For callers that cannot allocate device memory when they solve (work under stream capture,
 * tight serving loops, harnesses that forbid allocation): sgn_solve with every per-call working
 * buffer (scaled and permuted vectors, per-front solve vectors, split-k partials, pipelined-solve
 * tickets, refinement vectors, reduction partials, counters) in a static device array of the
 * library, 128 MiB per device, held from the first call on a device until the process ends.  The
 * factor, the assembled matrix and the symbolic tables stay in the context's workspace; d_rhs and
 * d_sol as in sgn_solve.  Call it with the context's device current.  Plain refinement only (no
 * FGMRES escalation): SGN_E_REFINE if max_ir sweeps do not reach solve_rtol.  SGN_E_NOMEM (with the
 * bytes needed in the message) when the system's working memory exceeds the array; SGN_E_HIP if
 * the array's address cannot be obtained.  No device memory is allocated or freed.  Every call on
 * one device shares that device's array: calls that overlap on one device (any contexts, any
 * streams) race and must be serialised by the caller. */
sgn_status sgn_solve_static(sgn_ctx ctx, const double* d_rhs, double* d_sol, sgn_solve_info* info);
/* One iteration of L-BFGS whose initial inverse Hessian is the Gauss-Newton one of the current
 * iterate (Sec. 4, "Combination with L-BFGS"): at the equilibrium (d_p, d_x) the adjoint gradient g
 * (eq. totalGradient) and K_SGN are assembled and factorised; the pair (s, y) = (p - p_prev,
 * g - g_prev) of the previous call enters the memory of the newest lbfgs_m pairs when
 * s^T y > 1e-12 |s| |y|; the two-loop recursion gives d = -H g with H0 q = H_GN^-1 q taken from one
 * saddle-point solve with right-hand side [0; q; 0]; then the Armijo backtracking of sgn_step along
 * d.  With no pairs (first call, restart != 0, or lbfgs_m = 0) d is the Gauss-Newton step.  The
 * memory lives in the workspace and persists across calls; restart != 0 clears it.  Needs solver
 * SGN_LDLT or SGN_BICGSTAB (SGN_E_STATE otherwise).  info as for sgn_step (grad_norm = |g|). */
sgn_status sgn_lbfgs_step(sgn_ctx ctx, double* d_p, double* d_x, int restart, sgn_step_info* info);
/* A batch of n independent problems (the batched form; each problem is the problem statement of
 * Sec. 3 on its own mesh) as one context: sgn_create of their disjoint union with n_components = n,
 * each problem's nodes, elements, free DOFs, parameters and targets stored in order, problem by
 * problem.  The problems must share dim, param_kind, E0, nu, target_w and reg_mu (SGN_E_ARG
 * otherwise, *out = NULL); the batch takes the largest length_scale of its problems, so each
 * problem's step is its Gauss-Newton step at that ell.  probs[i]->n_components must be 0 or 1;
 * NULL target_val / p_ref read as zeros.  Every other call works on the union (x, p, sol of length
 * n_x, n_p, N of the union, problems in order). */
sgn_status sgn_batch_create(int n, const sgn_problem* const* probs, const sgn_options* opt, void* stream,
                            sgn_ctx* out);
/* One outer iteration for every problem of a batch: d_p[k], d_x[k] (device, problem k's own layout,
 * an equilibrium on entry) are gathered into the union, the search directions of all problems come
 * from one assembly, factorisation and solve of the union (the union's K_SGN is block diagonal over
 * the problems, so each block of the solution is that problem's step), and each problem then takes
 * its own Armijo backtracking along its direction, f_k(alpha_k) <= f_k(0) + 1e-4 alpha_k g_k^T dp_k,
 * with the trials of all problems still searching solved together in one union equilibrium per
 * round (problems already accepted keep their state).  On success every d_p[k], d_x[k] is updated
 * in place.  info: NULL or an array of n entries (per-problem alpha, f0, f1, gtdp, halvings; shared
 * timings and solve info).  A problem stationary to working precision stays (alpha = 0, as sgn_step);
 * SGN_E_LINESEARCH if a problem finds no step (then nothing is written back).  Needs solver SGN_LDLT
 * or SGN_BICGSTAB and, for contexts not made by sgn_batch_create, log-modulus parameters stored
 * problem by problem (SGN_E_STATE otherwise). */
sgn_status sgn_batch_step(sgn_ctx ctx, double* const* d_p, double* const* d_x, sgn_step_info* info);
/* Block Gauss-Newton direction (Sec. 4 "Block Solve", Appendix B) at the equilibrium (d_x, d_p) into
 * d_sol ([N], block order [dx; dp; dlam]).  Only for contexts created with solver = SGN_BLOCK_GN, which
 * sgn_create accepts for rest-position parameters (Kp square), reg_mu = 0 (C = 0; B = 0 always) and
 * every free DOF a target exactly once (A = (w/ell^2) I invertible).  Then eq. sparseSystemGN reduces
 * by block substitution to dx = -A^-1 df/dx^T, Kp dp = -Kx dx (the appendix's sign) and, for the
 * adjoint right-hand side, dlam = Kx^-1 df/dx^T (the KKT form's multiplier block is 0): the same
 * step as the full solve when Kp is invertible.  K_SGN is assembled at (d_x, d_p) but never
 * factorised; Kp dp = -Kx dx is solved by restarted GMRES(30) (at most max_gmres cycles, at least
 * one) to a relative residual of min(1e-12, solve_rtol / 100), right-preconditioned by -Kx^-1 through
 * the Kx factor (the one sgn_equilibrium left, else a fresh one at this state).  info: sweeps and
 * gmres_iters = GMRES iterations, rel_res = raw_rel_res = final relative residual of the Kp system.
 * SGN_E_REFINE if GMRES does not reach it; SGN_E_PIVOT if a fresh Kx is not positive definite.
 * sgn_step with this solver uses the same direction. */
sgn_status sgn_block_step(sgn_ctx ctx, const double* d_x, const double* d_p, double* d_sol, sgn_solve_info* info);
/* One outer iteration: assemble + factor + solve for the step, then
 * backtracking p + alpha dp with one equilibrium per trial and Armijo
 * acceptance f(alpha) <= f(0) + 1e-4 alpha g^T dp.  (d_p, d_x) must be an
 * equilibrium on entry and are updated in place.  With rhs_kind = SGN_RHS_KKT
 * the step needs no adjoint solve (same dp, Appendix A, Theorem 2) and the
 * slope is df/dx dx + df/dp dp; info->grad_norm is then -1.  When every
 * trial fails while |g^T dp| <= 1e-12 |f(0)| (stationary to working
 * precision) the call succeeds with alpha = 0 and leaves (p, x) unchanged. */
sgn_status sgn_step(sgn_ctx ctx, double* d_p, double* d_x, sgn_step_info* info);
/* One outer iteration of Sparse Newton with inertia control (Sec. 4, "Generalization to Arbitrary
 * Objectives", eq. totalHessian; Appendix A, Theorem 2; Sec. 5, which tests positive definiteness on
 * the null space of the constraint Jacobian by the inertia of the LDL^T factorisation and adds
 * diagonal regularisation when it fails).  Needs a context created with hessian =
 * SGN_HESSIAN_NEWTON (SGN_E_STATE otherwise).  At the equilibrium (d_p, d_x) (solved first if the
 * context holds no Kx factor of it): lam = -Kx^-1 df/dx^T; the saddle-point matrix with
 *   A = d2f/dx2 + d2(lam^T c)/dx2,  B = d2(lam^T c)/dp dx,  C = d2f/dp2 + d2(lam^T c)/dp2
 * (element terms: the derivative of the element Hessian along lam, K_e lam_e, lam_e . g_e) is
 * factorised; while its inertia is not (n_x + n_p, n_x, 0), or a pivot was perturbed, delta I is
 * added to the x and p diagonal (which turns the reduced Hessian H into H + delta (I + S^T S)) and
 * it is factorised again, delta taking 0, then 1e-4 (or a third of the delta of the last call that
 * needed one, at least 1e-20), then eight times the previous value, up to 1e20 (SGN_E_PIVOT
 * beyond).  The step solves that system with [0; -g; 0] (refined as sgn_solve); the line search and
 * the stationary rule are those of sgn_step.  restart != 0 forgets the remembered delta.  info as
 * for sgn_step plus delta and inertia_trials. */
sgn_status sgn_newton_step(sgn_ctx ctx, double* d_p, double* d_x, int restart, sgn_step_info* info);

/* ---- Learned-preconditioner path.  The paper names preconditioning of the
 * saddle-point system and iterative saddle-point solvers as future work
 * (Sec. 6.1) after standard preconditioned Krylov solvers performed poorly
 * on its problems (Sec. 5); the operator below is this library's own.
 *
 * Reference factor: the factorisation left by the most recent sgn_factor (or
 * by a MINRES fallback), P (S K_ref S) P^T = L D L^T.  Preconditioner:
 *   M = S^-1 P^T L B L^T P S^-1,  B = blockdiag_i(R_i C_i C_i^T R_i^T),
 * over the node groups i (one free mesh node: its owned parameters, then x_v,
 * then lambda_v, in elimination order).  R_i R_i^T = |D_i| is the eigen-
 * absolute value of the group's 1x1 and 2x2 pivots (for a 2x2 pivot
 * [[a,b],[b,e]] the first position takes the eigenvalue (a+e)/2 + rho with
 * eigenvector (cos t, sin t), t = atan2(b, (a-e)/2)/2).  C_i is built from raw
 * FP32 corrections: exp(r) on each owned-parameter position, and on the
 * trailing 2d positions the lower-triangular block with diagonal exp(r_tt)
 * and off-diagonal r_ij.  Zero corrections give B = |D|.  M is symmetric
 * positive definite by construction. */

/* Set (or clear, with NULLs) the raw corrections: d_corr_node [n_nodes *
 * (2d)(2d+1)/2] float, per mesh node the lower triangle row by row (entry
 * (i,j), i >= j, at i(i+1)/2 + j; positions ordered x_v components then
 * lambda_v components); d_corr_par [n_p] float, per parameter.  Device
 * pointers, caller-owned, read by every later preconditioner application
 * until replaced; fixed nodes' entries are unused. */
sgn_status sgn_set_pc_correction(sgn_ctx ctx, const float* d_corr_node, const float* d_corr_par);
/* d_out = K_SGN d_in with the currently assembled matrix ([N] device arrays,
 * block order, distinct). */
sgn_status sgn_spmv(sgn_ctx ctx, const double* d_in, double* d_out);
/* d_out = M^-1 d_in ([N], block order; may alias).  d_fwd (optional, [N])
 * receives the forward-solve result L^-1 P S d_in in pivot order, the input
 * of sgn_pc_grad.  Needs a reference factor (SGN_E_STATE otherwise). */
sgn_status sgn_pc_apply(sgn_ctx ctx, const double* d_in, double* d_out, double* d_fwd);
/* d_fwd = L^-1 P S d_in (pivot order) without the block and backward solves. */
sgn_status sgn_pc_forward(sgn_ctx ctx, const double* d_in, double* d_fwd);
/* Accumulate weight * d(ya^T B^-1 yb)/d(raw corrections) into d_grad_node
 * (layout of d_corr_node) and d_grad_par (layout of d_corr_par; either may be
 * NULL), where ya, yb are sgn_pc_forward results.  For a scalar loss l with
 * dl/dy = g of y = M^-1 w, dl/dr = grad of fwd(g)^T B^-1 fwd(w).  Uses the
 * corrections currently set; deterministic (every entry has one writer). */
sgn_status sgn_pc_grad(sgn_ctx ctx, const double* d_fwd_a, const double* d_fwd_b, double weight,
                       float* d_grad_node, float* d_grad_par);
/* Solve K_SGN sol = rhs (assembled matrix) by preconditioned MINRES with the
 * reference factor's M, to the equilibrated relative residual solve_rtol
 * (row scaling of the current matrix).  Falls back to a fresh exact LDL^T
 * (which becomes the new reference) plus refined solve when there is no
 * reference factor, after max_minres iterations, or when the residual shrinks
 * less than tenfold over 50 iterations; info->fallback reports it and
 * info->sweeps counts MINRES iterations plus refinement sweeps.  sgn_step uses
 * this solve when options.solver == SGN_MINRES_LEARNED. */
sgn_status sgn_solve_minres(sgn_ctx ctx, const double* d_rhs, double* d_sol, sgn_solve_info* info);

/* ---- Preconditioner network (FP32 weights and activations).  A mesh graph
 * network maps the change from a reference state (x_a, p_a) to the current
 * state (x, p) to the raw corrections of sgn_set_pc_correction.  Graph: mesh
 * nodes, one directed edge each way between nodes sharing an element.
 * Inputs: per node (x - x_a)/ell, (x - X)/ell (zero on fixed nodes), a fixed
 * flag, and the mean over the node's elements of (p - p_a) and of p (log
 * modulus) or |p_v - p_a,v|/ell and |p_v|/ell (per-node parameters); per edge
 * (X_s - X_d)/hbar and ((x_s - x_d) - (X_s - X_d))/ell, hbar the mean rest edge
 * length.  Encoders to width 64 (tanh), three layers of
 *   e <- e + tanh(W [h_dst, h_src, e] + b),  h <- h + tanh(W [h, mean_in(e)] + b),
 * decoders: per node W h + b to the (2d)(2d+1)/2 block entries (then d
 * parameter corrections for per-node parameters), per element W mean(h) + b
 * (log modulus).  Weight vector layout: dense layers in the order enc_node,
 * enc_edge, (edge_l, node_l) for l = 0..2, dec_node, dec_elem, each as W
 * (K x N row-major) followed by b (N).  Every reduction has a fixed order:
 * results are bitwise reproducible.  All pointers are device pointers owned by
 * the caller; activations of the last forward pass live in the workspace. */

/* Number of FP32 weights of the context's network. */
sgn_status sgn_gnn_num_weights(sgn_ctx ctx, int64_t* n);
/* Glorot-uniform initial weights from a counter-based generator (splitmix64
 * of seed); the decoders start at zero (corrections 0, M uses |D|). */
sgn_status sgn_gnn_init(sgn_ctx ctx, float* d_w, uint64_t seed);
/* Forward pass: d_corr_node [n_nodes * (2d)(2d+1)/2], d_corr_par [n_p] (the
 * layouts of sgn_set_pc_correction).  d_x_ref, d_x [n_x] and d_p_ref, d_p
 * [n_p] are FP64 states; ell is the context's length scale. */
sgn_status sgn_gnn_forward(sgn_ctx ctx, const float* d_w, const double* d_x_ref, const double* d_p_ref,
                           const double* d_x, const double* d_p, float* d_corr_node, float* d_corr_par);
/* Backward pass of the last forward: d_gw [n_weights] += the gradient of
 * sum(d_gcorr_node * corr_node) + sum(d_gcorr_par * corr_par) (either
 * cotangent may be NULL).  SGN_E_STATE before any forward pass. */
sgn_status sgn_gnn_backward(sgn_ctx ctx, const float* d_w, const float* d_gcorr_node, const float* d_gcorr_par,
                            float* d_gw);
/* One Adam step with bias correction (step >= 1) on n FP32 weights; m and v
 * are the caller's moment buffers (zero before step 1).  Synchronises stream. */
sgn_status sgn_adam(int64_t n, float* d_w, const float* d_g, float* d_m, float* d_v, float lr, float beta1,
                    float beta2, float eps, int step, void* stream);

/* Use the network with weights d_w (caller-owned, device; NULL to stop):
 * every sgn_solve_minres (and sgn_step with SGN_MINRES_LEARNED) first
 * evaluates it for the move from the reference factor's state (the (x, p) of
 * the assembly that sgn_factor factorised) to the currently assembled state
 * and uses its corrections; sgn_pc_apply / sgn_pc_grad then read them too.
 * sgn_set_pc_correction replaces this with fixed corrections. */
sgn_status sgn_set_pc_weights(sgn_ctx ctx, const float* d_w);
/* Training loss of the network for the reference factor and the assembled
 * matrix K: *h_loss = mean over the probes u of
 *   min_gamma |gamma T^2 u - u|^2 / |u|^2 = 1 - (u^T T^2 u)^2 / (|u|^2 |T^2 u|^2)
 * with T = (R C)^-1 L^-1 P S K S P^T L^-T (R C)^-T, the symmetric matrix
 * similar to M^-1 K (its spectrum is what MINRES sees; with the reference
 * matrix itself and no correction T^2 = I).  The symmetric form keeps the
 * loss at the scale of the spectrum (M^-1 K itself is far from normal
 * because the restricted pivoting leaves L badly conditioned), and the free
 * gamma makes it blind to a scaling of M, as MINRES is.  d_gw [n_weights] +=
 * the loss's weight gradient.  d_probes: n_probes vectors of [N] in whitened
 * coordinates (pivot order), device; Gaussian probes are the intended use.
 * log_form = 1 adds the gradient of log(loss) instead (samples whose loss
 * spans many decades then weigh alike); *h_loss is the loss either way. */
sgn_status sgn_pc_train_loss(sgn_ctx ctx, const float* d_w, const double* d_probes, int n_probes, int log_form,
                             float* d_gw, double* h_loss);

/* One SGN step at (d_x, d_p) as a replayed HIP graph: element kernel and
 * assembly, the KKT right-hand side [-df/dx; -df/dp; 0] into d_rhs (same dp
 * as the adjoint form, Appendix A, Theorem 2), supernodal LDL^T, the solve and
 * exactly n_ir (0..16) refinement sweeps into d_sol ([N], block order), with
 * the final equilibrated relative residual and a done flag computed on the
 * device.  The first call (and any call with other pointers or n_ir) captures
 * the whole sequence once on a context-owned stream; later calls replay it
 * (the values behind the pointers may change between calls).  No host
 * synchronisation happens inside; the call waits for the context's stream
 * first and for the replay at the end.  *h_rel (optional) receives the
 * residual; SGN_E_REFINE if it exceeds solve_rtol, SGN_E_INVERTED if (x, p)
 * inverts an element.  Meant for batches of small problems (n_components),
 * where launch overhead dominates. */
sgn_status sgn_graph_step(sgn_ctx ctx, const double* d_x, const double* d_p, double* d_rhs, double* d_sol, int n_ir,
                          double* h_rel);

/* Sizes of a system: N, nnz of the lower CSR, number of supernodes, factor
 * entries sum(m*s) and dense front flops of one factorisation. */
sgn_status sgn_get_sizes(sgn_ctx ctx, int which, int64_t* n, int64_t* nnz, int64_t* n_supernodes,
                         int64_t* factor_entries, double* factor_flops);
/* Symbolic tables of a system (host arrays sized from sgn_get_sizes):
 * perm[new] = old [n], etree [n] (-1 = root), rowptr [n+1], colind [nnz]. */
sgn_status sgn_get_symbolic(sgn_ctx ctx, int which, int32_t* h_perm, int32_t* h_etree,
                            int64_t* h_rowptr, int32_t* h_colind);
/* Read back the assembled lower CSR values (host [nnz], new numbering). */
sgn_status sgn_get_values(sgn_ctx ctx, int which, double* h_vals);
/* Copy the stage measurements of the last calls into *out. */
sgn_status sgn_get_stats(sgn_ctx ctx, sgn_stats* out);
/* Self test of the matrix-core lane layout the factorisation kernels rely on:
 * d_out (16x16, row-major) = A (16x4, row-major d_a) * B (4x16, row-major d_b)
 * computed by one 16x16x4 MFMA in FP64 (prec 0) or FP32 (prec 1).  Device
 * pointers owned by the caller; synchronises the stream. */
sgn_status sgn_selftest_mfma(int prec, const double* d_a, const double* d_b, double* d_out, void* stream);
/* Last error message of the context (never NULL). */
const char* sgn_last_error(sgn_ctx ctx);
/* Release host state (the workspace stays owned by the caller). */
void sgn_destroy(sgn_ctx ctx);

/* Autotuner of the schedule's blocking, the batched form's requirement that the blocking per
 * front-size bucket be chosen by measurement (Sec. 5 reports the method's cost as time per step,
 * which is what is minimised).  For prob and the options *base, at the state (d_x [n_x], d_p [n_p],
 * device), each candidate setting runs in a context of its own (created, its workspace allocated
 * with hipMalloc on the current device, everything freed before the next) and is timed as the best
 * of `reps` (1..100) rounds of assembly + factorisation + solve of a right-hand side of ones, after
 * one warm-up round, in host wall milliseconds on `stream`.  Coordinate descent from *base: each
 * bucket's outer_panels in {1, 2, 4, 8, 16}, then seq_panels in {-1, 2, 4, 8}, then the panel
 * factorisation's wavefront policy panel_waves in {0, 8, 4}; a candidate replaces the incumbent only
 * if it is at least 1% faster.  *best receives *base with the chosen setting; h_ms (optional, host,
 * room for 24) the milliseconds of the candidates in the order tried, the first being *base itself;
 * *n_cand (optional) the number tried: 18 when *base's settings are among the candidates, up to 23
 * otherwise.  Errors of a candidate's
 * context (e.g. SGN_E_NOMEM when the device cannot hold it) end the search and are returned. */
sgn_status sgn_autotune(const sgn_problem* prob, const sgn_options* base, const double* d_x, const double* d_p,
                        int reps, void* stream, sgn_options* best, double* h_ms, int* n_cand);

#ifdef __cplusplus
}
#endif
#endif /* SGN_H */
