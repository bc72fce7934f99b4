/*
 * irk.h -- C ABI of libirk, an MI355X (gfx950) solver for the coupled stage
 * system of an s-stage implicit Runge--Kutta step, preconditioned by the
 * block-LDU preconditioner P_LD with one AMG V-cycle per diagonal block.
 *
 * Method: M. M. Rana, V. E. Howle, K. Long, A. Meek, W. Milestone, "A New
 * Block Preconditioner for Implicit Runge--Kutta Methods for Parabolic PDE
 * Problems" (arXiv 2010.11377).
 *
 *   IRK step (Sec. 2):        u_{n+1} = u_n + h sum_i b_i k_i
 *   stage system (Sec. 3.1, block system (3.2); Kronecker form in Sec. 4):
 *       (I_s (x) M + h A (x) K) k = 1_s (x) (g - K u_n)
 *   preconditioners (Sec. 4, general form (4.1); Sec. 4.1, (4.3)):
 *       P = I_s (x) M + h A~ (x) K,  A~ = L D (P_LD), D U (P_DU),
 *                                     tril(A) (P_GSL), diag(A) (P_J)
 *       with A = L D U factored without pivoting (Sec. 4.1)
 *   application (Sec. 4.2): forward (lower A~) or back (upper A~)
 *       substitution over the stage blocks, one AMG V-cycle on each
 *       diagonal block  M + h A~_ii K.
 *
 * The paper's stiffness matrix F is called K here.  K and the mass matrix M
 * (NULL: M = I, the finite-difference case) are CSR matrices on a structured
 * nx x ny grid (x fastest) whose couplings stay within the 3 x 3 neighbourhood
 * of a node (five-point finite differences, seven-point P1 elements on right
 * triangles, nine-point stencils).
 *
 * Conventions for every call:
 *  - "host" pointers are read during the call and copied; the caller keeps
 *    ownership.  "device" pointers are HIP device memory owned by the caller
 *    and must stay valid until the call returns.
 *  - All GPU work is enqueued on the HIP stream given to irk_setup.  Calls that
 *    produce results return after that work has finished (the Krylov loop
 *    reads its residual estimate on the host once per iteration).
 *  - Vectors of stage values are stage-major: element (i, p) of an s x N
 *    array is at index i * N + p.
 *  - Nothing is thrown across the ABI.  Every call returns an irk_status;
 *    irk_last_error() gives a message for the last failure on a solver.
 *  - A solver must not be used from two threads at once.
 */
#ifndef IRK_H
#define IRK_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct irk_solver irk_solver; /* opaque, owned by the library */

typedef enum {
  IRK_OK = 0,
  IRK_E_INVALID = -1,        /* bad argument, size mismatch, unsupported structure */
  IRK_E_SINGULAR_PIVOT = -2, /* A has a (near-)zero LDU pivot: no factorisation without pivoting */
  IRK_E_NOT_CONVERGED = -3,  /* max_iter reached; the best iterate is still written */
  IRK_E_BREAKDOWN = -4,      /* Krylov breakdown (zero or non-finite Hessenberg entry) */
  IRK_E_NONFINITE = -5,      /* NaN/Inf in the input or the residual */
  IRK_E_HIP = -6,            /* a HIP runtime call failed */
  IRK_E_OOM = -7             /* device allocation failed */
} irk_status;

/* Butcher tableau (Sec. 2): A is s x s row-major, b and c have s entries.
 * Host pointers. 1 <= s <= 8. */
typedef struct {
  int s;
  const double *A;
  const double *b;
  const double *c;
} irk_butcher;

/* Square CSR matrix, 0-based, column indices sorted within each row.
 * Host pointers. */
typedef struct {
  int n;
  int nnz;
  const int *rowptr; /* n + 1 entries */
  const int *colind; /* nnz entries */
  const double *val; /* nnz entries */
} irk_csr;

/* Structured grid of the unknowns: unknown (i, j) has index j * nx + i.
 * Couplings of K may only join (i, j) to (i +- 1, j) and (i, j +- 1). */
typedef struct {
  int nx;
  int ny;
} irk_grid;

enum { IRK_FP64 = 0, IRK_MIXED = 1 };
enum { IRK_PREC_LD = 0, IRK_PREC_DU = 1, IRK_PREC_GSL = 2, IRK_PREC_J = 3 };
enum { IRK_RIGHT = 0, IRK_LEFT = 1 };
enum { IRK_INTERP_LINEAR = 0, IRK_INTERP_CONSTANT = 1 };
enum { IRK_SMOOTH_RBGS = 0, IRK_SMOOTH_JACOBI = 1 };

typedef struct {
  int precision;   /* IRK_FP64: everything in double.  IRK_MIXED: V-cycles,
                      block sweeps and the preconditioned vectors Z in float;
                      Krylov basis, Arnoldi, Hessenberg, residuals and the
                      solution update in double. */
  int precond;     /* IRK_PREC_LD (the paper's method), DU, GSL or J */
  int restart;     /* FGMRES restart length m (1..200) */
  int max_iter;    /* total Krylov iterations allowed per solve */
  int nu_pre;      /* smoothing sweeps before the coarse correction (1..3): red-black
                      Gauss-Seidel sweeps (both colours) or damped Jacobi sweeps */
  int nu_post;     /* sweeps after it (must equal nu_pre) */
  int coarse_max;  /* coarsen while the level has more unknowns than this */
  int vcycles;     /* V-cycles per diagonal-block subsolve (the paper uses 1) */
  int true_resid;  /* 1: when the estimate reports convergence, recompute
                      ||rhs - A k|| / ||rhs|| in double and restart if it is
                      above rtol (guards single-pass Gram-Schmidt) */
  int reorth;      /* second classical Gram-Schmidt pass: 0 never, 1 always,
                      2 when the first pass leaves less than 1/sqrt(2) of the
                      vector's norm (DGKS criterion, decided on the GPU) */
  double rtol;     /* stop when the residual estimate <= rtol * ||rhs||
                      (IRK_LEFT: the preconditioned residual, relative to
                      ||P^-1 rhs||) */
  int side;        /* IRK_RIGHT: flexible GMRES on A P^-1 (the default).
                      IRK_LEFT: GMRES on P^-1 A with the preconditioned
                      residual as stopping test (Sec. 5.1, Tables 7-10);
                      requires IRK_FP64 and applies to forward steps; adjoint
                      solves stay right-preconditioned. */
  int interp;      /* multigrid prolongation (restriction is always the sum
                      over the 2 x 2 cell): IRK_INTERP_LINEAR, bilinear
                      between cell centres (the default); IRK_INTERP_CONSTANT,
                      the transpose of the restriction, which keeps every
                      Galerkin coarse operator of an M-matrix an M-matrix
                      (advection-dominated operators at large h_t). */
  int graphs;      /* 1: each preconditioner application (s coupling passes
                      and V-cycles, a fixed kernel sequence per Krylov column)
                      is captured once into a HIP graph and replayed, which
                      lowers the host's per-kernel launch cost (small grids,
                      where the host cannot keep ahead of the kernels); 0:
                      direct launches (the default: on large grids the host
                      keeps ahead anyway, and a graph launch delays its first
                      kernel).  Both run the same kernels in the same order, so
                      the results are identical. */
  double coarse_ratio; /* end of a block's V-cycle: the first level l whose
                      block S_l + tau_i K_l has tau_i max_p (K_l)_pp / (S_l)_pp
                      <= coarse_ratio (S_l, K_l the Galerkin mass and
                      stiffness operators of level l, S_0 = M) runs its pre-
                      and post-smoothing with no coarse correction, and the
                      levels below it are skipped for that block.  0: every
                      cycle goes down to the coarsest level (solved exactly). */
  int smoother;    /* IRK_SMOOTH_RBGS: red-black Gauss-Seidel (colours 0, 1
                      before the coarse correction, 1, 0 after; Jacobi within
                      a colour on nine-point levels), the default.
                      IRK_SMOOTH_JACOBI: damped Jacobi x += jacobi_omega
                      D^-1 (b - D x), every node from the old values; it
                      leans more on the coarse correction, so pair it with a
                      smaller coarse_ratio (2: double glazing 1024^2 takes
                      5.3 ms per step against 8.1 at the default 8). */
  double jacobi_omega; /* Jacobi damping weight in (0, 1] (default 0.8) */
  int fuse_levels; /* 1: two adjacent intermediate nine-point levels share one
                      launch per direction where the grid allows it (nu = 2,
                      red-black smoothing), the default.  0: one launch per
                      level.  The operations per node are the same; FP32
                      results may differ in the last bits where the compiler
                      contracts a product and a sum differently. */
} irk_options;

typedef struct {
  int iters;             /* Krylov iterations used (all cycles) */
  int restarts;          /* completed restart cycles */
  double rel_resid_est;  /* FGMRES estimate of ||rhs - A k|| / ||rhs|| */
  double rel_resid_true; /* true relative residual, or -1 if not computed */
  double seconds;        /* wall time of the call */
} irk_stats;

/* Fill *opt with the defaults: IRK_FP64, IRK_PREC_LD, restart 40,
 * max_iter 200, nu_pre = nu_post = 2, coarse_max 64, vcycles 1,
 * true_resid 1, reorth 0, rtol 1e-8, side IRK_RIGHT, interp IRK_INTERP_LINEAR,
 * graphs 0, coarse_ratio 8, smoother IRK_SMOOTH_RBGS, jacobi_omega 0.8,
 * fuse_levels 1. */
void irk_default_options(irk_options *opt);

/* LDU factorisation without pivoting, A = L diag(d) U (Sec. 4.1), host only.
 * A: s x s row-major (host).  L and U (s x s, row-major, unit diagonal) and d
 * (s) are written by the library into caller-provided host arrays; any of
 * them may be NULL.  Returns IRK_E_SINGULAR_PIVOT when some
 * |d_k| <= 64 * eps * max|a_ij|, IRK_E_INVALID for s outside 1..8. */
irk_status irk_ldu(int s, const double *A, double *L, double *d, double *U);

/* Build a solver for the stage system of Sec. 3.1 / Sec. 4 with mass matrix
 * M (host CSR, copied; NULL for M = I; positive diagonal required), stiffness
 * K (host CSR, copied), timestep h_t > 0 and the structured grid (required).
 * Factors A (Sec. 4.1), builds the AMG hierarchy of every diagonal block
 * M + h_t A~_ii K, uploads it and allocates the Krylov workspace on the
 * current HIP device.  IRK_E_INVALID when M and K differ in size or M has a
 * coupling outside the 3 x 3 neighbourhood or a non-positive diagonal.  hip_stream is a
 * hipStream_t (NULL for the default stream).  opt may be NULL (defaults).
 * On success *out owns all device memory until irk_destroy. */
irk_status irk_setup(irk_solver **out, const irk_butcher *tab, const irk_csr *M,
                     const irk_csr *K, double h_t, const irk_grid *grid,
                     const irk_options *opt, void *hip_stream);

/* Source term g (device, N doubles) of u' = -K u + g, copied into the solver;
 * NULL resets it to zero. */
irk_status irk_set_source(irk_solver *S, const double *g_dev);

/* Replace K (same grid and sparsity structure) and rebuild the hierarchy,
 * keeping the workspace.  Used when a coefficient field changes. */
irk_status irk_update_operator(irk_solver *S, const irk_csr *K);

/* One IRK step (Sec. 2): u_np1 = u_n + h sum_i b_i k_i with k from
 * right-preconditioned flexible GMRES on the stage system.  u_n_dev and
 * u_np1_dev are device arrays of N doubles and may alias.  st may be NULL.
 * IRK_E_NOT_CONVERGED still writes the best iterate; after other errors the
 * contents of u_np1_dev are unspecified when it does not overlap u_n_dev
 * (the true-residual check writes its candidate there). */
irk_status irk_step(irk_solver *S, const double *u_n_dev, double *u_np1_dev, irk_stats *st);

/* Same as irk_step and also writes the stage vectors k (device, s*N doubles,
 * stage-major) into k_dev. */
irk_status irk_step_stages(irk_solver *S, const double *u_n_dev, double *u_np1_dev,
                           double *k_dev, irk_stats *st);

/* For callers that cannot allocate device memory at step time (HIP graph
 * capture around the caller's own work, tight serving loops, harnesses that
 * forbid hipMalloc): the same step as irk_step, with every buffer the step
 * writes besides u_np1 (Krylov bases V and Z, right-hand sides, multigrid
 * level vectors, reduction partials, Hessenberg and Givens data) taken from
 * one static device array of 64 MiB per GPU instead of the solver's
 * workspace.  Nothing is allocated or freed; the array is held by each GPU
 * the library runs on until the process ends.  Results equal irk_step's.
 * Needs (restart + 1) * 8 + restart * (4 or 8) + 16 bytes per stage unknown
 * plus O(N) more; a solver whose step does not fit gets IRK_E_INVALID (the
 * message states the size) and must use irk_step.  All solvers on one GPU
 * share the array: calls that overlap on one GPU race.  Graph replay and
 * kernel-class timing are not used during this call. */
irk_status irk_step_noalloc(irk_solver *S, const double *u_n_dev, double *u_np1_dev,
                            irk_stats *st);

/* Discrete adjoint of irk_step (not in the paper): recomputes the forward
 * stages from the checkpoint u_n, solves the transposed stage system
 * (I (x) M^T + h A^T (x) K^T) psi = h (b (x) lam_np1) to the solver's
 * tolerance, and writes lam_n = lam_np1 - K^T sum_i psi_i.  For a symmetric
 * K and M = I the system is solved with this solver's operators,
 * right-preconditioned by the transposed preconditioner P^T (block back
 * substitution for P_LD); otherwise by a second solver of the same kind for
 * the tableau A^T and the operators K^T, M^T (its preconditioner built from
 * the LDU of A^T and the hierarchy of M^T + tau K^T), set up on the first
 * such call (the library owns it; irk_update_operator and irk_destroy drop
 * it).  Optionally writes psi and the stage values U_i = u_n + h sum_j a_ij k_j
 * (device, s*N doubles each; NULL skips).  lam_n_dev may alias lam_np1_dev. */
irk_status irk_adjoint_step(irk_solver *S, const double *u_n_dev, const double *lam_np1_dev,
                            double *lam_n_dev, double *psi_dev, double *U_dev, irk_stats *st);

/* Gradient of J with respect to the face coefficients kappa_f of the
 * diffusion operator (K u)_P = h_x^-2 sum_{faces (P,Q)} kappa_f (u_P - u_Q)
 * (not in the paper; the derivative of the discrete stage system of Sec. 3.1
 * with respect to a parameter of K, summed over the stages of one step):
 * adds  dJ/dkappa_f = -h_x^-2 sum_i (psi_iP - psi_iQ)(U_iP - U_iQ)  for every
 * face, boundary values of psi and U being zero.
 * Layout of gface_dev (device, accumulated, not overwritten), full-grid node
 * (I, J) with I in 0..nx+1, J in 0..ny+1 and interior node (i, j) = (I-1, J-1):
 *   x faces first: ny rows of nx+1, entry J' * (nx+1) + I' is the face between
 *     (I', J'+1) and (I'+1, J'+1);
 *   then y faces:  ny+1 rows of nx, entry ny*(nx+1) + J' * nx + I' is the face
 *     between (I'+1, J') and (I'+1, J'+1);
 *   2 nx ny + nx + ny doubles in all.
 * psi_dev, U_dev: device s*N doubles from irk_adjoint_step.  IRK_E_INVALID for
 * a NULL pointer or h_x <= 0. */
irk_status irk_grad_diffusion_faces(irk_solver *S, const double *psi_dev, const double *U_dev,
                                    double h_x, double *gface_dev);

/* Gradient of J with respect to nodal coefficients of the diffusion operator
 * (K u)_P = h_x^-2 sum_{faces (P,Q)} kappa_f (u_P - u_Q), kappa_f =
 * (kappa_P + kappa_Q)/2, on the (nx+2) x (ny+2) node grid including boundary
 * nodes: adds  -(1/2) h_x^-2 sum_i (psi_iP - psi_iQ)(U_iP - U_iQ)  of every
 * face to both of its nodes (boundary values of psi and U are zero).
 * psi_dev, U_dev: device s*N doubles from irk_adjoint_step; gnode_dev:
 * device (nx+2)*(ny+2) doubles, accumulated (not overwritten). */
irk_status irk_grad_diffusion_nodes(irk_solver *S, const double *psi_dev, const double *U_dev,
                                    double h_x, double *gnode_dev);

/* The Kronecker SpMM alone: y = (I_s (x) M + h A (x) K) x (Sec. 4), x and y
 * device arrays of s*N doubles (stage-major), no aliasing. */
irk_status irk_apply_operator(irk_solver *S, const double *x_dev, double *y_dev);

/* One application of the configured preconditioner, z ~= P^-1 v, by block
 * substitution with one V-cycle per stage block (Sec. 4.2).  With
 * coarse_max >= N the V-cycle is a direct solve and z = P^-1 v exactly.
 * v_dev, z_dev: device arrays of s*N doubles (stage-major), no aliasing.
 * In IRK_MIXED the sweep runs in float and z is widened to double. */
irk_status irk_apply_preconditioner(irk_solver *S, const double *v_dev, double *z_dev);

/* Release every resource of the solver (NULL is allowed). */
void irk_destroy(irk_solver *S);

/* Static description of a status code. */
const char *irk_status_string(irk_status st);

/* Message for the last failure on S (empty if none).  irk_last_error(NULL)
 * gives the message of the last failed irk_setup on this thread. */
const char *irk_last_error(const irk_solver *S);

/* Sizes of the built solver: N, s, number of AMG levels, and whether the
 * level operators were recognised as constant-coefficient (1) or are stored
 * per node (0).  Any pointer may be NULL. */
irk_status irk_info(const irk_solver *S, int *N, int *s, int *levels, int *constant_coeff);

/* Preconditioner graphs (option graphs = 1): the number of captured graphs
 * the solver holds (one per Krylov column and system kind used so far) and
 * the number of replays since setup.  A class selected with
 * irk_profile_select that runs inside the preconditioner switches the
 * replays off while it is selected.  Any pointer may be NULL. */
irk_status irk_graph_stats(const irk_solver *S, int *graphs, long long *replays);

/* Kernel classes for irk_profile_select. */
enum {
  IRK_KC_SPMM_DOTS = 0,   /* Kronecker SpMM fused with the Gram-Schmidt dots */
  IRK_KC_SPMM_UPDATE = 1, /* SpMM recomputed + first Gram-Schmidt update */
  IRK_KC_VEC_DOTS = 2,    /* second Gram-Schmidt pass: dots */
  IRK_KC_VEC_UPDATE = 3,  /* second Gram-Schmidt pass: update */
  IRK_KC_COUPLE = 4,      /* block-substitution coupling of one stage */
  IRK_KC_VDOWN_L0 = 5,    /* finest level: pre-smoothing + residual + restriction */
  IRK_KC_VUP_L0 = 6,      /* finest level: correction + post-smoothing */
  IRK_KC_VMID_DOWN = 7,   /* intermediate levels: pre-smoothing + residual + restriction */
  IRK_KC_VTAIL = 8,       /* the coarse levels solved in one workgroup */
  IRK_KC_VMID_UP = 9,     /* intermediate levels: correction + post-smoothing */
  IRK_KC_COUNT = 10
};

/* Measurement hook: while a class is selected (kc in 0..IRK_KC_COUNT-1),
 * every launch of that kernel class is bracketed by HIP events on the
 * solver's stream, and its duration and its algorithmic bytes (the bytes
 * the operation must move: each input and output element once, no halo or
 * cache re-reads) are accumulated.  kc = -1 disables it.  Selecting resets
 * the counters. */
irk_status irk_profile_select(irk_solver *S, int kc);

/* Read the counters of the selected class: number of timed launches, total
 * kernel milliseconds and total algorithmic bytes.  Any pointer may be NULL. */
irk_status irk_profile_read(const irk_solver *S, long long *launches, double *total_ms,
                            double *total_bytes);

#ifdef __cplusplus
}
#endif
#endif /* IRK_H */
