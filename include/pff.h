/*
 * pff.h -- C ABI of the matrix-free phase-field fracture Newton/GMG library (gfx950).
 *
 * The library implements one step of the primal-dual active-set (semi-smooth
 * Newton) method for the quasi-monolithic pressurized phase-field fracture
 * problem of Jodlbauer, Langer and Wick, "Matrix-free multigrid solvers for
 * phase-field fracture problems" (arXiv:1902.08112):
 *   - the semi-linear form A(u, phi) (Sec. 2.3, eq. semilinear, without a
 *     stress split or with the Miehe spectral split of Sec. 2.1, time-lagged
 *     extrapolation phi~ in the displacement equation) and its Jacobian
 *     G = A'(U) on Q1/Q2 quadrilaterals / hexahedra (Sec. 2.4);
 *   - the matrix-free cell-loop apply y = G~ x (Sec. 4.1) with rows and
 *     columns of the constrained DoFs eliminated (Algorithm 1, step 4);
 *   - coarse-level operators rediscretized at the injected linearization
 *     point G_l(U_l) with the injected active set (Sec. 4.2);
 *   - the monolithic geometric-multigrid V-cycle P_full = MG(G~) with a
 *     block-diagonal Chebyshev-Jacobi smoother and a Chebyshev coarse solve
 *     (Sec. 3.2, Sec. 3.3), and the block-diagonal alternative
 *     P_diag = diag(MG(U~), MG(P~)) of Sec. 3.3;
 *   - right-preconditioned FGMRES (Sec. 3, Sec. 5) inside one Newton step,
 *     the active-set loop to convergence and the steps of the time loop
 *     around it (extrapolation of phi~, the pressure of the loading);
 *   - the energies and boundary loads of Sec. 5 as reductions.
 *
 * Conventions shared by every call
 *   Vector layout: component-major blocks [u_1 | ... | u_d | phi]; each block
 *     covers the level's bounding-box node lattice, nn_k = p*N_k + 1 nodes per
 *     axis, x fastest, then y, then z.  A level vector has (d+1)*prod(nn_k)
 *     entries.  Lattice nodes of no active cell (the hole of the L-shaped
 *     domain) are stored, constrained in every component, and held at 0.
 *   Levels: l = 0 is the coarsest, l = n_levels-1 the finest; N_l = N_fine / 2^(L-1-l).
 *   Pointers marked d_ are device pointers on the current HIP device; they
 *     are owned by the caller.  The library never allocates or frees device
 *     memory: every device buffer it uses is carved from the caller's workspace.
 *   Streams: `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Calls are stream-ordered; only the calls documented as
 *     synchronizing wait for the stream.
 *   Errors: every call returns a pf_status; on failure pf_last_error() gives a
 *     message.  Arguments are validated before any device work; the library
 *     never aborts the process.
 *   Threads: one context per host thread.
 */
#ifndef PFF_H
#define PFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pf_status;
#define PF_OK 0
#define PF_ERR_INVALID_ARG 1
#define PF_ERR_UNSUPPORTED 2
#define PF_ERR_DEVICE 3
#define PF_ERR_WORKSPACE 4
#define PF_ERR_NOT_CONVERGED 5
#define PF_ERR_NONFINITE 6

#define PF_F64 0
#define PF_F32 1

/* Preconditioner structure (Sec. 3.3): PF_PREC_FULL = MG(G~), one multigrid on the whole
 * system with the block smoother; PF_PREC_DIAG = diag(MG(U~), MG(P~)), one multigrid per
 * diagonal block (every residual inside the cycle is formed with the block-diagonal B~, so
 * the coupling block G_phi,u is not seen by the preconditioner). */
#define PF_PREC_FULL 0
#define PF_PREC_DIAG 1

/* Energy split (Sec. 2.1): PF_SPLIT_NONE uses E_s^+ = E_s (the unsplit form); PF_SPLIT_MIEHE
 * uses the spectral split E_s^+ = lam/2 <tr e>_+^2 + mu tr(e_+^2) with sigma^+ = dE_s^+/de,
 * which makes the displacement equation nonlinear; its Jacobian is the consistent tangent
 * (the derivative of e -> e_+ by the divided differences of <.>_+ at the eigenvalue pairs;
 * d<x>_+/dx = 0 at x = 0, and an eigenvalue or tr e within 1e-13 of the spectral radius of
 * zero counts as zero).  In 2D the split acts on the in-plane strain of plane strain. */
#define PF_SPLIT_NONE 0
#define PF_SPLIT_MIEHE 1

#define PF_BOX 0
#define PF_LSHAPE 1 /* [0,1]^3 minus [0.5,1]x[0.5,1]x[0,1] (2D: the same without z), scaled by extent */

/* Per-node constraint bits (uint8): bit c < d constrains u_c, bit 3 constrains phi. */
#define PF_MASK_U(c) (1u << (c))
#define PF_MASK_PHI 8u

typedef struct pf_mesh {
  int dim;                  /* 2 or 3 */
  int degree;               /* 1 (Q1) or 2 (Q2) */
  int n_cells[3];           /* finest-level cells per axis (unused entries ignored) */
  double extent[3];         /* box edge lengths */
  int domain;               /* PF_BOX or PF_LSHAPE */
  int n_levels;             /* >= 1; n_cells divisible by 2^(n_levels-1) */
  unsigned dirichlet_faces; /* u = current value on faces: bit 2k = {x_k = 0}, bit 2k+1 = {x_k = extent_k} */
} pf_mesh;

/* Solver constants.  pf_default_options gives the paper's values:
 * Chebyshev degree 4 over [1.2 lam/5, 1.2 lam] with lam from 10 CG steps
 * (Sec. 3.2.1), coarse Chebyshev over [0.9 lam_min, 1.2 lam_max] (Sec. 3.2.2)
 * with 2 sweeps of degree 20, PDAS constant c = 100 (Sec. 3.1), FGMRES
 * restart 50 and relative tolerance 1e-8. */
typedef struct pf_options {
  int vcycle_precision;    /* PF_F64 or PF_F32 (V-cycle levels above the coarsest) */
  int cheb_degree;         /* smoother polynomial degree (operator applications per step) */
  double cheb_ratio;       /* lower end of the smoothing range = upper / ratio */
  double cheb_safety;      /* upper end = safety * estimated lam_max */
  int eig_cg_steps;        /* CG steps of the eigenvalue estimate */
  int coarse_degree;       /* Chebyshev degree of the coarse solve */
  int coarse_sweeps;       /* outer sweeps of the coarse solve */
  double coarse_lo_factor; /* coarse range lower end = factor * lam_min */
  int gmres_restart;       /* FGMRES restart length m (workspace grows with m) */
  int gmres_max_iter;      /* total FGMRES iteration cap */
  double gmres_rtol;       /* stop when ||R~ - G~ dU|| <= max(rtol ||R~||, atol) (true residual) */
  double pdas_c;           /* active-set constant c */
  uint64_t eig_seed;       /* SplitMix64 seed of the eigenvalue start vectors */
  double gmres_atol;       /* absolute floor of the FGMRES stop (default 0; the inexact solves of
                              Sec. 5 use rtol 1e-4 with a small floor) */
  int preconditioner;      /* PF_PREC_FULL (default, the paper's choice) or PF_PREC_DIAG */
  int stress_split;        /* PF_SPLIT_NONE (default) or PF_SPLIT_MIEHE: the model's energy split
                              (the batched solver evaluates the split on the fly in every mode) */
} pf_options;

typedef struct pf_newton_report {
  int gmres_iters;          /* FGMRES iterations of this step */
  int converged;            /* 1 if the true relative residual reached gmres_rtol */
  double rel_residual;      /* ||R~ - G~ dU|| / ||R~|| (FP64, recomputed) */
  double rhs_norm;          /* ||R~|| */
  int64_t n_active;         /* |A_k|: phase-field nodes in the active set */
  double t_residual_s;      /* wall time of step 1 (residual) */
  double t_setup_s;         /* wall time of steps 2-4 (active set, level data, diagonals, eigenvalues) */
  double t_solve_s;         /* wall time of step 5 (FGMRES) */
  double t_total_s;
} pf_newton_report;

typedef struct pf_pdas_report {
  int iterations;           /* linear solves done (Newton corrections) */
  int converged;            /* 1 if A_k = A_{k-1} and ||R~_k|| <= tol_as was reached */
  int gmres_iters_total;    /* FGMRES iterations summed over the corrections */
  int64_t n_active;         /* |A_k| of the last iteration */
  int64_t n_changed;        /* |A_k xor A_{k-1}| of the last iteration (-1 if k = 0) */
  double residual_norm;     /* ||R~_k|| of the last iteration (absolute, FP64) */
  double t_total_s;
} pf_pdas_report;

typedef struct pf_level_info {
  int n_cells[3];
  int n_nodes_axis[3];
  int64_t n_nodes;
  int64_t n_dofs;
  int64_t n_active_cells;
  double h[3];
  int precision;            /* arithmetic type of this level inside the V-cycle */
  int64_t n_domain_nodes;   /* lattice nodes that belong to an active cell (hole nodes excluded) */
} pf_level_info;

typedef struct pf_ctx pf_ctx;

/* Fill *opt with the paper's constants (see pf_options). */
void pf_default_options(pf_options* opt);

/* Device bytes of the workspace pf_setup needs for this mesh and options.
 * Errors: PF_ERR_INVALID_ARG (null pointer, bad mesh), PF_ERR_UNSUPPORTED (dim, degree). */
pf_status pf_workspace_size(const pf_mesh* mesh, const pf_options* opt, size_t* bytes);

/* Create a context.  Material (Sec. 2.1): Young's modulus E > 0, Poisson
 * ratio -1 < nu < 0.5 (mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu)) in 2D
 * and 3D), critical energy release rate G_c > 0, phase-field width eps > 0,
 * residual stiffness 0 <= kappa < 1, constant pressure p (finite).  opt may
 * be NULL (defaults).  d_workspace: device buffer of at least
 * pf_workspace_size bytes, 256-byte aligned, owned by the caller and kept
 * alive until pf_destroy.  Builds the level geometry, Dirichlet/hole masks and
 * the lumped mass (Sec. 3.1 remark, Gauss-Lobatto) on `stream`.
 * Errors: INVALID_ARG, UNSUPPORTED, WORKSPACE (too small / misaligned), DEVICE. */
pf_status pf_setup(const pf_mesh* mesh, double E, double nu, double G_c, double eps, double kappa,
                   double pressure, const pf_options* opt, void* d_workspace, size_t ws_bytes,
                   void* stream, pf_ctx** out);

/* Extra prescribed-displacement constraints on the finest level: one byte per
 * node, bit c constrains u_c (e.g. a loaded strip).  Coarser levels inherit
 * them by nodal injection.  d_bits may be NULL to clear. */
pf_status pf_set_constraints(pf_ctx* ctx, const uint8_t* d_bits, void* stream);

/* Set the linearization point on the finest level and build every level's
 * data: nodal injection of U, phi~ and the active indicator (Sec. 4.2),
 * constraint masks, matrix-free diagonals (Sec. 4.1 remark), FP32 copies, and
 * the eigenvalue estimates of every level and block (unless fixed by
 * pf_set_eig_bounds).  d_U: (d+1)*n_nodes FP64; d_phi_tilde: n_nodes FP64;
 * d_active: n_nodes bytes (nonzero = phi constrained), may be NULL.
 * Synchronizes the stream (reads back the Lanczos coefficients). */
pf_status pf_set_linearization(pf_ctx* ctx, const double* d_U, const double* d_phi_tilde,
                               const uint8_t* d_active, void* stream);

/* y = G~_l(U_l) x on level l: y = Pi_F G Pi_F x + Pi_C x (Sec. 4.1 eq. for
 * G u as a sum over cells; Algorithm 1 step 4 elimination).  prec PF_F64:
 * x, y are double*; PF_F32: float* (uses the FP32 copy of the level data).
 * Requires pf_set_linearization.  Asynchronous. */
pf_status pf_jacobian_apply(pf_ctx* ctx, int level, int prec, const void* d_x, void* d_y, void* stream);

/* Block-diagonal smoother operator B~_l x = diag(G_uu, G_phiphi) with the same
 * elimination (S_full of Sec. 3.3).  Same conventions as pf_jacobian_apply. */
pf_status pf_block_apply(pf_ctx* ctx, int level, int prec, const void* d_x, void* d_y, void* stream);

/* R = -A(U) on the finest level (Algorithm 1 step 1; Sec. 4.1 remark), no
 * constraints applied.  d_U: (d+1)*n_nodes, d_phi_tilde: n_nodes, d_R: (d+1)*n_nodes, FP64. */
pf_status pf_residual(pf_ctx* ctx, const double* d_U, const double* d_phi_tilde, double* d_R, void* stream);

/* Copy the diagonal of G~_l (1 on constrained rows) of level l into d_diag (FP64). */
pf_status pf_get_diagonal(pf_ctx* ctx, int level, double* d_diag, void* stream);

/* Copy the lumped mass of the finest level (n_nodes FP64) into d_M. */
pf_status pf_get_lumped_mass(pf_ctx* ctx, double* d_M, void* stream);

/* Copy the level's injected linearization point (d_U: (d+1)*n_nodes, may be NULL),
 * phi~ (n_nodes, may be NULL) and constraint mask bytes (n_nodes, may be NULL). */
pf_status pf_get_level_data(pf_ctx* ctx, int level, double* d_U, double* d_phi_tilde, uint8_t* d_mask,
                            void* stream);

/* Active-set decision (Algorithm 1 step 3): for every phase-field node that
 * is not otherwise constrained, v = R_phi/M + c (phi - phi^old); active iff
 * v > 0.  d_R: -A(U) (FP64, full vector), d_U, d_U_old: full vectors.
 * Writes d_active (n_nodes bytes, 1 = active), optionally d_v (n_nodes FP64,
 * 0 on skipped nodes), and the count into *n_active (synchronizes if non-NULL). */
pf_status pf_active_set(pf_ctx* ctx, const double* d_R, const double* d_U, const double* d_U_old,
                        uint8_t* d_active, double* d_v, int64_t* n_active, void* stream);

/* Transfers between level l (fine) and l-1 (coarse), FP64, whole vectors:
 * op 0: out_c = P^T in_f (restriction, Sec. 3.2), op 1: out_f = P in_c
 * (prolongation), op 2: out_c = nodal injection of in_f (Sec. 4.2).  No masks. */
pf_status pf_transfer(pf_ctx* ctx, int level, int op, const double* d_in, double* d_out, void* stream);

/* Eigenvalue estimates (raw Ritz values, before the safety factors) of
 * D^{-1} B~_bb per block on level l: out[0..3] = {lam_min_u, lam_max_u,
 * lam_min_phi, lam_max_phi}.  pf_set_eig_bounds fixes them (they are then
 * kept by pf_set_linearization until cleared with in == NULL). */
pf_status pf_get_eig_bounds(pf_ctx* ctx, int level, double out[4]);
pf_status pf_set_eig_bounds(pf_ctx* ctx, int level, const double in[4]);

/* z = P_full^{-1} r: one V-cycle (Sec. 3.3) with one pre- and one post-
 * smoothing step, prec = PF_F64 or PF_F32 for the levels above the coarsest
 * (the coarse solve is FP64).  r, z: fine-level FP64 vectors; z vanishes on
 * constrained DoFs and the constrained entries of r are ignored.  Asynchronous. */
pf_status pf_vcycle(pf_ctx* ctx, int prec, const double* d_r, double* d_z, void* stream);

/* One iteration k of Algorithm 1 (Sec. 3.1): residual, active set, level data,
 * FGMRES with the V-cycle (opt->vcycle_precision), update.  d_U (in/out):
 * U_k -> U_{k+1}; d_U_old: the previous time step (phi^old); d_phi_tilde:
 * extrapolated phase field for the displacement equation.  Dirichlet DoFs
 * keep their current values.  Synchronizes.  Returns PF_ERR_NOT_CONVERGED
 * (report filled, U updated with the last iterate) if gmres_max_iter is reached,
 * PF_ERR_NONFINITE if the residual is not finite (U unchanged). */
pf_status pf_newton_step(pf_ctx* ctx, double* d_U, const double* d_U_old, const double* d_phi_tilde,
                         pf_newton_report* rep, void* stream);

/* The primal-dual active-set loop (Algorithm 1 of Sec. 3.1 repeated): for
 * k = 0, 1, ... compute R_k, A_k and R~_k; stop when k > 0, A_k = A_{k-1}
 * and ||R~_k|| <= tol_as (absolute, the eps_as = 1e-10 of Sec. 5), else solve
 * and update as pf_newton_step.  At most max_iter corrections (>= 1).  The
 * check comes before the solve, so a converged iteration costs only the
 * residual.  d_U (in/out), d_U_old, d_phi_tilde as in pf_newton_step.
 * Synchronizes.  Returns PF_ERR_NOT_CONVERGED if max_iter corrections do not
 * converge or an FGMRES solve stops at gmres_max_iter (report filled, U holds
 * the last iterate), PF_ERR_NONFINITE on a non-finite residual. */
pf_status pf_pdas_solve(pf_ctx* ctx, double* d_U, const double* d_U_old, const double* d_phi_tilde, int max_iter,
                        double tol_as, pf_pdas_report* rep, void* stream);

/* Time-lagged extrapolation of the phase field for the displacement equation
 * (Sec. 2.3): d_out = phi_1 + theta (phi_1 - phi_2) on the finest level's
 * nodes (n_nodes entries each), with phi_1 = phi^{n-1}, phi_2 = phi^{n-2} and
 * theta = dt_n / dt_{n-1} (1 for a constant step; linear in time).  d_out may
 * alias neither input.  Hole nodes are copied from phi_1.  Asynchronous. */
pf_status pf_extrapolate(pf_ctx* ctx, const double* d_phi_1, const double* d_phi_2, double theta, double* d_out,
                         void* stream);

/* Quantities of interest of Sec. 5 for the state d_U = (u, phi) on the
 * finest level, as reductions over its cells (deterministic order):
 *   out[0] = crack energy  int G_c/2 ((1 - phi)^2 / eps + eps |grad phi|^2)
 *   out[1] = bulk energy   int g_kappa(phi) E_s^+(e(u)) + E_s^-(e(u)) + phi^2 p div u
 * (E_s^+ = E_s, E_s^- = 0 without a split; the Miehe parts with stress_split = PF_SPLIT_MIEHE)
 * at the cell Gauss points.  out is host memory.  Synchronizes. */
pf_status pf_energies(pf_ctx* ctx, const double* d_U, double out[2], void* stream);
/* For callers that cannot allocate memory while they run (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pf_energies
 * with d_out in DEVICE memory (2 doubles: crack energy, bulk energy), enqueued
 * on the stream without a read-back or a synchronization.  The call allocates
 * nothing: its per-block partial sums live in a static device array of the
 * library (16,448 bytes per GPU, held until the process ends; the array has
 * room for any mesh, as the reduction grid is capped at 1024 blocks), whose
 * address pf_setup resolves once per device.  All calls on one GPU share that
 * array: calls that overlap on one GPU (two streams or two host threads) race.
 * Errors: PF_ERR_INVALID_ARG for NULL pointers or when the current device is
 * not the one the context was set up on; PF_ERR_DEVICE for a launch failure. */
pf_status pf_energies_noalloc(pf_ctx* ctx, const double* d_U, double* d_out, void* stream);
/* Load on one face of the box: out[0..dim) = int_face (g_kappa(phi) sigma^+(u) + sigma^-(u)) n ds
 * (n the outward normal; the loading curve of Sec. 5 takes one component).
 * face = 2k for {x_k = 0}, 2k+1 for {x_k = extent_k}; only facets of active
 * cells count (the L-shape's hole is not part of the face).  p+1 Gauss points
 * per tangential direction.  out is host memory.  Synchronizes. */
pf_status pf_boundary_traction(pf_ctx* ctx, const double* d_U, int face, double* out, void* stream);

/* Set the crack pressure p of the loading (Sec. 5.1: p(t) = 1e3 t); finite.
 * Takes effect at the next operator, residual or set-up call. */
pf_status pf_set_pressure(pf_ctx* ctx, double pressure);

/* Level sizes. */
pf_status pf_get_level_info(pf_ctx* ctx, int level, pf_level_info* info);

/* Autotuner of the Q1 cell loop (the tensor-product apply of Sec. 4.1).  For
 * every level, precision and operator (mode 0: G~, mode 1: smoother block
 * B~) it times `reps` applies of each candidate kernel shape with HIP events
 * on `stream` and keeps in the context the first candidate (in the order
 * below) within 3% of the fastest, so that timing noise between near-equal
 * shapes does not flip the choice.  Candidates: variant 2 =
 * one thread per cell with atomic scatter; variant 4 = two threads per cell
 * (displacement / phase-field rows) with atomic scatter; variant 3 (3D) =
 * 256-thread bricks of cells staged through LDS with atomic scatter;
 * variant 0 / 1 = one wavefront per 8x8 / 16x4 tile of cells marching
 * through chunks of zc node planes with register carries (owner-computes,
 * deterministic); variant 5 (3D) = one 256-thread workgroup per 16x16 tile of
 * cells marching through chunks of zc node planes that stream through a ring
 * of three LDS planes one plane ahead (global-to-LDS loads), with the same
 * owner-computes combine (deterministic).  With stress_split = PF_SPLIT_MIEHE only variants 2 and 4
 * exist (the split's record-streaming loops).  Requires
 * pf_set_linearization; overwrites the V-cycle scratch vectors; synchronizes.
 * Q2 levels have one kernel and are skipped. */
pf_status pf_autotune(pf_ctx* ctx, int reps, void* stream);
/* HIP-event timing of the finest-level FP64 cell kernels of a Newton step.
 * enable is a combination of
 *   PF_KTIME_JACOBIAN  the Jacobian G~ (pf_jacobian_apply on the finest level, the FGMRES
 *                      operator applies, true residuals and smoother residuals), and
 *   PF_KTIME_BLOCK     the block operator B~ (the Chebyshev smoother's operator where it
 *                      is launched on its own, the eigenvalue CG, pf_block_apply on the
 *                      finest level), and
 *   PF_KTIME_BLOCK_CHEB the B~ launches that carry a fused Chebyshev step (see
 *                      pf_set_smoother_fusion).
 * A nonzero enable clears both records and, from then on, brackets every every-th
 * such launch of each record (the 1st, (every+1)-th, ...; every in [1, 1e6]) with two
 * events on the launch stream; the Pi_C start of y is outside the bracket.  At most
 * 1024 launches are recorded per record and period.  A bracket delays the stream by
 * a few microseconds (two event records), which a stride above 1 spreads thin;
 * enable = 0 stops recording and keeps the records (every is then ignored). */
#define PF_KTIME_JACOBIAN 1
#define PF_KTIME_BLOCK 2
#define PF_KTIME_BLOCK_CHEB 4
pf_status pf_set_kernel_timing(pf_ctx* ctx, int enable, int every);
/* One record (op = PF_KTIME_JACOBIAN, PF_KTIME_BLOCK or PF_KTIME_BLOCK_CHEB): the launches seen since it was
 * cleared (bracketed or not), the number bracketed and their mean / min / max duration
 * in seconds (waits for the last bracketed launch).  count = 0 gives zero durations. */
pf_status pf_get_kernel_timing_op(pf_ctx* ctx, int op, int64_t* launches, int* count, double* avg_s,
                                  double* min_s, double* max_s);
/* pf_get_kernel_timing_op with op = PF_KTIME_JACOBIAN. */
pf_status pf_get_kernel_timing(pf_ctx* ctx, int* count, double* avg_s, double* min_s, double* max_s);
/* Chebyshev smoother steps (Sec. 3.2.1) after the first one fused into the block-operator
 * apply on levels whose B~ runs as 3D Q1 marching tiles (autotuner variants 0 / 1 / 5), which
 * write every node exactly once: the step's vector update (residual, direction, iterate)
 * happens where the tile writes the node, and the separate vector pass disappears.  The
 * arithmetic per entry is the same as the separate pass's.
 *   PF_FUSE_OFF     never;
 *   PF_FUSE_TUNED   (default) on the levels and precisions where pf_autotune measured the
 *                   fused step faster than apply + vector pass by more than 3%, or where
 *                   pf_set_level_fusion chose it (untuned levels: not fused);
 *   PF_FUSE_ALWAYS  on every marching-tile level.
 * Drops captured V-cycle graphs.  Other shapes and levels are not affected. */
#define PF_FUSE_OFF 0
#define PF_FUSE_TUNED 1
#define PF_FUSE_ALWAYS 2
pf_status pf_set_smoother_fusion(pf_ctx* ctx, int mode);
/* The PF_FUSE_TUNED choice of one level and precision (fused = 0 or 1), as pf_autotune
 * would set it; used to restore cached tuning.  pf_tuning_report gives the autotuner's
 * choice ("fused") and its two step times ("step_us": unfused, fused) per block entry. */
pf_status pf_set_level_fusion(pf_ctx* ctx, int level, int prec, int fused);
/* Read / force the choice of one (level, prec, mode); variant -1 = size heuristic,
 * 0..5 as listed at pf_autotune, zc <= 0 = heuristic chunk.  Used to persist tuning results across runs. */
pf_status pf_get_tuning(pf_ctx* ctx, int level, int prec, int mode, int* variant, int* zc);
pf_status pf_set_tuning(pf_ctx* ctx, int level, int prec, int mode, int variant, int zc);
/* JSON text of the choices and measured candidate times (microseconds per apply). */
pf_status pf_tuning_report(pf_ctx* ctx, char* buf, size_t len);

/* Graph replay of the V-cycle: the first V-cycle after setup (or after a change
 * of pressure, kernel tuning, smoother fusion or coarse-solve path) is captured
 * into a hipGraph per precision on a private stream and replayed on the
 * caller's stream afterwards (pf_vcycle and the FGMRES of pf_newton_step).
 * Everything a new linearization or new eigenvalue bounds change -- level
 * data, diagonals, stored coefficients, the Chebyshev coefficients, the dense
 * coarse matrix -- is read by the kernels from device buffers with fixed
 * addresses, so one capture serves every later linearization.  enable = 0
 * launches every kernel directly (also while pf_set_kernel_timing is on).
 * Replays and direct launches compute the same operations; the atomic
 * scatters of some cell loops may order sums differently (rounding level).
 * Calls that overlap on one context race. */
pf_status pf_set_graphs(pf_ctx* ctx, int enable);
/* Number of V-cycle captures made by the context so far (both precisions). */
pf_status pf_get_graph_captures(pf_ctx* ctx, int64_t* n);

/* How the coarsest level's Chebyshev solve (Sec. 3.2.2) runs.  The solve is a fixed
 * polynomial in the level operator, so every mode computes the same linear map:
 *   PF_COARSE_AUTO  (default) for a Q1 coarsest level of at most 1024 DoFs without the
 *                   split, its dense matrix is formed at pf_set_linearization (one
 *                   workgroup per unit vector) and every V-cycle applies it as one
 *                   matvec; otherwise as PF_COARSE_FUSED;
 *   PF_COARSE_FUSED all sweeps in one single-workgroup launch (Q1 levels up to 4096 DoFs),
 *                   else as PF_COARSE_STEPS;
 *   PF_COARSE_STEPS one launch per operator apply and Chebyshev step.
 * New level-0 eigenvalue bounds rebuild the matrix on the stream of the next V-cycle; after
 * a change to AUTO or after pf_set_pressure the fused kernel serves until the next
 * pf_set_linearization rebuilds it. */
#define PF_COARSE_AUTO 0
#define PF_COARSE_FUSED 1
#define PF_COARSE_STEPS 2
pf_status pf_set_coarse_mode(pf_ctx* ctx, int mode);

/* Change the V-cycle precision used by pf_newton_step (PF_F64 or PF_F32). */
pf_status pf_set_vcycle_precision(pf_ctx* ctx, int prec);

/* Release the context (host memory only; the workspace stays the caller's). */
void pf_destroy(pf_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batches: n independent instances (own mesh sizes, extents, domains,
 * Dirichlet faces, materials, linearization points; common dim, degree and
 * n_levels) advanced together.  Every stage of the Newton step and V-cycle is
 * one launch over the whole batch, so many small problems fill the GPU.
 *
 * Packed layout: on each level the instances' vectors (each in the
 * single-instance layout above) are concatenated in instance order; instance b
 * occupies DoFs [dof_offsets[b], dof_offsets[b+1]) and nodes
 * [node_offsets[b], node_offsets[b+1]) of that level (pf_batch_layout).
 * ------------------------------------------------------------------------ */
typedef struct pf_batch pf_batch;

/* Workspace bytes for a batch (same validation as pf_workspace_size per instance;
 * all instances must share dim, degree and n_levels). */
pf_status pf_batch_workspace_size(const pf_mesh* meshes, int n, const pf_options* opt, size_t* bytes);
/* materials: host array of n*6 doubles {E, nu, G_c, eps, kappa, pressure} per
 * instance (ranges as in pf_setup).  Other arguments as in pf_setup. */
pf_status pf_batch_setup(const pf_mesh* meshes, const double* materials, int n, const pf_options* opt,
                         void* d_workspace, size_t ws_bytes, void* stream, pf_batch** out);
/* Host copies of the packed offsets of one level (n+1 entries each; either may be NULL). */
pf_status pf_batch_layout(pf_batch* b, int level, int64_t* dof_offsets, int64_t* node_offsets);
/* Extra displacement constraint bits on the finest level, packed by nodes (see pf_set_constraints). */
pf_status pf_batch_set_constraints(pf_batch* b, const uint8_t* d_bits, void* stream);
/* As pf_set_linearization, for every instance at once (packed finest-level vectors). */
pf_status pf_batch_set_linearization(pf_batch* b, const double* d_U, const double* d_phi_tilde,
                                     const uint8_t* d_active, void* stream);
/* y = G~_l x for every instance (packed level-l vectors; FP64 or FP32). */
pf_status pf_batch_jacobian_apply(pf_batch* b, int level, int prec, const void* d_x, void* d_y, void* stream);
/* One V-cycle for every instance (packed finest-level FP64 vectors). */
pf_status pf_batch_vcycle(pf_batch* b, int prec, const double* d_r, double* d_z, void* stream);
/* Raw Ritz estimates of instance inst on level l (as pf_get_eig_bounds). */
pf_status pf_batch_get_eig_bounds(pf_batch* b, int level, int inst, double out[4]);
/* Fix the bounds of instance inst on level l (as pf_set_eig_bounds: kept by
 * later pf_batch_set_linearization calls until cleared with in == NULL; the
 * device copy of the Chebyshev coefficients is rewritten at once, with a
 * synchronous copy, when a linearization is set).  Lets the oracle and the
 * batch run V-cycles with identical smoother intervals (Sec. 3.2.1). */
pf_status pf_batch_set_eig_bounds(pf_batch* b, int level, int inst, const double in[4]);
pf_status pf_batch_set_vcycle_precision(pf_batch* b, int prec);
/* Graph replay of the batched V-cycle (default on; see pf_set_graphs).  Its
 * coefficients are read from device memory, so one capture serves every step. */
pf_status pf_batch_set_graphs(pf_batch* b, int enable);
/* Autotuner of the batched Q1 cell loop (the tensor-product apply of Sec. 4.1, for every
 * instance at once).  For every level, precision and operator (mode 0: G~, 1: block B~) it
 * times `reps` applies of each candidate shape and keeps the first within 3% of the fastest:
 *   shape -1  one grid-stride launch over the cells of all instances (each cell finds its
 *             instance by a search of the packed offsets), atomic scatter;
 *   shape  2  a work table of (instance, 64 consecutive cells) items, atomic scatter;
 *   shape  0  a work table of (instance, marching tile) items: 3D 8x8 tiles / 2D 64-cell rows
 *             marching through zc node planes (rows), every node written once;
 *   shape  1  (3D) 16x4 marching tiles.
 * A table item's instance is uniform over its workgroup; the workgroups of one launch loop over
 * the table.  Candidates: -1, 2, 0 with zc = 4, 8, 16, 32, 1 with zc = 4, 8, 16 (Q1 only; the
 * split and Q2 keep shape -1).  Requires pf_batch_set_linearization; overwrites the V-cycle
 * scratch vectors; drops the captured V-cycles; synchronizes. */
pf_status pf_batch_autotune(pf_batch* b, int reps, void* stream);
/* The choice of one (level, prec, mode): shape and zc; us (NULL or 9 doubles): the autotuner's
 * time per apply of each candidate in the order above (-1 where not timed). */
pf_status pf_batch_get_tuning(pf_batch* b, int level, int prec, int mode, int* shape, int* zc, double* us);
/* Force a shape (-1, 0, 1, 2) and chunk for one (level, prec, mode), e.g. to restore cached
 * tuning; PF_ERR_WORKSPACE if its table exceeds the room set aside (chunks below 4). */
pf_status pf_batch_set_tuning(pf_batch* b, int level, int prec, int mode, int shape, int zc);
/* One Newton/active-set step (Algorithm 1) of every instance; reps: n reports
 * (may be NULL).  FGMRES advances all unconverged instances in lockstep and
 * stops each at its own tolerance.  Synchronizes.  PF_ERR_NOT_CONVERGED if any
 * instance hit gmres_max_iter (all reports filled, U updated). */
pf_status pf_batch_newton_step(pf_batch* b, double* d_U, const double* d_U_old, const double* d_phi_tilde,
                               pf_newton_report* reps, void* stream);
void pf_batch_destroy(pf_batch* b);

const char* pf_status_string(pf_status s);
/* Message of the last failed call on this thread ("" if none). */
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PFF_H */
