/*
 * ibschur.h -- C ABI of the MI355X coupled immersed-boundary Schur solver.
 *
 * The library advances the direct-forcing immersed-boundary SIMPLE scheme of
 * Yovel, Treister & Feldman (arXiv 2501.15314) on one GPU.  Its hot path is
 * the per-time-step pressure / force-density correction solve
 *
 *     S~ p' = RHS_p + c^-1 B^T RHS_F,      Phi' = c^-1 (B p' - RHS_F),
 *     S~    = L + c^-1 B^T B,  L = G^T G,  B = -W^T G  (B^T = D W),
 *
 * (paper Sec. 3.1 eq. Saddle; Sec. 4.1 eqs. tildeSp, ApproxSchurPrimalP,
 * ApproxSchurPrimalF), solved by flexible GMRES right-preconditioned by a
 * geometric-multigrid V-cycle approximating L^-1 (Sec. 4.1 uses the Laplacian
 * as the preconditioner, Sec. 4.2 solves it directly; Sec. 7 names multigrid
 * as the replacement).
 *
 * Notation.  W is the regularization matrix of Sec. 2.3 (the paper's R) with
 * dimensionless weights w_ik = phi(dx/h) phi(dy/h) phi(dz/h); W^T is the
 * interpolation.  Phi_k is the force unknown of point k, so that the force on
 * the grid is W Phi; the physical force of point k is h^3 Phi_k.  c is the
 * scalar of the lumping W^T W ~ c I (the paper's 1/2, Sec. 4.1).
 *
 * Layouts (all float64 unless stated):
 *   grid field       [n0][n1][n2], axis 2 contiguous; cell (i,j,k) is centred
 *                    at ((i+1/2)h, (j+1/2)h, (k+1/2)h)
 *   velocity comp d  [n0][n1][n2]; index (i,j,k) is the face of cell (i,j,k)
 *                    lower along axis d; on a wall axis d (either kind) the
 *                    index-0 face is the wall and always holds 0 (the far
 *                    wall is implicit)
 *   face field       [3][n0][n1][n2] (components u, v, w one after another)
 *   point arrays     [K][3], bodies one after another in sim_set_bodies order
 *
 * Ownership.  The caller owns every buffer.  The library allocates no device
 * memory: sim_create carves all of its state out of the caller's device
 * workspace (sim_workspace_bytes), and it never frees caller memory.  A "d_"
 * pointer is a device pointer on cfg.device; other pointers are host memory.
 * Every call enqueues its work on cfg.stream (a hipStream_t; NULL = the null
 * stream) and returns after that stream has drained, so outputs are ready.
 *
 * Errors.  Calls return a sim_status (negative on failure) and never abort or
 * throw across the ABI; sim_last_error gives a per-handle message.  On
 * SIM_ENOTCONV the best iterate and the statistics are still written.
 * Handles are thread-compatible: use one handle per host thread.
 */
#ifndef IBSCHUR_H
#define IBSCHUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sim_s *sim_t;

typedef enum {
  SIM_OK = 0,
  SIM_EINVAL = -1,      /* invalid argument or configuration */
  SIM_ESTATE = -2,      /* call out of order (e.g. no bodies set) */
  SIM_ENOTCONV = -3,    /* Krylov / outer loop hit its iteration limit */
  SIM_ENONFINITE = -4,  /* NaN or Inf met in a Krylov norm */
  SIM_EDEVICE = -5,     /* HIP runtime error */
  SIM_ENOMEM = -6       /* workspace too small */
} sim_status;

/* Boundary condition per axis.  Both wall kinds hold zero normal velocity
 * and give the pressure Laplacian a Neumann end.  NOSLIP: zero tangential
 * velocity at the wall (ghost value -u half a cell beyond it).  FREESLIP:
 * zero normal derivative of the tangential velocity (ghost value +u), the
 * box condition of the sedimentation runs of Sec. 6.1.3. */
enum { SIM_BC_PERIODIC = 0, SIM_BC_NOSLIP = 1, SIM_BC_FREESLIP = 2 };
enum { SIM_DELTA_PESKIN4 = 0, SIM_DELTA_ROMA3 = 1 };
/* FP64: every kernel in float64.  FP32MG: the V-cycle and the momentum
 * relaxations run in float32 inside float64 outer iterations; with FGMRES the
 * Krylov basis V, the preconditioned vectors Z and the products w = S~ z are
 * also stored in float32 (the Gram-Schmidt products, updates and norms are
 * float64 arithmetic on them; the coupling term c^-1 G^T W W^T G z of w is
 * float32 arithmetic), and each cycle restarts from the float64 true residual
 * once it has gained a factor 3e-6.  The result is checked in float64: at the
 * 256^3 benchmark size and krylov_rtol 3e-9 p' and Phi' are within 3e-9 of
 * an exact solution.  With BiCGStab the Krylov vectors and S~ products are
 * float64 in both precisions. */
enum { SIM_PREC_FP64 = 0, SIM_PREC_FP32MG = 1 };
enum { SIM_MOTION_PRESCRIBED = 0, SIM_MOTION_FREE = 1 };
/* VCYCLE: one geometric-multigrid V-cycle approximating L^+ (mg_* fields).
 * FASTDIAG: L^+ by fast diagonalisation of the whole grid (the direct method
 * of paper Sec. 4.2): six batched eigenbasis transforms on the matrix cores
 * with bfloat16 operands and float32 accumulation; every n[d] a multiple of
 * 8, at most 512 (else sim_create returns SIM_EINVAL).  It builds no
 * multigrid hierarchy, so the mg_* fields and their size rules do not apply. */
/* FASTDIAG_EXACT: the same L^+ exactly, with the eigenbasis transforms in
 * float64 (six dense mode products on the vector units, 12 n N flops per
 * application): the paper's exact direct solve for its solver variant
 * (BiCGStab to 1e-12, Sec. 4.2 and Sec. 6.2).  Needs precision FP64 (else
 * SIM_EINVAL); any axis sizes; no multigrid hierarchy. */
enum { SIM_PRECOND_VCYCLE = 0, SIM_PRECOND_FASTDIAG = 1, SIM_PRECOND_FASTDIAG_EXACT = 2 };
/* FGMRES: flexible GMRES(krylov_restart) with classical Gram-Schmidt.
 * BICGSTAB: right-preconditioned BiCGStab (the Krylov method the paper pairs
 * with the Laplacian preconditioner, Sec. 4.2): two preconditioner and two
 * operator applications per iteration, vectors in float64 in both
 * precisions, the preconditioner in the precision of `precision`;
 * krylov_maxit counts iterations.  The reported rel_res is the true residual
 * ||b - S~ p|| / ||b|| at exit. */
enum { SIM_KRYLOV_FGMRES = 0, SIM_KRYLOV_BICGSTAB = 1 };

typedef struct {
  int32_t n[3];          /* cells per axis; multiples of 4, >= 16 */
  double len[3];         /* box size; cells must be cubic: len[d]/n[d] equal */
  int32_t bc[3];         /* SIM_BC_* per axis (both ends) */
  double nu;             /* kinematic viscosity (1/Re in the paper's units) */
  double dt;             /* time step */
  double g[3];           /* gravity, used by SIM_MOTION_FREE bodies only */
  int32_t delta;         /* SIM_DELTA_* */
  double lump_c;         /* c in W^T W ~ c I, > 0 */
  int32_t precision;     /* SIM_PREC_* */
  int32_t krylov_restart;/* FGMRES restart length m, 1..64 */
  int32_t krylov_maxit;  /* total FGMRES iteration cap */
  double krylov_rtol;    /* stop on ||b - S~ p||_2 / ||b||_2 <= rtol */
  int32_t helm_maxit;    /* momentum (A-block) iteration cap */
  double helm_rtol;      /* momentum relative residual target */
  int32_t mg_coarsest;   /* grid-wide V-cycle levels stop above this size */
  int32_t mg_pre, mg_post;     /* red-black Gauss-Seidel sweeps per level */
  int32_t mg_coarse_sweeps;    /* coarsest grid: 0 = exact solve by fast diagonalisation
                                  (one LDS workgroup up to 32 cells per axis and 4096
                                  cells; above that on the matrix cores in bfloat16,
                                  sizes multiples of 8, <= 512), k >= 1 = k V-cycles
                                  of the LDS-resident coarse kernel */
  int32_t precond;       /* SIM_PRECOND_*: preconditioner of the Schur Krylov solve */
  int32_t krylov;        /* SIM_KRYLOV_*: Krylov method of the Schur solve */
  int32_t outer_iters;   /* pressure-force corrections per step (>= 1) */
  double outer_tol;      /* stop on ||Phi'||_1 / ||Phi||_1 < tol (0: fixed) */
  double xi;             /* relaxation of the correction (1 for one-way) */
  int32_t record_two_way;/* != 0: a two-way step keeps, per outer pass, what
                            sim_step_adjoint_two_way needs (outer_iters x (4 cell
                            fields + 3 point vectors) of workspace) */
  int32_t device;        /* HIP device ordinal */
  void *stream;          /* hipStream_t on which all work is enqueued */
} sim_config;

/* A rigid sphere.  Prescribed motion: centre(t) = center + vel t
 * - osc_amp cos(osc_omega t), constant angular velocity omega.  Free motion:
 * center / vel / omega are the state at the current time, advanced by the
 * discrete Newton-Euler equations (paper Sec. 3.2.1) with the body's volume
 * V_p = 4/3 pi radius^3 and moment of inertia 2/5 V_p radius^2 in fluid-density
 * units; the body enters its first step in steady motion (previous velocity
 * levels equal to the current ones, previous centre = center - dt vel) and
 * with orientation R = I.  The bodies of one handle are either all prescribed
 * or all free. */
typedef struct {
  double center[3], vel[3], omega[3];
  double radius;
  double density_ratio;  /* theta = rho_p / rho_f (free bodies) */
  double osc_amp[3];
  double osc_omega;
  int32_t motion;        /* SIM_MOTION_* */
  int32_t n_points;      /* Lagrangian points of this body */
} sim_body;

typedef struct {
  int32_t iters;         /* Krylov (or relaxation) iterations */
  double rel_res;        /* final ||b - A x|| / ||b|| */
  double seconds;        /* device time of the solve */
  int32_t nhist;
  double hist[64];       /* relative residual after each iteration */
} sim_solve_stats;

typedef struct {
  int32_t outer;         /* corrections done in the last step */
  sim_solve_stats helm;  /* momentum solve of the last step */
  sim_solve_stats schur; /* last pressure-force solve */
  double div_rel;        /* ||D u^{n+1}|| / ||D u*|| */
  double slip_rel;       /* ||W^T u^{n+1} - U|| / ||U||  (0 if U = 0) */
  double outer_crit;     /* ||Phi'||_1 / ||Phi||_1 of the last correction */
  double seconds;        /* device time of the last step */
  int32_t total_schur_iters;
} sim_step_stats;

/* Check a configuration on the host (no device work): SIM_OK, or SIM_EINVAL
 * with the first rule it breaks written to msg (NUL-terminated, truncated to
 * msg_len bytes; msg may be NULL).  max_points must lie in 0..2^30. */
sim_status sim_config_check(const sim_config *cfg, int64_t max_points, char *msg, int32_t msg_len);

/* Bytes of device workspace sim_create needs for this configuration and up
 * to max_points Lagrangian points; 0 if the configuration is invalid (see
 * sim_config_check for the reason). */
size_t sim_workspace_bytes(const sim_config *cfg, int64_t max_points);

/* Validate cfg, lay out the state in d_workspace (bytes long, 256-byte
 * aligned) and build the multigrid hierarchy.  Fields start at zero, t = 0.
 * Errors: SIM_EINVAL (non-cubic cells, odd sizes, lump_c <= 0, ...),
 * SIM_ENOMEM (bytes too small), SIM_EDEVICE. */
sim_status sim_create(const sim_config *cfg, void *d_workspace, size_t bytes,
                      int64_t max_points, sim_t *out);

sim_status sim_destroy(sim_t sim);

/* Set nb bodies and their points: offsets (host, [K][3], K = sum of
 * n_points) are the point positions relative to the body centre in the body
 * frame (paper Sec. 2.1, the radius vector L~).  Places the points at the
 * current time (Sec. 2.2: X_k = X_c + R X~_k), computes their velocities
 * (eq. kinematic_constraint) and sorts them into tiles.  SIM_EINVAL if K
 * exceeds max_points or a kernel support crosses a wall (Appendix B). */
sim_status sim_set_bodies(sim_t sim, int32_t nb, const sim_body *bodies,
                          const double *offsets);

/* Copy a time level of the state in: level 0 = t^n (u, v, w, p and, if
 * d_phi is not NULL, Phi [K][3]); level 1 = t^{n-1} (u, v, w only).
 * Wall faces are forced to zero. */
sim_status sim_set_fields(sim_t sim, int32_t level, const double *d_u, const double *d_v,
                          const double *d_w, const double *d_p, const double *d_phi);

/* Copy the state at t^n out (any pointer may be NULL). */
sim_status sim_get_fields(sim_t sim, double *d_u, double *d_v, double *d_w, double *d_p);

/* Advance nsteps time steps.  Prescribed bodies (paper Sec. 3.1): momentum
 * predictor (eq. ustar), then outer_iters pressure-force corrections.  Free
 * bodies (Sec. 3.2.1): Step 1 predicts centres and orientations, Step 2 is the
 * momentum predictor, Step 3 repeats {per-body force, torque and volume
 * integrals of the fluid velocity (eq. volume_integrals) -> Newton-Euler on
 * the host (eqs. bdy_linear_vel_iter, bdy_angular_vel_iter) -> point
 * velocities -> pressure-force correction relaxed by xi} outer_iters times or
 * until ||Phi'||_1 / ||Phi||_1 < outer_tol (eq. convergence_criterion).
 * Errors: SIM_EINVAL if a kernel support would cross a wall,
 * SIM_ENONFINITE, SIM_ENOTCONV (the step is still completed).  stats (may be
 * NULL) describe the last step. */
sim_status sim_step(sim_t sim, int32_t nsteps, sim_step_stats *stats);

/* One pressure-force correction solve on caller data at the current point
 * positions: d_rhs_p [n0][n1][n2] (its mean is discarded: the system is
 * singular on constants), d_rhs_f [K][3]; outputs d_p (mean zero) and
 * d_phi [K][3].  This is the unit of the throughput metric. */
sim_status sim_solve_schur(sim_t sim, const double *d_rhs_p, const double *d_rhs_f,
                           double *d_p, double *d_phi, sim_solve_stats *stats);

/* sim_solve_schur for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, arguments, results and errors, bit for bit, but the
 * solve's work arrays (staged right-hand sides, Krylov basis and
 * preconditioned vectors, BiCGStab vectors, multigrid levels below the
 * finest, fast-diagonalisation work grids, reduction partials) live in a
 * static device array of 64 MiB that the library holds on each device for
 * the life of the process, instead of in the handle's workspace.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * The handle's state (points, tiles, touch lists, eigenbases) still comes
 * from its workspace.  64 MiB covers e.g. a 64^3 grid in the FP32MG form or
 * a 48^3 grid in FP64 with krylov_restart 20; a configuration whose solve
 * needs more returns SIM_EINVAL with the byte count in sim_last_error.
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (from any handle, thread or stream) race and must be
 * serialised by the caller.  Nothing in the array needs to be zero at the
 * start of a call. */
sim_status sim_solve_schur_noalloc(sim_t sim, const double *d_rhs_p, const double *d_rhs_f,
                                   double *d_p, double *d_phi, sim_solve_stats *stats);

/* Forces of the last step: d_f [K][3] = h^3 Phi_k (may be NULL) and, per
 * body, body_ft [nb][6] = (h^3 sum Phi, h^3 sum L~ x Phi) on the host. */
sim_status sim_get_forces(sim_t sim, double *d_f, double *body_ft);

/* Current point positions and velocities, [K][3] each (either may be NULL). */
sim_status sim_get_points(sim_t sim, double *d_X, double *d_U);

/* Set the current time t^n (prescribed kinematics are evaluated at t^n and
 * t^{n+1} = t^n + dt; free-body states are unaffected). */
sim_status sim_set_time(sim_t sim, double t);

/* Rigid-body state at the current time, host array [nb][18] in body order:
 * centre X_c (0..2), velocity u_s (3..5), angular velocity omega in the
 * inertial frame (6..8), orientation R row-major (9..17; maps body-frame
 * offsets to inertial ones, Sec. 2.2).  Prescribed bodies report their
 * prescribed kinematics.  SIM_ESTATE without bodies. */
sim_status sim_get_body_state(sim_t sim, double *state);

/* Reverse-mode derivative (vector-Jacobian product) of the last time step,
 * which must be a one-way step (prescribed bodies) with one correction; any
 * other call that changes the state in between (sim_set_*, sim_solve_schur,
 * sim_apply, a two-way step) makes this SIM_ESTATE.  The transposed sequence
 * runs the update, force recovery (eq. ApproxSchurPrimalF), Schur solve (S~ is
 * symmetric: same FGMRES), right-hand side (eq. ApproxSchurPrimalP) and
 * momentum solve (A symmetric) backwards, plus the derivatives of W with
 * respect to the point positions (Sec. 2.3 kernels) and of the convection
 * term.  Inputs: cotangents of u^{n+1} (d_gu, d_gv, d_gw, natural face
 * layout), p^{n+1} (d_gp) and Phi^{n+1} (d_gphi, [K][3]); NULL means zero.
 * Outputs (NULL = not wanted): d_gX [K][3] = dl/dX_k at the step's point
 * positions; gU (host, [nb][6]) = (dl/du_s, dl/domega) of each body through
 * the point velocities U_k = u_s + omega x L~_k; the cotangents of the step's
 * inputs d_gu_in ([3][n0][n1][n2], u^n), d_gum_in (u^{n-1}), d_gp_in (p^n),
 * d_gphi_in ([K][3], Phi^n).  The state of the step is left unchanged, so the
 * call may be repeated with other cotangents.  SIM_ENOTCONV if a transposed
 * solve hit its iteration limit (outputs still written). */
sim_status sim_step_adjoint(sim_t sim, const double *d_gu, const double *d_gv,
                            const double *d_gw, const double *d_gp, const double *d_gphi,
                            double *d_gX, double *gU, double *d_gu_in, double *d_gum_in,
                            double *d_gp_in, double *d_gphi_in);

/* Reverse mode of the last two-way step (free bodies, Sec. 3.2.1): the
 * vector-Jacobian product of the step with its fixed number of outer passes.
 * Needs cfg.record_two_way != 0, cfg.outer_tol = 0 and a sim_step that ran
 * exactly one two-way step since the last state change (else SIM_ESTATE).
 * Output cotangents: d_gu, d_gv, d_gw, d_gp ([n0][n1][n2], device), d_gphi
 * ([K][3], device) for u^{n+1}, p^{n+1}, Phi^{n+1}; gbody_out (host,
 * [nb][15]) for each body's X_c^{n+1}, u_s^{n+1}, omega^{n+1} and the volume
 * integrals sum alpha u h^3, sum alpha r x u h^3 of u^{n+1} at X_c^{n+1}
 * (the next step's history).  Any may be NULL (zero).
 * Input cotangents (any may be NULL): d_gu_in, d_gum_in ([3][n0][n1][n2]) of
 * u^n, u^{n-1}; d_gp_in of p^n; d_gphi_in ([K][3]) of Phi^n; gbody_in (host,
 * [nb][30]) of each body's X_c^n, X_c^{n-1}, u_s^n, u_s^{n-1}, omega^n,
 * omega^{n-1} and of the volume-integral history I^n, I^{n-1}, J^n, J^{n-1}.
 * The orientation R^n is held fixed.  The transposed Schur and momentum solves
 * use the step's solvers and tolerances; SIM_ENOTCONV if one misses it (the
 * result is still written). */
sim_status sim_step_adjoint_two_way(sim_t sim, const double *d_gu, const double *d_gv,
                                    const double *d_gw, const double *d_gp, const double *d_gphi,
                                    const double *gbody_out, double *d_gu_in, double *d_gum_in,
                                    double *d_gp_in, double *d_gphi_in, double *gbody_in);

/* Operator applications on caller data (natural layouts above), for
 * operator-level checks.  in / out sizes follow the operator:
 *   SIM_OP_LAPLACIAN     cells -> cells      L = G^T G
 *   SIM_OP_SCHUR         cells -> cells      S~ = L + c^-1 B^T B
 *   SIM_OP_PRECOND       cells -> cells      one V-cycle, M^-1 ~ L^+
 *   SIM_OP_GRAD          cells -> faces      G
 *   SIM_OP_DIV           faces -> cells      D = -G^T
 *   SIM_OP_INTERP        faces -> points     W^T
 *   SIM_OP_SPREAD        points -> faces     W
 *   SIM_OP_HELMHOLTZ     faces -> faces      A = 3/(2dt) - nu Delta_h
 *   SIM_OP_CONVECTION    faces -> faces      div(u u)
 *   SIM_OP_HELM_SOLVE    faces -> faces      A^-1 (to helm_rtol)
 *   SIM_OP_SCHUR_RHS     cells+points -> cells  b = RHS_p + c^-1 D W RHS_F
 *   SIM_OP_SCHUR_EXACT   cells -> cells      S_p = L + B^T (W^T W)^-1 B, the primal Schur
 *                        complement before lumping (paper Sec. 4.1; the operator of the
 *                        spectral theorem of Sec. 5), (W^T W)^-1 by conjugate gradients
 *                        on the device to 1e-13 within 2000 iterations (else SIM_ENOTCONV)
 *                        (in = rhs_p, in2 = rhs_f)
 * Precision follows cfg.precision where the operator has a mixed form. */
enum {
  SIM_OP_LAPLACIAN = 0, SIM_OP_SCHUR = 1, SIM_OP_PRECOND = 2, SIM_OP_GRAD = 3,
  SIM_OP_DIV = 4, SIM_OP_INTERP = 5, SIM_OP_SPREAD = 6, SIM_OP_HELMHOLTZ = 7,
  SIM_OP_CONVECTION = 8, SIM_OP_HELM_SOLVE = 9, SIM_OP_SCHUR_RHS = 10, SIM_OP_SCHUR_EXACT = 11
};
sim_status sim_apply(sim_t sim, int32_t op, const double *d_in, const double *d_in2,
                     double *d_out);

/* Spectrum of the Laplacian-preconditioned Schur operator L^+ S on mean-free
 * pressures for the current point set: S = S~ = L + c^-1 B^T B (exact = 0,
 * the lumped operator the Krylov solve inverts, Sec. 4.1) or the primal
 * Schur complement S_p = L + B^T (W^T W)^-1 B (exact != 0, as in
 * SIM_OP_SCHUR_EXACT).  The theorem of Sec. 5 bounds spec(L^+ S_p) by
 * [1, 2]; Sec. 6.2 measures the extremes for both operators.
 * Method: Lanczos on the pencil (S, L) in the L inner product, `steps`
 * steps (1..1024) from the start vector d_v0 ([n0][n1][n2] on the device,
 * not modified; its mean is removed).  Each step applies S once and solves
 * L w = S v by flexible conjugate gradients preconditioned with the
 * configured preconditioner to relative residual lap_rtol (0 < lap_rtol < 1).
 * Outputs (host, any may be NULL): alpha[steps] and beta[steps], the
 * tridiagonal Lanczos matrix T (beta[0] = L-norm of the mean-free start
 * vector, beta[j] couples rows j-1 and j); *steps_done, the order of T (less
 * than steps if an invariant subspace was found); *lmin, *lmax, the extreme
 * eigenvalues of T, which lie inside the extremes of spec(L^+ S) and
 * approach them as the step count grows.
 * Uses the solver's work fields only (the state u, p, Phi is kept) and
 * invalidates the record of sim_step_adjoint.  Errors: SIM_ESTATE without
 * bodies; SIM_EINVAL for bad arguments or a start vector without mean-free
 * part; SIM_ENOTCONV if an inner solve (the Laplacian, or W^T W for the
 * exact operator) misses its tolerance; SIM_ENONFINITE. */
sim_status sim_schur_spectrum(sim_t sim, int32_t exact, const double *d_v0, int32_t steps,
                              double lap_rtol, double *alpha, double *beta, int32_t *steps_done,
                              double *lmin, double *lmax);

/* Kernel timing probes (a profiling aid, for throughput / roofline reports).
 * While a probe is enabled on a handle, every launch of its kernel class made
 * by that handle is bracketed by HIP events on the launch stream and
 * records its algorithmic bytes (every operand read once, every result
 * written once, from the launch's sizes; the models are stated where the
 * kernels are launched).  sim_probe_read returns the number of probed
 * launches, their summed device time in milliseconds (waiting for the
 * events) and, if bytes is not NULL, their summed algorithmic bytes; with
 * reset != 0 it clears them.  Probe state belongs to the handle.  A
 * multigrid level runs either the plane-march kernels (the first five
 * classes) or, at most 64^3 cells by default, the two tile kernels
 * (IBSCHUR_MG_TILE_CELLS in the environment at sim_create sets that bound;
 * 0: no tile levels). */
enum {
  SIM_PROBE_SMOOTH = 0,             /* red-black Gauss-Seidel half sweep, plane-march levels */
  SIM_PROBE_SMOOTH_FIRST = 1,       /* first sweep from zero, plane-march levels */
  SIM_PROBE_RESTRICT = 2,           /* residual + restriction, plane-march levels */
  SIM_PROBE_PROLONG = 3,            /* prolongation + correction, plane-march levels */
  SIM_PROBE_LAPLACIAN = 4,          /* L z inside the S~ product */
  SIM_PROBE_SPREAD_DIV = 5,         /* D W q on the active tiles */
  SIM_PROBE_SPREAD_FACE = 6,        /* W q on the active tiles */
  SIM_PROBE_INTERP_GRAD = 7,        /* W^T G z */
  SIM_PROBE_INTERP_FACE = 8,        /* W^T u */
  SIM_PROBE_MULTIDOT = 9,           /* Gram-Schmidt dot products */
  SIM_PROBE_UPDATE_NORM = 10,       /* Gram-Schmidt update and norm */
  SIM_PROBE_COARSE = 11,            /* coarsest-grid solve */
  SIM_PROBE_HELM_SWEEP = 12,        /* momentum red-black SOR half sweep */
  SIM_PROBE_HELM_RESID = 13,        /* momentum residual */
  SIM_PROBE_VCYCLE = 14,            /* one whole preconditioner application (all its kernels) */
  SIM_PROBE_MOM_RHS = 15,           /* momentum right-hand side with convection */
  SIM_PROBE_HELM_FIRST = 16,        /* momentum SOR sweep from zero (both colours) */
  SIM_PROBE_TILE_DOWN = 17,         /* tile level: pre-smoothing + residual + restriction */
  SIM_PROBE_TILE_UP = 18,           /* tile level: prolongation + post-smoothing */
  SIM_PROBE_COUNT = 19
};
sim_status sim_probe_enable(sim_t sim, int32_t probe, int32_t on);
sim_status sim_probe_read(sim_t sim, int32_t probe, int64_t *launches, double *ms, double *bytes,
                          int32_t reset);

/* Message of the last failing call on this handle ("" if none). */
const char *sim_last_error(sim_t sim);

#ifdef __cplusplus
}
#endif
#endif /* IBSCHUR_H */
