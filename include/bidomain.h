/*
 * bidomain.h -- C ABI of libbidomain: Newton-Krylov BDDC / FETI-DP deluxe
 * solver for the segregated implicit Bidomain time step on one MI355X.
 *
 * Method: Huynh, Pavarino, Scacchi, "Parallel Newton-Krylov-BDDC and FETI-DP
 * deluxe solvers for implicit time discretizations of the cardiac Bidomain
 * equations" (arXiv:2101.02959).  Section numbers below refer to that paper.
 *
 * Conventions (all calls):
 *   - Return 0 on success or a negative BDM_E_* code; bdm_last_error() gives
 *     a thread-local message for the last failure.  No C++ exception crosses
 *     this interface.
 *   - Global node numbering is lexicographic, x fastest:
 *       node(i,j,k) = i + (nx+1)*(j + (ny+1)*k),  N = (nx+1)(ny+1)(nz+1).
 *     "2N vectors" are blocked [v (N doubles) ; u_e (N doubles)].
 *   - Unknowns are (v, u_e) with v = u_i - u_e.  The library solves the
 *     congruent form T^T (F(T x) - G) = 0 of the paper's Step-2 system
 *     (Sec. 3b), T = [[I, I], [0, I]]: first row is the u_i equation, second
 *     row the sum of the two equations.  The Jacobian is symmetric positive
 *     semidefinite with kernel (v = 0, u_e = const); u_e is gauged to zero
 *     nodal mean.
 *   - Pointers marked "device" must be device memory of the context's GPU;
 *     work is ordered on the context's HIP stream and the call returns after
 *     the stream has been synchronised unless stated otherwise.  The caller
 *     owns every array passed in; the library owns the context and all of its
 *     workspace.
 *   - Unit system: cm, ms, mV, uA/cm^3; sigma in mS/cm; chi in 1/cm;
 *     C_m in uF/cm^2; G, eta_1 in mS/cm^2 (the ionic current per unit volume
 *     is chi * I_ion); eta_2 in 1/ms.
 */
#ifndef BIDOMAIN_H
#define BIDOMAIN_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BDM_OK = 0,
    BDM_E_ARG = -1,              /* invalid argument or unsupported layout   */
    BDM_E_OOM = -2,              /* device allocation failed                 */
    BDM_E_HIP = -3,              /* HIP runtime error                        */
    BDM_E_NOT_SPD = -4,          /* a local, deluxe or coarse factor failed  */
    BDM_E_KRYLOV_DIVERGED = -5,  /* ||r_k|| > dtol ||r_0||                   */
    BDM_E_KRYLOV_MAXIT = -6,     /* Krylov iteration limit reached           */
    BDM_E_NEWTON_MAXIT = -7,     /* Newton iteration limit reached           */
    BDM_E_COERCIVITY = -8,       /* reaction diagonal <= 0 (Sec. 3c lemma)   */
    BDM_E_STATE = -9,            /* call order violated (e.g. no linearize)  */
    BDM_E_LINESEARCH = -10       /* no step along a Newton direction passed  */
                                 /* the Armijo test within 20 trials         */
};

enum { BDM_SOLVER_BDDC = 0, BDM_SOLVER_FETIDP = 1 };
enum { BDM_PREC_FP64 = 0, BDM_PREC_MIXED = 1 };
enum { BDM_GUESS_PREV = 0, BDM_GUESS_EXTRAP = 1, BDM_GUESS_CNN = 2 };
/* Schedule of the batched per-subdomain triangular solves (uneven sizes):
 * QUEUE  one persistent launch per solve whose workgroups draw subdomains
 *        from a device work queue in decreasing factor size (LPT);
 * GRID   one workgroup per subdomain in subdomain order.
 * Both give bitwise identical results. */
enum { BDM_SCHED_QUEUE = 0, BDM_SCHED_GRID = 1 };
enum { BDM_FETI_F = 0, BDM_FETI_PRECOND = 1, BDM_FETI_RHS = 2, BDM_FETI_RECOVER = 3 };
/* Scaling of the dual (face and edge) dofs, Sec. 4.2:
 * DELUXE  u_* = (sum_m S_*^(m))^{-1} sum_m S_*^(m) u_*^(m) per face / edge;
 * RHO     u(x) = sum_j delta_j(x) u^(j)(x), with the pseudoinverse weights
 *         delta_j = sigma_M^(j) / sum_{k in N_x} sigma_M^(k) (sigma_M the
 *         largest principal conductivity, sigma^i for the v dofs and sigma^e
 *         for the u_e dofs); with the same tissue in every subdomain each
 *         weight is 1/|N_x|. */
enum { BDM_SCALING_DELUXE = 0, BDM_SCALING_RHO = 1 };
/* Primal space of BDDC and FETI-DP, Sec. 4.4 and the optimality test of
 * Sec. 6: the (v, u_e) values at the subdomain vertices, plus the averages
 * of v and of u_e over every edge (VE), or over every edge and face (VEF). */
enum { BDM_PRIMAL_VE = 0, BDM_PRIMAL_V = 1, BDM_PRIMAL_VEF = 2 };

/* Structured hexahedral Q1 mesh of nx*ny*nz box elements of size
 * h x hy x hz (Sec. 3a; hy <= 0 or hz <= 0 means h, i.e. cubes of side h)
 * and a tensor-product partition into non-overlapping box subdomains
 * (Sec. 4.1): cuts_x[0..px] are element indices with cuts_x[0] = 0,
 * cuts_x[px] = nx, strictly increasing; likewise y, z.  px, py, pz >= 2
 * (every subdomain must touch an interior cross point: every primal space
 * holds the vertex values).
 *
 * geometry = BDM_GEOM_ELLIPSOID maps the same logical grid onto the truncated
 * ellipsoid of Sec. 6, x = a(r) cos(theta) cos(phi), y = b(r) cos(theta)
 * sin(phi), z = c(r) sin(theta) (the printed z-component's sin(phi) read as
 * sin(theta)), with a(r) = a1 + r (a2 - a1) and likewise b, c; ellipsoid[] =
 * {a1, a2, b1, b2, c1, c2, theta_min, theta_max, phi_min, phi_max} (cm,
 * rad).  Node (i, j, k) sits at phi = phi_min + i (phi_max - phi_min) / nx,
 * theta = theta_min + j (theta_max - theta_min) / ny, r = k / nz.  Required:
 * 0 < a1 < a2, 0 < b1 < b2, 0 < c1 < c2, -pi/2 < theta_min < theta_max <
 * pi/2, phi_min < phi_max <= phi_min + 2 pi; else BDM_E_ARG.  Elements are
 * isoparametric Q1 (2x2x2 Gauss); the tensor of an element is that of
 * bdm_physics in the orthonormal frame at its parametric centre (e1 along
 * dX/dphi, e2 along dX/dtheta made orthogonal to e1, n = e1 x e2), with the
 * fibre angle at the centre's depth r.  h, hy and hz are unused. */
enum { BDM_GEOM_BOX = 0, BDM_GEOM_ELLIPSOID = 1 };
typedef struct bdm_mesh {
    int nx, ny, nz;
    double h;                   /* element size along x (cm)                 */
    int px, py, pz;
    const int* cuts_x;
    const int* cuts_y;
    const int* cuts_z;
    double hy, hz;              /* element sizes along y and z (cm; <= 0: h) */
    int geometry;               /* BDM_GEOM_*                                */
    double ellipsoid[10];       /* BDM_GEOM_ELLIPSOID parameters, see above  */
} bdm_mesh;

/* Conductivities along (l, t, n) (Sec. 2, D = sum sigma a a^T), fibre angle
 * rotating linearly in the xy-plane from theta0 at z = 0 to theta1 at the top,
 * evaluated at element centroids; Rogers-McCulloch parameters (Sec. 2). */
typedef struct bdm_physics {
    double sigma_i[3];
    double sigma_e[3];
    double theta0, theta1;
    double chi, Cm;
    double G, eta1, eta2, vth, vp;
} bdm_physics;

/* Time step and solver options (Sec. 3b-c, Sec. 6 tolerances). */
typedef struct bdm_opts {
    double dt;                  /* tau (ms)                                  */
    double newton_rtol;         /* stop: ||R(u^k)|| <= rtol ||R(u^n)||       */
    double newton_atol;         /*   or  ||R(u^k)|| <= atol                  */
    int newton_maxit;
    double krylov_rtol;         /* ||r_k||_2 <= rtol ||b||_2, b the Newton   */
                                /* right-hand side (BDDC), or the multiplier */
                                /* system's right-hand side (FETI-DP)        */
    double krylov_dtol;         /* divergence when ||r_k|| > dtol ||b||      */
    int krylov_maxit;
    int solver;                 /* BDM_SOLVER_*                              */
    int precision;              /* BDM_PREC_*: local factors in FP64 or FP32 */
    int guess;                  /* BDM_GUESS_*                               */
    int krylov_graph;           /* 1: each PCG iteration replays captured    */
                                /* HIP graphs (operator half, then the       */
                                /* preconditioner half while running) with   */
                                /* device scalars, same arithmetic and       */
                                /* iterates; 0: host-driven loop             */
    int schedule;               /* BDM_SCHED_*                               */
    int krylov_reduced;         /* BDDC only.  1: each Newton solve first    */
                                /* solves the subdomain interiors of its     */
                                /* right-hand side exactly (zero on the      */
                                /* interface, Sec. 4.1), so every PCG        */
                                /* residual vanishes on the interiors and    */
                                /* the preconditioner skips its condensation */
                                /* of r_I; the stopping test stays relative  */
                                /* to ||b||.  0: PCG on J s = b from zero.   */
                                /* Must be 0 or 1 (BDM_E_ARG otherwise).     */
    int scaling;                /* BDM_SCALING_* (BDM_E_ARG otherwise)       */
    int primal;                 /* BDM_PRIMAL_* (BDM_E_ARG otherwise)        */
} bdm_opts;

/* Per-step statistics filled by bdm_step (for its last step). */
typedef struct bdm_step_stats {
    int newton_its;
    int krylov_its[32];         /* per Newton iteration                      */
    double res_hist[33];        /* ||R|| before each Newton iteration        */
    double cond[32];            /* Lanczos estimate per Krylov solve         */
    double t_setup_ms;          /* preconditioner setup time (all Newton its)*/
    double t_krylov_ms;         /* Krylov loop time                          */
    double t_step_ms;           /* whole step                                */
    int bad_subdomain;          /* first subdomain whose factor failed or -1 */
    int guess_used;             /* 0 u^n, 1 extrapolation, 2 learned guess   */
    double guess_res_extrap;    /* ||R|| of the extrapolated guess (or -1)   */
    double guess_res_cnn;       /* ||R|| of the learned guess (or -1)        */
    double res_ref;             /* ||R(u^n)||, the reference of newton_rtol  */
    double krylov_true_res[32]; /* per Newton iteration: ||b - J s|| / ||b||  */
                                /* of the linear solve, recomputed in FP64   */
                                /* on the full system after the solve (the   */
                                /* error of the result under FP32 local      */
                                /* factors; b is the projected -R)           */
    double step_length[32];     /* per Newton iteration: the accepted step   */
                                /* length of the line search (1 = full       */
                                /* Newton step; Sec. 6 backtracking)         */
} bdm_step_stats;

typedef struct bdm_ctx bdm_ctx;

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (NULL = default stream).  Builds the partition, the N_x classification
 * into faces / edges / vertices (Sec. 4.1), index maps and element
 * matrices, and allocates all device workspace.  The state is set to rest
 * (v = u_e = w = 0), no stimulus. */
int bdm_create(const bdm_mesh* mesh, const bdm_physics* phys, const bdm_opts* opts,
               void* hip_stream, bdm_ctx** out);

/* Free every device allocation owned by the context. */
int bdm_destroy(bdm_ctx* ctx);

/* Copy the state (v, u_e, w: N doubles each, host or device pointers per
 * on_device) into / out of the context.  u_e is gauged to zero mean on input.
 * bdm_set_state starts a new trajectory: the previous-step history used for
 * extrapolated guesses is reset, and so is the step counter n that the
 * stimulus window of bdm_set_stimulus refers to (the next bdm_step takes
 * step n = 0). */
int bdm_set_state(bdm_ctx* ctx, const double* v, const double* ue, const double* w,
                  double t, int on_device);
int bdm_get_state(bdm_ctx* ctx, double* v, double* ue, double* w, double* t, int on_device);

/* Nodal transmembrane stimulus I_s (N doubles, uA/cm^3; host or device per
 * on_device), applied in the steps n with step_on <= n < step_off, evaluated
 * at t_{n+1}: it enters the first residual row as -tau * M * I_s. */
int bdm_set_stimulus(bdm_ctx* ctx, const double* Is, int step_on, int step_off, int on_device);

/* Step 1 of the decoupled scheme (Sec. 3b): w <- (w + tau eta_2 v / v_p) /
 * (1 + tau eta_2), the exact solution of w - tau R(v^n, w) = w^n. */
int bdm_ionic_update(bdm_ctx* ctx);

/* Residual R(v, u_e) of Step 2 (Sec. 3b) at the given iterate (device, N
 * each) with v^n, w^{n+1} and the stimulus taken from the context's state.
 * Outputs Rv, Re (device, N each). */
int bdm_residual(bdm_ctx* ctx, const double* v, const double* ue, double* Rv, double* Re);

/* Build the Jacobian (Sec. 3c) at (v_lin, w_lin) (device, N each) and every
 * preconditioner factor: local Dirichlet factors of K_II, local Schur
 * complements, constrained Neumann factors with the average constraints of
 * the primal space (opts.primal), the coarse basis and coarse matrix
 * (Sec. 4.4), and the face / edge scaling matrices (Sec. 4.2: deluxe
 * factors, or the rho weights).  Returns BDM_E_COERCIVITY if a reaction
 * diagonal is not positive and BDM_E_NOT_SPD if a factorisation fails. */
int bdm_linearize(bdm_ctx* ctx, const double* v_lin, const double* w_lin);

/* y = J x for 2N device vectors (matrix-free Q1 stencils, Sec. 3a-c). */
int bdm_jacobian_apply(bdm_ctx* ctx, const double* x, double* y);

/* z = M^{-1}_BDDC r on the full system (2N device vectors) at the last
 * linearisation (Sec. 4.4 with static condensation, Sec. 4.1): interior
 * Dirichlet correction, deluxe E_D^T, constrained local Neumann solves plus
 * coarse solve, deluxe E_D, discrete harmonic extension.  z is defined up to
 * the kernel (v = 0, u_e = const). */
int bdm_bddc_apply(bdm_ctx* ctx, const double* r, double* z);

/* Number of FETI-DP multipliers: one per face dof and one per dof and per
 * pair of subdomains sharing an edge (fully redundant), Sec. 4.3. */
int bdm_fetidp_size(bdm_ctx* ctx, long* n_lambda);

/* FETI-DP operators at the last linearisation (Sec. 4.3), device pointers:
 *   BDM_FETI_F        in = lambda (n_lambda), out = F lambda = B S~^{-1} B^T lambda
 *   BDM_FETI_PRECOND  in = lambda, out = B_D S_Gamma B_D^T lambda
 *   BDM_FETI_RHS      in = r (2N), out = d = B S~^{-1} f~ (n_lambda), where f~
 *                     is the interior-condensed residual split 1/|N_x|
 *   BDM_FETI_RECOVER  in = [r (2N) ; lambda (n_lambda)], out = z (2N):
 *                     w = S~^{-1}(f~ - B^T lambda), z_I by a Dirichlet solve */
int bdm_fetidp_apply(bdm_ctx* ctx, int op, const double* in, double* out);

/* Advance nsteps time steps: Step 1 then Newton with PCG preconditioned by
 * BDDC, or FETI-DP PCG on the multipliers plus recovery, per opts.solver.
 * Globalisation (Sec. 6, cubic backtracking): with f = ||R||^2 / 2 and
 * f'(0) = -||R||^2 along the Newton direction s, the step u + l s is
 * accepted when f(l) <= f(0) + 1e-4 l f'(0); the full step l = 1 is tried
 * first, then the minimiser of the quadratic model through f(0), f'(0),
 * f(l), then of the cubic model through f(0), f'(0) and the last two
 * trials, each new l clamped to [0.1, 0.5] of the previous; a trial whose
 * f is not finite halves l.  BDM_E_LINESEARCH after 20 failed trials.
 * stats may be NULL.
 * BDM_E_ARG for FETI-DP with FP32 local factors: the multiplier operator
 * B S~^{-1} B^T contains the local solves, and their FP32 round-off makes it
 * indefinite at scale (PCG breaks down); BDDC keeps the FP64 Jacobian as
 * its operator and takes FP32 factors in the preconditioner only.  The
 * FETI-DP operators themselves (bdm_fetidp_apply) work in either precision. */
int bdm_step(bdm_ctx* ctx, int nsteps, bdm_step_stats* stats);

/* Learned Newton initial guess (an addition to the paper's method: it only
 * changes the starting point of Newton; the tolerance and hence the converged
 * solution are unchanged).  A 3-D CNN on the node grid, four 3x3x3 zero-padded
 * convolutions with channels 4 -> 16 -> 16 -> 16 -> 2 and GELU after the first
 * three, FP16 weights and activations with FP32 accumulation.  Inputs
 * (v^n/s_v, u_e^n/s_e, (v^n - v^{n-1})/s_dv, (u_e^n - u_e^{n-1})/s_de); output
 * y; the guess is
 *   u^{(0)} = u^n + (u^n - u^{n-1}) + (s_yv y_0, s_ye y_1).
 * Parameters: one float vector, layer by layer, weights [Cout][Cin][27] (tap
 * dx + 3 dy + 9 dz) then biases; scales = {s_v, s_e, s_dv, s_de, s_yv, s_ye},
 * all positive (host, 6 doubles).
 * With opts.guess = BDM_GUESS_CNN, bdm_step evaluates the residual of the
 * learned and of the extrapolated guess and starts Newton from the smaller
 * (without weights it behaves as BDM_GUESS_EXTRAP).
 * The first bdm_predictor_set allocates the network's device buffers (about
 * 340 N bytes); set resets the Adam moments.  Errors: BDM_E_ARG for a
 * non-positive scale, learning rate or an order index outside [0, nsamples);
 * BDM_E_STATE for guess, loss_grad, train or get before weights were set;
 * BDM_E_OOM when the buffers cannot be allocated. */
long bdm_predictor_size(void);
int bdm_predictor_set(bdm_ctx* ctx, const float* params, const double* scales);   /* host */
int bdm_predictor_get(bdm_ctx* ctx, float* params, double* scales);               /* host */
/* guess (device, 2N) from v^n, u_e^n, v^{n-1}, u_e^{n-1} (device, N each) */
int bdm_predictor_guess(bdm_ctx* ctx, const double* vn, const double* uen, const double* vprev,
                        const double* ueprev, double* guess);
/* Mean-squared loss of one sample (device, 6N: v^n, u_e^n, v^{n-1}, u_e^{n-1},
 * v^{n+1}, u_e^{n+1}) against the target ((u^{n+1}-u^n)-(u^n-u^{n-1}))/s_y and
 * its gradient (host, bdm_predictor_size() floats). */
int bdm_predictor_loss_grad(bdm_ctx* ctx, const double* sample, float* grad, double* loss);
/* Adam (beta 0.9, 0.999, eps 1e-8, learning rate lr) over nsteps samples
 * samples + order[t] * 6N (device), losses (host, nsteps) before each update. */
int bdm_predictor_train(bdm_ctx* ctx, const double* samples, int nsamples, const int* order, int nsteps,
                        double lr, double* losses);

/* Kernel timing for roofline reports.  At the last linearisation, launches
 * one hot kernel reps times on the context stream, bracketed by HIP events,
 * and returns the mean duration of one launch in avg_ms and the kernel's
 * algorithmic work per launch in work (bytes for the bandwidth-bound kernels,
 * floating-point operations for the factorisation kernels):
 *   BDM_KERNEL_JACOBIAN         y = J x on 2N vectors; bytes = 40 N (read v,
 *                               u_e, reaction diagonal; write both outputs)
 *   BDM_KERNEL_TRSV_DIRICHLET   one forward Dirichlet solve L_II y = b over
 *                               all subdomains; bytes = lower triangles +
 *                               vectors
 *   BDM_KERNEL_TRSV_DIRICHLET_T the backward solve L_II^T x = y, same bytes
 *   BDM_KERNEL_POTRF_INTERIOR   the panel kernels of the interior elimination
 *                               (partial Cholesky through the interior
 *                               columns, right looking in 128-column panels,
 *                               Sec. 4.1) on the first setup chunk: the
 *                               diagonal-block factor and the row-block TRSM;
 *                               flops = divisions plus 2 per entry updated
 *                               inside the panels
 *   BDM_KERNEL_SYRK_UPDATE      the batched rank-k update kernel of the same
 *                               elimination: the trailing updates right of
 *                               each panel and the Schur update S_Gamma =
 *                               K_GG - L_GI L_GI^T; flops = 2 per updated
 *                               entry per inner index (lower triangles only)
 * For the last two, work and time are averaged over the kernel's launches in
 * one elimination (the launches differ in size); the local matrices of the
 * chunk are reassembled before each elimination (untimed).  The
 * preconditioner factors are left intact.  BDM_E_ARG for another id. */
enum {
    BDM_KERNEL_JACOBIAN = 0,
    BDM_KERNEL_TRSV_DIRICHLET = 1,
    BDM_KERNEL_POTRF_INTERIOR = 2,
    BDM_KERNEL_SYRK_UPDATE = 3,
    BDM_KERNEL_TRSV_DIRICHLET_T = 4
};
int bdm_profile_kernel(bdm_ctx* ctx, int kernel, int reps, double* avg_ms, double* work);

/* Autotuned kernel variants of the context (not part of the paper's method;
 * every variant computes the same operator).  Tuned families:
 *   "stencil"  tile shape of the fused 27-point stencil kernel, per mesh,
 *              chosen at bdm_create by timing the Jacobian apply;
 *   "syrk"     output tile and inner chunk of the batched rank-k update of
 *              the interior and r-block eliminations, per size class,
 *              chosen at the first bdm_linearize by timing the first setup
 *              chunk's updates (before its assembly).
 * If the environment variable BDM_TUNE_CACHE names a file, bdm_create reads
 * earlier results from it (JSON; a missing file is created) and new results
 * are written back, so a later context on the same device and sizes reuses
 * them without timing; an unreadable cache is BDM_E_ARG at bdm_create.
 * bdm_tune_report writes the JSON of the entries this context used (device,
 * family, size class, choice, time per variant in ms, cached flag) into the
 * caller's buffer buf of cap bytes, NUL-terminated, and sets *len to the
 * length without the NUL; if cap <= *len nothing is written and BDM_E_ARG is
 * returned, so a caller can size its buffer from *len. */
int bdm_tune_report(bdm_ctx* ctx, char* buf, long cap, long* len);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of bdm_residual without a context and without any device
 * allocation.  Inputs (device, N doubles each): the iterate v, u_e, the
 * previous potential v^n, the gating variable w^{n+1} and, when stim_on is
 * nonzero, the nodal stimulus Is (it may be NULL otherwise); outputs Rv, Re
 * (device, N each); mesh and physics as for bdm_create (the partition
 * arrays are not read) and the time step dt.  Work runs on hip_stream (a
 * hipStream_t, NULL = default) and the call returns after synchronising
 * it.  The coefficient tables the kernels read live in a static device
 * array of about 4 MB per GPU, held until the process ends: nz + 1 must not
 * exceed 1024 (BDM_E_ARG otherwise).  Calls on one GPU share that array and
 * are serialised by a host mutex; device work enqueued concurrently by
 * other code is not ordered against a call.  Box meshes only
 * (geometry = BDM_GEOM_BOX).  BDM_E_ARG for a null argument, another
 * geometry, or non-positive sizes, h or dt; BDM_E_HIP for a runtime
 * error. */
int bdm_residual_noalloc(const bdm_mesh* mesh, const bdm_physics* phys, double dt, const double* v,
                         const double* ue, const double* vn, const double* w, const double* Is, int stim_on,
                         double* Rv, double* Re, void* hip_stream);

/* Sizes for callers that allocate vectors: N, number of subdomains, global
 * primal (coarse) dimension. */
int bdm_sizes(bdm_ctx* ctx, long* n_nodes, long* n_sub, long* n_primal);

/* Thread-local message describing the last error ("" if none). */
const char* bdm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIDOMAIN_H */
