/*
 * jfnk.h — C ABI of the MI355X (gfx950) Jacobian-free Newton-Krylov hot path.
 *
 * Method (Pasquale & Markidis, "Robust Matrix-Free Newton-Krylov Solvers via
 * Automatic Differentiation"):
 *   - the discrete residual F(x^k, x*) of a PDE after space and time
 *     discretization (paper, Section 2; Appendix A);
 *   - the Newton step J(x^k) dx = -F(x^k), solved by restarted GMRES that sees
 *     J only through Jacobian-vector products (Section 2; Section 3.1);
 *   - the JVP either by forward-mode AD (value + tangent carried together
 *     through the residual, the paper's AD jvp pair) or by finite differences
 *     (F(x + eps v) - F(x)) / eps with eps from the paper's step-size rule;
 *   - the stopping test ||F(x^k)|| / ||F(x*)|| < tol_Newton and a backtracking
 *     line search x^{k+1} = x^k + alpha dx (Section 2).
 *
 * Everything runs on one GPU in hand-written HIP kernels; this header is the
 * whole boundary.  Conventions for every call:
 *   - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *     with the length n implied by the problem (see jfnk_problem) and the
 *     element type implied by the solver's precision:
 *        working vectors (x, v, F, Jv, rhs, dx):  double for JFNK_F64,
 *                                                 float  for JFNK_F32 / JFNK_F16S;
 *        state arrays (x_prev, source, Newton x): always double.
 *     Any alignment is accepted (16-byte alignment takes the vectorized path).
 *   - Layout of a state vector: 1D Burgers u[i]; two-field 2D problems as two
 *     row-major planes (field f, row j, column i at f*nx*ny + j*nx + i);
 *     Helmholtz-Kerr as interleaved complex (re, im) pairs at 2*(j*nx+i)+c.
 *   - No call retains a caller pointer after it returns.  The solver handle
 *     owns its workspace (Krylov basis, Hessenberg, scratch).
 *   - jfnk_residual and jfnk_jvp are asynchronous on the solver's HIP stream:
 *     the caller keeps the buffers alive until that stream is synchronized.
 *     jfnk_gmres and jfnk_newton_solve synchronize before returning.
 *   - Errors are status codes; nothing aborts and no exception crosses the
 *     ABI.  jfnk_last_error() describes the last failure of a handle.
 *   - A handle is not thread-safe; separate handles are independent.
 */
#ifndef JFNK_H
#define JFNK_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JFNK_OK = 0,
  JFNK_ERR_ARG = 1,           /* invalid argument or unsupported combination */
  JFNK_ERR_OOM = 2,           /* device or pinned-host allocation failed */
  JFNK_ERR_HIP = 3,           /* a HIP runtime call failed */
  JFNK_ERR_NONFINITE = 4,     /* NaN/Inf in a residual, Krylov quantity or update */
  JFNK_ERR_BREAKDOWN = 5,     /* Krylov breakdown that left no usable direction */
  JFNK_ERR_NOT_CONVERGED = 6  /* Newton iteration cap reached above tolerance */
} jfnk_status;

typedef enum { JFNK_JVP_AD = 0, JFNK_JVP_FD = 1 } jfnk_jvp_mode;

/* Working precision.  F16S: FP32 arithmetic, Krylov basis and JVP tangent
 * stored in FP16 with a per-vector power-of-two scale.  Givens rotations,
 * the Hessenberg least squares, dot-product accumulation, the Newton update
 * and the line-search merit norm are FP64 in every precision. */
typedef enum { JFNK_F64 = 0, JFNK_F32 = 1, JFNK_F16S = 2 } jfnk_precision;

/* FD step (paper, Section 2, step-size equation):
 *   PAPER:      eps = sqrt(eps_mach) * max(1, ||x||)
 *   NORMALIZED: eps = sqrt(eps_mach) * (1 + ||x||) / ||v||
 * eps_mach is that of the working arithmetic (2^-52 or 2^-23). */
typedef enum { JFNK_EPS_PAPER = 0, JFNK_EPS_NORMALIZED = 1 } jfnk_eps_rule;

typedef enum {
  JFNK_BURGERS1D = 0,   /* u_t + u u_x = nu u_xx, periodic; n = nx (ny = 1) */
  JFNK_BURGERS2D = 1,   /* (U.grad)U = nu Lap U (Appendix A.1), periodic; n = 2 nx ny */
  JFNK_GRAYSCOTT2D = 2, /* two-species reaction-diffusion, periodic; n = 2 nx ny */
  JFNK_KERR2D = 3,      /* -Lap E - k0^2 (eps_L + chi3 |E|^2) E = f, PEC nodes; n = 2 nx ny */
  JFNK_RD2D = 4,        /* u_t = D Lap u - u^3 (Appendix A.3), Dirichlet nodes; n = nx ny */
  JFNK_SUOLSON2D = 5,   /* Su-Olson radiation diffusion (Appendix A.2); n = 2 nx ny */
  JFNK_MAXWELL2D = 6    /* 2D TE Maxwell-Kerr (Appendix A.4), PEC nodes; n = 4 nx ny */
} jfnk_problem_id;

/* Problem description.  Time-dependent problems use the theta scheme
 *   F(x; x^n) = x - x^n + dt [theta N(x) + (1 - theta) N(x^n)] - dt s
 * (theta = 1/2 is the paper's Crank-Nicolson, 1 is backward Euler) with
 * N(u) = u D_x u - nu D_xx u (1D Burgers), Adv(U) - nu Lap(U) (2D Burgers),
 * (-D Lap u - u^2 v + (F+k) u, -Dv Lap v + u^2 v - F (1 - v)) (Gray-Scott),
 * -D Lap u + u^3 (reaction-diffusion, interior nodes; F = u on the boundary
 * nodes, which hold the homogeneous Dirichlet value), second-order central
 * differences.  Kerr: F = -Lap E - k0^2 (eps_L + chi3 |E|^2) E - f on
 * interior nodes and F = E on the boundary nodes.
 *   p[]: Burgers {nu}; Gray-Scott {D, Dv, F, k}; Kerr {k0, eps_re, eps_im, chi3};
 *   reaction-diffusion {D}; Su-Olson {xi, periodic_y}.
 * Su-Olson: N = (-(1/3) Lap U + (U - V), -xi (U - V)) on (U, V) planes at the
 * interior nodes, F = x at the boundary nodes; the source (Q, 0) enters as s.
 * Its two configurations (Appendix A.2): p[1] = 0, Dirichlet nodes all round
 * (the dynamic 2D case); p[1] = 1, the classic 1D profile on a 2D grid: the
 * rows are periodic (row 0 and row ny-1 are neighbours) and only the first
 * and last columns are boundary nodes.  Other p[1] values: JFNK_ERR_ARG.
 * Maxwell TE (planes Re Ex, Im Ex, Re Ey, Im Ey; mu0 = eps0 = 1):
 *   F = curl curl E - omega^2 (1 - i loss)(1 + chi |E|) E - f inside, F = E on
 *   the boundary nodes, with the mixed derivative from the diagonal
 *   neighbours and the AD tangent of |E| taken as 0 at E = 0;
 *   p[] = {omega, loss, chi}; f = i omega J is the source argument.
 * Grid: nx columns (contiguous) by ny rows, spacings hx, hy; nx >= 3, and
 * ny >= 3 for 2D problems (ny = 1 for 1D Burgers). */
typedef struct {
  int id;
  int nx, ny;
  double hx, hy;
  double dt, theta;
  double p[8];
} jfnk_problem;

/* Newton / GMRES options; jfnk_default_options() fills the paper's settings
 * (Section 3.3: FP64 tol_Newton 1e-6, tol_Krylov 1e-8; FP32 1e-4 / 1e-6;
 * at most 15 Newton iterations and 100 restart cycles; m = 30). */
typedef struct {
  int m;                 /* GMRES restart length, 1..32 (<= the m of jfnk_create) */
  int max_restarts;      /* restart cycles per Newton step */
  int max_newton;        /* Newton iterations, <= JFNK_MAX_ITERS */
  int ls_max_backtracks; /* line-search halvings (alpha down to 2^-ls_max_backtracks) */
  double tol_krylov;     /* relative to ||rhs|| = ||F(x^k)|| */
  double tol_newton;     /* on ||F(x^k)|| / ||F(x^0)|| */
  double ls_c;           /* Armijo constant: accept ||F(x+a dx)|| <= (1 - c a) ||F(x)|| */
  double fd_eps;         /* > 0: fixed FD step; otherwise eps_rule */
  double breakdown_tol;  /* happy breakdown when ||w|| <= breakdown_tol ||J v_j|| */
  int mode;              /* jfnk_jvp_mode */
  int eps_rule;          /* jfnk_eps_rule */
  double* history;       /* nullable DEVICE array of (max_newton + 1) * n doubles:
                            receives every Newton iterate x_k (k = 0, 1, ...) */
  int engine;            /* jfnk_engine */
  int krylov;            /* jfnk_krylov: the linear solver of each Newton step */
  int orth;              /* jfnk_orth: Gram-Schmidt form of GMRES on the MULTI_KERNEL engine */
  int precond;           /* jfnk_precond: right preconditioner of GMRES (default NONE) */
} jfnk_options;

/* Right preconditioner of GMRES (paper, Appendix A.4).  CSLP: the
 * block-diagonal complex shifted-Laplacian preconditioner of the Maxwell-Kerr
 * problem.  At each interior node the Ex pair (Re, Im) is divided, as one
 * complex number, by M_xx = 2/hy^2 - omega^2 eps_p and the Ey pair by
 * M_yy = 2/hx^2 - omega^2 eps_p, with the damped permittivity
 * eps_p = (1 - loss i)(1 + chi |E|)(1 - 0.5 i) of the current Newton iterate
 * (frozen for the linear solve); boundary nodes are left as they are.  GMRES
 * runs on J M^{-1} and returns dx = M^{-1} z, so its residual, tolerance and
 * reported norms are those of J dx = rhs.  Applied inside the JVP kernel (no
 * extra pass over memory) and once to the final update.  On the scalar
 * Helmholtz-Kerr workload (JFNK_KERR2D) the same construction: each interior
 * pair divided by M = 2/hx^2 + 2/hy^2 - k0^2 (eps_L + chi3 |E|^2)(1 - 0.5 i),
 * the diagonal of -Lap and the damped permittivity (the paper defines the
 * preconditioner for the TE problem only).  Only for JFNK_MAXWELL2D and
 * JFNK_KERR2D, with GMRES on the MULTI_KERNEL engine (AUTO picks it), and
 * with the FD JVP only under the paper's step rule or a fixed step; other
 * combinations return JFNK_ERR_ARG. */
typedef enum { JFNK_PRECOND_NONE = 0, JFNK_PRECOND_CSLP = 1 } jfnk_precond;

/* Gram-Schmidt form of the GMRES Arnoldi step (the paper fixes none; both
 * orthogonalize twice):
 *   CGS2:  w = J v_j is projected on the basis twice, in three passes over
 *          it (the first fused into the JVP);
 *   DCGS2: the second projection of each new vector is delayed by one step
 *          and fused into the next step's passes (its norm follows from
 *          ||u||^2 - ||V^T u||^2, the next JVP is applied to the once-
 *          projected vector and corrected through the Arnoldi relation):
 *          two passes over the basis per step.  Same basis and Hessenberg
 *          matrix in exact arithmetic.  With FP16 storage (F16S) the
 *          pending and the completed vector are each rounded to FP16 as they
 *          are written, and the second pass and the norms are taken over the
 *          stored values.  The SINGLE_WORKGROUP engine always runs CGS2.
 * The default is DCGS2 in every precision. */
typedef enum { JFNK_ORTH_CGS2 = 0, JFNK_ORTH_DCGS2 = 1 } jfnk_orth;

/* The Krylov method of each Newton step (paper, Section 2: GMRES(m) or
 * BiCGSTAB for nonsymmetric Jacobians, CG for symmetric positive-definite
 * ones such as the reaction-diffusion problem's).  BICGSTAB and CG take
 * max_restarts as their iteration cap (Section 3.3 gives every method the
 * same cap of 100), ignore m and breakdown_tol, and run on the MULTI_KERNEL
 * engine in FP64 or FP32 with a solver created with m >= 5 (BiCGSTAB) or
 * m >= 2 (CG). */
typedef enum { JFNK_KRYLOV_GMRES = 0, JFNK_KRYLOV_BICGSTAB = 1, JFNK_KRYLOV_CG = 2 } jfnk_krylov;

/* How jfnk_newton_solve runs the method (same algorithm, same options):
 *   AUTO:  SINGLE_WORKGROUP when the problem fits it, else MULTI_KERNEL;
 *   MULTI_KERNEL: one kernel per step of the method, the grid spread over
 *          the whole device (the throughput path);
 *   SINGLE_WORKGROUP: the whole solve in one launch of one workgroup with
 *          every vector in LDS (the latency path for small problems: about
 *          n (m + 6) * sizeof(working type) + 16 n bytes must fit the
 *          device's LDS per workgroup; FP64 and FP32 only).  Requesting it
 *          for a problem that does not fit returns JFNK_ERR_ARG;
 *   MULTI_KERNEL_GRAPH: the multi-kernel engine with each GMRES restart
 *          cycle (its m Arnoldi steps and the V y update) launched as one
 *          HIP graph, captured on first use per launch configuration and
 *          kept by the solver: one host launch per cycle instead of two or
 *          three per step, all m steps queued at once (steps after the one
 *          that stopped the cycle leave at once on the device), the same
 *          kernels in the same order, so the same results bit for bit as
 *          MULTI_KERNEL.  GMRES only (JFNK_ERR_ARG otherwise); a solver on the
 *          null stream, which cannot be captured, or with profiling on runs
 *          the cycles directly. */
typedef enum {
  JFNK_ENGINE_AUTO = 0,
  JFNK_ENGINE_MULTI_KERNEL = 1,
  JFNK_ENGINE_SINGLE_WORKGROUP = 2,
  JFNK_ENGINE_MULTI_KERNEL_GRAPH = 3
} jfnk_engine;

#define JFNK_MAX_ITERS 64

/* Per-solve record (paper, Section 3.4 metrics). */
typedef struct {
  int status;                      /* jfnk_status of the solve */
  int converged;                   /* Newton: rel. residual < tol; GMRES: ||r|| <= tol ||rhs|| */
  int newton_iters;
  int krylov_iters;                /* Arnoldi steps, all cycles and Newton steps */
  int restarts;                    /* restart cycles run */
  int ls_backtracks;
  int ls_failures;                 /* steps where no alpha passed the Armijo test */
  int lin_iters[JFNK_MAX_ITERS];   /* Arnoldi steps of each Newton step */
  double rel_res[JFNK_MAX_ITERS + 1]; /* ||F(x_k)|| / ||F(x_0)||, k = 0..newton_iters */
  double alpha[JFNK_MAX_ITERS];    /* accepted line-search step of each Newton step */
  double f0_norm;                  /* ||F(x_0)|| (FP64 merit norm) */
  double final_res;                /* GMRES: last true residual ||rhs - J dx|| */
  double seconds;                  /* wall time of the call */
} jfnk_info;

typedef struct jfnk_solver jfnk_solver;

/* Create a solver for one problem shape and precision on `hip_stream`
 * (a hipStream_t; NULL = the default stream) with workspace for GMRES(m),
 * 1 <= m <= 32.  Allocates jfnk_footprint_bytes() of device memory. */
jfnk_status jfnk_create(const jfnk_problem* problem, int precision, int m, void* hip_stream,
                        jfnk_solver** out);
jfnk_status jfnk_destroy(jfnk_solver* s);

/* Device bytes a solver of this shape allocates (for admission control). */
size_t jfnk_footprint_bytes(const jfnk_problem* problem, int precision, int m);

/* Number of real unknowns n of a problem (0 if the description is invalid). */
size_t jfnk_problem_size(const jfnk_problem* problem);

/* Fix x* for the next calls: the previous time level x^n (time-dependent
 * problems) and the optional source s / f (nullable; required for Kerr).
 * Both FP64 device arrays of length n.  Computes the constant part
 * x^n - (1 - theta) dt N(x^n) + dt s once (stream-ordered). */
jfnk_status jfnk_set_previous(jfnk_solver* s, const double* x_prev, const double* source);

/* F = F(x; x*) in the working precision (paper, Section 2). */
jfnk_status jfnk_residual(jfnk_solver* s, const void* x, void* F);

/* Jv = J(x) v (paper, Section 2: the JVP by forward-mode AD or by finite
 * differences).  mode AD: fused dual-number pass; if F_or_null is given it
 * also receives F(x).  mode FD: (F(x + eps v) - F(x)) / eps with both
 * residuals evaluated in one pass; eps > 0 is used as given, eps <= 0 takes
 * eps_rule (jfnk_eps_rule) with norms computed on the device.  On a
 * JFNK_F16S solver the tangent is stored in FP16 first, as Krylov vectors
 * are: v times the power of two sigma that maps ||v|| / sqrt(n) near 1,
 * rounded to nearest, read back divided by sigma (the normalized FD rule
 * takes ||v|| of the FP32 v). */
jfnk_status jfnk_jvp(jfnk_solver* s, const void* x, const void* v, void* Jv, void* F_or_null,
                     int mode, double eps, int eps_rule);

/* Solve J(x) dx = rhs by restarted GMRES(m) (paper, Section 2) from dx = 0,
 * with the Gram-Schmidt form set by jfnk_set_orthogonalization (DCGS2 by
 * default) and FP64 Givens least
 * squares; tolerance relative to ||rhs||.  Reaching the cycle cap returns
 * JFNK_OK with info->converged = 0. */
jfnk_status jfnk_gmres(jfnk_solver* s, const void* x, const void* rhs, void* dx, int m, double tol,
                       int max_restarts, int mode, double eps, int eps_rule, jfnk_info* info);

/* Unrotated Hessenberg matrix of the last restart cycle of the last GMRES
 * solve on the multi-kernel engine (paper, Section 2: the Arnoldi relation
 * J V_k = V_{k+1} H_k, column j holding V^T J v_j and ||w_j||), either
 * Gram-Schmidt form.  *k_out receives k, the cycle's Arnoldi steps; H (host,
 * column-major, leading dimension ldh >= k + 1, nullable when k = 0)
 * receives the (k + 1) x k matrix, zero below the subdiagonal.  With a
 * preconditioner it is that of J M^{-1}.  Synchronizes the solver's stream;
 * JFNK_ERR_ARG when H is too small. */
jfnk_status jfnk_gmres_hessenberg(jfnk_solver* s, double* H, int ldh, int* k_out);

/* Solve J(x) dx = rhs by BiCGSTAB (paper, Section 2: van der Vorst's
 * stabilized bi-conjugate gradients, two JVPs per iteration) from dx = 0
 * with shadow residual r^ = rhs; stops when ||s|| (half step) or ||r|| is at
 * most tol ||rhs||, after max_iters iterations, on a breakdown (rho,
 * (r^, J p) or ||J s||^2 exactly zero, or omega = 0) or on a non-finite
 * scalar.  x, rhs, dx: device arrays of n elements of the working precision
 * (FP64 or FP32 solvers created with m >= 5; the solver's first six basis
 * slots are its work vectors).  Returns JFNK_OK when converged or at the
 * cap (info->converged tells which), JFNK_ERR_BREAKDOWN, JFNK_ERR_NONFINITE
 * or JFNK_ERR_ARG; info (nullable) receives converged, krylov_iters (completed
 * iterations), final_res (last ||r||, or ||s|| at a half-step stop) and
 * f0_norm (||rhs||).  Synchronizes before returning. */
jfnk_status jfnk_bicgstab(jfnk_solver* s, const void* x, const void* rhs, void* dx, double tol, int max_iters,
                          int mode, double eps, int eps_rule, jfnk_info* info);

/* Solve J(x) dx = rhs by conjugate gradients (paper, Section 2: Hestenes
 * and Stiefel's method, for symmetric positive-definite J) from dx = 0; one
 * JVP per iteration; stops when ||r|| <= tol ||rhs||, after max_iters
 * iterations, on (p, J p) <= 0 (J not positive definite along p: breakdown)
 * or on a non-finite scalar.  Arguments, statuses and info as for
 * jfnk_bicgstab (FP64 or FP32 solvers created with m >= 2; the solver's
 * first three basis slots are its work vectors).  Synchronizes before
 * returning. */
jfnk_status jfnk_cg(jfnk_solver* s, const void* x, const void* rhs, void* dx, double tol, int max_iters, int mode,
                    double eps, int eps_rule, jfnk_info* info);

/* Newton with line search from x_inout (FP64 device array, overwritten with
 * the last iterate).  Returns JFNK_OK when converged, JFNK_ERR_NOT_CONVERGED
 * at the iteration cap, JFNK_ERR_NONFINITE on NaN/Inf; info is filled in all
 * three cases. */
jfnk_status jfnk_newton_solve(jfnk_solver* s, double* x_inout, const jfnk_options* opts,
                              jfnk_info* info);

/* Number of captured GMRES-cycle graphs the solver holds (one per launch
 * configuration the MULTI_KERNEL_GRAPH engine has met; released by
 * jfnk_destroy); -1 for a null solver. */
int jfnk_cycle_graphs(const jfnk_solver* s);

/* Frequency continuation of a frequency-domain problem (paper, Section 3.1:
 * the outer loop advances the angular frequency; Section 3.2 and Appendix
 * A.4: the initial guess is the Born solution, the problem linearized at
 * E = 0, i.e. the first Newton step from E = 0; Section 3.4: a run fails when
 * more than 20% of its frequency steps do not reach the Newton tolerance).
 * problems[0..count-1] are the frequencies in order (one unknown count n for
 * all; JFNK_ERR_ARG otherwise); sources[i] (nullable array, nullable
 * entries) host FP64 sources of n entries.  Frequency i starts from
 * frequency i-1's converged field; the first, and every frequency after one
 * that did not converge (cap, non-finite value or breakdown), starts from
 * E = 0.  fields (host, count * n FP64, frequency-major) receives each
 * frequency's last iterate, infos (nullable, count entries) each Newton
 * record, *run_failed the 20% rule.  One solver per frequency is created and
 * destroyed on hip_stream (device memory: one solver plus 2 n doubles at a
 * time).  Returns JFNK_OK when every frequency ran (converged or not), else
 * the first argument, allocation or HIP error. */
jfnk_status jfnk_frequency_sweep(const jfnk_problem* problems, const double* const* sources, int count,
                                 int precision, const jfnk_options* opts, void* hip_stream, double* fields,
                                 jfnk_info* infos, int* run_failed);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the Newton
 * solve of jfnk_newton_solve on the SINGLE_WORKGROUP engine without a solver
 * handle and without any allocation.  It computes the constant part from
 * x_prev and source (FP64 device arrays of n entries as for
 * jfnk_set_previous; x_prev may be NULL for Kerr and Maxwell) and runs the
 * solve from x_inout (FP64 device array, overwritten with the last iterate)
 * on `hip_stream` (a hipStream_t; NULL = the default stream), then
 * synchronizes that stream and fills info.  The constant part and the solve
 * record live in a static device array of 68 KiB per GPU (allocated with the
 * library's code object and held until the process ends), so the call
 * accepts at most 4096 unknowns, FP64 or FP32 (not FP16S), GMRES with no
 * preconditioner and an engine of AUTO or SINGLE_WORKGROUP, and the problem
 * must fit the engine's LDS; otherwise it returns JFNK_ERR_ARG and
 * jfnk_last_error(NULL) says why.  Results are bitwise those of
 * jfnk_newton_solve on the same engine.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other threads or streams) race and
 * must be serialized by the caller.  Statuses as for jfnk_newton_solve. */
jfnk_status jfnk_newton_solve_noalloc(const jfnk_problem* problem, int precision, const double* x_prev,
                                      const double* source, double* x_inout, const jfnk_options* opts,
                                      jfnk_info* info, void* hip_stream);

/* Gram-Schmidt form (jfnk_orth) of later jfnk_gmres calls on this solver
 * (default DCGS2); jfnk_newton_solve takes it from its options instead
 * (jfnk_default_options: the same).  An unknown form returns JFNK_ERR_ARG. */
jfnk_status jfnk_set_orthogonalization(jfnk_solver* s, int orth);

/* Preconditioner (jfnk_precond) of later jfnk_gmres calls on this solver
 * (default NONE); jfnk_newton_solve takes it from its options instead.
 * CSLP on a problem other than JFNK_MAXWELL2D or JFNK_KERR2D returns
 * JFNK_ERR_ARG, and a later jfnk_gmres call with the FD JVP under the
 * normalized step rule does too. */
jfnk_status jfnk_set_preconditioner(jfnk_solver* s, int precond);

/* Move a solver to another stream (a hipStream_t; NULL = the default stream)
 * for its later calls.  The caller orders any work still pending on the old
 * stream (the solver keeps no pointer to it). */
jfnk_status jfnk_set_stream(jfnk_solver* s, void* hip_stream);

/* The paper's defaults for a precision (see jfnk_options). */
void jfnk_default_options(int precision, jfnk_options* out);

const char* jfnk_status_string(int status);
const char* jfnk_last_error(const jfnk_solver* s);

/* Kernel timing with HIP events on the solver's stream (off by default).
 * kernel: 0 residual, 1 AD JVP, 2 FD JVP, 3 CGS pass A (V^T w), 4 CGS pass B
 * (update + dot), 5 CGS pass C (update + norm + Givens), 6 V y update,
 * 7 cycle start, 8 Newton trial update, 9 single-workgroup whole solve,
 * 10 BiCGSTAB streaming kernels, 11 CG streaming kernels (the JVPs of both
 * count as 1 or 2), 12 update pass of the DCGS2 Arnoldi step.  Reports the
 * launches timed since the last reset, their summed duration (ms) and their
 * algorithmic HBM bytes. */
jfnk_status jfnk_profile_enable(jfnk_solver* s, int on);
jfnk_status jfnk_profile_read(jfnk_solver* s, int kernel, long long* launches, double* total_ms,
                              double* bytes);
jfnk_status jfnk_profile_reset(jfnk_solver* s);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent implicit-step solves.
 *
 * A batch owns `max_slots` worker threads, each with its own HIP stream, and a
 * device-memory budget.  Requests (one Newton solve each: problem, previous
 * state, options) are admitted first come, first served as soon as a slot is
 * free and the request's workspace fits the budget; admitted requests run
 * concurrently on their slots' streams, so their kernels overlap on the
 * device.  Solver workspaces stay on the device between requests of the same
 * shape (least recently used ones are released when the budget needs room).
 * Device memory is returned only while no request is on the device (a device
 * free waits for every stream): a workspace to be released is held, its
 * bytes still counted, until the running requests have finished, and a
 * request that needs that room waits for it.
 * Every kernel's launch shape depends only on the problem, so a request's
 * result is bitwise the same whether it runs alone or in a mix.
 * ------------------------------------------------------------------------ */
typedef struct jfnk_batch jfnk_batch;

typedef struct {
  size_t budget_bytes;  /* device memory for solver workspaces (running + cached) */
  int max_slots;        /* requests on the device at once, 1..64 */
  int precision;        /* jfnk_precision of every request */
  int m;                /* GMRES restart length of every request, 1..32 */
  int keep_workspaces;  /* 1: cache idle workspaces by shape; 0: free after each request */
} jfnk_batch_config;

typedef struct {
  long long submitted, completed, failed;
  long long workspaces_created, workspaces_released;
  int max_running;          /* most requests seen on the device at once */
  size_t bytes_in_use;      /* workspaces held now */
  size_t peak_bytes;        /* most workspace bytes held at once (never above the budget) */
  long long frees_while_running; /* device frees made while a request was on the device (0) */
} jfnk_batch_stats;

/* Create a batch; the calling thread's current device is used. */
jfnk_status jfnk_batch_create(const jfnk_batch_config* cfg, jfnk_batch** out);

/* Wait for running requests, drop queued ones, free everything. */
jfnk_status jfnk_batch_destroy(jfnk_batch* b);

/* Queue one solve.  x_prev (and source, nullable; Kerr only) are host FP64
 * arrays of jfnk_problem_size() entries, copied before the call returns; the
 * Newton iteration starts from x_prev.  opts NULL = jfnk_default_options.
 * Returns JFNK_ERR_ARG for an invalid problem and JFNK_ERR_OOM when the
 * request alone exceeds the budget.  Thread-safe. */
jfnk_status jfnk_batch_submit(jfnk_batch* b, const jfnk_problem* problem, const double* x_prev,
                              const double* source, const jfnk_options* opts, long long* ticket);

/* 1 when the request has finished, 0 while queued or running, -1 for an
 * unknown ticket.  Thread-safe. */
int jfnk_batch_poll(jfnk_batch* b, long long ticket);

/* Block until the request finishes, copy its last iterate to x_out (host,
 * nullable) and its info (nullable), and retire the ticket.  times (nullable,
 * 3 doubles): submit, start and finish time in seconds on the batch clock.
 * Returns the request's Newton status (jfnk_newton_solve's). */
jfnk_status jfnk_batch_wait(jfnk_batch* b, long long ticket, double* x_out, jfnk_info* info,
                            double* times);

/* Seconds since jfnk_batch_create on the clock used by jfnk_batch_wait. */
double jfnk_batch_clock(const jfnk_batch* b);

jfnk_status jfnk_batch_get_stats(jfnk_batch* b, jfnk_batch_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* JFNK_H */
