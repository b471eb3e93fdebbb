/*
 * kfbi.h -- C ABI of the MI355X (gfx950) kernel-free boundary integral library.
 *
 * The library solves the interior Dirichlet problem of the modified Helmholtz
 * equation  Lap u - kappa u = f  in Omega,  u = g  on Gamma = dOmega  (kappa >= 0)
 * by the kernel-free boundary integral (KFBI) method of Tan, Huang & Ying,
 * "A GPU-accelerated Cartesian grid method for PDEs on irregular domain"
 * (arXiv 2404.15249):
 *   - Sec. 2.1 (second-kind equation): phi/2 + W phi + Y f = g on Gamma, and
 *     u = W phi + Y f in Omega.  K_D = I/2 + W is the interior one-sided limit
 *     of the double-layer potential.
 *   - Sec. 2.2 (interface problem and the table under it): W phi and Y f are the
 *     solution of  Lap v - kappa v = F  off Gamma, [v] = Phi, [d_n v] = 0,
 *     v = 0 on the box, with (F, Phi) = (0, phi) or (f~, 0).
 *   - Alg. 1-4: jumps, correction of the 5-point system at irregular nodes,
 *     fast sine-transform solve, interpolation to the boundary samples.
 *   - Alg. 5: restarted GMRES with K_D as the matrix-vector product.
 *
 * Conventions shared by every entry point
 *   Box B = [lo, hi]^2 split into n intervals per axis (h = (hi-lo)/n); node
 *   (i, j) sits at (lo + i h, lo + j h).  A "grid" array holds the (n+1)^2 node
 *   values row by row: element j*(n+1) + i (row j is the line y = lo + j h).
 *   Gamma is given by M >= 3 samples x_m (counter-clockwise, no repeated end
 *   point) and represented by the periodic cubic spline through them in the
 *   sample index; densities and f on Gamma are sampled at the same points and
 *   splined the same way.  The samples are the GMRES unknowns (the paper's
 *   control points).
 *
 *   Unless a parameter says "host", array pointers are DEVICE pointers on the
 *   context's device, FP64, owned by the caller, and must stay valid until the
 *   work enqueued by the call has finished on the context stream.  Calls enqueue
 *   on the context stream and return without synchronising unless stated.
 *   The library owns only its handles and the device workspace it allocates in
 *   kfbi_prob_create.  A problem or batch handle must not be used by two host
 *   threads at the same time; different handles on one context may be used
 *   from different threads (e.g. problems created by a preparation thread while
 *   another thread steps a batch): the library builds its graphs node by node,
 *   never by stream capture, so no call ever runs inside a capture.
 *
 * Errors: every call returns a kfbi_status; on error no output is written (for
 * enqueueing calls: nothing is enqueued) and kfbi_last_error() returns a
 * message for the calling thread.
 *
 * Non-finite data: the device checks what it computes from the caller's data.
 * kfbi_apply, kfbi_apply_neumann and kfbi3_apply check the density first
 * (and so wait for the check); the solves and outer iterations (GMRES,
 * BiCGSTAB, Richardson, in every form) stop at the first residual or
 * Arnoldi norm that comes out NaN or Inf -- a NaN or Inf anywhere in f inside
 * Omega, f on Gamma, g or the initial density reaches it -- and return
 * KFBI_ERR_NONFINITE with none of their outputs written.
 */
#ifndef KFBI_H
#define KFBI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int kfbi_status;
#define KFBI_OK 0
#define KFBI_NOT_CONVERGED 1       /* warning: outputs hold the last iterate */
#define KFBI_ERR_ARG (-1)          /* bad argument (null pointer, size out of range) */
#define KFBI_ERR_GEOMETRY (-2)     /* curve too close to the box, grid edge crossed twice, ... */
#define KFBI_ERR_OOM (-3)          /* device allocation failed */
#define KFBI_ERR_DEVICE (-4)       /* HIP runtime error */
#define KFBI_ERR_BUDGET (-5)       /* request can never fit the batch's memory budget */
#define KFBI_ERR_NONFINITE (-6)    /* NaN or Inf met in the data */
#define KFBI_ERR_UNSUPPORTED (-7)  /* configuration outside what the library handles */

typedef struct kfbi_ctx kfbi_ctx;
typedef struct kfbi_prob kfbi_prob;

/* Problem description (all host memory). */
typedef struct {
    double lo, hi;        /* box [lo, hi]^2 */
    int n;                /* intervals per axis; power of two, 64 <= n <= 4096 */
    double kappa;         /* >= 0, the operator is Lap - kappa (Sec. 2, modified Helmholtz) */
    int m;                /* number of boundary samples, 3 <= m <= 12288 */
    const double* xy;     /* host, m x 2 (x0, y0, x1, y1, ...), counter-clockwise */
    double tol;           /* GMRES relative residual tolerance (Sec. 5 uses 1e-8); <= 0: 1e-10 */
    int restart;          /* GMRES restart length; <= 0: 50; capped at 64 */
    int max_iter;         /* cap on K_D applications inside GMRES; <= 0: 500 */
    int precision;        /* arithmetic of the dense grid solves (volume potential,
                             final solution, kfbi_fast_solve and the interface
                             solves): KFBI_FP64, or KFBI_FP32_REFINED */
    int refine_steps;     /* KFBI_FP32_REFINED only: FP64 residual corrections after
                             the first FP32 solve, 0..4; < 0: 1 */
} kfbi_desc;

/* Precision of the dense grid solves.  KFBI_FP32_REFINED runs the two column
 * sine transforms of Alg. 4 in FP32 arithmetic with FP32 storage between them
 * (the tridiagonal solves along x and the transforms' running sums stay FP64),
 * then refines: r = rhs - (L_h - kappa) v in FP64, v += FP32 solve of r, per
 * refine step.  GMRES, the jumps, corrections and interpolation, and the
 * K_D apply of the iteration stay FP64 in both modes. */
#define KFBI_FP64 0
#define KFBI_FP32_REFINED 1

/* ---------------------------------------------------------------- contexts */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (NULL: the library creates its own stream with default flags and
 * priority).  The caller keeps ownership of a stream it passes in. */
kfbi_status kfbi_ctx_create(int device, void* hip_stream, kfbi_ctx** out);
kfbi_status kfbi_ctx_destroy(kfbi_ctx* ctx);
/* Block until all work enqueued on the context stream has finished. */
kfbi_status kfbi_ctx_sync(kfbi_ctx* ctx);

/* ---------------------------------------------------------------- problems */

/* Build the geometry plan on the host (spline of Gamma, classification of the
 * nodes by horizontal scan lines, grid-line crossings, irregular nodes and
 * their arms, six-point interpolation stencils: Alg. 1 steps 1-3 and the
 * Procedure 1 list of Sec. 4.2) and upload it with the workspace of the solve.
 * Fails with KFBI_ERR_GEOMETRY when the curve comes within 2h of the box, when
 * an edge whose end nodes differ holds other than one crossing, or when an edge
 * is crossed twice.  Synchronous. */
kfbi_status kfbi_prob_create(kfbi_ctx* ctx, const kfbi_desc* desc, kfbi_prob** out);
kfbi_status kfbi_prob_destroy(kfbi_prob* prob);

/* Sizes: samples M, crossings Q, irregular nodes I, device bytes held. */
kfbi_status kfbi_prob_info(const kfbi_prob* prob, int* m, int* q, int* n_irregular,
                           size_t* device_bytes);
/* host, (n+1)^2 bytes: 1 where the node lies in Omega (or on Gamma). */
kfbi_status kfbi_prob_mask(const kfbi_prob* prob, unsigned char* inside);
/* host, plan export: for each crossing its axis (0: on a line y = const, 1: on a
 * line x = const), its two end nodes (i0, j0, i1, j1), its spline parameter and
 * its position (x, y).  Any pointer may be NULL. */
kfbi_status kfbi_prob_crossings(const kfbi_prob* prob, int* axis, int* nodes, double* t, double* xy);
/* host, I x 2: the irregular nodes (i, j) in the library's internal order. */
kfbi_status kfbi_prob_irregular(const kfbi_prob* prob, int* ij);
/* host, M x 2 each (either may be NULL): the control points where g, f on
 * Gamma and the density live -- the samples as given, since Sec. 2.1 takes the
 * density at the boundary points the curve is described by -- and the unit
 * outward normal of the spline curve there (the normal of the jump formulas
 * and of d_n v+; Neumann data are g_n = grad u . normal at these points). */
kfbi_status kfbi_prob_points(const kfbi_prob* prob, double* xy, double* normal);

/* ---------------------------------------------------------------- hot path */

/* K_D phi = (I/2 + W) phi at the M samples: one interface solve with [v] = phi,
 * F = 0 (Alg. 1 steps 4-6).  Jumps and corrections at the irregular nodes
 * (Alg. 2), a sine-transform solve along y with a tridiagonal solve along x
 * (Alg. 4) evaluated only where the interpolation needs it, and the
 * interpolation (Alg. 3).  phi, out: device, M doubles.  Waits for the check
 * of phi (KFBI_ERR_NONFINITE, out untouched, if it holds a NaN or Inf). */
kfbi_status kfbi_apply(kfbi_prob* prob, const double* phi, double* out);

/* kfbi_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and the same result, with the apply's scratch (spline second
 * derivatives, corrections, partial sums: 256 + 8 M + 512 T + 8 G M bytes,
 * rounded up to 256-byte blocks) taken from a 32 MiB array of static device
 * memory that each GPU holds for the life of the process, in place of the
 * problem's workspace.  Allocates nothing and enqueues only: it does not wait,
 * so a NaN or Inf in phi leaves out untouched but is not reported (kfbi_apply
 * reports it).  KFBI_ERR_UNSUPPORTED, with nothing enqueued, when the problem
 * needs more scratch than the array holds (the 2048^2 grid with 1024 samples
 * needs about 2.1 MiB).  Every call on one GPU shares that GPU's array: calls
 * that overlap on a GPU (on two streams, or from two threads) race, so
 * serialise them.  phi, out: device, M doubles, as kfbi_apply. */
kfbi_status kfbi_apply_noalloc(kfbi_prob* prob, const double* phi, double* out);

/* Full Dirichlet solve (Sec. 2.1): g^ = g - (Y f)^+, GMRES (Alg. 5) on
 * K_D phi = g^ until the relative residual drops below tol, then u = W phi + Y f.
 *   f_grid : device grid, f at every node (values outside Omega are ignored)
 *   f_gamma: device, M: f at the samples (the jump of F across Gamma)
 *   g      : device, M: Dirichlet data at the samples
 *   u_grid : device grid out: u at nodes in Omega, 0 elsewhere
 *   u_gamma: device, M out: the interior limit u+ at the samples
 *   phi    : device, M in/out: initial guess in, density out
 *   iters  : host out, K_D applications made by GMRES (may be NULL)
 *   rel_res: host out, final true relative residual (may be NULL)
 * Synchronises.  Returns KFBI_NOT_CONVERGED when max_iter was reached. */
kfbi_status kfbi_solve(kfbi_prob* prob, const double* f_grid, const double* f_gamma,
                       const double* g, double* u_grid, double* u_gamma, double* phi,
                       int* iters, double* rel_res);

/* Alg. 5 alone: restarted GMRES on K_D phi = rhs, fully device resident (the
 * Hessenberg least-squares problem is solved on the device, so nothing crosses
 * to the host inside the iteration).  rhs: device M; phi: device M, initial
 * guess in, iterate out.  Stops when the true relative residual drops below
 * tol, or after max_iter Arnoldi steps; tol <= 0 never stops early (fixed
 * work, for timing).  iters: Arnoldi steps made; applies: all K_D
 * applications (Arnoldi steps, one residual apply at the end of every cycle,
 * and one at the start unless the initial guess is zero: K_D 0 = 0);
 * rel_res: last relative residual (true residual at cycle ends, Givens
 * estimate otherwise).  Host outputs may be NULL.  Synchronises. */
kfbi_status kfbi_gmres(kfbi_prob* prob, const double* rhs, double* phi, double tol, int max_iter,
                       int* iters, int* applies, double* rel_res);

/* ---------------------------------------------------------------- other outer iterations (Table 2) */
/* The paper compares GMRES with the Richardson iteration of Sec. 2.1 and with
 * BiCGSTAB on the same boundary equation (Table 2).  Both run device resident
 * on the K_D apply of kfbi_apply, with GMRES's stopping rule: the relative
 * residual |rhs - K_D x| / |rhs - K_D x0| below tol, or max_iter reached.
 * rhs: device M; phi: device M, initial guess in, iterate out.  Host outputs
 * may be NULL.  Synchronise; KFBI_NOT_CONVERGED at the cap. */

/* x <- x + gamma (rhs - K_D x) (Sec. 2.1; the paper shows convergence for
 * gamma in (0, 1]).  iters: updates made (one K_D apply each, plus the initial
 * residual); rel_res: the relative residual of the final iterate. */
kfbi_status kfbi_richardson(kfbi_prob* prob, const double* rhs, double* phi, double gamma, double tol,
                            int max_iter, int* iters, double* rel_res);

/* Unpreconditioned BiCGSTAB (van der Vorst), shadow residual r0.  iters:
 * iterations begun; applies: all K_D applications; rel_res: the true relative
 * residual of the final iterate. */
kfbi_status kfbi_bicgstab(kfbi_prob* prob, const double* rhs, double* phi, double tol, int max_iter,
                          int* iters, int* applies, double* rel_res);

#define KFBI_GMRES 0
#define KFBI_BICGSTAB 1
#define KFBI_RICHARDSON 2

/* kfbi_solve with the outer iteration chosen: KFBI_GMRES (exactly kfbi_solve),
 * KFBI_BICGSTAB or KFBI_RICHARDSON (relax = gamma), with the problem's
 * tolerance and cap.  iters as the chosen method reports them. */
kfbi_status kfbi_solve_method(kfbi_prob* prob, int method, double relax, const double* f_grid,
                              const double* f_gamma, const double* g, double* u_grid, double* u_gamma,
                              double* phi, int* iters, double* rel_res);

/* ---------------------------------------------------------------- the Neumann problem */
/* The paper names the Neumann problem (its Sec. 4 procedure extracts d_n u in
 * place of u+) without stating its form.  Here the density psi is the jump of
 * the normal derivative: v_psi solves the interface problem of Sec. 2.2 with
 * [v] = 0, [d_n v] = psi (n the outward normal of Omega), and u = v_psi + Y f.
 * The jumps at a point of Gamma are then [v_n] = psi, [v_tautau] = c psi,
 * [v_taun] = psi_s and [v_nn] = [F] - c psi (c the curvature); correction, fast
 * solve and interpolation are those of the Dirichlet path, and d_n v+ is the
 * gradient of the same six-point quadratic (Alg. 3) along the spline's outward
 * normal at the sample.  All arrays are device memory, same layouts as above. */

/* K_N psi = d_n v+ at the M samples for [v] = 0, [d_n v] = psi, F = 0 (sparse
 * path, as kfbi_apply).  psi, out: device, M doubles. */
kfbi_status kfbi_apply_neumann(kfbi_prob* prob, const double* psi, double* out);

/* One full-grid interface solve with [v] = 0, [d_n v] = psi (NULL: 0),
 * F = ftilde (used as given; NULL: 0) and [F] = f_gamma (NULL: 0).  Outputs,
 * each may be NULL but not all: vgrid (grid), vz (v+ at the samples), dnz
 * (d_n v+ at the samples). */
kfbi_status kfbi_interface_solve_neumann(kfbi_prob* prob, const double* psi, const double* ftilde,
                                         const double* f_gamma, double* vgrid, double* vz, double* dnz);

/* Restarted GMRES on K_N psi = rhs, as kfbi_gmres. */
kfbi_status kfbi_gmres_neumann(kfbi_prob* prob, const double* rhs, double* psi, double tol, int max_iter,
                               int* iters, int* applies, double* rel_res);

/* Full Neumann solve of Lap u - kappa u = f in Omega, d_n u = g_n on Gamma:
 * g^ = g_n - d_n (Y f)^+, GMRES on K_N psi = g^ (tolerance and cap of the
 * problem's descriptor), then u = v_psi + Y f.  Needs kappa > 0 (for kappa = 0
 * the constants solve the homogeneous problem): KFBI_ERR_ARG otherwise.
 *   f_grid, f_gamma: as kfbi_solve;  g_n: device M, Neumann data at the samples
 *   u_grid  : grid out, u at nodes in Omega, 0 elsewhere
 *   u_gamma : M out, the trace u+ at the samples
 *   dn_gamma: M out, d_n u+ at the samples (g_n to the solver tolerance)
 *   psi     : M in/out, initial guess in, density out
 *   iters, rel_res: host out (may be NULL).
 * Synchronises.  Returns KFBI_NOT_CONVERGED when max_iter was reached. */
kfbi_status kfbi_solve_neumann(kfbi_prob* prob, const double* f_grid, const double* f_gamma,
                               const double* g_n, double* u_grid, double* u_gamma, double* dn_gamma,
                               double* psi, int* iters, double* rel_res);

/* ---------------------------------------------------------------- Gray-Scott time stepping */
/* Example 3 of the paper: u_t = eps1 Lap u + (gamma (1-u) - u v^2)/eps0,
 * v_t = eps2 Lap v + (u v^2 - (gamma + kill) v)/eps0 in Omega, d_n u = d_n v = 0
 * on Gamma, by second-order Strang splitting (the paper names the splitting; the
 * rest is this library's reading): each step is R(dt/2) D(dt) R(dt/2), with R one
 * classical Runge-Kutta step of the pointwise reaction at the grid nodes in
 * Omega and at the boundary samples, and D Crank-Nicolson as w <- 2 z - w, z the
 * solution of the Neumann problem Lap z - kappa z = -kappa w, d_n z = 0,
 * kappa = 2/(eps dt) (kfbi_solve_neumann, GMRES warm-started from the previous
 * step's density).  z is solved as c + z', c the mean of w's trace at the
 * samples and z' the Neumann solution for the right-hand side -kappa (w - c):
 * the same z, but the zero extension of the right-hand side outside Omega then
 * jumps across Gamma by kappa (w - c) only, so a uniform state stays uniform.
 * The state is a grid of (n+1)^2 values (zero outside Omega) and the trace at
 * the M boundary samples, per species. */
typedef struct kfbi_gs kfbi_gs;

typedef struct {
    double lo, hi;        /* box [lo, hi]^2 */
    int n;                /* intervals per axis, as kfbi_desc */
    int m;                /* boundary samples */
    const double* xy;     /* host, m x 2, counter-clockwise (read during create only) */
    double gamma, kill;   /* feed and removal rates (the paper's gamma and kappa) */
    double eps0, eps1, eps2;
    double dt;            /* time step */
    double tol;           /* GMRES tolerance of each solve (the paper: 1e-8); <= 0: 1e-10 */
    int restart, max_iter;   /* as kfbi_desc (<= 0: defaults) */
} kfbi_gs_desc;

/* Two Neumann problems on one geometry (kappa = 2/(eps1 dt) and 2/(eps2 dt))
 * and the state buffers, all zero.  Geometry errors as kfbi_prob_create. */
kfbi_status kfbi_gs_create(kfbi_ctx* ctx, const kfbi_gs_desc* desc, kfbi_gs** out);
kfbi_status kfbi_gs_destroy(kfbi_gs* gs);
/* host out (each may be NULL): samples M, steps taken, GMRES iterations of all solves */
kfbi_status kfbi_gs_info(const kfbi_gs* gs, int* m, int* steps, long long* gmres_iters);
/* Copy in the state (device: grids (n+1)^2, zero outside Omega; traces M) and
 * reset the warm starts and counters. */
kfbi_status kfbi_gs_set_state(kfbi_gs* gs, const double* u_grid, const double* v_grid,
                              const double* u_gamma, const double* v_gamma);
/* Copy out the state (device; each pointer may be NULL).  Synchronises. */
kfbi_status kfbi_gs_get_state(kfbi_gs* gs, double* u_grid, double* v_grid, double* u_gamma, double* v_gamma);
/* Advance nsteps steps (two Neumann solves each).  Synchronises; returns
 * KFBI_NOT_CONVERGED if a solve hit its iteration cap (the step count then
 * stops at the step that failed). */
kfbi_status kfbi_gs_step(kfbi_gs* gs, int nsteps);

/* ---------------------------------------------------------------- steps (for tests and tools) */

/* Gram-Schmidt of the GMRES steps (kfbi_gmres, kfbi_solve and their Neumann
 * and batched forms): one classical pass, and a second one over the new
 * vector only when its norm after the first pass is below eta times its norm
 * before (the cancellation that would cost orthogonality).  eta in [0, 1]:
 * 0 never, 1 always; default 1e-3.  Takes effect at the next GMRES run. */
kfbi_status kfbi_prob_set_reorth(kfbi_prob* prob, double eta);

/* Alg. 2 alone: the correction of the right-hand side at every irregular node
 * for [v] = phi and [F] = f_gamma (f_gamma may be NULL: [F] = 0).  corr: device,
 * I doubles in the order of kfbi_prob_irregular. */
kfbi_status kfbi_correct(kfbi_prob* prob, const double* phi, const double* f_gamma, double* corr);

/* Alg. 4 alone: solve (L_h - kappa) v = rhs on the interior nodes with v = 0 on
 * the box.  rhs, v: device grids (only interior nodes of rhs are read; the box
 * rows and columns of v are written 0).  rhs and v may alias. */
kfbi_status kfbi_fast_solve(kfbi_prob* prob, const double* rhs, double* v);

/* One interface solve with the full grid: [v] = phi, F = ftilde (already zero
 * outside Omega), [F] = f_gamma (may be NULL).  vgrid: device grid out, vz:
 * device M out (v+ at the samples).  phi may be NULL (Phi = 0). */
kfbi_status kfbi_interface_solve(kfbi_prob* prob, const double* phi, const double* ftilde,
                                 const double* f_gamma, double* vgrid, double* vz);

/* As kfbi_interface_solve but with the Cartesian jumps given directly:
 * jq: device Q x 6 at the crossings, jz: device M x 6 at the samples, each row
 * ([v], [v_x], [v_y], [v_xx], [v_xy], [v_yy]).  Used to check that correction,
 * fast solve and interpolation are exact on quadratics. */
kfbi_status kfbi_interface_solve_jumps(kfbi_prob* prob, const double* jq, const double* jz,
                                       const double* ftilde, double* vgrid, double* vz);

/* ---------------------------------------------------------------- tile shapes and the autotuner */

/* Launch shapes of a problem's kernels. */
typedef struct {
    int modes_per_group;  /* sparse fast solve: sine modes per workgroup, 1/2/4/8/16 */
    int modes_groups;     /* sparse fast solve: workgroups, ceil((n-1) / modes_per_group) (output only) */
    int dst_cols;         /* column sine transforms: columns per workgroup, 4/8/16 (32/64 in FP64) */
    double apply_us;      /* autotune output: mean K_D apply time with this shape */
    double grid_solve_us; /* autotune output: mean dense grid solve time (transforms + row solves) */
} kfbi_tiles;

/* Time the candidate shapes on this problem (each K_D apply and grid solve
 * candidate `reps` times, after one warm-up, with HIP events on the context
 * stream), keep the fastest and return it in *out.  Candidates: half, the same
 * and twice the default modes per workgroup (where the local data share holds
 * them); every valid column tile.  Overwrites the problem's scratch vectors
 * (not its results).  Synchronises.  reps <= 0: 10. */
kfbi_status kfbi_prob_autotune(kfbi_prob* prob, int reps, kfbi_tiles* out);
/* The shapes in use (the times are those of the last autotune, else 0). */
kfbi_status kfbi_prob_get_tiles(const kfbi_prob* prob, kfbi_tiles* out);
/* Use the given shapes (e.g. from a cache of earlier autotune results);
 * KFBI_ERR_ARG if a value is not a valid candidate for this problem.  The
 * apply's result changes only by the grouping of its partial sums. */
kfbi_status kfbi_prob_set_tiles(kfbi_prob* prob, const kfbi_tiles* tiles);

/* ---------------------------------------------------------------- batches (many problems, one launch per step) */

/* A batch advances the GMRES iterations of up to max_slots problems together:
 * every stage of an iteration (correction, sparse fast solve, interpolation,
 * Gram-Schmidt/Givens) is one persistent launch over a device-resident work
 * list of all live problems, replayed as a captured graph.  Problems may have
 * different grids (n <= 4096) and sample counts (m <= m_max); a problem's
 * arithmetic is split into the same blocks whatever else is in the batch, so
 * its result is the same alone and in the mix.  hbm_budget bounds the device
 * bytes of the admitted problems (0: no bound).  For callers that serve solve
 * requests: admit when a slot and memory are free, step, poll, finish. */
typedef struct kfbi_batch kfbi_batch;
kfbi_status kfbi_batch_create(kfbi_ctx* ctx, int max_slots, int m_max, size_t hbm_budget, kfbi_batch** out);
/* Destroys the batch; problems still admitted are released, not destroyed. */
kfbi_status kfbi_batch_destroy(kfbi_batch* batch);
/* Device bytes a problem with grid n, m samples and restart length would hold
 * once admitted to a batch (plan, workspace and batch buffers), as an upper
 * bound computed before its plan exists: for admission control. */
kfbi_status kfbi_batch_estimate_bytes(int n, int m, int restart, size_t* bytes);
/* Admit a problem: enqueue its volume potential (Sec. 2.1, g^ = g - (Y f)^+)
 * and start its GMRES iteration.  f_grid, f_gamma and g (device, as in
 * kfbi_solve) must stay valid until kfbi_batch_finish returns.  Returns the
 * slot id.  KFBI_ERR_BUDGET: no free slot, or the budget cannot take it now
 * (retry after a finish); KFBI_ERR_UNSUPPORTED: it can never fit this batch. */
kfbi_status kfbi_batch_admit(kfbi_batch* batch, kfbi_prob* prob, const double* f_grid, const double* f_gamma,
                             const double* g, int* slot);
/* Enqueue nsteps GMRES iterations of every live problem (no synchronisation). */
kfbi_status kfbi_batch_step(kfbi_batch* batch, int nsteps);
/* Synchronise and report per slot (host arrays of max_slots entries, any may be
 * NULL): state 1 converged, -1 iteration cap reached, 0 running, -2 empty slot,
 * -3 stopped on a NaN or Inf in the request's data; Arnoldi steps made; last
 * relative residual. */
kfbi_status kfbi_batch_poll(kfbi_batch* batch, int* state, int* iters, double* rel_res);
/* Final solve u = W phi + Y f of a slot (outputs as in kfbi_solve) and release
 * the slot.  Enqueues; the outputs are ready after the next synchronisation.
 * A slot the last poll reported as -3 is released with nothing written and
 * KFBI_ERR_NONFINITE returned. */
kfbi_status kfbi_batch_finish(kfbi_batch* batch, int slot, double* u_grid, double* u_gamma, double* phi);
/* Live problems and the device bytes they hold. */
kfbi_status kfbi_batch_info(const kfbi_batch* batch, int* live, size_t* bytes_in_use);

/* ---------------------------------------------------------------- three dimensions */

/* The same Dirichlet problem in the ellipsoid
 *   Omega = { x^2/a^2 + y^2/b^2 + z^2/c^2 < 1 }
 * inside the cube B = [lo, hi]^3, on the 7-point grid of n intervals per axis
 * (Sec. 2 and Alg. 1-5 with the stencil, transforms and interpolation taken to
 * three dimensions; the paper gives the method in two).  Node (i, j, k) sits at
 * (lo + i h, lo + j h, lo + k h); a 3D grid array holds the (n+1)^3 node values,
 * element (k (n+1) + j) (n+1) + i.  A node is in Omega iff the level function
 * above is negative there.  The control points (the GMRES unknowns, where g and
 * f on the surface are sampled and phi lives) are all crossings of grid edges
 * with the surface, M of them, in the order kfbi3_prob_points reports.
 * Surface derivatives of a density come from weighted least-squares
 * tangent-plane quadratics over the control points within 2.5 h; jumps use the
 * surface's shape operator; v+ at a control point is the quadratic through
 * ten nodes around it (the 7-point cross plus three diagonals toward it).
 * Conventions as above (device FP64 arrays, context stream, errors). */
typedef struct kfbi_prob3 kfbi_prob3;

typedef struct {
    int n;              /* intervals per axis: 64, 128 or 256 */
    double lo, hi;      /* the cube */
    double kappa;       /* >= 0 */
    double axes[3];     /* semi-axes a, b, c of the ellipsoid, centred at the origin;
                           it must keep two cells away from the box */
    double tol;         /* GMRES relative residual tolerance (<= 0: 1e-10) */
    int restart;        /* GMRES restart length (<= 0: 50; at most 64) */
    int max_iter;       /* GMRES iteration cap (<= 0: 500) */
} kfbi_desc3;

/* Builds the plan on the host (classification, crossings, fits, stencils) and
 * uploads it.  KFBI_ERR_GEOMETRY: the ellipsoid reaches within two cells of the
 * box, or n is not supported.  Synchronises. */
kfbi_status kfbi3_prob_create(kfbi_ctx* ctx, const kfbi_desc3* desc, kfbi_prob3** out);
kfbi_status kfbi3_prob_destroy(kfbi_prob3* prob);
/* M control points, irregular nodes, device bytes held (host outputs, may be NULL). */
kfbi_status kfbi3_prob_info(const kfbi_prob3* prob, int* M, int* n_irregular, size_t* device_bytes);
/* pts: host M x 3 control point coordinates; axis: host M, the axis (0 x, 1 y,
 * 2 z) of the grid edge each lies on.  Either may be NULL. */
kfbi_status kfbi3_prob_points(const kfbi_prob3* prob, double* pts, int* axis);
/* inside: host (n+1)^3 bytes, 1 for nodes in Omega. */
kfbi_status kfbi3_prob_mask(const kfbi_prob3* prob, unsigned char* inside);
/* node: host, one per irregular node: ((k-1) n + (j-1)) n + (i-1), in the
 * order of increasing (k, j, i). */
kfbi_status kfbi3_prob_irregular(const kfbi_prob3* prob, int* node);
/* The Cartesian jumps at every control point for [v] = phi, [F] = f_gamma
 * (NULL: 0) and [d_n v] = 0.  J: device 10 M, component-major: J[c M + m] for
 * c = [v], [v_x], [v_y], [v_z], [v_xx], [v_yy], [v_zz], [v_xy], [v_xz], [v_yz]. */
kfbi_status kfbi3_jumps(kfbi_prob3* prob, const double* phi, const double* f_gamma, double* J);
/* K_D phi = (I/2 + W) phi at the control points.  phi, Kphi: device M. */
kfbi_status kfbi3_apply(kfbi_prob3* prob, const double* phi, double* Kphi);
/* One interface solve with [v] = phi (NULL: 0), F = f_grid masked to Omega
 * (NULL: 0) and [F] = f_gamma (NULL: 0): the grid solution (vgrid, device
 * (n+1)^3, may be NULL) and v+ at the control points (vz, device M, may be NULL). */
kfbi_status kfbi3_interface_solve(kfbi_prob3* prob, const double* phi, const double* f_grid,
                                  const double* f_gamma, double* vgrid, double* vz);
/* The whole solve, as kfbi_solve: f_grid device (n+1)^3, f_gamma and g device M
 * at the control points; u_grid (zero outside Omega) and u_gamma outputs; phi
 * device M, initial guess in, density out.  Synchronises. */
kfbi_status kfbi3_solve(kfbi_prob3* prob, const double* f_grid, const double* f_gamma, const double* g,
                        double* u_grid, double* u_gamma, double* phi, int* iters, double* rel_res);
/* Alg. 5 alone, as kfbi_gmres.  Synchronises. */
kfbi_status kfbi3_gmres(kfbi_prob3* prob, const double* rhs, double* phi, double tol, int max_iter,
                        int* iters, int* applies, double* rel_res);

/* ---------------------------------------------------------------- diagnostics */

const char* kfbi_status_str(kfbi_status s);
const char* kfbi_last_error(void);
/* Kernel timing of the K_D apply.  While timing is on, every apply (also the
 * ones inside kfbi_gmres and kfbi_solve) launches its three kernels directly
 * on the context stream (no graph), each recording a start and an end HIP event
 * from its own dispatch packet, without synchronising; kfbi_apply_timing
 * synchronises and returns the average duration in microseconds of the
 * correction (Alg. 2), the sparse fast solve (Alg. 4) and the interpolation
 * (Alg. 3) launches over the applies recorded since timing was switched on
 * (at most 4096).  kfbi_set_timing(prob, 1) also clears the record. */
kfbi_status kfbi_set_timing(kfbi_prob* prob, int on);
kfbi_status kfbi_apply_timing(kfbi_prob* prob, double* us_correct, double* us_modes,
                              double* us_interp, int* count);

#ifdef __cplusplus
}
#endif
#endif /* KFBI_H */
