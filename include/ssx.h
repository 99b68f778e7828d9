/*
 * ssx.h -- C ABI of the surface-source subproblem library (libssx.so).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the operators
 * of the surface-source subproblem of W. W. Symes, "Efficient Computation
 * of Extended Surface Sources" (arXiv 2203.16573):
 *
 *   F    pressure source on the line z = z_s  ->  pressure traces on z = z_r
 *        (the operator S of the Operators section, eqn sdef);
 *   F^T  its exact discrete transpose (eqn sadj1, Appendix A);
 *   A    multiplication by the lateral distance |x - x_s| (eqn penop);
 *   M^-1 = D W^-1 D, D = (I + a^2 A^T A)^(-1/2), W^-1 the thin-slab
 *        symmetrised pressure-to-source operator (eqns defprecond,
 *        winvcomp, lamnear);
 *   and Algorithm 1 (preconditioned CG) on N h = F^T d,
 *   N = F^T F + alpha^2 A^T A (the penalised problem esisp);
 *   and the same in the weighted norms of the Accelerated Iterative
 *   Inversion section: N_w h = F^T W_d d, N_w = F^T W_d F + alpha^2 A^T W_m A
 *   (the normpart system), W_d and W_m thin-slab weights;
 *   the other blocks of the vector modelling operator (V: normal load to
 *   normal velocity, eqn vdef), the time-reversal inverse 4 V^T (eqn
 *   approxinv), Lambda~ and its transpose (eqns lamtilde, lamtransp);
 *   and the gradient in kappa of the data misfit, by the adjoint state of
 *   the discrete scheme (the variable-projection outer problem).
 *
 * Discretisation: 2D staggered grid (p on nodes, v_x and v_z on half
 * nodes), order 2 in time and 4 or 8 in space, split-field PML of npml
 * cells added outside the physical grid, linear interpolation for sampling
 * and its transpose (divided by h) for injection (Numerical Examples,
 * "Synthetic models and simulation").  Time alignment: source sample n
 * enters the update p^n -> p^{n+1}; pressure trace sample n is p^{n+1};
 * normal-velocity trace sample n is v_z^{n+1/2}.
 *
 * Conventions for every entry point below:
 *  - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *    row-major, of the context's vector dtype (double for SSX_F64 fields,
 *    float otherwise).  Trace arrays are [nshots][nt][n] with the trace
 *    index fastest.  The library never frees caller memory and keeps no
 *    reference to it after the call returns.
 *  - All device work is ordered on the stream given to ssx_create (work
 *    the library forks to a stream of its own is joined back into it
 *    before the call returns, see SSX_OPT_OVERLAP); calls return before the
 *    work finishes unless stated otherwise.
 *  - Inputs and outputs must not overlap unless stated otherwise.
 *  - Errors are returned as ssx_status; no exception crosses the ABI.  On an
 *    error the outputs are unspecified and the context stays usable, except
 *    after SSX_ERR_HIP.  ssx_last_error() describes the last error of the
 *    calling thread.
 */
#ifndef SSX_H
#define SSX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssx_ctx ssx_ctx;

typedef enum {
  SSX_OK = 0,
  SSX_ERR_ARG = 1,        /* invalid argument or geometry                 */
  SSX_ERR_CFL = 2,        /* dt above the stability bound                 */
  SSX_ERR_OOM = 3,        /* device allocation failed / workspace too small*/
  SSX_ERR_HIP = 4,        /* HIP runtime error (context no longer usable)  */
  SSX_ERR_BREAKDOWN = 5,  /* PCG: <g,r> or <p,q> became zero               */
  SSX_ERR_NONFINITE = 6   /* PCG: a non-finite scalar appeared             */
} ssx_status;

typedef enum { SSX_F64 = 0, SSX_F32 = 1, SSX_F16 = 2, SSX_BF16 = 3 } ssx_dtype;

/* penalty operators for ssx_penalty */
typedef enum {
  SSX_PEN_A = 0,      /* y = A x,                      A = |x_k - x_s|     */
  SSX_PEN_ATA = 1,    /* y = A^T A x                                        */
  SSX_PEN_DHALF = 2   /* y = (1 + a^2 A^T A)^(-1/2) x  (a = argument a)     */
} ssx_penalty_op;

/*
 * Problem description.  Physical grid nz x nx (z slow, x fast), spacing h
 * (metres) in both directions, node (i, j) at depth i h and lateral
 * position j h.  npml absorbing cells are added on every side; pml_R is the
 * target reflection coefficient of the layer.  Source line: ns samples at
 * depth z_src, lateral positions x_src0 + k h (k < ns); receiver line
 * likewise.  Lateral positions must lie on grid columns; depths may fall
 * between rows (linear interpolation).  slab_dz: signed offset, in cells,
 * of the thin-slab datum from the source line (positive = deeper), used by
 * the preconditioner.  nshots subproblems share the model and both lines
 * and differ in their physical point x_s (given to ssx_create) and data.
 * field_dtype: wavefield storage (F64, F32, F16, BF16); vec_dtype: traces
 * and Krylov vectors, which must be F64 for F64 fields and F32 otherwise.
 * rslab_dz: signed offset, in cells, of the datum of a second thin slab
 * around the receiver line (positive = deeper), which carries the
 * data-space weight W_d of the weighted entry points; 0 leaves that slab
 * out (the weighted entry points then return SSX_ERR_ARG).
 */
typedef struct {
  int32_t nz, nx;
  double h, dt;
  int32_t nt;
  int32_t order;        /* 4 or 8 */
  int32_t npml;
  double pml_R;
  double z_src, x_src0;
  int32_t ns;
  double z_rec, x_rec0;
  int32_t nr;
  int32_t slab_dz;
  int32_t nshots;
  int32_t field_dtype;  /* ssx_dtype */
  int32_t vec_dtype;    /* ssx_dtype */
  int32_t rslab_dz;     /* 0: no receiver-side slab */
} ssx_problem;

/* Host-only check of a problem and model (no device work).  Rejects:
 * nz or nx below order+1; order not 4 or 8; negative npml; non-positive h,
 * dt, nt, ns, nr or nshots; lines off grid columns or outside the physical
 * grid; slab_dz == 0; dtype combinations other than F64/F64 and
 * {F32,F16,BF16}/F32; non-finite or non-positive kappa or rho (ARG); and
 * c_max dt / h above 1 / (sqrt(2) sum_m |c_m|) (CFL).  kappa_host may be
 * NULL to check the problem alone (the CFL test is then skipped). */
ssx_status ssx_validate(const ssx_problem* prob, const double* kappa_host, double rho);

/* Device bytes a context for this problem needs (all fields, coefficients,
 * slab, PCG vectors and scratch); 0 if the problem is invalid. */
size_t ssx_footprint(const ssx_problem* prob);

/* Create a context.  kappa_host: HOST array [nz][nx] of bulk modulus (Pa),
 * read during the call only; rho: constant density (kg/m^3) (see
 * ssx_create_density for a density array); xs_host: HOST
 * array [nshots] of the physical point of each shot (lateral position, m).
 * stream: hipStream_t for all work of this context (NULL = default stream).
 * workspace: optional DEVICE buffer of at least ssx_footprint(prob) bytes,
 * owned by the caller and used for every internal buffer (then the library
 * allocates no device memory); NULL makes the library allocate it.  The
 * call synchronises the stream once (coefficient upload). */
ssx_status ssx_create(const ssx_problem* prob, const double* kappa_host, double rho,
                      const double* xs_host, void* stream, void* workspace,
                      size_t workspace_bytes, ssx_ctx** out);

/* The same for a model with variable density (the operators of the paper
 * carry both kappa and rho): rho_host, HOST array [nz][nx] of density at
 * the pressure nodes (kg/m^3), read during the call only.  Each velocity
 * update uses the mean density of its two nodes (a half node beyond the
 * last node takes that node's value); the stability bound uses the largest
 * sqrt(kappa / rho).  Such a context runs the split kernels or the fused
 * one-step kernel with one tile per workgroup: SSX_OPT_TILE_LOOP and 4 or
 * 8 slab steps per launch return SSX_ERR_ARG.  SSX_ERR_ARG for a null
 * rho_host or non-finite or non-positive values. */
ssx_status ssx_create_density(const ssx_problem* prob, const double* kappa_host,
                              const double* rho_host, const double* xs_host, void* stream,
                              void* workspace, size_t workspace_bytes, ssx_ctx** out);

/* Release the context (waits for its stream).  NULL is ignored. */
void ssx_destroy(ssx_ctx* ctx);

/* d = F h (Operators section, eqn sdef; one full simulation per shot).
 * h: [nshots][nt][ns] -> d: [nshots][nt][nr]. */
ssx_status ssx_fwd(ssx_ctx* ctx, const void* h, void* d);

/* g = F^T r, the exact transpose of ssx_fwd (eqn sadj1, Appendix A): a
 * reverse-time sweep driven by the residual traces, no stored forward
 * states.  r: [nshots][nt][nr] -> g: [nshots][nt][ns]. */
ssx_status ssx_adj(ssx_ctx* ctx, const void* r, void* g);

/* Thin-slab vector operator X (eqns fwd, lamnear): normal-load source f on
 * the source line of the slab, pressure P and normal velocity V recorded on
 * the datum z_s + slab_dz h.  f: [nshots][nt][ns] -> P, V: [nshots][nt][ns]. */
ssx_status ssx_slab_fwd(ssx_ctx* ctx, const void* f, void* P, void* V);

/* Exact transpose of ssx_slab_fwd: a enters the pressure-trace slot, b the
 * normal-velocity slot; f: the normal-load source slot. */
ssx_status ssx_slab_adj(ssx_ctx* ctx, const void* a, const void* b, void* f);

/* Diagonal operators of the penalty (eqn penop; the outer factors of eqn
 * defprecond), per shot with its own x_s: see ssx_penalty_op.  x and y may
 * be the same array.  x, y: [nshots][nt][ns]. */
ssx_status ssx_penalty(ssx_ctx* ctx, int op, double a, const void* x, void* y);

/* g = M^-1 r = D W^-1 D r with D = (1 + alpha_hat^2 A^T A)^(-1/2) and
 * W^-1 = s X^T J X, J (P, V) = (V, P), s = 4 sign(slab_dz) (eqns
 * defprecond and winvcomp: one forward and one adjoint thin-slab
 * simulation).  r, g: [nshots][nt][ns]. */
ssx_status ssx_precond(ssx_ctx* ctx, double alpha_hat, const void* r, void* g);

/* q = N p = F^T F p + alpha^2 A^T A p (the normal operator of esisp), and
 * Fp = F p if Fp is not NULL.  p, q: [nshots][nt][ns]; Fp: [nshots][nt][nr]. */
ssx_status ssx_normal(ssx_ctx* ctx, double alpha, const void* p, void* q, void* Fp);

/* Per-shot FP64 inner products <x, y> over n elements per shot (shots at
 * stride n), deterministic reduction order.  out_host: HOST [nshots];
 * synchronises the stream. */
ssx_status ssx_dot(ssx_ctx* ctx, const void* x, const void* y, int64_t n,
                   double* out_host);

/* Allocation-free per-shot FP64 inner products, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and reduction order as
 * ssx_dot, without a context.  x, y: DEVICE arrays of nshots vectors of n
 * elements (shots at stride n) of vec_dtype (SSX_F64 or SSX_F32); out_dev:
 * DEVICE [nshots] doubles receiving <x, y> per shot.  Stream-ordered on
 * `stream` (hipStream_t, NULL = default stream), no synchronisation.  The
 * partial sums live in a static device array of the library (one per GPU,
 * SSX_DOT_STATIC_MAX_SHOTS x 256 doubles, 128 KiB, held until the process
 * ends); no memory is allocated.  Calls that overlap on one GPU share that
 * array and race: order them on one stream.  SSX_ERR_ARG for null pointers,
 * n < 0, nshots outside [1, SSX_DOT_STATIC_MAX_SHOTS] or another dtype. */
#define SSX_DOT_STATIC_MAX_SHOTS 64
ssx_status ssx_dot_static(const void* x, const void* y, int64_t n, int32_t nshots,
                          int32_t vec_dtype, double* out_dev, void* stream);

/* Algorithm 1 (standard PCG, h_0 = 0) on N h = F^T d for every shot:
 * alpha = alpha_rel ||F^T d|| / ||d|| per shot; M^-1 as ssx_precond with
 * alpha_hat = alpha_rel when use_precond != 0, M = I otherwise (plain CG).
 * Step lengths, beta and all inner products are FP64 on the device.  Runs
 * maxit iterations, or stops early once every shot has ||r_k|| <=
 * rtol ||r_0|| (rtol > 0 only).  d: [nshots][nt][nr]; h_out:
 * [nshots][nt][ns].  hist_host: HOST [nshots][maxit+1][4] or NULL, row k =
 * (||r_k||, ||g_k||, <g_k, r_k>, ||F h_k - d||).  iters_host: HOST, the
 * iterations run.  Synchronises the stream before returning.  Algorithm 1
 * is run as stated: a change of sign of <g,r> (M^-1 indefinite on that
 * residual) does not stop it (hist records <g,r>).  Returns
 * SSX_ERR_BREAKDOWN / SSX_ERR_NONFINITE if <g,r> or <p,q> became zero or
 * non-finite for any shot (that shot's iterate is frozen at its last valid
 * value). */
ssx_status ssx_pcg_solve(ssx_ctx* ctx, const void* d, double alpha_rel, int32_t maxit,
                         double rtol, int32_t use_precond, void* h_out,
                         double* hist_host, int32_t* iters_host);

/* Heterogeneous batch (serving several requests at once): contexts of any
 * grid sizes, record lengths, shot counts, lines and models -- one stencil
 * order, one field type, one vector type, one stream -- solved together.
 * ssx_batch_create takes n >= 1 distinct contexts (the batch keeps the
 * pointers: destroy the batch before any of them; it owns no device memory
 * beyond its captured graphs).  SSX_ERR_ARG for a null or repeated context
 * or contexts that differ in order, types or stream.
 *
 * ssx_batch_pcg_solve runs Algorithm 1 for every member as ssx_pcg_solve
 * does (d[i], h_out[i]: DEVICE, member i's layouts; alpha_rel[i] per member;
 * hist_host[i]: HOST [nshots_i][maxit+1][4] or NULL, hist_host itself may
 * be NULL; iters_host, status_host: HOST [n] or NULL, each member's
 * iterations and the status its own solve would return), with its
 * propagations merged:
 * the members' solves advance in lockstep, and each propagation stage they
 * reach together runs as one sequence of launches in which every time
 * step advances every member's grid (members with shorter records drop out
 * of the later steps), up to 6 grids per launch of the fused step kernel
 * (tile height 16, one tile per workgroup, every shot of a member in the
 * same launch).  Each member's results are bitwise those of its own
 * ssx_pcg_solve, whatever its launch options (every launch form evaluates
 * the same expressions).  A member stopping early (rtol, an error) leaves
 * the lockstep; the others go on.  Synchronises the stream before
 * returning; returns the first member's error (the others' results stay
 * valid), its message naming the member.  The members' own stream-ordered work must not run concurrently
 * with the batch solve. */
typedef struct ssx_batch ssx_batch;
ssx_status ssx_batch_create(int32_t n, ssx_ctx* const* ctxs, ssx_batch** out);
ssx_status ssx_batch_pcg_solve(ssx_batch* batch, const void* const* d, const double* alpha_rel,
                               int32_t maxit, double rtol, int32_t use_precond,
                               void* const* h_out, double* const* hist_host,
                               int32_t* iters_host, int32_t* status_host);
void ssx_batch_destroy(ssx_batch* batch);

/* ---- weighted normal equations (Accelerated Iterative Inversion, the
 * normpart system S* = S^T W_d, A* = A^T W_m; weights of Computing and
 * Symmetrizing Lambda).  All return SSX_ERR_ARG when the context was
 * created with rslab_dz == 0. */

/* y = W_d r: the symmetrised pressure-to-source operator of the receiver
 * surface (the "similar definition" beside eqn winvcomp), computed like
 * W^-1 on the receiver-side slab: normal load on z_rec, pressure and normal
 * velocity recorded on the datum z_rec + rslab_dz h, exchanged, and the
 * transposed sweep read from the normal-load slot, scaled by
 * 4 sign(rslab_dz).  Two slab simulations.  r, y: [nshots][nt][nr]. */
ssx_status ssx_weight_d(ssx_ctx* ctx, const void* r, void* y);

/* y = W_m x: the symmetrised inverse pressure-to-source operator (eqn wcomp)
 * on the source-side slab: a pressure source on z_src instead of a normal
 * load, the same exchange on the datum, read back from the pressure-source
 * slot and scaled by sign(slab_dz), so that W_m is positive and inverse to
 * W^-1 on laterally uniform input.  Two slab simulations.
 * x, y: [nshots][nt][ns]. */
ssx_status ssx_weight_m(ssx_ctx* ctx, const void* x, void* y);

/* q = N_w p = F^T W_d F p + alpha^2 A^T W_m A p, and Fp = F p if Fp is not
 * NULL (the W_m term is skipped when alpha == 0).  p, q: [nshots][nt][ns];
 * Fp: [nshots][nt][nr]. */
ssx_status ssx_normal_w(ssx_ctx* ctx, double alpha, const void* p, void* q, void* Fp);

/* Algorithm 1 on N_w h = F^T W_d d for every shot, as ssx_pcg_solve except
 * that alpha (per metre, the weighted norms making F nearly unitary) is
 * used as given, both in N_w and as alpha_hat of M^-1 = D W^-1 D (eqn
 * defprecond); use_precond == 0 runs M = I.  hist rows as in ssx_pcg_solve
 * (||r_k||, ||g_k||, <g_k, r_k>, ||F h_k - d||); ||g_k|| with M^-1 applied
 * is the normal residual of the norm1 form.  Same return codes. */
ssx_status ssx_pcg_solve_w(ssx_ctx* ctx, const void* d, double alpha, int32_t maxit,
                           double rtol, int32_t use_precond, void* h_out,
                           double* hist_host, int32_t* iters_host);

/* The subproblem with the normal load as the unknown (the source vector's
 * second component, observed as normal velocity on the receiver line):
 * min_f ||V f - d||^2 + alpha^2 ||A f||^2, Algorithm 1 on N_v f = V^T d,
 * N_v = V^T V + alpha^2 A^T A, alpha = alpha_rel ||V^T d|| / ||d||, with
 * M = I (the paper derives no preconditioner for this form).  d:
 * [nshots][nt][nr] normal-velocity traces; f_out: [nshots][nt][ns]; hist
 * and return codes as ssx_pcg_solve (column 4: ||V f_k - d||).  Needs the
 * normal-velocity rows of ssx_fwd_v (SSX_ERR_ARG otherwise). */
ssx_status ssx_pcg_solve_v(ssx_ctx* ctx, const void* d, double alpha_rel, int32_t maxit,
                           double rtol, void* f_out, double* hist_host, int32_t* iters_host);

/* ---- V, the time-reversal inverse and Lambda~ (Time Reversal, Unitarity,
 * Computing and Symmetrizing Lambda). */

/* y = V f (eqn vdef): normal load f on the source line (normal-velocity
 * rows at z_src), normal velocity sampled on the receiver line (rows at
 * z_rec); one full simulation.  f: [nshots][nt][ns] -> y: [nshots][nt][nr].
 * SSX_ERR_ARG when z_src or z_rec has no pair of normal-velocity rows
 * inside the physical grid (a line on its last row). */
ssx_status ssx_fwd_v(ssx_ctx* ctx, const void* f, void* y);

/* g = V^T r, the exact transpose of ssx_fwd_v (reverse-time sweep).
 * r: [nshots][nt][nr] -> g: [nshots][nt][ns]. */
ssx_status ssx_adj_v(ssx_ctx* ctx, const void* r, void* g);

/* h = 4 V^T d: the time-reversal approximate inverse of F (eqn approxinv,
 * V^T F ~ I/4 for downgoing fields; the normal velocity of a normal load
 * has the same sign on both of its sides, so the factor does not depend on
 * whether the receivers lie above or below the sources).
 * d: [nshots][nt][nr] -> h: [nshots][nt][ns]. */
ssx_status ssx_tr_inverse(ssx_ctx* ctx, const void* d, void* h);

/* y = B x, B a block of the vector modelling operator (Operators section:
 * the source vector (h, f) on z_src to the traces (P_r p, P_r v_z) on z_rec):
 * src 0 a pressure source, 1 a normal load on the source line; rec 0
 * pressure, 1 normal velocity on the receiver line; with transpose != 0,
 * y = B^T x.  Block (0, 0) is ssx_fwd / ssx_adj, block (1, 1) ssx_fwd_v /
 * ssx_adj_v.  x: [nshots][nt][ns] (or [nshots][nt][nr] transposed), y the
 * other.  Blocks other than (0, 0) need the normal-velocity rows of
 * ssx_fwd_v (SSX_ERR_ARG otherwise). */
ssx_status ssx_block(ssx_ctx* ctx, int32_t src, int32_t rec, int32_t transpose, const void* x,
                     void* y);

/* Gradient of the data misfit J = 1/2 ||F h - d||^2 with respect to the
 * bulk modulus at fixed h (the derivative that the variable-projection
 * outer problem of the Introduction needs: at the subproblem's minimiser
 * h the reduced objective's gradient is this partial gradient), by the
 * adjoint state of the discrete scheme: g = (1/kappa) sum_n P~^{n+1} r^n,
 * r^n = E_h h^n - D^- v^{n+1/2} stored by a forward sweep, P~ the
 * transposed pressure of the sweep driven by F h - d.  g covers the
 * physical grid, [nshots][nz][nx] (row-major, vector dtype); the absorbing
 * layer's coefficients (copies of the edge values, damping profile) are
 * held fixed.  J_host: HOST [nshots] or NULL (then the call does not
 * synchronise).  h: [nshots][nt][ns]; d: [nshots][nt][nr].  F64 and F32
 * fields only (SSX_ERR_ARG otherwise).  The first call allocates the step
 * history, nt * nshots * nz * nx' field values plus an FP64 accumulator
 * of nshots * nz * nx' (nx' = nx rounded out to the grid's aligned groups
 * of four columns, at most nx + 6), held until ssx_destroy (also for contexts made with a workspace);
 * SSX_ERR_OOM if that fails.  Two full simulations, one step per launch
 * (replayed as one captured graph when graphs are on). */
ssx_status ssx_misfit_gradient(ssx_ctx* ctx, const void* h, const void* d, void* g,
                               double* J_host);

/* y = Lambda~ x (eqn lamtilde) or, with transpose != 0, its transpose (eqn
 * lamtransp), on the source-side slab (side 0, x and y [nshots][nt][ns]) or
 * the receiver-side one (side 1, [nshots][nt][nr]; needs rslab_dz != 0):
 * 2 s X^T (0, P) or 2 s X^T (V, 0) with (P, V) = X x and s = 4 sign(dz) of
 * that slab, so that half the sum of the two is ssx_precond's W^-1 (side 0,
 * alpha_hat = 0) or W_d (side 1), eqn winvcomp.  Two slab simulations. */
ssx_status ssx_lambda(ssx_ctx* ctx, int32_t side, int32_t transpose, const void* x, void* y);

/* Execution options (results do not depend on them, see each value):
 *   SSX_OPT_GRAPHS      1 (default): replay each whole propagation as a
 *                       captured HIP graph; 0: plain stream launches.
 *   SSX_OPT_STEP_KERNEL 1 (default): one fused launch per time step
 *                       (velocity and pressure on an LDS-staged tile);
 *                       0: one velocity and one pressure launch per step.
 *   SSX_OPT_TILE_Z      tile height of the fused kernel on the full grid
 *                       and the thin slab: 8, 16 or 32 (32 not for F64
 *                       fields); 0 picks a default from the grid size.
 *   SSX_OPT_TILE_Z_SLAB the same for the thin slab only.
 *   SSX_OPT_STEPS_PER_LAUNCH      time steps per launch on the full
 *                       grid: 1 (default), the fused one-step kernel; 2, 4
 *                       or 8, the multi-step kernel: each workgroup holds
 *                       a region of at most 56 rows and one strip of
 *                       columns in LDS and advances it that many steps,
 *                       recomputing a halo of that many stencil reaches
 *                       on each side; a grid taller than 56 rows is cut
 *                       into overlapping windows (order 4: 2, 4 or 8
 *                       steps; order 8: 2 steps, or any of them for a grid
 *                       of at most 56 rows).  F64 fields and density
 *                       arrays take 64-column strips.
 *   SSX_OPT_STEPS_PER_LAUNCH_SLAB the same for the thin slabs.
 *   SSX_OPT_STRIP       strip width in columns of the multi-step kernel on
 *                       the full grid, halo included: 64 or 128; 0 (the
 *                       default): 64 for F64 fields and density arrays,
 *                       else 128.  Order 8 with 8 steps needs 128.
 *   SSX_OPT_SLAB_STRIP  the same for the thin slabs.
 *   SSX_OPT_SHOT_GROUP  shots advanced together by one launch on the full
 *                       grid and the thin slab: the shots are split into
 *                       balanced groups of at most this many, and each
 *                       group runs its whole record before the next one;
 *                       0 (default) picks the largest group whose per-step
 *                       traffic fits the last-level cache (176 MiB at 6
 *                       field values and one coefficient per cell).
 *   SSX_OPT_SHOT_GROUP_SLAB the same for the thin slab only.
 *   SSX_OPT_TILE_LOOP   one-step fused kernel on the full grid: 0
 *                       (default) one tile per workgroup; 1 one workgroup
 *                       per tile of the absorbing frame, line rows and grid
 *                       edges, and for the interior tiles a set of
 *                       workgroups the device holds at once, each taking
 *                       tiles in turn and loading the next one while it
 *                       computes the current one; a value of 8 or more
 *                       also caps that set at the value rounded down to a
 *                       multiple of 8.
 *   SSX_OPT_OVERLAP     1 (default): the weighted normal operator runs its
 *                       model-space term (W_m, two slab simulations) on a
 *                       second stream of the library's, concurrently with
 *                       F, W_d and F^T, and joins it into the context's
 *                       stream before summing; 0: all on the context's
 *                       stream.
 * Returns SSX_ERR_ARG for an unknown option or value, or a value that does
 * not combine with the context's problem or with the other options set
 * (steps per launch and strip width are checked together). */
typedef enum {
  SSX_OPT_GRAPHS = 0,
  SSX_OPT_STEP_KERNEL = 1,
  SSX_OPT_TILE_Z = 2,
  SSX_OPT_TILE_Z_SLAB = 3,
  SSX_OPT_STEPS_PER_LAUNCH = 4,
  SSX_OPT_STEPS_PER_LAUNCH_SLAB = 5,
  SSX_OPT_SHOT_GROUP = 6,
  SSX_OPT_SHOT_GROUP_SLAB = 7,
  SSX_OPT_SLAB_STRIP = 8,
  SSX_OPT_TILE_LOOP = 9,
  SSX_OPT_OVERLAP = 10,
  SSX_OPT_STRIP = 11
} ssx_option;
ssx_status ssx_set_option(ssx_ctx* ctx, int option, int value);

/* Message for the last error on the calling thread ("" if none). */
const char* ssx_last_error(void);

/* Name of the kernel that dominates a full-grid propagation, and the
 * number of grid cells one of its launches advances by one time step
 * (the shots of one group, see SSX_OPT_SHOT_GROUP), for throughput
 * accounting. */
const char* ssx_step_kernel_name(ssx_ctx* ctx);
int64_t ssx_cells_per_launch(ssx_ctx* ctx);

/* Launch shape of the full-grid step as the next propagation will run it:
 * shape[0] tile height, shape[1] time steps per launch, shape[2] shots per
 * launch, shape[3] the tile-loop setting (options resolved, defaults
 * included).  shape is a host array of four; SSX_ERR_ARG for a null
 * argument. */
ssx_status ssx_launch_shape(ssx_ctx* ctx, int32_t* shape);

/* ======================================================================
 * Three dimensions (the 3D form of the Operators section's acoustic
 * system, the generalisation the closing remarks name): F maps a pressure
 * source on the plane z = z_src to pressure traces on the plane z = z_rec,
 * F^T is its exact discrete transpose (eqns sdef and sadj1, Appendix A);
 * with the penalty, the thin-slab preconditioner and Algorithm 1 on the
 * same plane geometry.
 * Staggered grid (p on nodes, v_x, v_y, v_z on the half nodes of their
 * axis), order 2 in time and 4 or 8 in space, the split-field absorbing
 * layer of npml cells on every side, constant density; sampling and
 * injection as in 2D (linear interpolation in z, transpose divided by h).
 * Time alignment as in 2D: source sample n enters p^n -> p^{n+1}, trace
 * sample n is p^{n+1}.
 * ==================================================================== */
typedef struct ssx3_ctx ssx3_ctx;

/*
 * Physical grid nz x ny x nx (z slowest, x fastest), spacing h in every
 * direction, node (i, k, j) at depth i h, y = k h, x = j h.  Source plane:
 * nsx x nsy traces at depth z_src, lateral positions (x_src0 + a h,
 * y_src0 + b h), trace index b nsx + a; receiver plane likewise.  Lateral
 * positions must lie on grid nodes; depths may fall between nodes.
 * field_dtype: SSX_F64 or SSX_F32, also the type of every trace array.
 * slab_dz and (x_s, y_s) play the roles of the 2D slab_dz and x_s: the
 * thin slab of M^-1 around z_src with its datum slab_dz cells away, and
 * the point from which A measures lateral distance, sqrt((x - x_s)^2 +
 * (y - y_s)^2).
 */
typedef struct {
  int32_t nz, ny, nx;
  double h, dt;
  int32_t nt;
  int32_t order;        /* 4 or 8 */
  int32_t npml;
  double pml_R;
  double z_src, x_src0, y_src0;
  int32_t nsx, nsy;
  double z_rec, x_rec0, y_rec0;
  int32_t nrx, nry;
  int32_t field_dtype;  /* SSX_F64 or SSX_F32 */
  int32_t slab_dz;      /* signed thin-slab datum offset (cells), nonzero */
  double x_s, y_s;      /* the physical point, for the penalty A */
} ssx3_problem;

/* Host-only check (no device work).  Rejects (ARG): a grid below order + 1
 * nodes on an axis; order not 4 or 8; negative npml; non-positive h, dt, nt
 * or trace counts; pml_R outside (0, 1); planes off grid nodes or outside
 * the physical grid; a padded grid with more than 65535 planes in z; field
 * types other than F64 and F32; non-finite or non-positive kappa or rho.
 * CFL: c_max dt / h above 1 / (sqrt(3) sum_m |c_m|).  kappa_host (HOST,
 * [nz][ny][nx], Pa) may be NULL to check the problem alone. */
ssx_status ssx3_validate(const ssx3_problem* prob, const double* kappa_host, double rho);

/* Device bytes a 3D context owns (the full grid's and the thin slab's ten
 * fields and coefficients, ten trace vectors, FP64 scalars); 0 if the
 * problem is invalid. */
size_t ssx3_footprint(const ssx3_problem* prob);

/* Create a 3D context: kappa_host HOST [nz][ny][nx] bulk modulus (Pa), read
 * during the call only; rho constant density (kg/m^3); stream the
 * hipStream_t of all its work (NULL = default stream).  Allocates
 * ssx3_footprint(prob) bytes of device memory (SSX_ERR_OOM on failure). */
ssx_status ssx3_create(const ssx3_problem* prob, const double* kappa_host, double rho,
                       void* stream, ssx3_ctx** out);

/* d = F h.  h: DEVICE [nt][nsy][nsx], d: DEVICE [nt][nry][nrx], both of the
 * field type; asynchronous on the context's stream; one call at a time per
 * context (the fields are the context's). */
ssx_status ssx3_fwd(ssx3_ctx* ctx, const void* h, void* d);

/* g = F^T r.  r: DEVICE [nt][nry][nrx], g: DEVICE [nt][nsy][nsx]. */
ssx_status ssx3_adj(ssx3_ctx* ctx, const void* r, void* g);

/* y = op(x) on source-plane traces [nt][nsy][nsx], op as ssx_penalty's with
 * the 3D lateral distance (eqn penop; defprecond for SSX_PEN_DHALF with
 * a = alpha_hat); x and y may be the same array. */
ssx_status ssx3_penalty(ssx3_ctx* ctx, int op, double a, const void* x, void* y);

/* g = M^-1 r = D W^-1 D r (eqns defprecond, winvcomp): W^-1 = s X^T J X on
 * the thin slab, X a normal load on z_src recorded as pressure and normal
 * velocity on the datum plane, J their exchange, s = 4 sign(slab_dz),
 * D = (1 + alpha_hat^2 A^T A)^(-1/2).  r, g: DEVICE [nt][nsy][nsx], not
 * overlapping; alpha_hat >= 0. */
ssx_status ssx3_precond(ssx3_ctx* ctx, double alpha_hat, const void* r, void* g);

/* Algorithm 1 on N h = F^T d, N = F^T F + alpha^2 A^T A, alpha = alpha_rel
 * ||F^T d|| / ||d||, M^-1 as ssx3_precond with alpha_hat = alpha_rel
 * (use_precond != 0) or M = I; h_0 = 0, maxit iterations (0..4096).
 * d: DEVICE [nt][nry][nrx]; h_out: DEVICE [nt][nsy][nsx]; hist_host: HOST
 * [maxit + 1][4] (||r_k||, ||g_k||, <g_k, r_k>, ||F h_k - d||) or NULL;
 * iters_host: HOST or NULL.  FP64 inner products; the call synchronises
 * the stream once per inner product.  SSX_ERR_BREAKDOWN /
 * SSX_ERR_NONFINITE if <g, r> or <p, q> becomes zero / non-finite (the
 * iterate so far is in h_out). */
ssx_status ssx3_pcg_solve(ssx3_ctx* ctx, const void* d, double alpha_rel, int32_t maxit,
                          int32_t use_precond, void* h_out, double* hist_host,
                          int32_t* iters_host);

/* Release a 3D context (waits for its stream). */
void ssx3_destroy(ssx3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SSX_H */
