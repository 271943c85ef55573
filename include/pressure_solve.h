/*
 * pressure_solve.h -- C ABI of the MI355X (gfx950) direct FFT pressure solve.
 *
 * The method (paper Section 2.1, "Direct FFT"): a forward Fourier transform
 * of every horizontal level turns the pressure equation into one vertical
 * ODE per horizontal wavenumber; each ODE is a tridiagonal system solved by
 * a sweep up and down its column, independently of every other column; a
 * backward transform gives the pressure.  As in the paper, the problem is
 * described once to a plan (FFTW-style planning, Section 2.1) and the plan,
 * with its reusable buffers (the decomposition plan of Section 2.1, last
 * paragraphs), is executed every timestep.
 *
 * Discrete problem solved (a reading of the paper, which names only a
 * Poisson-like elliptic equation, lateral periodicity and vertical
 * tridiagonal columns):
 *   A p = b - mu,   sum(p) = 0,
 *   A = periodic 3-point second differences in x and y (spacings dx, dy)
 *     + V, (V p)_k = [f_{k+1/2}(p_{k+1}-p_k) - f_{k-1/2}(p_k-p_{k-1})] / D_k,
 *   f_{k+1/2} = (rho_k + rho_{k+1})/2 / ((dz_k + dz_{k+1})/2),
 *   D_k = rho_k dz_k, zero flux through the bottom and the top,
 *   mu = the D-weighted mean of b (projection onto the range of A).
 * This is the p-block of [[A,1],[1^T,0]] [p; mu] = [b; 0].
 *
 * Layout of every field argument: level-major C order [nz][ny][nx], x
 * fastest, device memory, element type double for PS_FP64 plans and float
 * for every other precision.  Fields are owned by the caller; the plan owns
 * its workspace and tables.
 *
 * Execution: every call that takes device pointers only enqueues work on
 * the plan's HIP stream and returns; it does not synchronise.  A plan is not
 * reentrant: at most one call per plan may be in flight on its stream, and
 * calls on one plan from several host threads must be serialised by the
 * caller.  Every argument is validated on the host before any device work
 * is enqueued, so an error return means nothing was enqueued.
 *
 * Errors: every function returns a ps_status.  PS_EHIP means a HIP runtime
 * call failed; ps_last_error() then describes it (per host thread).
 */
#ifndef PRESSURE_SOLVE_H
#define PRESSURE_SOLVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_plan ps_plan;
typedef struct ps_batch ps_batch;

typedef enum ps_status {
    PS_OK = 0,
    PS_EINVAL = 1,        /* null/aliased pointer, non-positive spacing or coefficient, NaN/inf */
    PS_EUNSUPPORTED = 2,  /* grid size or precision this library does not implement */
    PS_ENOMEM = 3,        /* device or host allocation failed */
    PS_EHIP = 4,          /* a HIP runtime call failed; see ps_last_error() */
    PS_ESTATE = 5         /* call not valid in the object's current state */
} ps_status;

typedef enum ps_precision {
    /* FP64 transforms and FP64 column solves throughout. */
    PS_FP64 = 0,
    /* FP32 transforms and FP32 column solves; the singular mean column and
     * every near-singular column (lateral eigenvalue below tau times the
     * largest vertical diagonal) are solved in FP64; level sums in FP64. */
    PS_FP32 = 1,
    /* PS_FP32 plus one refinement of every FP32 column solve: the residual
     * of the tridiagonal system is formed in FP64 in registers and one
     * correction sweep is applied. */
    PS_FP32_R2 = 2,
    /* PS_FP32 plus one step of iterative refinement on the 3D residual:
     * r = b - A p is formed with FP64 accumulation, A d = r is solved in
     * PS_FP32 form, and p += d.  Needs rhs and p not to alias. */
    PS_FP32_R1 = 3
} ps_precision;

/* Supported sizes: nx even with nx/2 = 2^a 3^b, 1 <= nx/2 <= 1024;
 * ny = 2^a 3^b, 1 <= ny <= 1024; 1 <= nz <= 256.  Other sizes give
 * PS_EUNSUPPORTED (the CPU oracle accepts any size). */
#define PS_MAX_NX 2048
#define PS_MAX_NY 1024
#define PS_MAX_NZ 256

/* Create a plan (the one-off planning phase of Section 2.1).
 *   out        : receives the plan handle (host pointer, must not be NULL).
 *   nx, ny, nz : grid points in x, y (periodic) and levels in z.
 *   dx, dy     : lateral spacings, > 0.
 *   dz         : host array of nz level thicknesses, each > 0 (copied).
 *   rho        : host array of nz per-level densities rho_k > 0 (copied).
 *   precision  : a ps_precision value.
 *   tau        : near-singular threshold for the FP64 columns of the FP32
 *                forms; <= 0 selects the default 1e-3.  Ignored for PS_FP64.
 *   stream     : hipStream_t to enqueue on (NULL = the null stream).
 * Allocates the device workspace (ps_workspace_bytes) on the current
 * device and uploads the tables; this call synchronises.  Errors:
 * PS_EINVAL, PS_EUNSUPPORTED, PS_ENOMEM, PS_EHIP; *out is NULL on error. */
int ps_plan_create(ps_plan **out, int nx, int ny, int nz, double dx, double dy,
                   const double *dz, const double *rho, int precision, double tau,
                   void *stream);

/* Release the plan and its device memory (synchronises its stream).  NULL is
 * accepted and ignored. */
int ps_plan_destroy(ps_plan *plan);

/* Change the stream later calls enqueue on. */
int ps_plan_set_stream(ps_plan *plan, void *stream);

/* Replace the per-level densities (host array of nz values > 0) without
 * reallocating; synchronises the device first (work enqueued earlier on any
 * stream may still read the tables).  The set of columns solved in FP64 by
 * the FP32 forms stays the one chosen at planning. */
int ps_plan_set_coeffs(ps_plan *plan, const double *rho);

/* Solve A p = b - mu, sum(p) = 0 (Section 2.1: forward transform, one
 * tridiagonal solve per wavenumber column, backward transform).
 *   rhs : device [nz][ny][nx], read only.
 *   p   : device [nz][ny][nx], written.  May alias rhs except for
 *         PS_FP32_R1 (PS_EINVAL).  rhs is not modified.
 * ps_solve, ps_solve_adjoint and ps_grad_coeffs only enqueue kernels and
 * event records / waits on the plan's stream (the FP64 columns fork onto the
 * plan's second stream and join back): no allocation, no memset, no
 * synchronisation, so a caller may capture them into a HIP graph on that
 * stream and replay it with the same pointers. */
int ps_solve(ps_plan *plan, const void *rhs, void *p);

/* ps_solve (adjoint = 0) or ps_solve_adjoint (adjoint != 0) for fields in
 * MONC's own layout p%data(z,y,x) (Section 2.2's Fortran field, z fastest):
 * element (i, j, k) at (i ny + j) nz + k, element type as for ps_solve.  No
 * extra pass over HBM: with the register-resident transforms (the plan's x
 * and y variants >= 1) the x passes move between the field and a plan-owned
 * [kx][j][k] buffer (loads and stores along k, staged in LDS) and the y
 * passes between that buffer and the spectrum; otherwise the x passes
 * transpose between columns and rows in LDS around ps_solve's y and column
 * passes.  The first call on a plan of the first kind allocates that buffer
 * (the size of the spectrum; synchronises): call it once before capturing
 * it into a graph.  PS_FP32_R1: the refinement's residual b - A p is formed
 * in a pass of its own (FP64 accumulation, into a plan-owned field
 * allocated on the first such call), solved, and accumulated into p by the
 * last backward x pass.  rhs and p may alias, except for PS_FP32_R1
 * (PS_EINVAL). */
int ps_solve_zyx(ps_plan *plan, const void *rhs, void *p, int adjoint);

/* One pressure-projection step of the dynamical core around the solve
 * (Section 1: the source terms feed the solve, its pressure corrects the
 * flow).  u, v, w: device [nz][ny][nx] fields of the plan's element type,
 * the provisional velocity on the staggered grid -- u[k][j][i] on the
 * x-face between cells i-1 and i, v on the y-face between rows j-1 and j,
 * w on the face between levels k-1 and k (level 0's w is the bottom
 * boundary, no flux: neither read nor written); no flux through the top.
 * Solves A p = div(u, v, w)/dt (p written to the device field p), with
 *   div = (u_{i+1}-u_i)/dx + (v_{j+1}-v_j)/dy
 *       + (rho_{k+1/2} w_{k+1} - rho_{k-1/2} w_k)/(rho_k dz_k),
 * the divergence formed inside the forward x pass (no right-hand-side
 * field); then, if correct != 0, subtracts dt times the pressure gradient
 * (p_i-p_{i-1})/dx, (p_j-p_{j-1})/dy, (p_k-p_{k-1})/h_{k-1/2} from u, v and w
 * in one further pass, after which div(u, v, w) = 0 up to rounding (div of
 * the gradient is A).  In the PS_FP32_R1 form the refinement's residual
 * div/dt - A p is formed again from u, v, w and p (FP64 accumulation) inside
 * the second solve's forward x pass, so it refers to the FP64 divergence.
 * dt finite and > 0; u, v, w, p distinct.  Asynchronous on the plan's
 * stream. */
int ps_project(ps_plan *plan, void *u, void *v, void *w, double dt, void *p, int correct);

/* Adjoint solve: grhs = S^T gp, the lambda-block of
 * [[A^T,1],[1^T,0]] [lambda; nu] = [gp; 0] -- the gradient of <gp, p> with
 * respect to rhs.  Same layout and aliasing rules as ps_solve (refinement
 * forms run the adjoint in their base FP32 form plus the same refinement). */
int ps_solve_adjoint(ps_plan *plan, const void *gp, void *grhs);

/* Gradient of L = <w, p> with respect to the per-level densities, given
 * lam = S^T w (from ps_solve_adjoint) and the solution p (from ps_solve):
 * grho[k] = -lam^T (dA/drho_k) p.  lam and p are device fields of the
 * plan's element type; grho is a device array of nz doubles, written.
 * Deterministic (fixed-order reductions, no atomics). */
int ps_grad_coeffs(ps_plan *plan, const void *lam, const void *p, double *grho);

/* ps_grad_coeffs for callers that cannot allocate device memory during the
 * call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and the same result, with the
 * per-block partial sums in a fixed device array of the library (2 MiB per
 * GPU, held until the process ends; every valid plan fits, larger needs
 * would give PS_EUNSUPPORTED) instead of the plan's buffer.  Allocates
 * nothing.  All calls on one GPU share that GPU's array: calls that overlap
 * on one GPU (on different streams, or from several host threads) race. */
int ps_grad_coeffs_noalloc(ps_plan *plan, const void *lam, const void *p, double *grho);

/* Device workspace owned by the plan, in bytes. */
size_t ps_workspace_bytes(const ps_plan *plan);

typedef struct ps_plan_info {
    int nx, ny, nz, precision;
    int fp64_columns;     /* near-singular columns solved in FP64 (FP32 forms) */
    double tau;           /* threshold in effect */
    int fft_variant_x;    /* transform kernels chosen by planning / autotuning: */
    int fft_variant_y;    /* forward x, y, ... */
    size_t spectrum_elems;/* complex elements of the spectral layout, nz*(nx/2)*ny */
    int column_variant;   /* column-solve kernel chosen by planning / autotuning */
    int chunks;           /* kx ranges the y / column / y passes are split into */
    int fft_variant_xi;   /* ... and backward x */
    int special_variant;  /* FP64-column kernel: 0 one lane per task through an HBM
                             workspace, 1 staged in LDS */
    int zyx_kc;           /* z-fastest-layout x passes: levels per tile (capped by the
                             tile's rows); with the register-resident passes >= 32
                             selects the wide blocks */
    int fp64_beside;      /* where the FP64 columns (packed kx = 0 row, mean column,
                             near-singular columns) run: the tune cache's fp64_beside */
    int xy_chunks;        /* level ranges in which the forward x + y and backward
                             y + x passes run pairwise (1: whole-field passes) */
} ps_plan_info;

int ps_plan_query(const ps_plan *plan, ps_plan_info *info);

/* Time the implemented kernel variants (x transform, y transform, column
 * solve) for this plan on its stream by coordinate descent, each candidate
 * in two interleaved rounds of reps timed solves (the faster round counts),
 * and keep the fastest.  Uses two temporary device fields
 * of the plan's size.  Choices are cached per (device architecture, nx, ny,
 * nz, precision) for the life of the process -- a later autotune of an equal
 * plan just applies them -- and can be saved to / loaded from a text file
 * (one line per entry: arch nx ny nz precision x_variant y_variant
 * column_variant [fp64_beside [chunks [xi_variant [special_variant [zyx_kc
 * [xy_chunks]]]]]]:
 * fp64_beside where the FP64 columns run: 0 on the plan's stream before the
 * main column kernel, 1 on a second stream beside it (that stream also
 * transforms their rows in y), 2 on a second stream forked after the whole
 * y pass; chunks the number of kx ranges the y / column / y passes are
 * taken in (with fp64_beside 1 only); both defaulting to 1; xi_variant the backward x
 * pass's, defaulting to x_variant; special_variant the FP64-column kernel's
 * (0 or 1), defaulting to 1; zyx_kc the levels per tile of the z-fastest
 * layout's x passes (1..256), defaulting to 64 -- with the register-resident
 * passes, values of 32 or more select blocks of twice the standard levels
 * (32 FP32, 16 FP64) -- timed with ps_solve_zyx); xy_chunks (1..64,
 * default 1) the number of level ranges in which the forward x and y passes,
 * and the backward y and x passes, run pairwise, so that each second pass
 * reads what the first has just written while it is still in the
 * last-level cache (with the register-resident passes; with fp64_beside 1
 * the second stream transforms the FP64 rows of each range after its x
 * pass; the result is the same bit for bit; the autotuner searches it
 * jointly with fp64_beside).
 * Synchronises. */
int ps_plan_autotune(ps_plan *plan, int reps);
int ps_tune_cache_save(const char *path);
int ps_tune_cache_load(const char *path);

/* ---- per-kernel timing ---------------------------------------------------
 * While enabled, every kernel the plan enqueues is bracketed by a pair of HIP
 * events recorded on the plan's stream, and the elapsed times are
 * accumulated per kernel.  ps_plan_profile(plan, 1) clears the totals and
 * starts recording; ps_plan_profile(plan, 0) stops.  ps_plan_profile_report
 * synchronises the stream and returns, for kernel index idx = 0, 1, ...,
 * its name, total milliseconds and number of launches; PS_EINVAL past the
 * last index.  Profiling adds an event pair per launch, so time steps with it
 * disabled when the whole-step rate matters. */
int ps_plan_profile(ps_plan *plan, int enable);
int ps_plan_profile_report(ps_plan *plan, int idx, const char **name, double *total_ms,
                           int *launches);

/* ---- stages, for testing each kernel on its own ------------------------
 * spectrum: device buffer of spectrum_elems complex values of the plan's
 * element type (interleaved re, im) in the packed, transposed layout
 *   spec[k][kx][ky], kx in [0, nx/2), ky in [0, ny),
 * where for kx >= 1 the entry is the 2D DFT coefficient (kx, ky) of level k,
 * and the kx = 0 row packs two real-input transforms: along y it holds
 * DFT_y(X_0 + i X_{nx/2}), X_0 and X_{nx/2} being the x-DC and x-Nyquist
 * coefficients of each row.  Unnormalised forward transform. */
int ps_forward_transform(ps_plan *plan, const void *rhs, void *spectrum);
/* Column solves on a spectrum produced by ps_forward_transform from the same
 * rhs (in place; adjoint != 0 selects the adjoint solve).  The mean column
 * uses the level sums recorded by the preceding ps_forward_transform. */
int ps_spectral_solve(ps_plan *plan, void *spectrum, int adjoint);
/* Backward transform of a solved spectrum (the 1/(nx*ny) factor is applied
 * inside ps_spectral_solve). */
int ps_inverse_transform(ps_plan *plan, const void *spectrum, void *p);

/* ---- batched: many independent solves of uneven sizes ------------------
 * Describe count problems once and solve all of them with one call, replayed
 * from captured hipGraphs (the uneven-decomposition plan of Section 2.1: one
 * plan with reusable buffers per problem, made once and executed every
 * timestep).  Each problem is planned as by ps_plan_create (its size limits
 * apply) with the planning defaults, so a batched solve gives exactly the
 * result of that problem's standalone ps_solve.
 * Mode PS_BATCH_LANES (the only mode): the problems are dealt to `lanes`
 * streams, most points first, each to the lane with the fewest points so
 * far; each lane's solves are captured one after another into one graph on
 * its stream, and a solve forks the lanes from the caller's stream,
 * launches the graphs side by side and joins them back.  Each problem's FP64
 * columns run in order on its lane by default (ps_batch_set_fp64_order).
 *   nx, ny, nz, dx, dy : host arrays of count values.
 *   dz, rho            : host arrays of count host pointers to nz[i] values.
 *   precision          : a ps_precision value, shared by every problem.
 *   stream             : hipStream_t the solves are ordered on (NULL = null
 *                        stream); see ps_batch_set_stream.
 * Allocates every problem's workspace (synchronises).  Errors as
 * ps_plan_create (the message names the failing problem). */
int ps_batch_create(ps_batch **out, int count, const int *nx, const int *ny,
                    const int *nz, const double *dx, const double *dy,
                    const double *const *dz, const double *const *rho,
                    int precision, void *stream);
/* rhs, p: host arrays of count device pointers ([nz][ny][nx] fields of the
 * batch's element type; rhs[i] must not alias p[i] in the PS_FP32_R1 form).
 * The first call, and any call with other pointers, synchronises the
 * stream, solves every problem once eagerly on its lane and captures the
 * lane graphs (allocating graph resources); later calls with the same
 * pointers only replay them, asynchronously after the work already on the
 * stream, and later work on the stream waits for them.  One solve in flight
 * per batch. */
int ps_batch_solve(ps_batch *batch, const void *const *rhs, void *const *p);
int ps_batch_set_stream(ps_batch *batch, void *stream);
/* Number of lanes, 1..8 (default 4; PS_EINVAL otherwise).  Synchronises
 * and drops the captured graphs when it changes. */
int ps_batch_set_lanes(ps_batch *batch, int lanes);
/* PS_BATCH_LANES is accepted.  The earlier forms are refused with
 * PS_EUNSUPPORTED: PS_BATCH_PERSISTENT (one persistent launch over
 * (problem, phase, tile) tickets: did not complete on the GPU),
 * PS_BATCH_PHASES (one launch per phase over the same tiles: withdrawn with
 * it) and PS_BATCH_PLANS (one graph over forked plan streams: a host fault
 * during its capture). */
enum { PS_BATCH_PHASES = 0, PS_BATCH_PERSISTENT = 1, PS_BATCH_PLANS = 2, PS_BATCH_LANES = 3 };
int ps_batch_set_mode(ps_batch *batch, int mode);
/* in_order 1 (the default): every problem's FP64 columns (the packed
 * kx = 0 row, the mean column and the near-singular columns) run on its
 * lane before its main column kernel, so each lane's graph is a single chain
 * on one stream; 0: each plan keeps its own placement (ps_plan_info's
 * fp64_beside), forking them onto the plan's second stream.  The result is
 * the same bit for bit.  PS_EINVAL for other values; synchronises and drops
 * the captured graphs when it changes. */
int ps_batch_set_fp64_order(ps_batch *batch, int in_order);
/* Autotune every problem's plan (ps_plan_autotune, reps repetitions; equal
 * shapes share the tune-cache entry), then time 1, 2, 4 and 8 lanes, each
 * with the FP64 columns in order and with each plan's own placement, over
 * reps replays each on the given fields (which are written) and keep the
 * fastest pair.  Synchronises. */
int ps_batch_autotune(ps_batch *batch, const void *const *rhs, void *const *p, int reps);
/* count of problems, the number of lanes and the FP64-column order (1: in
 * order on the lanes).  Any pointer may be NULL. */
int ps_batch_query(const ps_batch *batch, int *count, int *lanes, int *fp64_in_order);
/* Synchronise the batch's streams; PS_OK, or PS_EHIP if an earlier solve
 * failed on the device. */
int ps_batch_status(ps_batch *batch);
int ps_batch_destroy(ps_batch *batch);

/* ---- matrix-free conjugate gradients -----------------------------------
 * The paper's iterative alternative to the direct solve (Section 2.2: a
 * bespoke matrix-free Krylov solver with a hard-coded operator, several
 * inner products reduced together, terminated on the relative residual;
 * Table 1 compares its accuracy and cost with the FFT solve), on the same
 * discrete operator A and the same bordered-system result as ps_solve.
 * CG runs on M = -D A (D_k = rho_k dz_k), which is symmetric positive
 * semi-definite, with the right-hand side -D (b - mu), mu the D-weighted
 * mean of b; the result is shifted to zero mean.  FP64 throughout. */
typedef struct ps_cg ps_cg;
enum { PS_CG_NONE = 0, PS_CG_JACOBI = 1 }; /* preconditioner: none, diagonal of M */
/* nx, ny, nz >= 1 (fewer than 2^31 points), dx, dy > 0, dz and rho host
 * arrays of nz values > 0 (copied).  Allocates three FP64 fields of
 * workspace (synchronises).  Errors: PS_EINVAL, PS_EUNSUPPORTED, PS_ENOMEM,
 * PS_EHIP. */
int ps_cg_create(ps_cg **out, int nx, int ny, int nz, double dx, double dy, const double *dz,
                 const double *rho, int precond, void *stream);
/* Solve from the initial guess in x (device, [nz][ny][nx] doubles, read
 * and overwritten; the previous timestep's pressure is a warm start) for
 * rhs (device, not aliasing x) until |r| <= rtol |-D (b - mu)| (2-norms of
 * the residual of the symmetrised system, as updated by the recurrence) or
 * max_iter iterations.  iters and rel_res (host, may be NULL) receive the
 * iterations done and the final relative residual.  Synchronises: the host
 * reads the device-side convergence flag every 16 iterations, so this call
 * cannot be captured into a graph. */
int ps_cg_solve(ps_cg *cg, const double *rhs, double *x, double rtol, int max_iter, int *iters,
                double *rel_res);
/* Krylov method of the object: PS_KRYLOV_CG (default) as above, or
 * PS_KRYLOV_BICGSTAB, the paper's other bespoke solver (Section 2.2; its
 * Table 2 compares the two): stabilised bi-conjugate gradients on A itself,
 * which it does not need to be symmetric, with the projected right-hand side
 * b' = b - mu, post-conditioned as the paper's is (right preconditioning by
 * K, the diagonal of A for PS_CG_JACOBI or the identity: it solves
 * A K^-1 y = b' and x = K^-1 y, so its residual is that of A x = b'); it
 * stops when |b' - A x| <= rtol |b'| (the recurrence residual, tested after
 * each half step) or after max_iter iterations of two operator applications
 * each; the result is shifted to zero mean.  A breakdown (a zero inner
 * product in a denominator) also stops it, with rel_res above rtol.
 * Selecting BiCGStab the first time allocates its two further FP64 fields
 * (synchronises).  Errors: PS_EINVAL (NULL, unknown method), PS_ENOMEM,
 * PS_EHIP. */
enum { PS_KRYLOV_CG = 0, PS_KRYLOV_BICGSTAB = 1 };
int ps_cg_set_method(ps_cg *cg, int method);
int ps_cg_set_stream(ps_cg *cg, void *stream);
size_t ps_cg_workspace_bytes(const ps_cg *cg);
int ps_cg_destroy(ps_cg *cg);

const char *ps_status_string(int status);
const char *ps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRESSURE_SOLVE_H */
