/*
 * psv.h -- C ABI of the eigenexpansion pressure solve for variable-density
 * two-phase flow (Dalla Barba et al., "An interface capturing method for
 * liquid-gas flows at low-Mach number", arXiv:2005.11806).
 *
 * Problem (Sec. 3.3, Eq. lap_p): div(rho^-1 grad p) = f on a marker-and-cell
 * grid (Sec. 3: p and all scalars at cell centres), periodic in x and y,
 * walls in z where the pressure obeys the homogeneous Neumann condition that
 * the eigenexpansion needs (Sec. 3.3.1). f is the user's right-hand side,
 * i.e. (div u* - div u^{n+1}) / dt.
 *
 * Method I (Sec. 3.3.1, Eq. poisson_me1) recasts it with a constant
 * coefficient; one step is
 *     lap p^{s+1} = D[(1 - rho0/rho_face) G p^s] + rho0 f,   rho0 = min(rho),
 * solved exactly by eigenexpansion: real FFT along x, FFT along y, one
 * tridiagonal solve per wavenumber pair along z (uniform or stretched z),
 * inverse FFTs, with the singular (0,0) mode projected (volume-weighted mean
 * of the right-hand side removed) and gauged (volume-weighted mean of p = 0).
 * The density on a face is the arithmetic mean of its two cells.
 *
 * Conventions for every call:
 *  - Field pointers are DEVICE pointers to contiguous float64 arrays in
 *    C order [nz][ny][nx] (x fastest), 16-byte aligned (the passes move
 *    pairs of doubles; PSV_ERR_INVALID_ARG otherwise), owned by the caller;
 *    the library never frees or retains them beyond the call's stream work.
 *  - `stream` is a hipStream_t (NULL = the default stream). Work is enqueued
 *    asynchronously; a call returns before the GPU finishes unless it
 *    documents a synchronisation.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    non-OK status means nothing was enqueued (except PSV_ERR_HIP, and the
 *    data-dependent checks of `check_inputs`, which synchronise).
 *  - No exception crosses the ABI. psv_last_error_message() gives a
 *    thread-local description of the last non-OK status.
 *  - A plan owns one workspace: calls on one plan must not overlap in time
 *    (serialise them on one stream).
 */
#ifndef PSV_H
#define PSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSV_OK = 0,
    PSV_ERR_INVALID_ARG = 1,      /* bad pointer, size, option or input value */
    PSV_ERR_UNSUPPORTED_SIZE = 2, /* nx or ny (other than ny = 1) not even or not 2^a 3^b, or too large */
    PSV_ERR_HIP = 3,              /* a HIP runtime call failed */
    PSV_ERR_NONFINITE = 4,        /* check_inputs found NaN/Inf in an input */
    PSV_ERR_NOT_CONVERGED = 5,    /* mixed precision hit max_refine; p holds the last iterate */
    PSV_ERR_OOM = 6               /* device or host allocation failed */
} psv_status;

typedef enum { PSV_FP64 = 0, PSV_MIXED = 1 } psv_precision;

typedef enum {
    PSV_CONST = 0,      /* constant coefficient: p = S(f), rho unused */
    PSV_SPLIT_RHO0 = 1  /* Method I, Eq. poisson_me1 */
} psv_method;

typedef enum { PSV_BC_WALL_NEUMANN = 0 } psv_bc_z;

/* Grid (Sec. 3). x and y periodic with nx, ny even and of the form 2^a 3^b,
 * 4 <= nx, ny <= 1024, or ny = 1 for a two-dimensional x-z problem (the
 * paper's own cases); nz >= 2. zf: HOST array of nz+1 strictly increasing
 * z-face positions with zf[0] = 0 and zf[nz] = lz (copied at plan creation),
 * or NULL for uniform spacing lz/nz. Cell centres are face midpoints. */
typedef struct {
    int32_t nx, ny, nz;
    double lx, ly, lz;
    const double* zf;
    psv_bc_z bc_z;
} psv_grid;

typedef struct {
    psv_precision precision; /* FP64, or MIXED: FP32 transforms and tridiagonal
                                sweeps, FP64 residual refinement */
    psv_method method;
    double tol;              /* MIXED: target relative residual; <= 0 selects 1e-10 */
    int32_t max_refine;      /* MIXED: maximum refinement sweeps; <= 0 selects 4 */
    int32_t check_inputs;    /* 1: scan inputs for NaN/Inf and rho <= 0 (synchronises) */
    int32_t autotune;        /* launch shapes (x lines per block, chunk rows, stencil variant):
                                0 built-in; 1 from the autotune cache when it holds the plan's
                                (arch, grid, precision, method), else built-in; 2 as 1, but
                                when the cache has no entry the candidates are timed at plan
                                creation (on synthetic data, synchronising) and the choice is
                                added. The cache lives in the process and, when the
                                environment variable PSV_AUTOTUNE_CACHE names a file, in that
                                file (read once, appended to). Batches tune each problem's
                                plan the same way and run every tile in its plan's shape. */
    int32_t batch_executor;  /* batches: 0 default (per-pass launches), 1 per-pass launches,
                                2 one persistent launch over the task queue */
    int32_t chunk_rows;      /* rows per chunk of the wall-normal partition (planes per y
                                tile): 0 automatic (tuned when autotune >= 1), else 4, 8
                                or 16 (PSV_ERR_UNSUPPORTED_SIZE if its tile does not fit) */
    int32_t x_stencil;       /* neighbours of the forward x pass's stencil: 0 automatic
                                (staged unless the autotuner finds direct loads faster),
                                1 rows staged in LDS, 2 loaded directly (cache-served) */
} psv_opts;

#define PSV_RELRES_HISTORY 8
typedef struct {
    int32_t refine_steps;    /* refinement sweeps applied (MIXED) */
    double relres;           /* ||r - L p||_2 / ||r||_2 of the last step, r = projected RHS */
    double rhs_mean_removed; /* volume-weighted mean of the last step's RHS removed by projection */
    double rho0_used;        /* the rho0 of the splitting */
    double relres_sweep[PSV_RELRES_HISTORY]; /* MIXED, last step of psv_solve: relres after the
                                FP32 solve (entry 0) and after each refinement sweep (entry i);
                                NaN past the last sweep, and in FP64 or batched solves */
} psv_info;

typedef struct psv_plan psv_plan;
typedef struct psv_batch psv_batch;

/* Fills *opts with the defaults (FP64, Method I, tol 1e-10, max_refine 4). */
void psv_opts_default(psv_opts* opts);

/* Host-only validation of a grid (no GPU needed). */
psv_status psv_grid_validate(const psv_grid* grid);

/* Builds the plan: validates, then allocates device tables (twiddles,
 * eigenvalues lx[m] = -4 sin^2(pi m/nx)/dx^2 and ly, z-tridiagonal
 * coefficients) and the workspace on the current device. */
psv_status psv_plan_create(const psv_grid* grid, const psv_opts* opts, psv_plan** out);
psv_status psv_plan_workspace_size(const psv_plan* plan, size_t* bytes);
/* Launch shape the plan runs with (after autotuning): x lines per block and
 * rows per chunk of the wall-normal partition (= planes per y tile; the z
 * solve has 2 ceil(nz / chunk_rows) interface rows per wavenumber pair).
 * Either output pointer may be NULL. */
psv_status psv_plan_shape(const psv_plan* plan, int* lines_x, int* chunk_rows);

/* Every launch-shape field of a plan. */
typedef struct {
    int32_t lines_x;        /* x lines per block of the forward x pass (divides ny) */
    int32_t lines_x_inv;    /* x lines per block of the inverse x pass (divides ny) */
    int32_t chunk_rows;     /* rows per chunk of the wall-normal partition: 4, 8 or 16 */
    int32_t x_staged;       /* forward x pass: 1 stencil rows staged in LDS, 0 loaded directly */
    int32_t x_order;        /* forward x pass tile order: 1 each XCD takes a window of lines
                               through all planes (where the tiles per plane, ny / lines_x, are a
                               multiple of 8; plane ranges otherwise), 0 each XCD takes a
                               contiguous range of planes */
} psv_shape;
/* psv_plan_get_shape reads the shape the plan runs with; psv_plan_set_shape
 * replaces it (host-side checks first: PSV_ERR_INVALID_ARG for a field out of
 * range, PSV_ERR_UNSUPPORTED_SIZE when a tile does not fit the LDS of a block;
 * a new chunk_rows recomputes the interface factor table and synchronises the
 * device). Results do not depend on the shape beyond rounding. */
psv_status psv_plan_get_shape(const psv_plan* plan, psv_shape* shape);
psv_status psv_plan_set_shape(psv_plan* plan, const psv_shape* shape);
psv_status psv_plan_destroy(psv_plan* plan);

/* One or more chained solves (Sec. 3.3.1, Eq. poisson_me1).
 *  PSV_CONST:      p_out = S(f); rho and p_prev unused (may be NULL); n_steps must be 1.
 *  PSV_SPLIT_RHO0: p_1 = S(rho0 f + D((1 - rho0/rho_f) G p_prev)), then n_steps-1 more
 *                  steps with p_prev <- p; rho required; p_prev NULL means zero.
 * rho0 > 0 is used as given; rho0 <= 0 selects min(rho), computed on the device.
 * p_prev may alias p_out. If info != NULL the call synchronises `stream` and
 * fills *info for the last step (relres is computed only then, or always in
 * MIXED precision).
 * MIXED refinement: each sweep is one fused pass (FP64 residual, its norm, and
 * the FP32 x transform of the residual), a device-side check of relres
 * against tol, and the FP32 correction. With info == NULL nothing waits on
 * the host: max_refine sweeps are enqueued and those after convergence return
 * on the device at once, so the call can be captured in a graph; a miss of
 * tol then leaves p at the last iterate without an error. With info != NULL
 * the host reads the check after every sweep, stops enqueueing at
 * convergence and returns PSV_ERR_NOT_CONVERGED on a miss. */
psv_status psv_solve(psv_plan* plan, const double* f, const double* rho, double rho0,
                     const double* p_prev, double* p_out, int32_t n_steps, void* stream,
                     psv_info* info);

/* Adjoint of ONE Method-I step for loss = sum(w * p_out): gradients with respect
 * to f, rho and p_prev (any output may be NULL to skip it). With rho0 > 0, rho0
 * is an independent input: grad_rho is the partial derivative and
 * d loss/d rho0 = sum(lambda f) - sum_faces gface/rho_f is written to
 * *grad_rho0_host (f is then required). With rho0 <= 0 (rho0 = min rho),
 * that derivative is added to grad_rho at the first cell holding the minimum
 * (a subgradient), and also reported through grad_rho0_host if non-NULL.
 * Synchronises `stream` only if grad_rho0_host != NULL. PSV_CONST plans return
 * grad_f = S^T w and ignore the rest. */
psv_status psv_solve_adjoint(psv_plan* plan, const double* w, const double* f, const double* rho,
                             double rho0, const double* p_prev, double* grad_f, double* grad_rho,
                             double* grad_p_prev, double* grad_rho0_host, void* stream);

/* Method III (Sec. 3.3.1, Eq. new_poisson) solved with its loop (Algorithm 1):
 *     lap p^{s+1} = (1/dt) [ D(rho u*) - rho div_target - u^s . grad rho ],
 *     u^{s+1}     = u* - dt rho_f^-1 G p^{s+1}          (Eq. corr),
 * from u^0 = u* (or from the pressure p_init), until
 *     eps = sum over cells of |div u^{s+1} - div_target| <= eps_t
 * or max_iter solves. rho_f is the arithmetic mean of the two cells of a face
 * and u . grad rho the discrete product-rule remainder D(rho_f u) - rho D u,
 * which makes the recast exact on the grid: a converged u meets div_target
 * in every cell, and p solves div(rho^-1 grad p) = (div u* - div_target)/dt.
 * Each iteration is the eigenexpansion solve of the plan (FP64, or FP32 for a
 * MIXED plan: the loop itself corrects the FP32 solves). Uses the plan's
 * workspace. The residual is tested on the device after every solve; the host
 * reads it every few iterations (as many as the observed contraction predicts
 * are still needed, at most 32), so the call synchronises a few times.
 *   ux, uy     [nz][ny][nx]   u* on the x face between cells i and i+1 (and
 *                             the y face between j and j+1), periodic
 *   uz         [nz+1][ny][nx] u* on the z face below cell k; the planes 0 and
 *                             nz are the walls (normal velocity 0)
 *   div_target [nz][ny][nx]   div u^{n+1}; its volume-weighted mean must be 0
 *                             (a closed domain cannot meet the mean part)
 *   rho        [nz][ny][nx]   density > 0;  dt > 0
 *   eps_t >= 0 absolute threshold on eps; max_iter in [1, 100000]
 *   p_init     optional starting pressure (may equal p_out); NULL starts
 *              from u* (p = 0)
 *   p_out      pressure (zero volume-weighted mean)
 *   ux_out, uy_out, uz_out  the corrected velocity u^{n+1}, same layouts as
 *              u*: all three or none (NULL); must not alias u*
 * Stops without error when max_iter is reached (info->converged = 0). */
typedef struct {
    int32_t iterations;      /* eigenexpansion solves performed */
    int32_t converged;       /* 1 when eps <= eps_t */
    double eps;              /* eps of the returned p and u */
    double eps_start;        /* eps of u* itself (NaN when p_init is given) */
} psv_m3_info;

psv_status psv_solve_method3(psv_plan* plan, const double* ux, const double* uy, const double* uz,
                             const double* div_target, const double* rho, double dt, double eps_t,
                             int32_t max_iter, const double* p_init, double* p_out,
                             double* ux_out, double* uy_out, double* uz_out, void* stream,
                             psv_m3_info* info);

/* The converged variable-density solve: the fixed point that Methods I, II and
 * III all iterate towards (Sec. 3.3.1; Eq. lap_p with f given directly),
 *     D(rho_f^-1 G p) = f - mean_V(f),
 * reached by iterating, in pressure form,
 *     p <- p + S[omega (f - mean_V(f) - D(rho_f^-1 G p))],
 * S the plan's eigenexpansion solve, with
 *   PSV_ITER_METHOD1: omega = min rho (Eq. poisson_me1; robust at any density
 *                     ratio, slow),
 *   PSV_ITER_METHOD2: omega = 2 a b / (a + b), the harmonic mean of a = min rho
 *                     and b = max rho, standing for the two phase densities
 *                     (Eq. poisson_laizet; converges while max/min rho stays
 *                     moderate),
 *   PSV_ITER_METHOD3: omega = rho in each cell (Eq. new_poisson; fewest
 *                     iterations; may diverge at large density ratios on
 *                     fine grids),
 * until
 *     eps = sum over cells of |f - mean_V(f) - D(rho_f^-1 G p)| <= eps_t
 * or max_iter solves. mean_V is the volume-weighted mean.
 *   f, rho [nz][ny][nx] device fields, rho > 0
 *   p_init optional starting pressure (may equal p_out); p_out keeps its
 *          volume-weighted mean (zero when p_init is NULL)
 *   p_out  must not alias f or rho
 * info (may be NULL; the call then does not synchronise at its end):
 * iterations = solves performed, eps of the returned p, eps_start = eps of
 * p = 0 (NaN when p_init is given). MIXED plans run FP32 solves inside the
 * loop, which corrects them. Stops without error at max_iter
 * (info->converged = 0). Synchronises every few iterations, as Method III does. */
typedef enum { PSV_ITER_METHOD1 = 1, PSV_ITER_METHOD2 = 2, PSV_ITER_METHOD3 = 3 } psv_iteration;
psv_status psv_solve_converged(psv_plan* plan, const double* f, const double* rho,
                               int32_t iteration, double eps_t, int32_t max_iter,
                               const double* p_init, double* p_out, void* stream,
                               psv_m3_info* info);

/* Implicit adjoint of psv_solve_converged for loss = sum(w * p): V A is
 * symmetric (A = D(rho_f^-1 G), V the cell volumes), so the gradients take one
 * more converged solve instead of differentiating the iterations:
 *     lambda      = A^+ (V^-1 w), zero volume-weighted mean (same iteration,
 *                   eps_t and max_iter; eps is measured on V^-1 w's system)
 *     grad_f      = V lambda
 *     grad_rho[c] = sum over the faces F of cell c of
 *                   (D^T V lambda)_F (G p)_F / (2 rho_F^2),
 * with (D^T mu)_F = mu_L/h_L - mu_R/h_R across F and rho_F the arithmetic
 * mean of the two cells of F.
 *   w, rho [nz][ny][nx]; p = the converged pressure of the forward call
 *   (required for grad_rho). grad_f / grad_rho may be NULL to skip them; they
 *   must not alias rho or p (grad_f may alias w). Uses the plan's workspace.
 * info describes the adjoint solve. */
psv_status psv_solve_converged_adjoint(psv_plan* plan, const double* w, const double* rho,
                                       const double* p, int32_t iteration, double eps_t,
                                       int32_t max_iter, double* grad_f, double* grad_rho,
                                       void* stream, psv_m3_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): psv_solve
 * without a plan. The plan's tables (twiddles, eigenvalues, z geometry,
 * interface factors) and its workspace (spectrum, partial sums, device scalars
 * and flags) are carved out of one static device array of
 * PSV_STATIC_SCRATCH_BYTES per GPU, which the library holds until the process
 * ends; each call refills the tables from kernel arguments and clears the
 * scalars and flags with kernels. The call allocates nothing, on the host or
 * the device, and records no memset. Arguments and results as psv_solve
 * (FP64, built-in launch shapes: the same passes and bits as a plan created
 * with autotune = 0), without info. opts may be NULL (defaults); it must have
 * precision PSV_FP64, autotune 0 and check_inputs 0 (PSV_ERR_INVALID_ARG);
 * chunk_rows and x_stencil are honoured. Tables and workspace must fit the
 * array (about 5 million cells; 128^3 takes about 24 MB of it):
 * PSV_ERR_UNSUPPORTED_SIZE otherwise, before any device work when the
 * spectrum alone is too large. Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and give wrong results, so serialise them. */
#define PSV_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
psv_status psv_solve_static(const psv_grid* grid, const psv_opts* opts, const double* f,
                            const double* rho, double rho0, const double* p_prev, double* p_out,
                            int32_t n_steps, void* stream);

/* Mixture density of Sec. 2.2, Eq. eq_22, with the colour Phi = 1 in gas:
 * rho = rho_gas * Phi + rho_liq * (1 - Phi). phi and rho_gas are device fields. */
psv_status psv_density_from_colour(const psv_plan* plan, const double* phi, const double* rho_gas,
                                   double rho_liq, double* rho_out, void* stream);

/* Discrete divergence of a face field (the D of the 7-point operator):
 * ux, uy [nz][ny][nx] hold the faces i+1/2 and j+1/2 (periodic), uz [nz+1][ny][nx]
 * the z faces at zf[k] (uz[0] and uz[nz] are the wall values). */
psv_status psv_divergence(const psv_plan* plan, const double* ux, const double* uy,
                          const double* uz, double* div_out, void* stream);

/* Relative residual ||r - L p||_2 / ||r - mean_V r||_2 of a constant-coefficient
 * system, FP64 7-point operator; synchronises and writes *relres. */
psv_status psv_relres(psv_plan* plan, const double* r, const double* p, void* stream,
                      double* relres);

/* Batched uneven problems (one grid per problem, x/y periodic, z walls) solved
 * together: per pass, one launch over the tiles of every problem
 * (opts.batch_executor 0 or 1), or one persistent-kernel launch over a task
 * queue (2); the launches are captured in a HIP graph on the first call and
 * replayed after. Pointer arrays are HOST arrays of DEVICE pointers; rho0 is
 * a HOST array (<= 0 selects min(rho)). Each call copies its pointer table to
 * the device on `stream` and, before rewriting that table, waits on the host
 * until the previous call's copy has run. Calls on one batch share its
 * workspace: the caller orders calls made on different streams. */
psv_status psv_batch_create(int32_t n, const psv_grid* grids, const psv_opts* opts,
                            psv_batch** out);
psv_status psv_batch_solve(psv_batch* batch, const double* const* f, const double* const* rho,
                           const double* rho0, const double* const* p_prev, double* const* p_out,
                           void* stream, psv_info* infos);
psv_status psv_batch_destroy(psv_batch* batch);

/* Per-kernel timing (profiling aid): with enable = 1 every kernel the plan
 * launches is bracketed by two hipEvents on its launch stream, recorded
 * without a system-scope fence (hipEventDisableSystemFence), so that timing
 * does not write back and invalidate the caches between kernels. The
 * timings describe eager calls: enable the trace outside stream capture.
 * psv_trace_summary synchronises on the recorded events, writes a JSON object
 * {"kernel": [launches, total_ms], ...} (NUL-terminated, truncated to `len`)
 * into buf, stores the untruncated length in *needed (may be NULL) and
 * clears the records. */
psv_status psv_trace_enable(psv_plan* plan, int32_t enable);
psv_status psv_trace_summary(psv_plan* plan, char* buf, size_t len, size_t* needed);

const char* psv_status_string(psv_status s);
const char* psv_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* PSV_H */
