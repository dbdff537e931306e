/*
 * pdd.h -- C ABI of the MI355X (gfx950) Monte Carlo assembler of the
 * PDDSparse interfacial system G u = b (Bernal, Moron-Vidal, Acebron,
 * arXiv 2301.05780).
 *
 * Conventions shared by every entry point
 *   - Plain C types only.  "device" pointers are HIP device memory (for
 *     example the data pointer of a torch tensor on cuda:0); "host" pointers
 *     are ordinary CPU memory.
 *   - Ownership: the caller allocates and owns every input and output; the
 *     library borrows them for the duration of the call (or, for enqueued
 *     device work, until that work has completed on the context's stream).
 *     The library owns only context-internal scratch, released by pdd_destroy.
 *   - Asynchrony: device work is enqueued on the context's stream and the call
 *     returns; results are valid after pdd_sync or after the caller
 *     synchronises that stream.  pdd_solve is the exception: it reads back
 *     convergence scalars and therefore returns after the solve has finished;
 *     a float32 table assembly waits for its table scan (see pdd_assemble).
 *   - Errors: host-side validation fails fast with PDD_EINVAL before touching
 *     any output; HIP failures give PDD_EDEVICE (asynchronous kernel faults
 *     surface at the next synchronising call).  pdd_last_error returns a
 *     message for the last non-OK status of a context.  Nothing is printed
 *     and no exception or abort crosses the ABI.
 *   - Threads: a context may be used by one host thread at a time.
 */
#ifndef PDD_H
#define PDD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pdd_status {
  PDD_OK = 0,
  PDD_EINVAL = 1,        /* invalid argument (nothing was written) */
  PDD_ENOMEM = 2,        /* device or host allocation failed */
  PDD_EDEVICE = 3,       /* a HIP runtime call or kernel failed */
  PDD_ENOTCONV = 4,      /* iterative solve stopped before the tolerance */
  PDD_EUNSUPPORTED = 5   /* combination of options not implemented */
} pdd_status;

typedef struct pdd_ctx pdd_ctx;

/* ---- problem description ------------------------------------------------ */

/* Coefficient families of problem (6) (Sec. 2.2): the diffusion sigma (taken
 * symmetric, A = sigma sigma^T as in eq. 7), drift d, reaction c <= 0, source
 * f and Dirichlet datum g.
 *   POISSON    sigma = sqrt(2) I, d = 0, c = 0, u* = sin(pi x) sin(pi y) + x^2 y,
 *              f = Laplacian of u*, g = u*
 *   VARCOEF    sigma = diag(sqrt(2 + sin 2 pi x), sqrt(2 + cos 2 pi y)),
 *              d = (sin 2 pi y, cos 2 pi x), c = -(1 + x^2), u* = e^x cos 2y,
 *              f = L u*, g = u*
 *   AMPLITUDE  sigma = diag(sqrt(2 (1 + a sin 2 pi x)), sqrt(2 (1 + a cos 2 pi y))),
 *              a = param[0] in [0, 1), d = 0, c = 0, u* as POISSON, f = L u*
 *   LUT        the seven fields (sxx, sxy, syy, dx, dy, c, f) read by bilinear
 *              interpolation from a float32 table on an lut_n x lut_n grid of
 *              nodes spanning the partition's domain, node (i, j) at
 *              (x0 + i (x1-x0)/(lut_n-1), y0 + j (y1-y0)/(lut_n-1)); layout
 *              lut[(j * lut_n + i) * PDD_LUT_STRIDE + field], device pointer;
 *              g = u* of POISSON.  The table must give a positive definite
 *              A = sigma sigma^T.  Under PDD_EXIT_GM each assembly first
 *              reads the whole table once (max |sxx|, |sxy|, |syy|) to bound
 *              the shift; the exact shift uses a_nn at the projection.
 *              Float32 production reads a cell-major copy of the table
 *              ((lut_n - 1)^2 cells of 128 B, which must stay below 4 GiB:
 *              lut_n <= 5793, else PDD_EUNSUPPORTED), of only the varying
 *              fields when at most two vary (pdd_set_table_read).  The
 *              table pointer must be 16-byte aligned (PDD_EINVAL).
 *   CONSTSOL   sigma, d, c of VARCOEF, f = c, g = 1 (u = 1 is the solution)
 *   EXITTIME   sigma = sqrt(2) I, d = 0, c = 0, f = -1, g = 0 (u = mean exit
 *              time, eq. 26)
 *   EQ43       the Poisson problem of the Sec. 5 experiment (eq. 42): sigma =
 *              sqrt(2) I, d = 0, c = 0, u* of eq. 43, f = Lap u*, g = u* */
enum {
  PDD_COEF_POISSON = 0,
  PDD_COEF_VARCOEF = 1,
  PDD_COEF_AMPLITUDE = 2,
  PDD_COEF_LUT = 3,
  PDD_COEF_CONSTSOL = 4,
  PDD_COEF_EXITTIME = 5,
  PDD_COEF_EQ43 = 6
};
enum { PDD_LUT_STRIDE = 8 };

typedef struct pdd_coeffs {
  int32_t kind;          /* PDD_COEF_* */
  int32_t lut_n;         /* LUT nodes per direction (>= 2), LUT kind only */
  double param[4];       /* family parameters (AMPLITUDE: param[0] = a) */
  const float* lut;      /* device, LUT kind only */
} pdd_coeffs;

/* Omega = [x0, x1] x [y0, y1] cut into H x H subdomains (eq. 12). */
typedef struct pdd_partition {
  double x0, x1, y0, y1;
  int32_t H;             /* >= 2 */
  int32_t _pad;
} pdd_partition;

/* Knots (Sec. 3.1): m lattice intervals per subdomain side, so the knot
 * spacing is (x1 - x0) / (H m); knots are the lattice points inside Omega on
 * grid lines, crossings included.  Unknowns are numbered in lexicographic
 * (y, x) order.  Each interface side's stencil (eq. 17) is its line's knots
 * within the side widened by ext lattice units at both ends, clipped to the
 * domain (Sec. 5.1 widens by half a segment; Sec. 3.3 beyond corners). */
typedef struct pdd_knots {
  int32_t m;             /* >= 1 */
  int32_t ext;           /* >= 0 */
} pdd_knots;

/* ---- run options --------------------------------------------------------- */

enum {
  PDD_FP64_SAME_STREAM = 0,  /* float64 paths: matches the CPU definition to rounding */
  PDD_FP32_PRODUCTION = 1    /* float32 paths, float64 accumulation of G and b */
};
enum {
  PDD_EXIT_NAIVE = 0,        /* exit when strictly outside the closed patch (Sec. 2.3) */
  PDD_EXIT_GM = 1            /* Gobet-Menozzi inward shift 0.5826 sqrt(a_nn h) (Sec. 2.3) */
};
enum {
  PDD_CV_NONE = 0,
  PDD_CV_NETWORK = 1,        /* grad v of the 2-64-64-1 tanh network at every step */
  PDD_CV_GRAD_LUT = 2        /* grad v baked into a float32 table, bilinear read */
};
enum {
  PDD_INTERP_HAT = 0,        /* linear (hat) weights on the two nearest lattice points (footnote 8) */
  PDD_INTERP_RBF_IMQ = 1     /* cardinal functions of the inverse multiquadric on the side's whole
                                stencil (eqs. 1-5, 21) */
};
enum { PDD_DIAG_WIDTH = 8 };   /* per knot: sum K, N, exits E/N/W/S, sum s, sum s^2 */
enum { PDD_DUMP_WIDTH = 8 };   /* per dumped path: K, x_K, y_K, Y_K, Z_K, Xi_K, knot, path */
enum { PDD_MLP_WIDTH = 64, PDD_MLP_PARAMS = 4417 };
#define PDD_COLLECT_STREAM 0x40000000u /* added to run.instance by pdd_collect_training */
enum { PDD_CAL_WIDTH = 8 };    /* per knot: sum(phi_EM - phi_GM), sum phi_GM, sum phi_GM^2, sum xi,
                                  sum xi^2, sum phi_GM xi, sum K_GM, sum K_EM */

/* Control variate of eqs. (37)-(38): Xi accumulates -Y (sigma^T grad v) . dW
 * and is added to b only; the mean of the estimator is unchanged for any v.
 * NETWORK: params = float32[PDD_MLP_PARAMS] laid out W1[64][2], b1[64],
 * W2[64][64] (out, in), b2[64], w3[64], b3 (device).  The network's input is
 * the point in the domain's unit coordinates ((x - x0)/(x1 - x0),
 * (y - y0)/(y1 - y0)), so one architecture serves any domain; grad v is
 * taken with respect to x and y (chain rule).
 * GRAD_LUT: grad_lut = float32 [lut_n][lut_n][2] node-centred over the domain
 * (device, 8-byte aligned, else PDD_EINVAL; float32 runs take lut_n <= 23170,
 * else PDD_EUNSUPPORTED). */
typedef struct pdd_cv {
  int32_t mode;              /* PDD_CV_* */
  int32_t lut_n;
  const float* params;
  const float* grad_lut;
} pdd_cv;

typedef struct pdd_run {
  uint64_t seed;                   /* Philox key = (seed lo 32 bits, seed hi 32 bits) */
  uint32_t instance;               /* fourth Philox counter word (assemblies: below 2^30 keeps
                                      the stream apart from the training pairs' and the point
                                      evaluations', which add PDD_COLLECT_STREAM and 2^31) */
  int32_t precision;               /* PDD_FP64_SAME_STREAM | PDD_FP32_PRODUCTION */
  int32_t exit_rule;               /* PDD_EXIT_NAIVE | PDD_EXIT_GM */
  int32_t dump_paths;              /* >0: record the first dump_paths paths of every knot */
  int64_t n_paths;                 /* paths per knot when n_paths_per_knot is NULL */
  const int32_t* n_paths_per_knot; /* host, length n, entries >= 1; nullable */
  double h;                        /* Euler-Maruyama time step, > 0 */
  const pdd_cv* cv;                /* nullable: plain estimator */
  const double* u_ref;             /* device, length n, nullable: knot values used in
                                      the per-path score diagnostics (sum s, sum s^2) */
  double* dump;                    /* device, n * dump_paths * PDD_DUMP_WIDTH, when dump_paths > 0 */
  int32_t interp;                  /* PDD_INTERP_HAT (0) | PDD_INTERP_RBF_IMQ: interface-side interpolation */
  double rbf_c;                    /* RBF_IMQ: shape parameter c > 0 of phi_c(r) = 1 / sqrt(r^2 + c^2),
                                      in domain units (pdd_rbf_shape picks it by condition number) */
  const double* h_per_knot;        /* host, length n, nullable: per-knot time steps h_i (eq. 40), each
                                      finite and > 0, used for knot i's paths instead of h (pdd_assemble
                                      only; PDD_EUNSUPPORTED elsewhere) */
} pdd_run;

/* ---- context ------------------------------------------------------------- */

/* Create a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the null stream).  *ctx receives the handle. */
pdd_status pdd_create(pdd_ctx** ctx, int32_t device, void* stream);
void pdd_destroy(pdd_ctx* ctx);
pdd_status pdd_set_stream(pdd_ctx* ctx, void* stream);
/* Block until all work enqueued on the context's stream has finished. */
pdd_status pdd_sync(pdd_ctx* ctx);
/* Message of the last non-OK status of ctx (ctx may be NULL for failures of
 * calls that take no context); never NULL, valid until the next call. */
const char* pdd_last_error(const pdd_ctx* ctx);

/* ---- discretisation (host only, no device work) -------------------------- */

/* Sizes of the system and, when row_ptr/col_idx are non-NULL, its sparsity
 * pattern: row k holds column k and the stencil of every interface side of
 * knot k's patch (support of eq. 24), ascending, structural zeros kept.
 * row_ptr: host int32[n + 1]; col_idx: host int32[nnz]. */
pdd_status pdd_pattern(const pdd_partition* part, const pdd_knots* knots,
                       int64_t* n, int64_t* nnz, int32_t* row_ptr, int32_t* col_idx);

/* Work decomposition of pdd_assemble (host only; needs no device or
 * context): the tickets (knot, path range) that a single-instance assembly
 * hands to its waves, the order in which the waves claim them, and the split
 * of that order over the eight XCDs.
 *   n_paths_per_knot: host, one entry >= 1 per knot in canonical order.
 *   paths_per_ticket >= 1: knot k's paths are cut into
 *     ceil(N_k / paths_per_ticket) near-equal contiguous ranges.
 *   spatial != 0: the order used with tabulated coefficients, the tickets
 *     sorted by the Morton (Z) index of their knot's subdomain; else the
 *     longest expected work first (patch area x paths, the mean exit time
 *     growing with the patch area, eq. 26).  Both sorts are stable.
 *   grid: workgroups of the launch, for the XCD split (workgroup b runs on
 *     XCD b mod 8; XCD x takes order positions [xcd_begin[x], xcd_begin[x+1])
 *     with the share of the expected cost that matches its share of
 *     workgroups).  Only with spatial != 0 and grid >= 8.
 * Outputs (host, nullable): *n_tickets; tickets[3 n_tickets] = (knot, first
 * path, end path) by ticket index; order[n_tickets]; xcd_begin[9].  Call
 * with tickets = order = xcd_begin = NULL to size the arrays. */
pdd_status pdd_plan_tickets(const pdd_partition* part, const pdd_knots* knots, const int32_t* n_paths_per_knot,
                            int32_t paths_per_ticket, int32_t spatial, int32_t grid, int64_t* n_tickets,
                            int32_t* tickets, int32_t* order, int32_t* xcd_begin);

/* Knot coordinates in canonical order: xy = host double[2 n] (x0, y0, x1, y1, ...). */
pdd_status pdd_knot_xy(const pdd_partition* part, const pdd_knots* knots, double* xy);

/* ---- assembly (eqs. 20-25) ------------------------------------------------ */

/* Monte Carlo assembly of G (CSR) and b: for every knot k, N_k paths of the
 * diffusion (9) start at x_k and are integrated by Euler-Maruyama until they
 * first leave the knot's patch (eq. 15); the exit point is projected onto the
 * closest tripped side line and interpolated onto that line's knot lattice
 * (eq. 21): linearly (footnote 8's scheme, run->interp = PDD_INTERP_HAT) or
 * with the inverse-multiquadric cardinal functions of the side's whole
 * extended stencil (eqs. 1-5, run->interp = PDD_INTERP_RBF_IMQ; float64
 * evaluation in both precision modes, as the interpolation matrix is
 * ill-conditioned by design).  Row k: G_kk = 1,
 * G_kj = -mean(Y_K w_j), b_k = mean(Z_K + Xi_K + Y_K * boundary data reached).
 * The RBF mode takes no u_ref and no network control variate
 * (PDD_EUNSUPPORTED); its results equal the per-path definition up to
 * rounding amplified by the condition number of the interpolation matrix.
 * Random numbers: Philox4x32-10, counter = (draw j, path p, knot k, instance),
 * draw j feeding steps 2j and 2j+1 through Box-Muller.
 * Outputs (device): row_ptr int32[n+1], col_idx int32[nnz], val double[nnz],
 * b double[n], diag double[n * PDD_DIAG_WIDTH] (nullable).
 * A float32 assembly of the LUT family (without the network control
 * variate) synchronises the context's stream once, after the table scan, to
 * choose its kernel (pdd_set_table_read); while the stream is captured into
 * a graph it keeps the previous eager call's choice instead. */
pdd_status pdd_assemble(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                        const pdd_knots* knots, const pdd_run* run,
                        int32_t* row_ptr, int32_t* col_idx, double* val, double* b,
                        double* diag);

/* ---- batched assembly -------------------------------------------------------- */

/* One BVP instance of a batch: its problem, discretisation, run options and
 * its own device outputs (as for pdd_assemble). */
typedef struct pdd_instance {
  pdd_coeffs coeffs;
  pdd_partition part;
  pdd_knots knots;
  pdd_run run;
  int32_t* row_ptr;
  int32_t* col_idx;
  double* val;
  double* b;
  double* diag;          /* nullable */
} pdd_instance;

/* Assemble n_inst independent instances in ONE persistent launch: the tickets
 * of all instances form a single work list ordered longest-expected-first
 * (paths x patch area / h), so instances of uneven size and uneven path
 * lengths share the machine.  Every instance's result equals what
 * pdd_assemble gives it alone, up to float64 summation order.  Restrictions:
 * all instances share precision, exit rule, coefficient family (POISSON,
 * VARCOEF or AMPLITUDE) and seed; no u_ref, dump or RBF interpolation.  A control variate is
 * allowed when every instance names the same one (same mode and the same
 * table or parameter pointers) and the instances share the domain; the
 * network mode is float32 only here.  Instances are told apart in the random
 * stream by run.instance (e.g. independent replicas of one problem). */
pdd_status pdd_assemble_batch(pdd_ctx* ctx, int32_t n_inst, const pdd_instance* inst);

/* ---- graph capture ---------------------------------------------------------- */

/* Capture the device work that the context enqueues between pdd_graph_begin
 * and pdd_graph_end into a HIP graph, then replay it with pdd_graph_launch.
 * Only cached work can be captured: run the same pdd_assemble /
 * pdd_assemble_batch call once before capturing (a call that needs new
 * tables during capture fails with PDD_EINVAL).  The graph uses the
 * context's scratch as sized then: a later call that needs more (a larger
 * table, more tickets) reallocates it, after which the graph must be
 * captured again.  Captured work must not call pdd_solve.  *n_nodes receives
 * the node count of the graph (nullable). */
pdd_status pdd_graph_begin(pdd_ctx* ctx);
pdd_status pdd_graph_end(pdd_ctx* ctx, int32_t* n_nodes);
pdd_status pdd_graph_launch(pdd_ctx* ctx);

/* ---- autotuning ----------------------------------------------------------- */

/* Time the assembly of the given instance(s) (n_inst == 1: pdd_assemble;
 * otherwise pdd_assemble_batch) over a grid of launch shapes -- threads per
 * block, workgroups per compute unit, paths per ticket, static or dynamic
 * schedule -- then, on the fastest, refill thresholds (pdd_set_refill) and
 * spare tally rows with larger tickets (pdd_set_spare_rows), with `reps`
 * timed repetitions each, and keep the fastest as the context's launch shape
 * (pdd_set_launch, pdd_set_refill, pdd_set_spare_rows).  A shape's time is
 * the device time of the assembly kernel and of the row sums after it (which
 * grow with the ticket count); *best_ms receives the chosen shape's mean
 * time; `report` (nullable, report_len bytes) a text table of every
 * shape tried.  Results are cached per workload signature in the context.
 * The call ends with one assembly in the chosen shape (also on a cache hit),
 * so pdd_last_launch reports it and its tables are ready for graph capture. */
pdd_status pdd_autotune(pdd_ctx* ctx, int32_t n_inst, const pdd_instance* inst, int32_t reps, double* best_ms,
                        char* report, int32_t report_len);

/* ---- solve (eq. 23) -------------------------------------------------------- */

/* Solve G u = b for a CSR matrix (device arrays; row_ptr int32[n+1], col_idx
 * int32[nnz], val double[nnz], b double[n]; u double[n] receives the
 * solution, starting from u = 0).  Iterative refinement: the residual
 * b - G u is formed in float64; each correction is computed by BiCGStab on
 * float32 vectors (float64 dot products) until the float64 relative residual
 * ||b - G u||_2 / ||b||_2 <= tol.  *iters receives the BiCGStab iterations
 * used, *relres the final relative residual (host pointers).  Returns
 * PDD_ENOTCONV, with the best iterate in u, if max_iter BiCGStab iterations
 * do not reach tol.  Synchronises the context's stream. */
pdd_status pdd_solve(pdd_ctx* ctx, int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                     const double* val, const double* b, double* u, double tol, int32_t max_iter,
                     int32_t* iters, double* relres);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * solve of pdd_solve, same arguments, results and errors, on a static device
 * scratch array of 128 MiB that the library holds on every GPU it runs on
 * (looked up once per device by pdd_create) instead of context scratch.  It
 * allocates nothing.  Sizes beyond the array give PDD_EINVAL before any
 * kernel runs: 4 (nnz + 7 n) + 8 n bytes plus 7 KiB must fit 128 MiB
 * (nnz = row_ptr[n]; about 31 M nonzeros at n = 65,536).  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (several
 * contexts or streams) race; calls in sequence do not. */
pdd_status pdd_solve_noalloc(pdd_ctx* ctx, int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                             const double* val, const double* b, double* u, double tol, int32_t max_iter,
                             int32_t* iters, double* relres);

/* ---- values inside the subdomains (Sec. 3.3; eq. 8 on each square) ------- */

/* u at n_pts points from the knot values: each subdomain square is a
 * Dirichlet problem whose sides carry the knot values interpolated along the
 * grid lines (hat functions, the along-side coordinate clamped to the side)
 * on interfaces and g on the domain boundary; u(x) is the Feynman-Kac mean of
 * Z + Y u(exit) over run.n_paths paths from x absorbed at the square's
 * boundary, with the assembly's step, exit rule and side choice.  The square
 * of (x, y) has lower-left corner index min(floor((x - x0) / s), H - 1) per
 * direction, s the subdomain side; a point exactly on a grid line of its
 * square gets the line value itself (se = 0).  Points outside the closed
 * domain give NaN.
 * Inputs (device): u_knots[n] (canonical knot order, e.g. from pdd_solve),
 * xy[2 n_pts] float64 interleaved.  Outputs (device): u[n_pts], se[n_pts]
 * (nullable) the Monte Carlo standard error of each value.  n_pts = 0 does
 * nothing (xy and u may then be NULL).
 * run: seed, instance (< 2^31), precision, exit_rule, n_paths (paths per
 * point), h; cv, n_paths_per_knot and dump must be unset and interp must be
 * PDD_INTERP_HAT (else PDD_EUNSUPPORTED).  Path p of point i
 * draws from the Philox counter (draw, p, i, instance + 2^31), disjoint from
 * the knot streams of assemblies with instance < 2^31. */
pdd_status pdd_eval_subdomain(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                              const pdd_knots* knots, const double* u_knots, int64_t n_pts, const double* xy,
                              const pdd_run* run, double* u, double* se);

/* ---- pseudospectral subdomain solves and the global u0(x) (Sec. 3.3) ---- */

/* Once the knot values are known, every subdomain square is an independent
 * Dirichlet problem for (6) (Sec. 3.3), which the paper solves with the
 * pseudospectral method (Sec. 3.3, 5.1); the solutions together give the
 * global u0(x) of Phase I (Sec. 4.3) and the control variate F =
 * sigma^T grad u0 kept on a look-up table (Sec. 4.2, eq. 37).
 *
 * Discretisation: on each square the tensor grid of the p + 1
 * Chebyshev-Gauss-Lobatto points per direction, t_j = -cos(pi j / p),
 * j = 0..p (ascending), mapped onto the square; collocation of (6) at the
 * interior points, u = side value at the boundary points.  Side values: g on
 * the domain boundary; on an interface, the line's lattice values (knot
 * values u_knots, g at the two lattice points on the domain boundary)
 * interpolated over the side's stencil, the line's lattice points from the
 * side's lower end minus knots->ext to its upper end plus knots->ext clipped
 * to the domain: hat weights (interp = PDD_INTERP_HAT) or the
 * inverse-multiquadric cardinal functions of that stencil with shape
 * parameter rbf_c (PDD_INTERP_RBF_IMQ, eqs. 1-5).  The four corners of a
 * square take the values of its horizontal (lower and upper) sides.
 * Operators: constant coefficients with diagonal sigma and no drift (POISSON,
 * EXITTIME, EQ43, or a LUT whose sigma, drift and reaction fields are
 * constant over the table, checked on the device: the call then
 * synchronises the stream); others give PDD_EUNSUPPORTED.  The interior
 * system is solved by diagonalising the second-derivative block (the
 * decomposition computed once per p on the host in extended precision):
 * results equal the direct solve of the collocation system to float64
 * rounding amplified by the eigenvector conditioning (about 1e-10 relative
 * at p = 63).
 * grid (device, float64, caller-owned): H^2 * 3 * (p+1)^2 doubles,
 * grid[((s * 3 + f) * (p+1) + i) * (p+1) + j] for square s = a + H c (a, c
 * its column and row), field f = 0 (u), 1 (du/dx), 2 (du/dy), at the point
 * (x_a + S (t_i + 1) / 2, y_c + S (t_j + 1) / 2), S the side length.
 * u_knots: device double[n] in canonical order.  2 <= p <= 63. */
pdd_status pdd_spectral_solve(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                              const pdd_knots* knots, int32_t p, int32_t interp, double rbf_c, const double* u_knots,
                              double* grid);

/* u0 and grad u0 at n_pts points from a grid of pdd_spectral_solve (same
 * partition and p): 2-D barycentric Chebyshev interpolation on the point's
 * square, the square with lower-left corner index min(floor((x - x0) / S),
 * H - 1) per direction (points outside the domain extrapolate from the
 * nearest square).  Device arrays: xy[2 n_pts], u[n_pts] and grad[2 n_pts]
 * (each nullable, not both). */
pdd_status pdd_spectral_eval(pdd_ctx* ctx, const pdd_partition* part, int32_t p, const double* grid, int64_t n_pts,
                             const double* xy, double* u, double* grad);

/* grad u0 on the lut_n x lut_n node grid of the domain, the table read by
 * PDD_CV_GRAD_LUT (the paper's F = sigma^T grad u0 on a look-up table, eq.
 * 37; the assembly applies sigma^T): grad_lut[(j lut_n + i) 2 + d] (device
 * float32), node (i, j) at (x0 + i (x1 - x0) / (lut_n - 1), y0 + j (y1 -
 * y0) / (lut_n - 1)), each node evaluated on its square as pdd_spectral_eval
 * does. */
pdd_status pdd_spectral_grad_lut(pdd_ctx* ctx, const pdd_partition* part, int32_t p, const double* grid, int32_t lut_n,
                                 float* grad_lut);

/* Host only: accuracy of the degree-p diagonalisation that pdd_spectral_solve
 * uses, max |E V - V diag(lam)| / max |E| and max |V V^{-1} - I| (E the
 * interior block of the second-derivative collocation matrix).  PDD_EINVAL
 * outside 2 <= p <= 63 or when the decomposition fails. */
pdd_status pdd_spectral_tables(int32_t p, double* decomp_residual, double* inverse_residual);

/* ---- Phase II calibration (Sec. 4.1-4.2, eqs. 32-41) ----------------------- */

/* Mixed Gobet-Menozzi / Euler-Maruyama trajectories (Sec. 4.1): for every
 * knot, run->n_paths paths of step run->h (h0') start at the knot and run
 * until they leave the closed patch (the naive exit); the first step at
 * which a path is no longer strictly inside the Gobet-Menozzi-shrunk patch is
 * its GM exit.  Both exits are resolved as in pdd_assemble and scored with
 * the warm-up solution, phi = Z_K + Y_K u0(P_K): u0 interpolated from
 * u_knots (device double[n], e.g. pdd_solve of a warm-up assembly) on
 * interface sides and the boundary datum g on the domain boundary.  With
 * run->cv in gradient-table mode, xi (eq. 37) is drawn alongside and taken
 * at the GM exit (run->cv NULL: xi = 0).  With run->interp =
 * PDD_INTERP_RBF_IMQ, u0 at an interface exit is the RBF interpolant of the
 * side's stencil values (as pdd_assemble interpolates; float64, n * 4 *
 * stencil-length doubles of extra scratch).  The network mode and
 * h_per_knot are not accepted (PDD_EINVAL, PDD_EUNSUPPORTED).
 * Path p of knot k draws from the Philox counter (draw, p, k, run->instance)
 * with key run->seed; run->exit_rule, n_paths_per_knot and dump are not used.
 * stats: device double[n * PDD_CAL_WIDTH], the per-knot sums listed at
 * PDD_CAL_WIDTH, each summed over the knot's paths in a fixed order.  Needs
 * n * n_paths * 40 bytes (plus 512) of scratch, at most 16 GiB. */
pdd_status pdd_calibrate(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part, const pdd_knots* knots,
                         const pdd_run* run, const double* u_knots, double* stats);

/* Per-knot parameters from the calibration sums (host only; all arrays host):
 * with N = n_paths, h0_cal the calibration step h0' that pdd_calibrate ran
 * with (run->h), h0 the production cap (0 < h0 <= h0_cal, Sec. 4.2; the
 * Sec. 4.3 pseudocode takes h0_cal = h0) and the means over the knot's paths,
 *   bias[i] = |mean(phi_EM - phi_GM)| / 2                     (eqs. 35-36)
 *   var[i]  = mean(phi_GM^2) - mean(phi_GM)^2 (>= 0)
 *   rho2[i] = cov(phi_GM, xi)^2 / (var(phi_GM) var(xi)) (0 if a variance is 0)
 *   h[i]    = min(h0, 2 h0_cal eps / (3 |mean(phi_GM - phi_EM)|)) (eq. 40; h0 if 0)
 *   paths[i]= 9 var (1 - rho2) / eps^2 rounded to the closest k n_job, k >= 1
 *                                                              (eq. 41)
 * stats: double[n * PDD_CAL_WIDTH] (pdd_calibrate's, copied to the host);
 * h, paths: outputs of n entries; bias, var, rho2 nullable. */
pdd_status pdd_calibration_plan(int64_t n, const double* stats, int64_t n_paths, double h0_cal, double h0, double eps,
                                int32_t n_job, double* h, int32_t* paths, double* bias, double* var, double* rho2);

/* Shape parameter of the inverse multiquadric (Sec. 5.1 picks it so that the
 * interpolation matrix has a spectral condition number of about 1e10), host
 * only: the c at which the matrix Phi_ij = phi_c(|i - j| spacing) of n_nodes
 * equispaced points reaches condition number target_cond, found by bisection
 * on log c in [1e-3, 1e3] spacing to a relative width of 1e-12 (eigenvalues
 * by cyclic Jacobi).  PDD_EINVAL for n_nodes < 2 or > 256, spacing <= 0,
 * target_cond outside (1, 1e14] (beyond, float64 cannot resolve it) or
 * outside the range reached in that interval. */
pdd_status pdd_rbf_shape(int32_t n_nodes, double spacing, double target_cond, double* c);

/* ---- control-variate network (eqs. 11, 37-38) ---------------------------- */

/* Initial parameters (device params[PDD_MLP_PARAMS]): zero biases and
 * Glorot-uniform weights, W1, W2 and w3 each uniform on (-lim, lim) with
 * lim = sqrt(6 / (fan_in + fan_out)); parameter i draws the first word of
 * Philox4x32-10 at counter (i, 0, 0, 0), key (seed lo, seed hi). */
pdd_status pdd_mlp_init(pdd_ctx* ctx, float* params, uint64_t seed);

/* v and/or grad v of the 2-64-64-1 tanh network at n points (float32, device
 * arrays: params[PDD_MLP_PARAMS], xy[2n], v[n] nullable, grad[2n] nullable;
 * n = 0 does nothing, and xy, v and grad may then all be NULL).  xy and grad
 * are in the network's own (unit) coordinates, as pdd_collect_training
 * writes them. */
pdd_status pdd_mlp_eval(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* v, float* grad);

/* grad v of the network at n points through the routine that the float32
 * network control variate (PDD_CV_NETWORK, PDD_FP32_PRODUCTION) runs at every
 * Euler step of pdd_assemble (eq. 37's F = sigma^T grad v): bf16 operands on
 * the matrix cores with float32 accumulation, layer 1 and the final
 * contraction from hi/lo bf16 splits, tanh on the vector units.  Arguments as
 * for pdd_mlp_eval (device: params[PDD_MLP_PARAMS], xy[2n] and grad[2n]
 * float32 in the network's unit coordinates; n = 0 does nothing).  Results
 * equal the float64 definition within the rounding of the bf16 operands
 * (about 2^-9 of each product term); pdd_mlp_eval gives the float32 form. */
pdd_status pdd_mlp_grad_bf16(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* grad);

/* Gradient of the loss L = mean_i (v(x_i) - t_i)^2 / 2 over the n points with
 * respect to all parameters (device: grad[PDD_MLP_PARAMS]; loss[1] nullable),
 * computed by the trainer's forward and backward pass in float32. */
pdd_status pdd_mlp_grad(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, const float* target,
                        float* grad, float* loss);

/* `steps` Adam updates (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, the
 * step counter continuing from step0) of params in place; step s uses the
 * points order[(s batch + i) mod n_order], i < batch, of the n_points pairs
 * (xy[2 n_points], target[n_points]; order entries outside [0, n_points) are
 * skipped; the loss is still averaged over `batch`).  adam_m / adam_s are
 * the moment vectors (device, PDD_MLP_PARAMS each, zero before the first
 * call); losses[steps] (nullable) receives each step's loss.  Up to a batch
 * of 1024 one workgroup runs the whole sequence (the steps are sequential);
 * larger batches spread each step over workgroups of 256 points, whose
 * gradients are summed in workgroup order before the update (two launches
 * per step; scratch of about 18 KB per workgroup). */
pdd_status pdd_mlp_train(pdd_ctx* ctx, float* params, float* adam_m, float* adam_s, int64_t n_points,
                         const float* xy, const float* target, const int32_t* order, int64_t n_order, int32_t batch,
                         int32_t steps, int32_t step0, float lr, float* losses);

/* grad v on the lut_n x lut_n node grid of the partition's domain, the table
 * read by PDD_CV_GRAD_LUT: grad_lut[(j lut_n + i) 2 + d] (device); node
 * (i, j) is the network input (i, j)/(lut_n - 1), and the gradient is scaled
 * to the domain's coordinates. */
pdd_status pdd_mlp_bake_grad_lut(pdd_ctx* ctx, const float* params, const pdd_partition* part, int32_t lut_n,
                                 float* grad_lut);

/* Training pairs from the method's own paths: for every knot k and path
 * p < paths_per_knot (the float32 step of the production assembly; the
 * Philox counter (draw, p, k, run.instance + PDD_COLLECT_STREAM) with key
 * run.seed, run.instance < 2^30, so the pairs never share paths with an
 * assembly whose instance word is below 2^30: a network fitted on them stays
 * adapted to the assembly's Brownian increments, eq. 38; an assembly with
 * instance word run.instance + PDD_COLLECT_STREAM replays the same paths),
 * the first points_per_path iterates X_n receive the tail score
 * (Z_K + Y_K u(exit) - Z_n) / Y_n, u at the exit interpolated from u0 (device,
 * the solved knot values) or the boundary datum.  Outputs (device, slot
 * (k paths_per_knot + p) points_per_path + n): xy[2 slots] (the iterate in
 * the domain's unit coordinates, the network's input), target[slots];
 * slots past a path's exit get a NaN target.  run.cv must be NULL and
 * run.interp PDD_INTERP_HAT (else PDD_EUNSUPPORTED). */
pdd_status pdd_collect_training(pdd_ctx* ctx, const pdd_coeffs* coeffs, const pdd_partition* part,
                                const pdd_knots* knots, const pdd_run* run, const double* u0, int32_t paths_per_knot,
                                int32_t points_per_path, float* xy, float* target);

/* ---- launch control and measurement ------------------------------------ */

/* Ticket schedules: STATIC gives wave w the tickets w, w + W, w + 2W, ...
 * (bitwise reproducible sums for a fixed launch shape); DYNAMIC lets waves
 * claim tickets from a device counter (better balance; float64 sums then
 * vary at rounding level between runs). */
enum { PDD_SCHEDULE_STATIC = 0, PDD_SCHEDULE_DYNAMIC = 1 };

/* Override the assembly launch shape (0 = automatic): threads per block (a
 * multiple of 64, at most 256), workgroups in the persistent grid, paths per
 * ticket (the unit a wave takes from the work list) and the ticket schedule.
 * Results do not depend on these except through float64 summation order. */
pdd_status pdd_set_launch(pdd_ctx* ctx, int32_t block, int32_t grid, int32_t paths_per_ticket,
                          int32_t schedule);
/* Deferred refill: a wave refills the lanes whose paths have exited only once
 * at least min_idle of its 64 lanes are idle, or none is running (1, the
 * default, refills at once; at most 64).  Larger values trade idle lanes for
 * fewer refill passes.  Results do not depend on it except through float64
 * summation order.  pdd_autotune also tries 8, 16 and 32 on its best shape
 * and leaves the winner set. */
pdd_status pdd_set_refill(pdd_ctx* ctx, int32_t min_idle);
/* Tally rows of an assembly workgroup (batched launches and the LUT family;
 * other single-instance assemblies keep two rows per wave): its waves share
 * a pool of one row per wave plus `spare` more (at most one more per wave;
 * -1, the default: one more per wave, so every wave can hold its current and
 * its draining ticket at once).  Fewer rows use less LDS per wave, so more waves fit on a CU; a
 * wave that finds no free row for its next ticket keeps stepping its running
 * paths, or, with none running, waits for another wave of the workgroup to
 * flush one.  Results do not depend on it except through float64 summation
 * order.  pdd_autotune also tries 2, 1 and 0 on its best block size and
 * schedule, with tickets of 1024 to 4096 paths. */
pdd_status pdd_set_spare_rows(pdd_ctx* ctx, int32_t spare);
/* The context's current spare-row setting (-1: one per wave). */
pdd_status pdd_get_spare_rows(const pdd_ctx* ctx, int32_t* spare);
/* The context's current refill threshold (as set by pdd_set_refill or chosen
 * by pdd_autotune). */
pdd_status pdd_get_refill(const pdd_ctx* ctx, int32_t* min_idle);
/* Table reads of the float32 LUT assembly.  With read_all = 0 (the
 * default) every assembly first scans the table for fields that hold the
 * same finite value at every node; when at most two of the seven fields
 * vary, the cell-major copy keeps only their bilinear forms and the kernel
 * reads them one lane per path, taking the constant fields from the
 * table's first node.  read_all = 1 keeps the full eight-form copy and the
 * cooperative read.  Both give the same bits (the bilinear form of a
 * constant field evaluates to the constant exactly). */
pdd_status pdd_set_table_read(pdd_ctx* ctx, int32_t read_all);
/* After an assembly of the LUT family in float32 production (waits for the
 * context's stream): *varying receives bit q set for each field q (sxx, sxy,
 * syy, dx, dy, c, f) the scan found varying or not finite; *lane_read 1 when
 * the lane-per-path read of the varying fields ran, 0 for the full read. */
pdd_status pdd_table_fields(pdd_ctx* ctx, uint32_t* varying, int32_t* lane_read);
/* Shape of the last assembly launch: grid, block and number of tickets. */
pdd_status pdd_last_launch(const pdd_ctx* ctx, int32_t* grid, int32_t* block, int64_t* tickets);
/* enable != 0: bracket every assembly kernel launched from now on with a pair
 * of HIP events on the context's stream (up to 4096 launches; the list is
 * cleared by every call of pdd_set_timing).  pdd_kernel_ms waits for the
 * recorded launches and returns the summed kernel time in milliseconds and
 * the number of launches timed. */
pdd_status pdd_set_timing(pdd_ctx* ctx, int32_t enable);
pdd_status pdd_kernel_ms(pdd_ctx* ctx, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* PDD_H */
