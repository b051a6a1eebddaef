/*
 * uvadmm.h -- C ABI of the MI355X (gfx950) UV-decomposition ADMM conic solver.
 *
 * Solves  minimize c'x  subject to  A x = b,  x in K            (Section II,
 * eq. prob_primal) with K = R_+^{n_orthant} x K_{s_1} x ... x K_{s_q}, a
 * product of Lorentz cones K_s = { w in R^s : w_1 >= ||(w_2..w_s)||_2 } (the
 * orthant coordinates are cones of size 1), by the two-block ADMM on the
 * UV-decomposed reformulation (Section IV, eq. prob_reform, Algorithm 1).
 *
 * Every iteration is a closed-form sweep (Algorithm 1, repeat block):
 *   x-step (Block 1, eq. vvt), y-step with the matrix inversion lemma
 *   (Block 2), z-step = projection onto K (eq. proj), dual updates.
 * The library runs it in an algebraically equivalent reduced form that keeps
 * no per-nonzero vectors: gamma = -U'lambda holds after every iteration, so
 * y and gamma are never stored, and an iteration is one pass over A in
 * column-major order (A'u, x-step, projection, delta update) and one in
 * row-major order (A x, lambda update).
 *
 * Conventions for every entry point:
 *  - All pointers passed in are HOST pointers unless stated otherwise.  The
 *    library copies what it needs during the call; the caller keeps
 *    ownership of its buffers and may free them as soon as the call returns.
 *  - Every int-returning function returns UV_OK (0) or a negative UV_E* code;
 *    solver_strerror() names it.  On error no state is changed unless stated.
 *  - The returned multiplier lambda is the paper's: it multiplies U y = b in
 *    the augmented Lagrangian (eq. lll), so the textbook dual variable of
 *    A x = b is -lambda, the dual objective is -b'lambda and the gap is
 *    c'x + b'lambda.
 *  - Device work is ordered on one HIP stream (opts.hip_stream, or a stream
 *    the library creates when it is NULL).  A solver handle must not be used
 *    from two host threads at once.
 */
#ifndef UVADMM_H
#define UVADMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define UV_OK        0
#define UV_EINVAL   -1  /* null pointer, mu <= 0, m < 1, n < 1, bad option */
#define UV_EBADCSR  -2  /* row_ptr not starting at 0 / not monotone / not ending
                           at nnz, column index out of range, or column indices
                           not strictly increasing within a row */
#define UV_ECONE    -3  /* cone sizes do not sum to n, a size < 1, or a
                           second-order cone larger than UV_MAX_CONE */
#define UV_ENOMEM   -4  /* device or pinned-host allocation failed */
#define UV_EHIP     -5  /* a HIP runtime call failed */
#define UV_ENUMERIC -6  /* NaN or Inf met in a residual check (non-finite
                           b or c are accepted at create and end the run
                           at its first check with this code) */
#define UV_ETOOBIG  -7  /* nnz >= 2^31 (device indices are 32-bit) */
#define UV_ENOSCRATCH -8  /* the problem does not fit solver_solve_noalloc */

/* Largest second-order cone handled (one workgroup projects a cone). */
#define UV_MAX_CONE 1024

/* Arithmetic of the sweep. */
#define UV_FP64  0   /* everything in FP64 */
#define UV_MIXED 1   /* A, x, z, u, b, c in FP32 for the sweep; lambda and
                        delta accumulate in FP64; residuals in FP64 with the
                        FP64 values of A */

/* Solver status (uv_residuals.status). */
#define UV_STATUS_RUNNING   0
#define UV_STATUS_CONVERGED 1  /* kkt <= eps_kkt at a check */
#define UV_STATUS_MAX_ITER  2  /* max_iter reached without convergence */
#define UV_STATUS_NUMERIC   3  /* NaN/Inf seen at a check; iteration stopped */

/* A in compressed sparse row form: row i holds the entries
 * col_idx[row_ptr[i] .. row_ptr[i+1]-1] with values val[...].  Column
 * indices strictly increase within a row.  Explicitly stored zeros are kept
 * as entries (they are still a valid UV decomposition: their column of U is
 * zero and they count in V V'). */
typedef struct {
    int32_t m, n;            /* rows (constraints), columns (variables) */
    int64_t nnz;             /* stored entries, row_ptr[m] */
    const int64_t *row_ptr;  /* m + 1 entries */
    const int32_t *col_idx;  /* nnz entries */
    const double *val;       /* nnz entries */
} uv_csr;

/* K: the first n_orthant coordinates are nonnegative; then n_soc Lorentz
 * cones of sizes soc_sizes[0..n_soc-1] follow in order, each with its
 * "t" coordinate first (Section II).  n_orthant + sum(soc_sizes) == n. */
typedef struct {
    int32_t n_orthant;
    int32_t n_soc;
    const int32_t *soc_sizes;
} uv_cones;

typedef struct {
    double mu;            /* ADMM penalty, > 0 (Algorithm 1 takes a fixed mu) */
    int32_t precision;    /* UV_FP64 or UV_MIXED */
    int32_t check_every;  /* residual check every this many iterations (>= 1) */
    double eps_kkt;       /* stop when kkt <= eps_kkt at a check (0 = never) */
    int64_t max_iter;     /* cap on the total iteration count (0 = none) */
    void *hip_stream;     /* hipStream_t to order all device work on, or NULL */
    int32_t lanes_row;    /* lanes per row in the A x pass without slabs or
                             with slab_kernel 2 (0 = automatic; else 1, 2,
                             4, 8, 16, 32 or 64); the chunked slab passes do
                             not use lanes_* or unroll_* */
    int32_t lanes_col;    /* lanes per column in the A'u pass (same values) */
    int32_t use_graph;    /* 1 = replay check_every iterations as one captured
                             HIP graph; 0 = launch kernels one by one */
    int32_t unroll_row;   /* gathers in flight per lane in the A x pass
                             (0 = automatic; else 1, 2, 4 or 8) */
    int32_t unroll_col;   /* same for the A'u pass */
    int32_t slabs_row;    /* XCD slabs of x in the A x pass: 0 = automatic
                             (none up to 2 MiB of x, two up to 6 MiB, else
                             four), 1 = none, 2, 4, 8 */
    int32_t slabs_col;    /* XCD slabs of u in the A'u pass: 0 = automatic
                             (none up to 2 MiB of u, two up to 16 MiB, else
                             four), 1 = none, 2, 4, 8 */
    int32_t criterion;    /* UV_CRIT_KKT, UV_CRIT_INF or UV_CRIT_POGS */
    double eps_abs;       /* absolute tolerance of UV_CRIT_INF; the bound
                             on ||A x - b||_2 of UV_CRIT_POGS */
    int32_t slab_kernel;  /* slab passes: 0 = automatic (= 1), 1 = 64-segment
                             chunks per wavefront (eight 64-entry steps in
                             flight), 2 = lane group per segment, 3 = chunks
                             with four steps in flight */
    double eps_gap;       /* bound on |c'x + b'lambda| of UV_CRIT_POGS, and
                             an extra condition of UV_CRIT_INF when > 0
                             (0 = none); >= 0 */
    int32_t resident;     /* 0 = automatic: a problem whose cones all have
                             size 1, with m, n < 65536 and small enough for
                             one CU's LDS (about 150 KiB: x, z, u, delta,
                             lambda and both copies of A with 16-bit row and
                             column numbers) runs on the resident path, one
                             workgroup iterating in LDS with the checks in
                             the same launch, unless lanes_*, unroll_*,
                             slabs_* or slab_kernel force a shape of the
                             sweep kernels; 1 = never; 2 = required
                             (UV_EINVAL at create when it does not apply) */
    int32_t history;      /* residual history: the last `history` checks of
                             the iteration are recorded on the device (0 =
                             none; at most 2^24); see solver_history */
    int32_t full_checks;  /* 0 = a check of the iteration evaluates its
                             primal half first (the row residuals, which
                             the row pass forms anyway) and its column half
                             (A'lambda: the dual residual, c'z, the gap) only
                             when the primal half passes the stopping test,
                             since otherwise the check cannot stop the run:
                             the same stopping iteration, status and
                             iterates, and a NaN on the dual side alone shows
                             at the next check whose primal half passes or
                             whose primal residual is NaN; 1 = every check
                             evaluates both halves.  Checks are always whole
                             with a residual history, in the family solver
                             and in solver_residuals; the resident path, the
                             batched solver and the standard-ADMM baseline
                             gate their checks the same way */
} uv_opts;

/* Stopping tests (Section V): UV_CRIT_KKT stops when kkt <= eps_kkt (the
 * SCS-form relative residuals of Section V-B); UV_CRIT_INF stops when
 * prim_inf <= eps_abs + eps_kkt * scale_p and dual_inf <= eps_abs +
 * eps_kkt * scale_d (the infinity-norm test of the OSQP comparison, Section
 * V-A1), and, when eps_gap > 0, gap_x < eps_gap (that comparison's gap
 * condition); UV_CRIT_POGS stops when res_ax_b < eps_abs and gap_x <
 * eps_gap (the test of the POGS comparison, Section V-A2, eq. stopcri, whose
 * two bounds are the competitor's ||A x - b||_2 and |c'x + b'lambda|, given
 * here by the caller).  Each is evaluated at the checks only. */
#define UV_CRIT_KKT  0
#define UV_CRIT_INF  1
#define UV_CRIT_POGS 2

/* Residuals at the last check, evaluated at (z, lambda, delta), all FP64
 * (the SCS-form test of Section V-B, with the dual residual taken for
 * x in K and an absolute gap):
 *   r_prim = ||A z - b|| / (1 + ||b||)
 *   r_dual = ||A'lambda + c - delta|| / (1 + ||c||)
 *   r_gap  = |c'z + b'lambda| / (1 + |c'z| + |b'lambda|)
 *   kkt    = max(r_prim, r_dual, r_gap)
 * pobj = c'z, dobj = -b'lambda, res_ax_b = ||A x - b|| (at x, as printed),
 * pobj_x = c'x and gap_x = |c'x + b'lambda| (the gap at x of Section V-A). */
typedef struct {
    double r_prim, r_dual, r_gap, kkt;
    double pobj, dobj;
    double res_ax_b;
    double prim_inf;      /* ||A z - b||_inf */
    double dual_inf;      /* ||A'lambda + c - delta||_inf */
    double scale_p;       /* max(||A z||_inf, ||b||_inf) */
    double scale_d;       /* max(||A'lambda||_inf, ||c||_inf) */
    int64_t iter;         /* iterations done when these were evaluated */
    int32_t status;       /* UV_STATUS_* */
    double pobj_x;        /* c'x */
    double gap_x;         /* |c'x + b'lambda| */
} uv_residuals;

typedef struct uv_solver uv_solver;

/* Test hook for the out-of-memory paths: after `after` more successful
 * device or pinned-host allocations made by the library, the next one fails
 * as if memory were exhausted (the entry point then returns UV_ENOMEM and
 * frees what it had taken); the hook then disarms itself.  A negative value
 * disarms it.  Process-wide; not for use while other threads call the
 * library. */
void uv_test_fail_alloc(int64_t after);

/* Fills *o with the defaults: mu = 1, UV_FP64, check_every = 10,
 * eps_kkt = 1e-4, max_iter = 0, NULL stream, automatic lanes, graphs on. */
void uv_default_opts(uv_opts *o);

/* Validates and copies the problem to the device, builds the column-major
 * copy of A and the diagonal factors F_U = (I + U U')^{-1} and
 * F_V = (I + V V')^{-1} (the set-up of Algorithm 1; U U' = diag of the squared
 * row norms of A and V V' = diag of the column counts), and sets the zero
 * start.  b has m entries, c has n.  opts may be NULL (defaults).  On
 * success *out owns device memory until solver_destroy. */
int solver_create(const uv_csr *A, const double *b, const double *c,
                  const uv_cones *K, const uv_opts *opts, uv_solver **out);

/* Sets the starting point (Algorithm 1's "initial points"): x, z, delta
 * (n entries) and lambda (m entries), any of them NULL for zero.  The
 * per-nonzero variables start at y = V'x and gamma = -U'lambda.  Resets the
 * iteration count and the status. */
int solver_set_start(uv_solver *s, const double *x, const double *z,
                     const double *delta, const double *lambda);

/* Restores a state returned by solver_solution so that iterating continues
 * the interrupted run (checkpoint / resume).  The iterate (x, z, delta,
 * lambda) at the end of an iteration fixes the per-nonzero variables too:
 * gamma = -U'lambda, and y is the y-step's output at x with that gamma,
 * y = (I - U'F_U U)(U'b + V'x) (Block 2 with the matrix inversion lemma).
 * (solver_set_start instead takes y = V'x, the plain starting point.)
 * Resets the iteration count and the status; NULL means zero. */
int solver_resume(uv_solver *s, const double *x, const double *z,
                  const double *delta, const double *lambda);

/* Replaces the right-hand side b (m doubles, host; every entry finite, else
 * UV_EINVAL) of problem eq. prob_primal, keeping A, c, the cones, the
 * factors F_U, F_V and the device set-up: one handle serves a family of
 * problems that differ in b.  The iterate belongs to the old b, so the next
 * iteration needs a new start: solver_iterate returns UV_EINVAL until
 * solver_set_start or solver_resume is called (with the state of a run on
 * this b, solver_resume continues that run).  Residual queries evaluate
 * against the new b. */
int solver_set_rhs(uv_solver *s, const double *b);

/* Runs up to k iterations (fewer if kkt <= eps_kkt at a check, or max_iter
 * is reached) and waits for them.  Checks happen when the total iteration
 * count is a multiple of check_every.  *done (may be NULL) is set to 1 when
 * the solver has stopped (converged, max_iter, or numeric failure). */
int solver_iterate(uv_solver *s, int64_t k, int32_t *done);

/* Residuals of the current iterate (evaluated now if the state changed
 * since the last check).  An evaluation made here, between checks, only
 * reports: the status and the stopping decision change at the iteration's
 * own checks alone, so polling does not change the trajectory. */
int solver_residuals(uv_solver *s, uv_residuals *r);

/* Copies the current iterate to caller-owned host buffers: x, z, delta
 * (n doubles each), lambda (m doubles); any may be NULL. */
int solver_solution(uv_solver *s, double *x, double *z, double *lambda,
                    double *delta);

/* Frees everything the handle owns.  NULL is ignored. */
void solver_destroy(uv_solver *s);

/* Static string for a UV_E* code. */
const char *solver_strerror(int code);

/* One record of the residual history: a check of the iteration (Section
 * V-B's residuals, as in uv_residuals), with the GPU time since the start
 * (solver_set_start or solver_resume) at which it was taken. */
typedef struct {
    int64_t iter;
    double seconds;
    double r_prim, r_dual, r_gap, kkt, pobj, dobj, res_ax_b, gap_x;
} uv_history;

/* The latest min(max, recorded, opts.history) checks of the residual
 * history into out[0..*count-1], oldest first (host buffer of max records);
 * *count = 0 when opts.history was 0.  Residual queries between checks are
 * not recorded; a new start (solver_set_start, solver_resume) begins a new
 * history.  The one-call solves keep none. */
int solver_history(uv_solver *s, int32_t max, uv_history *out, int32_t *count);

/* One call: solver_create, iterations from the zero start until the
 * stopping test holds at a check or `iters` iterations (or max_iter) are
 * done, solver_solution (any output may be NULL) and solver_residuals of the
 * final iterate into *r (may be NULL), then solver_destroy.  Returns what
 * solver_create or solver_iterate returned (UV_ENUMERIC with the outputs
 * filled on a numeric stop), else the first failing call's code. */
int solver_solve(const uv_csr *A, const double *b, const double *c,
                 const uv_cones *K, const uv_opts *opts, int64_t iters,
                 double *x, double *z, double *lambda, double *delta,
                 uv_residuals *r);

/* solver_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments and results (bitwise the same outputs as solver_solve),
 * and no device, pinned-host or host heap allocation -- every device buffer
 * is carved from one fixed 2 MiB array per GPU, which each GPU keeps until
 * the process ends.  It serves the problems of the resident path: every
 * cone of size 1, m, n < 65536, small enough for one CU's LDS (about
 * 158 KiB) and for the fixed array; others return UV_ENOSCRATCH before any
 * device work (UV_EINVAL with opts.resident = 1).  Inputs and outputs are
 * host buffers as for solver_solve; the work is ordered on opts.hip_stream
 * (NULL: the null stream) and the call returns when it is done.  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (two host
 * threads, or two streams) race and must not be made; a call overwrites all
 * it reads of the array before reading it. */
int solver_solve_noalloc(const uv_csr *A, const double *b, const double *c,
                         const uv_cones *K, const uv_opts *opts,
                         int64_t iters, double *x, double *z,
                         double *lambda, double *delta, uv_residuals *r);

/* Measurement: runs `iters` iterations (no residual checks), timing every
 * kernel launch with HIP events on the solver's stream, and returns the
 * average duration in milliseconds of the column pass (A'u, x-step,
 * projection, delta update) and of the row pass (A x, lambda update). */
int solver_time_kernels(uv_solver *s, int32_t iters, double *ms_col,
                        double *ms_row);

/* The resolved launch shape: shape[0] lanes per row and shape[1] gathers in
 * flight per lane in the row pass, shape[2], shape[3] the same for the
 * column pass, shape[4], shape[5] the XCD slab counts of the row and column
 * passes, shape[6] 1 on the resident path (shape holds 7 entries).  On the
 * resident path solver_iterate runs the resident kernel; the other calls
 * (residual queries between checks, resume, solver_time_kernels) use the
 * sweep kernels on the same state. */
int solver_launch_shape(const uv_solver *s, int32_t *shape);

/* ------------------------------------------------------------------------
 * Batched solver: many independent problems with the orthant cone
 * (min c_i'x s.t. A_i x = b_i, x >= 0), solved together.  One persistent
 * launch (replayed as a captured HIP graph) gives each workgroup one
 * instance at a time, longest first; x and u of the instance live in LDS,
 * so (m_i + n_i) * 4 bytes (UV_MIXED) or * 8 bytes (UV_FP64) must fit in
 * 159 KiB (a CU's 160 KiB less the kernel's own reduction slots); when
 * (m_i + 3 n_i) values fit for every instance, z and c are kept there too.
 * Row and column numbers are held instance-local in 16 bits, which that
 * bound always allows.  The iteration, residuals and stopping rule are those of the
 * single-problem solver; each instance keeps its own iteration count and
 * status, and an instance that has stopped is skipped by later launches.
 * ------------------------------------------------------------------------ */
typedef struct uv_batch uv_batch;

/* count instances; A[i] in CSR, b[i] (A[i].m doubles), c[i] (A[i].n
 * doubles).  opts as for solver_create (lanes and unroll fields unused; the
 * tiles below set the lanes).  Everything is copied.  UV_ETOOBIG if an
 * instance's x and u do not fit in LDS or the totals reach 2^31. */
int batch_create(int32_t count, const uv_csr *A, const double *const *b,
                 const double *const *c, const uv_opts *opts, uv_batch **out);

/* Runs up to k more iterations of every running instance; *n_active (may
 * be NULL) receives the number still running afterwards. */
int batch_iterate(uv_batch *h, int64_t k, int32_t *n_active);

/* Residuals / status of instance i at its last whole check (see
 * uv_residuals; the infinity-norm fields, pobj_x and gap_x are not evaluated
 * by the batched solver and read 0).  With opts.full_checks = 0 a check whose
 * r_prim exceeds eps_kkt (it cannot stop the instance) skips its column half
 * and records nothing; the check that stops an instance is always whole.  Returns UV_ENUMERIC (with *r filled) when that instance stopped on a
 * NaN or Inf. */
int batch_residuals(uv_batch *h, int32_t i, uv_residuals *r);

/* Iterate of instance i into caller-owned host buffers (any may be NULL):
 * x, z, delta (n_i doubles), lambda (m_i doubles). */
int batch_solution(uv_batch *h, int32_t i, double *x, double *z,
                   double *lambda, double *delta);

/* Starting point of instance i (as solver_set_start); resets its iteration
 * count and status so later launches run it again. */
int batch_set_start(uv_batch *h, int32_t i, const double *x, const double *z,
                    const double *delta, const double *lambda);

/* Launch tiles: threads per workgroup (64..1024, a power of two) and
 * lanes[8] = (lanes per row, lanes per column) for the four size buckets
 * m < 128, m < 512, m < 2048, m >= 2048 (powers of two, <= threads).
 * Lanes per column 0 selects the sliced column copy: a wavefront per 64
 * columns whose t-th entries are stored side by side, so every entry load
 * is one coalesced access; the sums are those of one lane per column, bit
 * for bit.  UV_EINVAL for any other value. */
int batch_set_tiles(uv_batch *h, int32_t threads, const int32_t *lanes);
int batch_get_tiles(const uv_batch *h, int32_t *threads, int32_t *lanes);

/* Measurement for the tile search: duration (ms) of one launch running
 * `iters` iterations of the instances of one size bucket (0..3, or -1 for
 * all) with the current tiles.  The state is saved before and restored
 * after, so timing does not advance any instance. */
int batch_time(uv_batch *h, int32_t bucket, int32_t iters, double *ms);

/* info[0..5] = count, total rows, total columns, total nonzeros,
 * workgroups per launch, LDS bytes per workgroup. */
int batch_info(const uv_batch *h, int64_t *info);

void batch_destroy(uv_batch *h);

/* ------------------------------------------------------------------------
 * Parametric family: one A and c (orthant cone), B right-hand sides
 * b_1..b_B iterated together.  Per-instance vectors live instance-fastest on
 * the device (entry j of instance l at j * B + l), so every nonzero of A is
 * read once per 64 instances and its gather is one contiguous line.  Each
 * instance is checked every check_every iterations and frozen once it stops.
 * Host arrays below are instance-major: instance l's vector starts at
 * l * length.
 * ------------------------------------------------------------------------ */
typedef struct uv_family uv_family;

/* B: instances per launch, a multiple of 64 in [64, 1024].  opts as for
 * solver_create (lanes/unroll unused).  A and c are copied. */
int family_create(const uv_csr *A, const double *c, int32_t B,
                  const uv_opts *opts, uv_family **out);

/* Right-hand sides of the first nb <= B instances (nb x m doubles) and the
 * zero start for all of them; instances nb..B-1 stay idle. */
int family_set_rhs(uv_family *h, int32_t nb, const double *b);

/* Start of the current nb instances (nb x n for x, z, delta; nb x m for
 * lambda; NULL = zero), with y = V'x and gamma = -U'lambda as in
 * solver_set_start; resets iteration counts and statuses. */
int family_set_start(uv_family *h, const double *x, const double *z,
                     const double *delta, const double *lambda);

/* Start from predicted primal-dual points held on the DEVICE: row l of
 * xl_dev (FP32, row stride ld >= n + m) is [x (n) ; lambda (m)].  Sets
 * z = max(x, 0) and delta = max(c + A'lambda, 0) (the stationarity
 * condition c + A'lambda - delta = 0 projected on the dual cone).  parts:
 * 1 = use the predicted x only (lambda = 0), 2 = lambda only (x = 0),
 * 3 = both. */
int family_set_start_predicted(uv_family *h, const float *xl_dev, int64_t ld,
                               int32_t parts);

/* New members into stopped slots, so that a slot does not idle until the
 * slowest member of its group stops: slots[0..count-1] (distinct, < nb,
 * each holding a member that has stopped, else UV_EINVAL) take the
 * right-hand sides b (count x m, host, instance-major) and either the zero
 * start (xl_dev NULL) or the predicted start of family_set_start_predicted
 * from the device FP32 rows xl_dev + q * ld, q < count (ld >= n + m; parts
 * as there).  Each entering member counts its own iterations from here, is
 * checked at the family's checks and is capped by max_iter on its own count
 * (after a refill that cap takes effect at the first check at or past it).
 * The other members are untouched; a member's iterates do not depend on the
 * slot it runs in or on the other members. */
int family_refill(uv_family *h, int32_t count, const int32_t *slots,
                  const double *b, const float *xl_dev, int64_t ld,
                  int32_t parts);

/* Up to k more iterations; *n_active = instances still running. */
int family_iterate(uv_family *h, int64_t k, int32_t *n_active);

/* Residuals of the nb current instances into r[0..nb-1] (infinity-norm
 * fields, pobj_x and gap_x not evaluated: 0).  Returns UV_ENUMERIC (with r filled) when any of
 * them stopped on a NaN or Inf. */
int family_residuals(uv_family *h, uv_residuals *r);

/* Iterates of the nb instances into host buffers (instance-major; any may
 * be NULL): x, z, delta (nb x n), lambda (nb x m). */
int family_solution(uv_family *h, double *x, double *z, double *lambda,
                    double *delta);

/* Iterate of the member in one slot (< nb) into host buffers (any may be
 * NULL): x, z, delta (n doubles), lambda (m doubles) -- the state that
 * solver_resume takes, so a member can continue its run on a solver_create
 * handle of the same A and c (its b set by solver_set_rhs), for instance
 * once few members are left running and the group's iteration costs more
 * than the single problem's. */
int family_member_state(uv_family *h, int32_t slot, double *x, double *z,
                        double *lambda, double *delta);

/* FP32 rows [z (n) ; lambda (m)] of the nb instances into a DEVICE matrix
 * with row stride ld >= n + m (training data for a learned start). */
int family_solution_device(uv_family *h, float *dst_dev, int64_t ld);

void family_destroy(uv_family *h);

/* ------------------------------------------------------------------------
 * Algorithm 1 as printed (FP64, orthant cone): y and gamma (one entry per
 * stored nonzero, eq. prob_reform) are stored and updated, U, U', V, V'
 * applied as sums over the nonzero index (eqs. UU, VV).  The ablation of the
 * reduced form and a second GPU implementation of the same iteration; zero
 * start, no residual checks.
 * ------------------------------------------------------------------------ */
typedef struct uv_literal uv_literal;
int literal_create(const uv_csr *A, const double *b, const double *c,
                   const uv_opts *opts, uv_literal **out);
int literal_iterate(uv_literal *h, int64_t k);
/* x, z, delta (n), lambda (m), y, gamma (nnz, CSR order); any may be NULL. */
int literal_solution(uv_literal *h, double *x, double *z, double *lambda,
                     double *delta, double *y, double *gamma);
/* Average duration (ms) of the column and row passes over `iters` iterations. */
int literal_time(uv_literal *h, int32_t iters, double *ms_col, double *ms_row);
void literal_destroy(uv_literal *h);

/* ------------------------------------------------------------------------
 * Baseline: standard two-block ADMM on the splitting x1 = x2 (Section II-B:
 * f the cone indicator, g the objective on {A x = b}) with the block system
 * eq. lin solved indirectly every iteration (Section III-B): conjugate
 * gradients on (A A') nu = A (w0 - c/mu) - b, warm-started from the previous
 * nu.  FP64, K as for solver_create.  Per iteration:
 *   x1 = proj_K(x2 - lam/mu);  delta = lam + mu (x1 - x2)
 *   CG: at most cg_iters steps, stopping once ||r||_2 <= cg_tol (1 + ||b||_2)
 *       or when p'A A'p is not positive
 *   x2 = x1 + lam/mu - c/mu - A'nu;  lam += mu (x1 - x2)
 * Residuals (uv_residuals, SCS form as for solver_residuals) at z = x1 with
 * the multiplier lambda_A = mu nu of A x = b and delta of the cone; the
 * fields r_prim, r_dual, r_gap, kkt, pobj, dobj, iter, status are set, the
 * others are zero.
 *
 * standard_create: A, b, c as for solver_create (host, copied; invalid CSR
 *   -> UV_EBADCSR); K as for solver_create, or NULL for the orthant (cone
 *   sizes not summing to n or below 1 -> UV_ECONE; one thread projects a
 *   cone, so very large cones are slow but allowed); opts: mu, check_every,
 *   eps_kkt, max_iter, hip_stream, use_graph, slabs_row / slabs_col (0, 1,
 *   2 or 4; 0 = the solver's rule);
 *   precision must be UV_FP64 (else UV_EINVAL); cg_iters >= 0,
 *   cg_tol >= 0 (else UV_EINVAL).  Zero start.
 * standard_set_state: x2, lam (n) and the CG start nu (m), host, any NULL =
 *   zero; resets the iteration count and status.
 * standard_iterate / standard_residuals: as solver_iterate /
 *   solver_residuals; *cg_steps (may be NULL) receives the CG steps taken.
 * standard_solution: x1, x2, lam, delta (n), nu (m) into host buffers; any
 *   may be NULL.
 * ------------------------------------------------------------------------ */
typedef struct uv_standard uv_standard;
int standard_create(const uv_csr *A, const double *b, const double *c,
                    const uv_cones *K, const uv_opts *opts, int32_t cg_iters,
                    double cg_tol, uv_standard **out);
int standard_set_state(uv_standard *h, const double *x2, const double *lam,
                       const double *nu);
int standard_iterate(uv_standard *h, int64_t k, int32_t *done);
int standard_residuals(uv_standard *h, uv_residuals *r, int64_t *cg_steps);
int standard_solution(uv_standard *h, double *x1, double *x2, double *lam,
                      double *nu, double *delta);
/* Slab counts of the row and column products (either may be NULL). */
int standard_launch_shape(uv_standard *h, int32_t *slabs_row, int32_t *slabs_col);
void standard_destroy(uv_standard *h);

/* ------------------------------------------------------------------------
 * Measurement: random-gather rate of the chip, the practical bound of the
 * sweep's sparse products (each stored entry of A is one gather of a vector
 * entry at an address no cache line is shared with).  Streams nnz
 * (int32 index, value) pairs, gathers a table of table_len entries
 * (fp64 != 0: FP64, else FP32) at uniform random positions, workgroup w
 * confined to table part w % slabs (slabs in 1..8, table_len / slabs
 * entries each), eight pairs per thread, one sum stored per thread.  *ms
 * receives the average kernel duration over reps launches after one
 * warm-up.  Allocates and frees its own device buffers (about
 * 12 nnz + 8 table_len bytes); nnz in [1, 2^31), else UV_EINVAL.
 * ------------------------------------------------------------------------ */
int probe_gather(int64_t nnz, int64_t table_len, int32_t slabs, int32_t fp64,
                 int32_t reps, uint64_t seed, double *ms);

/* ------------------------------------------------------------------------
 * Learned warm start: dense kernels.  Pointers marked _dev are DEVICE
 * pointers (for instance from framework tensors); the stream argument may be
 * NULL (the default stream).  All of these wait for their work to finish.
 * ------------------------------------------------------------------------ */

/* C = alpha * A B + beta * C in FP32: A(i,k) = A[i*a_rs + k*a_cs],
 * B(k,j) = B[k*b_rs + j*b_cs], C row-major with leading dimension ldc; all
 * device pointers. */
int gemm_f32(int32_t M, int32_t N, int32_t K, const float *A_dev, int64_t a_rs,
             int64_t a_cs, const float *B_dev, int64_t b_rs, int64_t b_cs,
             float *C_dev, int64_t ldc, float alpha, float beta, void *stream);

/* Y (N x D, leading dimension ld, device) += v (D, device) on every row. */
int add_row_vector(int64_t N, int64_t D, float *Y_dev, int64_t ld,
                   const float *v_dev, void *stream);

/* Y (N x D, leading dimension ld, device) *= v (D, device) column-wise on
 * every row (the standardisation of PCA coefficients). */
int mul_row_vector(int64_t N, int64_t D, float *Y_dev, int64_t ld,
                   const float *v_dev, void *stream);

/* Principal components of the rows of Y (N x D, leading dimension ld,
 * device; CENTERED IN PLACE): mean_dev (D), basis_dev (k x D, orthonormal
 * rows, the top-k right singular vectors of the centered Y) and sv (k
 * singular values, host), by a randomized range finder with power_iters
 * power iterations and k + oversample (<= 1024) probe vectors. */
int pca_fit(float *Y_dev, int64_t N, int64_t D, int64_t ld, int32_t k,
            int32_t oversample, int32_t power_iters, uint64_t seed,
            float *mean_dev, float *basis_dev, float *sv, void *stream);

/* Symmetric eigen-decomposition (host): S (l x l row-major, destroyed) ->
 * eigenvalues w (descending) and eigenvectors in the columns of V. */
int uvla_sym_eig(int32_t l, double *S, double *w, double *V);

/* Multilayer perceptron dims[0] -> dims[1] -> ... -> dims[nlayers], ReLU
 * between layers, linear output; every width a multiple of 16.  GEMMs on
 * the BF16 matrix cores with FP32 accumulation; FP32 master weights
 * (He-uniform initialisation from seed) and Adam state. */
typedef struct uv_mlp uv_mlp;
int mlp_create(int32_t nlayers, const int32_t *dims, int32_t max_batch,
               uint64_t seed, void *stream, uv_mlp **out);
/* All weights (layer by layer, each dims[l] x dims[l+1] row-major) and
 * biases as flat host arrays. */
int mlp_get_params(uv_mlp *h, float *w, float *b);
int mlp_set_params(uv_mlp *h, const float *w, const float *b);
/* y_dev (batch x dims[nlayers]) = net(x_dev (batch x dims[0])); batch a
 * multiple of 16, <= max_batch; device pointers. */
int mlp_forward(uv_mlp *h, int32_t batch, const float *x_dev, float *y_dev);
/* Gradients of the mean squared error mean((net(x) - t)^2) into host
 * arrays laid out as in mlp_get_params, and the loss; no update. */
int mlp_gradients(uv_mlp *h, int32_t batch, const float *x_dev,
                  const float *t_dev, float *gw, float *gb, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss; *loss (may
 * be NULL) receives the loss before the step. */
int mlp_train_step(uv_mlp *h, int32_t batch, const float *x_dev,
                   const float *t_dev, float lr, float *loss);
void mlp_destroy(uv_mlp *h);

/* C (FP32) = A B on BF16 operands (raw bit patterns), strides as gemm_f32;
 * M, N, K multiples of 16 -- the MLP's matrix-core kernel on its own. */
int mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A_dev,
                  int64_t a_rs, int64_t a_cs, const uint16_t *B_dev,
                  int64_t b_rs, int64_t b_cs, float *C_dev, int64_t ldc,
                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* UVADMM_H */
