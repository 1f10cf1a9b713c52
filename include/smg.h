/*
 * smg.h -- C ABI of the MI355X (gfx950) SMG-preconditioned Krylov library.
 *
 * Problem (Section 2 of Bouwmeester, Dougherty and Knyazev, "Nonsymmetric
 * multigrid preconditioning for conjugate gradient methods"): the 7-point
 * negative Laplacian A on an nx*ny*nz brick with homogeneous Dirichlet
 * boundary,
 *     (A x)_{ijk} = cx(2x_{ijk} - x_{i-1jk} - x_{i+1jk}) + cy(...j...) + cz(...k...),
 * neighbours outside the brick counted as zero.  The paper uses unit grid
 * size (cx = cy = cz = 1); a unit cube with n interior points per axis has
 * c = (n+1)^2.
 *
 * Preconditioner T (Section 3): one V-cycle of semicoarsening multigrid
 * (SMG) from a zero initial guess, with plane relaxation as the smoother at
 * every level and independent pre- and post-smoothing counts:
 *   - z is coarsened by two (coarse planes are the odd fine planes), with
 *     linear prolongation P, restriction P^T and Galerkin operators P^T A P;
 *   - a smoothing step is one zebra sweep: every plane of one colour gets the
 *     correction x_k += V2_k((b - A x)_k), then the other colour; pre-sweeps
 *     take the colours in the order F (even) then C (odd), post-sweeps in
 *     reverse, so that equal counts give a symmetric operator (Section 1);
 *   - V2_k is one 2D V-cycle of the same construction in y on plane k's
 *     operator, with x-lines relaxed zebra-wise by exact tridiagonal solves
 *     and one exact line solve on its coarsest level.
 * pre = post gives a symmetric positive definite T; post = 0 gives the
 * nonsymmetric preconditioner that the paper studies.
 *
 * Solvers: Algorithm 1 of Section 2 with beta from equation (1) (pcg_solve),
 * equation (2) (fpcg_solve) or beta = 0 (psd_solve); LOBPCG (Section 4) for
 * the m smallest eigenpairs.
 *
 * Memory: every vector argument is a DEVICE pointer to FP64 data laid out
 * with index i + nx*(j + ny*k) (x fastest); a block of nrhs vectors is
 * column-major with leading dimension ld >= nx*ny*nz.  The caller owns every
 * buffer, including the device workspace handed to smg_setup; the library
 * never frees caller memory and allocates no device memory of its own.
 * `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue work
 * on `stream`; solvers synchronise it before returning their info.
 * A handle is not thread-safe; distinct handles are independent.
 *
 * Return codes: SMG_OK (0); SMG_NOT_CONVERGED (1, outputs valid);
 * SMG_EINVAL (-1); SMG_EWORKSPACE (-2); SMG_EHIP (-3); SMG_EBREAKDOWN (-4, a
 * zero or non-finite denominator in the recurrence); SMG_ENONFINITE (-5, a
 * non-finite input).  No exception or abort crosses this interface.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SMG_OK = 0,
    SMG_NOT_CONVERGED = 1,
    SMG_EINVAL = -1,
    SMG_EWORKSPACE = -2,
    SMG_EHIP = -3,
    SMG_EBREAKDOWN = -4,
    SMG_ENONFINITE = -5
};

/* Storage/arithmetic precision of the SMG hierarchy.  The Krylov recurrences,
 * dot products and LOBPCG's Rayleigh-Ritz always run in FP64; with F32 or
 * BF16 the preconditioner converts r to that precision on entry and s back to
 * FP64 on exit (BF16: bfloat16 storage, FP32 arithmetic). */
enum { SMG_PREC_F64 = 0, SMG_PREC_F32 = 1, SMG_PREC_BF16 = 2 };

enum { SMG_PRECOND_SMG = 0, SMG_PRECOND_NONE = 1 };

typedef struct smg_grid {
    int32_t nx, ny, nz;     /* brick size, each >= 1, nx <= 512 */
    double cx, cy, cz;      /* axis coefficients, each > 0 */
} smg_grid;

typedef struct smg_opts {
    int32_t pre, post;              /* 3D smoothing counts, 0..8 each */
    int32_t inner_pre, inner_post;  /* 2D plane-cycle counts; -1 inherits pre/post */
    int32_t order;                  /* 0: pre F then C (default); 1: pre C then F */
    int32_t precision;              /* SMG_PREC_* */
    int32_t kernel_mode;            /* 0: fused schedule where it applies (default);
                                       1: one launch per stage (reference schedule);
                                       2: the fused schedule with its streaming
                                          kernels at one point per thread (the
                                          same arithmetic, for comparison) */
} smg_opts;

enum { SMG_STOP_2NORM = 0, SMG_STOP_CNORM = 1 };

typedef struct krylov_opts {
    double rtol;            /* stopping threshold, see stop_norm */
    int32_t max_iter;       /* >= 0 */
    int32_t precond;        /* SMG_PRECOND_SMG or SMG_PRECOND_NONE (T = I) */
    int32_t x0_zero;        /* 1: ignore the contents of x and start from 0 */
    int32_t stop_norm;      /* SMG_STOP_2NORM: stop when ||r_k||_2 <= rtol ||b||_2 (recursive r_k);
                               SMG_STOP_CNORM: stop when sqrt|(T r_k, r_k)| <= rtol sqrt|(T b, b)|, the
                               ratio the paper plots (Figs. 2 and 5), tested once s_k = T r_k is formed */
    double *history;        /* HOST, nullable, max_iter+1 entries: ||r_k||_2/||b||_2 */
    double *history_c;      /* HOST, nullable, max_iter entries: sqrt|(s_k,r_k)| / sqrt|(T b, b)| */
    /* Per-step diagnostics of Section 5 (all nullable; they cost two extra
     * stencil passes and a host round trip per iteration):
     *   xstar      DEVICE, the exact solution A^{-1} b (e.g. from a tighter solve);
     *   diag_work  DEVICE, 2*nx*ny*nz doubles of scratch, required with xstar;
     *   err_a      HOST, max_iter+1 entries: ||x* - x_k||_A / ||x* - x_0||_A, which
     *              equals ||r_k||_{A^{-1}} / ||r_0||_{A^{-1}} (needs xstar);
     *   sin_angle  HOST, max_iter entries: sin of the A^{-1}-angle between r_k and
     *              A T r_k, cos = |(r_k, T r_k)| / (||r_k||_{A^{-1}} ||A T r_k||_{A^{-1}})
     *              (Theorem 1: for PSD err_a[k+1]/err_a[k] equals it; flexible PCG,
     *              being locally optimal, is never slower) (needs xstar). */
    const double *xstar;
    double *diag_work;
    double *err_a;
    double *sin_angle;
} krylov_opts;

typedef struct krylov_info {
    int32_t iters;          /* number of x updates performed */
    int32_t status;         /* same value as the return code */
    double rel_res;         /* ||r||_2/||b||_2 of the recursive residual */
    double true_rel_res;    /* ||b - A x||_2/||b||_2 recomputed at exit */
    double solve_seconds;   /* wall time of the iteration, host clock */
    double rel_res_c;       /* sqrt|(T r, r)| / sqrt|(T b, b)| of the last residual T was applied to
                               (the final one with SMG_STOP_CNORM); NaN when T was never applied */
} krylov_info;

typedef struct smg_handle smg_handle;

/* Bytes of device workspace smg_setup needs for this grid and options when
 * smg_apply is called with up to max_nrhs right-hand sides at once (the
 * single-vector Krylov solvers need max_nrhs >= 1).  Host-only; no GPU work. */
int smg_workspace_bytes(const smg_grid *g, const smg_opts *o, int32_t max_nrhs, size_t *bytes);

/* Builds the SMG hierarchy (Galerkin coefficients in z and, per plane, in y;
 * Thomas factor tables of every distinct line operator) inside the caller's
 * device workspace `ws` of `ws_bytes` bytes (>= smg_workspace_bytes) and
 * returns a handle in *out.  The workspace must stay valid and untouched
 * until smg_destroy. */
int smg_setup(const smg_grid *g, const smg_opts *o, int32_t max_nrhs, void *ws, size_t ws_bytes,
              void *stream, smg_handle **out);

/* s = T r for nrhs vectors (1 <= nrhs <= max_nrhs), leading dimension ld.
 * r is read only; r and s must not overlap. */
int smg_apply(smg_handle *h, const double *r, double *s, int32_t nrhs, int64_t ld, void *stream);

/* For callers that cannot allocate device memory (graph-captured code, tight
 * serving loops, harnesses that forbid hipMalloc): s = T r exactly as
 * smg_apply computes it for a handle set up with (g, o) and max_nrhs = nrhs
 * (same kernels, bitwise equal results), with no handle and no workspace
 * argument.  The hierarchy is rebuilt on every call inside a static device
 * scratch array of 64 MiB that each GPU the library runs on holds until the
 * process ends, so the call allocates no device or pinned host memory (its
 * host-side tables live on the host heap during the call).  The workspace
 * smg_workspace_bytes reports for (g, o, nrhs) must fit in 64 MiB (e.g. an
 * FP64 cube of 94^3 with one right-hand side); a larger request returns
 * SMG_EWORKSPACE before any device work.  All calls on one GPU share its
 * array: calls on one stream are ordered, calls that overlap on one GPU from
 * different streams or unordered host threads race.  The call synchronises
 * `stream` once (after uploading the tables) and returns with the V-cycle
 * enqueued on it. */
int smg_apply_static(const smg_grid *g, const smg_opts *o, const double *r, double *s, int32_t nrhs, int64_t ld,
                     void *stream);

/* y = A x for nrhs vectors; x and y must not overlap. */
int smg_matvec(smg_handle *h, const double *x, double *y, int32_t nrhs, int64_t ld, void *stream);

/* Algorithm 1, Section 2.  b and x are single device vectors of nx*ny*nz
 * doubles; x holds x0 on entry (unless o->x0_zero) and the iterate on exit.
 * pcg_solve: beta from equation (1); fpcg_solve: equation (2), evaluated as
 * -alpha_{k-1} (s_k, A p_{k-1}) = (s_k, r_k - r_{k-1}); psd_solve: beta = 0.
 * Returns SMG_OK when converged, SMG_NOT_CONVERGED when max_iter was reached. */
int pcg_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream);
int fpcg_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream);
int psd_solve(smg_handle *h, const double *b, double *x, const krylov_opts *o, krylov_info *info, void *stream);

typedef struct lobpcg_opts {
    double rtol;            /* per-column ||A x - theta x||_2 / (|theta| ||x||_2) target */
    int32_t max_iter;       /* >= 0 */
    int32_t precond;        /* SMG_PRECOND_SMG or SMG_PRECOND_NONE */
    int32_t guard;          /* >= 0 extra block columns iterated but not required to
                               converge; they keep near-degenerate eigenvalues just
                               above the m-th from slowing the last wanted columns */
    int32_t reserved;
} lobpcg_opts;

typedef struct lobpcg_info {
    int32_t iters;          /* iterations (block updates) performed */
    int32_t nconv;          /* columns meeting rtol at exit */
    int32_t status;         /* same value as the return code */
    int32_t reserved;
    double seconds;         /* wall time, host clock */
} lobpcg_info;

/* Bytes of device workspace lobpcg_solve needs for block size mb (the wanted
 * m plus the guard columns): six N x 3mb blocks (basis S = [X W P], A S and
 * their scratch copies), three N x mb blocks and small Gram buffers.  Host-only. */
int lobpcg_workspace_bytes(smg_handle *h, int32_t mb, size_t *bytes);

/* LOBPCG (Section 4) for the m smallest eigenpairs of A, preconditioned by
 * the handle's SMG V-cycle (requires max_nrhs >= m + guard at setup) or
 * unpreconditioned.  The block holds mb = m + o->guard columns.
 * X: device, mb columns of nx*ny*nz doubles (ld = nx*ny*nz), the initial
 * block on entry (must have full column rank) and the orthonormal Ritz vectors
 * on exit.  lambda: host[mb], Ritz values ascending.  resnorms: host[mb],
 * nullable, final relative residuals.  ws: device workspace of ws_bytes bytes
 * (>= lobpcg_workspace_bytes(h, mb)).  Method: Rayleigh-Ritz on span{X, T R, P}
 * with Cholesky-QR orthonormalisation; converged columns stay in the basis
 * but stop generating directions.  Returns SMG_OK when the first m columns
 * meet rtol, SMG_NOT_CONVERGED at max_iter. */
int lobpcg_solve(smg_handle *h, int32_t m, double *X, double *lambda, double *resnorms, void *ws,
                 size_t ws_bytes, const lobpcg_opts *o, lobpcg_info *info, void *stream);

/* Batched flexible PCG over nbox independent bricks (each with its own handle,
 * grid and right-hand side), all advanced together: every stage of the
 * V-cycle and of the recurrence is one grouped launch over all boxes, the
 * stopping test (||r_k||/||b|| <= rtol or max_iter) runs on the device, and
 * one iteration is captured as a HIP graph and replayed (use_graph = 1).
 * Per box, the kernels, their arguments and their order are those of
 * fpcg_solve, so each box's result equals its single-box fpcg_solve bitwise.
 * Handles must be FP64 (SMG_PREC_F64), distinct, and not used elsewhere while
 * the batch exists.  b[i], x[i]: device vectors of box i (host arrays of nbox
 * device pointers, bound at creation).  ws: caller-owned device workspace of
 * ws_bytes >= smg_batch_workspace_bytes (launch tables).  The batch runs on a
 * private stream ordered after and before the caller's `stream`. */
typedef struct smg_batch smg_batch;
int smg_batch_workspace_bytes(smg_handle *const *hs, int32_t nbox, size_t *bytes);
int smg_batch_create(smg_handle *const *hs, int32_t nbox, const double *const *b, double *const *x, void *ws,
                     size_t ws_bytes, int32_t use_graph, void *stream, smg_batch **out);
/* One batched solve with options o (history and diagnostic pointers must be
 * NULL, precond SMG_PRECOND_SMG, stop_norm SMG_STOP_2NORM); infos: host, nbox
 * entries (rel_res_c is NaN).  Returns SMG_OK when every box
 * converged, else the most severe status among the boxes. */
int smg_batch_fpcg(smg_batch *bt, const krylov_opts *o, krylov_info *infos, void *stream);
/* Grouped launches per iteration (steps) and the per-box launches they
 * replace (the sum over boxes of each box's launches per iteration). */
int smg_batch_stats(const smg_batch *bt, int32_t *steps_per_iteration, int32_t *launches_per_iteration);
int smg_batch_destroy(smg_batch *bt);

/* Autotuner of the fused V-cycle schedule: times `reps` V-cycles s = T r for
 * each distinct schedule given by candidate LDS budgets (which 2D levels the
 * LDS-resident coarse kernel absorbs, and the strip heights of the wide-line
 * kernels), keeps the fastest in the handle and reports it in info
 * (nullable).  Every schedule computes the same V-cycle (up to rounding
 * order).  s is overwritten.  Synchronises the stream. */
typedef struct smg_tune_info {
    int32_t candidates;     /* schedules timed, including the default */
    int32_t l0;             /* first 2D level handled by the coarse kernel */
    int32_t s_down, s_up;   /* strip heights */
    int32_t march_waves;    /* lines up to 256 points: a pre-smoothing launch gives each wave a run of
                               2, 4 or 8 coarse lines while it keeps >= march_waves waves (0: never) */
    int32_t reserved;
    int64_t coarse_lds;     /* LDS bytes of the coarse kernel */
    double default_ms;      /* V-cycle time of the schedule before tuning */
    double best_ms;         /* V-cycle time of the chosen schedule */
} smg_tune_info;
int smg_autotune(smg_handle *h, const double *r, double *s, int32_t reps, void *stream, smg_tune_info *info);
/* The handle's current schedule (l0, s_down, s_up, march_waves, coarse_lds;
 * the timing fields are zero).  Host-only. */
int smg_get_schedule(const smg_handle *h, smg_tune_info *info);
/* Sets the marching threshold of the register-only pre-smoothing kernels
 * (march_waves >= 0; 0: one wave per coarse line everywhere).  Every value
 * computes the same V-cycle up to rounding.  Host-only; SMG_EINVAL for a
 * negative value. */
int smg_set_march(smg_handle *h, int32_t march_waves);

/* Measurement: the Gram product G = S^T S of LOBPCG's FP64 MFMA kernels for an
 * N x k block (k <= 3m) held in a workspace sized by lobpcg_workspace_bytes(h,
 * m) (the block is filled with a constant first).  Returns the mean time of
 * one product (partial products and the fixed-order reduction) over reps. */
int lobpcg_profile_gram(smg_handle *h, int32_t m, int32_t k, void *ws, size_t ws_bytes, int32_t reps, void *stream,
                        double *ms);

/* Variable coefficients.  SMG was designed for general structured-grid
 * operators (Section 1 cites Schaffer's semicoarsening multigrid); these
 * entry points build the same V-cycle for a symmetric 7-point operator given
 * per point (device arrays of nx*ny*nz doubles, index i + nx*(j + ny*k)):
 *     (A x)_p = diag[p] x_p - sum over axes e of (a_e[p] x_{p+e} + a_e[p-e] x_{p-e}),
 * a_e[p] being ignored where p+e is outside the brick (for a diffusion
 * operator, a_e is the coupling across the face between p and p+e and diag
 * the sum of the six face couplings).  The operator should be symmetric
 * positive definite.  Per 3D level the Galerkin operator P^T A P is stored per
 * point (15-point: 5 in-plane points on 3 planes), every plane has its own
 * 2D hierarchy (9-point) and every x-line its own LU factors.  Prolongation
 * weights of an even (F) plane from its two C-plane neighbours:
 * SMG_INTERP_LINEAR: 1/2 each; SMG_INTERP_OPERATOR: from the F-point's
 * collapsed couplings a (to the plane below) and b (above), a/(a+b) and
 * b/(a+b), following jumps of the coefficients across planes (1/2 each where
 * they are not both positive); the same rule in y inside planes.  With
 * constant coefficients both give the model problem's V-cycle.
 * The returned handle is used like smg_setup's with smg_apply, smg_matvec,
 * pcg_solve, fpcg_solve, psd_solve, lobpcg_solve and the Section 5
 * diagnostics; opts->precision must be SMG_PREC_F64 (kernel_mode is
 * ignored).  smg_autotune, smg_profile_kernel, smg_profile_levels, the
 * batched solver and the learned post-smoother reject such handles
 * (SMG_EINVAL).  The caller's
 * coefficient arrays are read during setup only. */
enum { SMG_INTERP_LINEAR = 0, SMG_INTERP_OPERATOR = 1 };
int smgv_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const smg_opts *o, int32_t interp, int32_t max_nrhs,
                         size_t *bytes);
int smgv_setup(int32_t nx, int32_t ny, int32_t nz, const double *diag, const double *ax, const double *ay,
               const double *az, int32_t interp, const smg_opts *o, int32_t max_nrhs, void *ws, size_t ws_bytes,
               void *stream, smg_handle **out);
/* Number of 3D levels and of 2D levels per plane of a variable handle. */
int smgv_levels(const smg_handle *h, int32_t *nlev3, int32_t *nlev2);
/* Copies the stored operator of 3D level `level` into the device buffer out:
 * with level2 = -1, eight arrays of nz_l*nx*ny doubles (the entries of the
 * in-plane block C_k: centre, to (i+1,j), to (i,j+1); of the coupling U_k
 * from plane k to plane k+1: to (i,j), (i+1,j), (i-1,j), (i,j+1), (i,j-1));
 * with level2 >= 0, the 2D level of every plane of that 3D level, five arrays
 * of nz_l*ny_l2*nx doubles (line block: centre, to i+1; coupling of line j to
 * line j+1: to i, i+1, i-1).  Matrix entries, not negated.  Synchronises. */
int smgv_export(smg_handle *h, int32_t level, int32_t level2, double *out, void *stream);

/* Section 5 diagnostics.  Assumption (4) of the convergence bound (3) for PSD
 * reads ||I - c A T||_{A^{-1}} <= delta < 1; with r = A e this is the operator
 * norm ||I - c T A||_A.  Power iteration on E# E, where E = I - c T A and
 * E# = I - c T^T A is its adjoint in the A inner product, gives Rayleigh
 * quotients that increase to delta(c)^2.
 *
 * smg_delta: delta(c) for the preconditioner of h after `iters` (>= 1) power
 * steps from the device vector v0 (nx*ny*nz doubles, nonzero).  ht must hold
 * T's transpose: the same grid and options with pre and post swapped (the
 * transposed V-cycle runs the adjoint sweeps in reverse order; with the
 * restriction P^T of the prolongation P the result is exact), or h itself
 * when pre = post.  work: device, 5*nx*ny*nz doubles.  Each step costs two
 * V-cycles and two stencil passes and synchronises the stream.
 * smg_delta_min: min over c in [c_lo, c_hi] of delta(c) (golden-section
 * search to relative width tol; delta(c) is convex in c), the best c in
 * *c_best: the scaling-free form of assumption (4).
 * smg_spectrum: for an SPD T (pre = post), the extreme eigenvalues of T A
 * (self-adjoint in the A inner product) by power iteration on T A and then on
 * lambda_max I - T A, `iters` steps each; work: 3*nx*ny*nz doubles.  With
 * Theorem 2's prescaling c = 2 / (lambda_min + lambda_max), delta(c) =
 * (kappa - 1) / (kappa + 1), kappa = lambda_max / lambda_min. */
int smg_delta(smg_handle *h, smg_handle *ht, double c, const double *v0, int32_t iters, double *work, double *delta,
              void *stream);
int smg_delta_min(smg_handle *h, smg_handle *ht, double c_lo, double c_hi, double tol, const double *v0,
                  int32_t iters, double *work, double *c_best, double *delta, void *stream);
int smg_spectrum(smg_handle *h, const double *v0, int32_t iters, double *work, double *lmin, double *lmax,
                 void *stream);

/* Releases the host-side handle (the caller's workspace is not freed). */
int smg_destroy(smg_handle *h);

/* Static message for a return code. */
const char *smg_strerror(int status);

/* Kernel families of one V-cycle, for smg_profile_kernel. */
enum {
    SMG_KERNEL_LINE_RELAX = 0,  /* zebra x-line relaxation, one colour of one 2D level */
    SMG_KERNEL_RESTRICT2 = 1,   /* 2D residual + restriction */
    SMG_KERNEL_PROLONG2 = 2,    /* 2D prolongation + correction */
    SMG_KERNEL_RESID3 = 3,      /* 3D residual of one plane colour */
    SMG_KERNEL_CORRECT3 = 4,    /* 3D correction x_k += y_k */
    SMG_KERNEL_RESTRICT3 = 5,   /* 3D residual + restriction */
    SMG_KERNEL_PROLONG3 = 6,    /* 3D prolongation + correction */
    SMG_KERNEL_DOWN2 = 7,       /* fused pre-smoothing + residual + restriction of a 2D level */
    SMG_KERNEL_COARSE2 = 8,     /* LDS-resident 2D sub-cycle on the small levels */
    SMG_KERNEL_CHAIN2 = 9,      /* 2D prolongation chain + 3D correction */
    SMG_KERNEL_UP2 = 10,        /* fused prolongation + post-smoothing of a 2D level */
    SMG_KERNEL_CHAIN3 = 11,     /* 3D prolongation chain */
    SMG_KERNEL_COUNT = 12
};

/* Measurement: runs `reps` single-vector V-cycles s = T r and times every
 * launch of kernel family `family` with dispatch-stamped HIP events on
 * `stream`.  Returns the launches per V-cycle, their summed duration in ms
 * per V-cycle, and their algorithmic bytes per V-cycle (every value a launch
 * must read or write, counted once).  s is overwritten. */
int smg_profile_kernel(smg_handle *h, int32_t family, const double *r, double *s, int32_t reps, void *stream,
                       int32_t *launches, double *kernel_ms, double *bytes);

/* Measurement: the same V-cycles with every launch of kernel family `family`
 * (every launch when family is -1) stamped, summed per 3D level of the
 * z-semicoarsening hierarchy (Section 3).  Row l (0 = finest)
 * holds the launches that work on level l: its zebra sweeps with their plane
 * solves and colour residuals, its restriction to level l + 1, and its
 * prolongation and post-smoothing when there are any; the last row (index
 * nlev3) holds the single prolongation chain of a V-cycle without
 * post-smoothing, which spans every level (empty otherwise).  On return
 * *nrows = nlev3 + 1 and launches[i], kernel_ms[i] (summed durations per
 * V-cycle) and bytes[i] (algorithmic bytes per V-cycle) are filled for each
 * row.  The arrays are caller-owned, of max_rows entries; SMG_EINVAL when
 * max_rows < nlev3 + 1, for a family outside -1 .. SMG_KERNEL_COUNT - 1, a
 * variable-coefficient handle or a null pointer.
 * s is overwritten. */
int smg_profile_levels(smg_handle *h, int32_t family, const double *r, double *s, int32_t reps, void *stream,
                       int32_t max_rows, int32_t *nrows, int32_t *launches, double *kernel_ms, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* SMG_H */
