/*
 * qp.h - C ABI of the MI355X (gfx950) projection-method solver.
 *
 * The library solves the lifted Fourier-Galerkin system of the projection
 * method (PM) for quasiperiodic elliptic problems
 *
 *     -div( a(x) grad u(x) ) = f(x),   x in R^d,   a(x) = A(P^T x),
 *     A(y) = sum_{m in S} Ahat_m exp(i m.y),   y in T^n,
 *
 * (Jiang, Li, Zhang, Zhang, "Projection method for quasiperiodic elliptic
 * equations and application to quasiperiodic homogenization", Sec. 2-4), and
 * the corrector problems and homogenized coefficient of Sec. 5.2.
 *
 * Discrete system (Sec. 3.1, eq. n-discrete and eq. linear_system):
 *     Q U = F,   Q_ij = Ahat_{k_V -_N k_U} (P k_V).(P k_U),
 * over the frequency grid K_N^n = {k in Z^n : -N/2 <= k_t < N/2}, D = N^n.
 *
 * Conventions shared by every entry point
 *   - Complex vectors have D entries stored as interleaved (re, im) pairs
 *     (double: 16 bytes per entry, float: 8 bytes), in the tensor-to-vector
 *     order C of Sec. 3.1.2: entry i holds k with
 *         i = sum_t (k_t mod N) * N^(n-1-t),  k_1 slowest (FFT order per axis).
 *   - The zero frequency is not an unknown (zero-mean trial and test space,
 *     Sec. 3.1.1): solutions have U[C(0)] = 0 and rhs[C(0)] is ignored.
 *   - "_d" entry points take device pointers (hipMalloc'ed or torch CUDA
 *     tensors on the problem's device); the others take host pointers.
 *     Every pointer is owned by the caller and must stay valid for the call.
 *   - Calls are synchronous with respect to the host: on return, outputs are
 *     written (the work is queued on the problem's stream and waited for).
 *   - Errors: every function returns a qp_status; QP_OK is 0 and errors are
 *     negative.  qp_last_error() returns a message for the calling thread.
 *     A failed call leaves the problem usable unless it returned QP_EDEVICE.
 *   - Calls on the same qp_problem must not overlap (one stream, one
 *     workspace); distinct problems are independent.
 */
#ifndef QP_H
#define QP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qp_problem qp_problem;

typedef enum qp_status {
    QP_OK = 0,
    QP_EINVAL = -1,        /* invalid argument (see qp_create)                    */
    QP_ENOTELLIPTIC = -2,  /* coefficient negative on the collocation grid        */
    QP_ENOTSPD = -3,       /* PCG breakdown: (Q h, h) <= 0                         */
    QP_ENOCONV = -4,       /* iteration limit reached; best iterate is returned    */
    QP_ENOMEM = -5,        /* device allocation failed or workspace too small      */
    QP_EDEVICE = -6,       /* HIP runtime error or no usable gfx950 device         */
    QP_ENONFINITE = -7     /* NaN or Inf in an input or in the residual            */
} qp_status;

/* Compile-time limits of the library. */
#define QP_MAX_DIM_N 8     /* parent dimension n  */
#define QP_MAX_DIM_D 4     /* physical dimension d */
#define QP_MAX_MODES 64    /* coefficient modes g  */

enum { QP_PREC_FP64 = 0, QP_PREC_FP32_IR = 1 };
enum { QP_PRECOND_PAPER = 0, QP_PRECOND_JACOBI = 1 };

/* qp_solve_info.flags bits */
enum {
    QP_FLAG_DEGENERATE = 1,  /* min of A on the grid is 0 (within 1e-12 max|A|)  */
    QP_FLAG_F0_IGNORED = 2,  /* |rhs[C(0)]| > 1e-14 ||rhs||; it was ignored       */
    QP_FLAG_INDEFINITE = 4   /* A is negative on the grid (allow_indefinite)    */
};

typedef struct qp_options {
    int precision;      /* QP_PREC_FP64 (default) or QP_PREC_FP32_IR: float
                           vectors, stiffness product and preconditioner inside
                           FP64 refinement (the float residual is replaced by
                           the FP64 residual of the FP64 solution); scalars,
                           dot products, residuals and A* stay FP64              */
    int precond;        /* QP_PRECOND_PAPER (default): M of eq. precond;
                           QP_PRECOND_JACOBI: 1 / q_kk                            */
    int maxit;          /* PCG iteration limit; default 10000                     */
    double inner_tol;   /* FP32-IR: replace the float residual once it has
                           dropped by this factor since the last replacement;
                           default 1e-5 (float rounding limits it to about
                           1e-6: below that the recursion drifts and restarts) */
    int poll_every;     /* iterations queued between convergence polls (FP32-IR:
                           each batch ends with the replacement steps, which act
                           on the right-hand sides that reached inner_tol);
                           0 = 12, rounded up to an even count, at most 64      */
    int profile;        /* nonzero: time every stiffness-product launch with a
                           HIP event pair that the launch itself records (kernel
                           start and end); totals reported in qp_solve_info.
                           Batches are then launched directly (no graph replay) */
    void *stream;       /* hipStream_t to run on; NULL = a stream the library
                           creates and owns                                      */
    void *workspace;    /* optional device buffer of qp_workspace_bytes() bytes;
                           NULL = the library allocates its own                  */
    size_t workspace_bytes;
    int graphs;         /* nonzero (default): each full batch of poll_every
                           iterations is captured once as a HIP graph and
                           replayed; 0 = launch every kernel directly            */
    int gather64;       /* nonzero: the stiffness product forms 64-bit neighbour
                           addresses and serves one right-hand side per launch.
                           Always on when N^n * max(2, d) * 8 >= 2^32 (a family
                           of vectors of 4 GiB or more, beyond the 32-bit
                           record offsets of the default gathers); default 0  */
    int autotune;       /* nonzero: qp_create times the candidate work layouts
                           of the plane-tile stiffness product (tiles per wave
                           item, workgroups, item order) on this problem and
                           keeps the fastest (qp_product_layout reports it).
                           The choice is kept per problem shape and precision
                           for the life of the process and reused.  Output
                           values of the product do not depend on the layout;
                           which workgroup sums which partial dot product does,
                           so iterates can differ from an untuned problem's in
                           the last bits.  Default 0 (fixed heuristics)      */
    int allow_indefinite; /* nonzero: qp_create accepts a coefficient that is
                           negative on the collocation grid (flag
                           QP_FLAG_INDEFINITE) instead of failing with
                           QP_ENOTELLIPTIC.  Q is then indefinite and a solve
                           may stop with QP_ENOTSPD ((Q h, h) <= 0, Alg. 2
                           breakdown; u holds the last iterate); default 0  */
    int half_storage;   /* nonzero: Hermitian half storage (Sec. 2.3: the
                           coefficients of a real function satisfy
                           u_{-k} = conj(u_k), and with a real coefficient Q
                           keeps that symmetry).  Odd N, a real scalar
                           coefficient and n >= 2, N <= 32 (QP_EINVAL
                           otherwise).  Every vector of the problem's calls
                           (right-hand sides, solutions, correctors, products,
                           preconditioner, multi-indices) then holds the
                           (N^n + 1)/2 stored entries in the half layout of
                           qp_matvec_half_d, qp_dim returns that count, and
                           the solves move about half the bytes.  A
                           right-hand side must be the half of a Hermitian
                           vector (e.g. the coefficients of a real source).
                           The stored-matrix calls are not available, the
                           problem cannot join grouped calls, and a server
                           rejects the option.  Fixed at creation; default 0 */
    int small_dim;      /* FP64 solves of problems with at most this many
                           unknowns (and at most 2048; scalar coefficient,
                           full storage) run the whole PCG loop in one launch,
                           one workgroup per right-hand side holding its
                           vectors in registers and LDS, instead of three
                           launches per iteration: the same recurrences and
                           state (status, iterations, condition estimate),
                           with the sums formed in the workgroup's order.  Not
                           with the profile option (which times every product
                           launch).  0 = never; default 2048 (above about
                           that size the three-launch loop, spread over the
                           whole device, is faster)                         */
} qp_options;

typedef struct qp_solve_info {
    int status;           /* qp_status of the solve                              */
    int iters;            /* PCG iterations (float iterations for FP32-IR)       */
    int outer_iters;      /* FP32-IR: FP64 residual replacements (0 for FP64)    */
    int flags;            /* QP_FLAG_* bits                                      */
    double rel_resid;     /* final ||r||_2 / ||F'||_2: the PCG residual for FP64,
                             the true FP64 residual F' - Q U for FP32-IR         */
    double seconds;       /* time of the solve on the device stream              */
    int matvec_launches;  /* profile only: FP64 stiffness products that ran      */
    double matvec_ms;     /*   and their summed event-timed duration             */
    int matvec32_launches;/* profile only: float stiffness products that ran     */
    double matvec32_ms;
    int matvec_rhs;       /* profile only: right-hand sides those FP64 launches
                             served (a launch serves every unfinished one)       */
    int matvec32_rhs;     /* the same for the float launches                     */
    double kappa_est;     /* condition estimate of the preconditioned operator
                             M^(1/2) Q M^(1/2): the ratio of the extreme
                             eigenvalues of the Lanczos tridiagonal matrix that
                             the PCG coefficients define (diagonal 1/alpha_j +
                             beta_(j-1)/alpha_(j-1), off-diagonal
                             sqrt(beta_j)/alpha_j; the first 1024 iterations;
                             FP32-IR: the float iterations, each run between
                             two residual replacements a separate Lanczos
                             segment).  In FP64 it approaches the true ratio
                             from below as the iterations grow (Sec. 4.3
                             discusses cond(QM)); float rounding perturbs the
                             FP32-IR recurrence, whose estimate can exceed the
                             FP64 one for ill-conditioned operators (14% at a
                             ratio of 1e4).  0 when no iteration ran           */
    double bytes_moved;   /* algorithmic device bytes of the solve's kernels for
                             this right-hand side: each vector a kernel touches
                             read or written once (16 B per FP64 complex entry,
                             8 B float; 8 / 4 B per preconditioner entry), from
                             the iteration and replacement counts; cache and
                             refetch traffic are not counted                   */
} qp_solve_info;

/* Work layout of the stiffness product (see qp_options.autotune): one for
 * the float launches and one for the FP64 launches. */
typedef struct qp_layout {
    int item_tiles;     /* float launches: plane tiles per wave work item
                           (line tiles: 1)                                     */
    int workgroups;     /* float launches: grid of the product                 */
    int xcd_front;      /* 1: each of the 8 XCDs sweeps a contiguous share of
                           the work items; 2: the same, with the slowest axis
                           varying fastest inside each share (when the shares
                           are whole values of it, n >= 3; else as 1); 3: the
                           same shares swept in blocks of the axes after the
                           second one, each block through every value of the
                           second axis (n >= 5; else as 2);
                           0: items in plain order                             */
    int tuned;          /* 0: fixed heuristics; 1: timed on this problem;
                           2: reused from an earlier problem of the same shape */
    int candidates;     /* layouts timed (tuned == 1)                          */
    double default_us;  /* float product (FP32-IR problems): mean launch of the
                           heuristic layout (tuned == 1)                       */
    double best_us;     /* ... and of the chosen layout                        */
    int item_tiles64;   /* the same three for the FP64 launches (FP64 solves,  */
    int workgroups64;   /* the residual replacements of FP32-IR, qp_matvec_d); */
    int xcd_front64;    /* workgroups64 = 0 in qp_set_product_layout: as float */
    double default64_us;/* FP64 product (the residual product for FP32-IR):    */
    double best64_us;   /* mean launch of the heuristic and the chosen layout  */
} qp_layout;

/* Fill *opt with the defaults listed above. */
void qp_default_options(qp_options *opt);

/* Device bytes a problem of this shape needs when the caller supplies the
 * workspace (qp_options.workspace).  Host-only; no device call. */
size_t qp_workspace_bytes(int d, int n, int N, int g);

/*
 * Create a problem (Sec. 3.1: P, the coefficient modes and N define Q).
 *   d, n    physical and parent dimensions, 1 <= d <= n, d <= QP_MAX_DIM_D,
 *           n <= QP_MAX_DIM_N
 *   P       d x n projection matrix, row-major, host (Def. 2.1)
 *   g       number of coefficient modes, 1 <= g <= QP_MAX_MODES
 *   modes   g x n int32 modes m, host; every |m_t| < N/2 (no aliasing)
 *   coef    g complex Ahat_m as (re, im) pairs, host
 *   N       points per parent dimension (N >= 2, N^n < 2^31)
 *   opt     options or NULL for the defaults
 * Returns QP_EINVAL for: a size outside the limits, non-finite P or coef,
 * a repeated mode, |m_t| >= N/2, a missing or non-positive Ahat_0, a field
 * that is not real (Ahat_{-m} != conj(Ahat_m) beyond 1e-14 max|Ahat|), or P
 * with P k = 0 for some nonzero k in K_N^n (|P k| < 1e-12 |P|).
 * QP_ENOTELLIPTIC if min over the collocation grid of A is below
 * -1e-12 max|A|.  On success *out owns device memory until qp_destroy.
 * Argument checks run on the host before any device call.
 */
qp_status qp_create(qp_problem **out, int d, int n, const double *P, int g,
                    const int32_t *modes, const double *coef, int N,
                    const qp_options *opt);

/*
 * Create a problem with a diagonal coefficient A = diag(a_1, ..., a_d)
 * (App. D): every a_l is a real quasiperiodic function with the same P, and
 *   Q = sum_l A^l o W^l,  A^l_{k_V k_U} = Ahat of a_l at k_V -_N k_U,
 *   W^l_{k_V k_U} = (P k_V)_l (P k_U)_l.
 * The d entries share one mode list:
 *   modes   g x n int32, host, as for qp_create (the union of the entries'
 *           modes; a mode absent from a_l has coefficient 0 there)
 *   coefs   d x g complex (re, im) pairs, host: a_l's Ahat at mode r is
 *           element l * g + r
 * Every other argument, and every later call, is as for a problem from
 * qp_create; the corrector source of axis j is d a_j / d x_j
 * (F_k = i (P k)_j Ahat of a_j at k) and A*_ij = mean{a_i (delta_ij +
 * d_{x_i} chi_j)} (App. D, eqs. homcoefficient11-22).  Each a_l must pass
 * qp_create's checks (real field, positive Ahat_0); QP_ENOTELLIPTIC if the
 * minimum over the collocation grid of any a_l is below -1e-12 max|a|.
 * QP_EINVAL for a null coefs.
 */
qp_status qp_create_diag(qp_problem **out, int d, int n, const double *P, int g,
                         const int32_t *modes, const double *coefs, int N,
                         const qp_options *opt);

/* Release the problem and everything it owns.  NULL is ignored. */
void qp_destroy(qp_problem *p);

/* Entries of the problem's vectors: D = N^n, or (N^n + 1)/2 with half
 * storage. */
int64_t qp_dim(const qp_problem *p);

/* Replace the solver options (precision, preconditioner, limits, profile).
 * The stream, workspace and half_storage of a created problem cannot change
 * (the values passed for them are ignored).  A change of
 * precision waits for the problem's stream and re-derives the grid of the
 * vector kernels (chosen per precision). */
qp_status qp_set_options(qp_problem *p, const qp_options *opt);

/* The stiffness product's work layout of p (host-only; no device call).
 * QP_EINVAL for null arguments. */
qp_status qp_product_layout(const qp_problem *p, qp_layout *out);

/* Set the stiffness product's work layouts (item_tiles, workgroups and
 * xcd_front of *layout for the float launches; item_tiles64, workgroups64
 * and xcd_front64 for the FP64 launches, or the float ones when workgroups64
 * is 0; the other fields are ignored), e.g. ones that
 * qp_product_layout reported in an earlier process, so that the partial sums,
 * and with them the iterates, repeat bitwise.  Waits for the problem's stream
 * and drops its captured batches.  QP_EINVAL unless item_tiles is 1, 2 or 4
 * (1 for line tiles, N > 32 or n = 1), 1 <= workgroups <= 1024 and xcd_front
 * is 0, 1, 2 or 3. */
qp_status qp_set_product_layout(qp_problem *p, const qp_layout *layout);

/*
 * Solve Q U = F' by C-PCG (Alg. 2) with the diagonal preconditioner M of
 * eq. precond applied as z = M r, from U_0 = 0, until
 * ||F' - Q U||_2 <= tol ||F'||_2 (F' = rhs without its zero frequency).
 * rhs, u: D complex each (host for qp_solve, device for qp_solve_d); they
 * must not overlap.  info may be NULL.  On QP_ENOCONV u holds the last
 * iterate.  QP_ENONFINITE if rhs holds NaN/Inf.
 */
qp_status qp_solve(qp_problem *p, const double *rhs, double *u, double tol,
                   qp_solve_info *info);
qp_status qp_solve_d(qp_problem *p, const double *rhs, double *u, double tol,
                     qp_solve_info *info);

/*
 * K independent solves with the same operator (1 <= K <= d), run together:
 * one stiffness-product launch serves every right-hand side that has not
 * converged, so each (entry, mode) weight is computed once for all of them.
 * rhs, u: device, K consecutive vectors of D complex (vector r at element
 * r * D); they must not overlap.  infos: host array of K entries, or NULL.
 * Each right-hand side stops at its own tolerance; the iterates are the same
 * as those of K separate qp_solve_d calls.  Returns the first non-QP_OK status.
 */
qp_status qp_solve_multi_d(qp_problem *p, int K, const double *rhs, double *u, double tol,
                           qp_solve_info *infos);

/*
 * Corrector chi_j, 0 <= j < d, of the corrector equation
 * -div(a(e_j + grad chi_j)) = 0 (Sec. 5.2, eq. corrector), i.e. the solve
 * with F_k = i (P k)_j Ahat_k (the coefficients of d a / d x_j, App. D).
 * chi: D complex (host / device), or NULL.  The result is also kept in the
 * problem's corrector slot j until the next qp_corrector* call with that j.
 */
qp_status qp_corrector(qp_problem *p, int j, double *chi, double tol,
                       qp_solve_info *info);
qp_status qp_corrector_d(qp_problem *p, int j, double *chi, double tol,
                         qp_solve_info *info);

/*
 * Homogenized coefficient A* (Sec. 5.2, eq. homcoefficient; App. D):
 *     A*_ij = mean{ e_i . a (e_j + grad chi_j) }
 * solving the d correctors to `tol` first.  With the discrete mean over the
 * collocation grid this is Ahat_0 delta_ij + sum_m Ahat_m i(P(-m))_i chi_j[-m].
 * Astar: host d*d row-major (flux form above).  Astar_energy (host d*d, may be
 * NULL): the symmetric energy form Ahat_0 delta_ij - chi_i^H Q chi_j.
 * info: host array of d entries (one per corrector), may be NULL.  The d
 * correctors are solved together (as by qp_solve_multi_d).
 */
qp_status qp_homogenized(qp_problem *p, double *Astar, double tol,
                         qp_solve_info *info);
qp_status qp_homogenized_ex(qp_problem *p, double *Astar, double *Astar_energy,
                            double tol, qp_solve_info *info);

/*
 * Homogenize several problems together (a batch of coefficient instances):
 * each problem's result is the one qp_homogenized computes (same launches,
 * same values), and the host keeps every problem's batches of iterations
 * queued on that problem's stream, advancing whichever has a poll ready, so
 * the device runs the problems' kernels concurrently.
 *   problems  count distinct problems (count >= 1).  Their solves overlap
 *             only if they run on different streams (qp_options.stream NULL
 *             at creation gives each its own).
 *   Astar     host, sum over i of d_i^2 doubles: problem i's d_i x d_i
 *             coefficient (flux form, row-major) follows those of problems
 *             0 .. i-1
 *   infos     host, sum of d_i entries in the same order, or NULL
 * Blocks until every problem has finished.  Returns QP_EINVAL for a null or
 * repeated problem; otherwise the first non-QP_OK status in problem order
 * (every problem is still run to its end).
 */
qp_status qp_homogenized_batch(qp_problem *const *problems, int count, double *Astar, double tol,
                               qp_solve_info *infos);

/*
 * Homogenize several FP32-IR problems with one launch per solver step for
 * the whole group: each launch of the float product, update, direction and
 * of the residual replacement covers the workgroups of every problem, each
 * workgroup computing what it computes in that problem's own launch, so
 * every A* equals qp_homogenized's on the problem alone.  The replacement
 * steps follow every second iteration; the host polls every poll_every
 * iterations (problem 0's options).
 *   problems  count distinct problems created with precision
 *             QP_PREC_FP32_IR, the same d (2 or 3), a scalar coefficient
 *             (all real or all complex), plane tiles (N <= 32, n >= 2) with
 *             the default 32-bit gathers, on one device, with equal maxit;
 *             N, n, P, modes and g may differ
 *   Astar, infos  as for qp_homogenized_batch
 * Runs on problem 0's stream after waiting for every problem's stream.
 * Calls from several host threads are serialized (the group tables are
 * shared: up to count * (160 + 4 * workgroups) bytes of device memory and
 * 3 * count * d states of pinned memory, allocated on first use and kept).
 * Returns QP_EINVAL (naming the problem and the reason) when a problem
 * cannot join; otherwise the first non-QP_OK corrector status.
 */
qp_status qp_homogenized_grouped(qp_problem *const *problems, int count, double *Astar, double tol,
                                 qp_solve_info *infos);

/*
 * qp_homogenized_grouped for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launches and results (every A*, iteration count and status equals
 * qp_homogenized_grouped's on the same problems), with the group table, the
 * owner arrays and the poll words in a static device array of 4 MiB that the
 * library holds on each device until the process ends, instead of memory
 * allocated on first use.  The call makes no device, pinned or host heap
 * allocation: it polls one done bit per problem into problem 0's pinned
 * words and reads the final states into each problem's own pinned slot,
 * all made by qp_create.
 *   problems, count, Astar, tol, infos   as for qp_homogenized_grouped;
 *             count <= 4096.
 * Returns QP_EINVAL, naming the sizes, when the group table (about 170 bytes
 * per problem plus 4 bytes per workgroup of its float product, FP64 product
 * and vector launches) exceeds the array, and otherwise as
 * qp_homogenized_grouped.  The array keeps the last call's contents (every
 * call writes what it reads).  Calls from several host threads of one
 * process are serialized with qp_homogenized_grouped's; calls that overlap
 * on one device through another route (e.g. a second copy of the library
 * loaded into the process) would share the array and race.
 */
qp_status qp_homogenized_grouped_noalloc(qp_problem *const *problems, int count, double *Astar,
                                         double tol, qp_solve_info *infos);

/*
 * A batch with its small problems grouped: the problems with at most
 * group_max_dim unknowns (qp_dim) that can join a group with the first of
 * them (the conditions of qp_homogenized_grouped) run as one group, with one
 * launch per solver step on that first problem's stream, while every other
 * problem runs on its own stream as in qp_homogenized_batch; the host
 * advances the group and the other problems together.  Small problems are
 * bound by launch latency, which the group shares out, and large ones by
 * memory traffic, which per-problem streams keep cache-resident.  Every A*,
 * iteration count and status equals qp_homogenized's on the problem alone.
 *   problems, count, Astar, tol, infos   as for qp_homogenized_batch
 *   group_max_dim  the size limit of the group's members; with 0, or with
 *             fewer than two problems that qualify, no group is formed and
 *             the call is qp_homogenized_batch
 * Allocates as qp_homogenized_grouped does (shared group tables; calls from
 * several host threads are serialized while a group runs).  Returns
 * QP_EINVAL for a null or repeated problem or a negative group_max_dim;
 * otherwise the first non-QP_OK status in problem order.
 */
qp_status qp_homogenized_batch_mixed(qp_problem *const *problems, int count, double *Astar,
                                     double tol, qp_solve_info *infos, int64_t group_max_dim);

/* ---- serving: a request queue over a cache of problems ---- */

/*
 * A server runs homogenization requests as they arrive.  It creates the
 * problems the requests describe and keeps them (workspace, tables,
 * preconditioner) in a cache whose device bytes (qp_workspace_bytes of each)
 * stay within hbm_budget.  Requests are admitted in arrival order: when
 * their problem is cached and idle, or when it can be created within the
 * budget after evicting idle problems (least recently used first); a
 * request whose problem does not fit yet stops the creation of problems for
 * the requests behind it.  Every admitted request runs on its problem's own
 * stream; requests join and leave while the others keep iterating, and each
 * result equals that of qp_homogenized on the same problem alone.
 * opt: the problems' options (precision, preconditioner, limits; stream and
 * workspace are ignored: every problem gets its own), NULL for the defaults.
 * A server is used from one host thread at a time.
 */
typedef struct qp_server qp_server;
qp_status qp_server_create(qp_server **out, size_t hbm_budget, const qp_options *opt);

/*
 * Queue a homogenization (as qp_homogenized) of the problem (d, n, P, g,
 * modes, coefficient, N): coef as for qp_create, or coefs as for
 * qp_create_diag (exactly one of the two is used: coefs when not NULL).
 * The arrays are copied.  Astar (host, d*d) and infos (host, d entries, or
 * NULL) receive the result and must stay valid until the request's ticket
 * is returned by qp_server_progress.  *ticket: a positive request id.
 * Returns QP_EINVAL for invalid arguments (the checks of qp_create that need
 * no device) and QP_ENOMEM when the problem alone exceeds the budget;
 * device-side checks (ellipticity, dependent P) surface as the request's
 * status.
 */
qp_status qp_server_submit(qp_server *s, int d, int n, const double *P, int g,
                           const int32_t *modes, const double *coef, const double *coefs, int N,
                           double tol, double *Astar, qp_solve_info *infos, int64_t *ticket);

/*
 * Admit what fits and advance every running request, for at most wait_us
 * microseconds or until some request has finished (or nothing is left).
 * The finished tickets (up to max_done) go to done[] with their statuses in
 * done_status[] (may be NULL); *ndone is their count.  Tickets not returned
 * yet are returned by a later call.
 */
qp_status qp_server_progress(qp_server *s, int wait_us, int64_t *done, qp_status *done_status,
                             int max_done, int *ndone);

/* Requests queued, running, or finished but not yet returned. */
int qp_server_pending(const qp_server *s);

/* Device bytes held by the cached problems. */
size_t qp_server_bytes(const qp_server *s);

/* Finish the running requests, release every cached problem and the server. */
void qp_server_destroy(qp_server *s);

/* ---- sampled inputs: discrete Fourier-Bohr coefficients (Sec. 2.3) ---- */

/*
 * n-dimensional DFT on the collocation grid T_N^n, in the storage order of
 * Sec. 3.1.2 (which is also the sample order of y_j = 2 pi j / N, first
 * axis slowest):
 *   forward (inverse = 0):  out_k = (1/D) sum_j in_j exp(-i k.y_j)
 *                           (the discrete coefficients of sampled values),
 *   inverse (inverse != 0): out_j = sum_k in_k exp(i k.y_j)  (the samples).
 * in, out: device, D = N^n complex (re, im) doubles; out may equal in.
 * 1 <= n <= QP_MAX_DIM_N, 1 <= N <= 1024, N^n < 2^31.  stream: hipStream_t
 * or NULL (the null stream); returns after the transform has finished.
 * A forward transform of sampled right-hand-side values gives the F of
 * qp_solve_d.
 */
qp_status qp_dft_d(int n, int N, const double *in, double *out, int inverse, void *stream);

/*
 * The coefficient modes of a sampled real coefficient: from its spectrum
 * (host, D complex, e.g. qp_dft_d of the samples copied back), keep every k
 * with |spec_k| or |spec_{-k}| above rel_tol * max|spec| (and k = 0), so
 * that modes come in +-pairs, and store Hermitian-symmetrized coefficients
 * (spec_k + conj(spec_{-k})) / 2.  modes (host, max_modes * n int32, signed
 * in K_N) and coef (host, max_modes complex) receive *g entries in storage
 * order, ready for qp_create.  QP_EINVAL when more than max_modes modes
 * qualify, when a retained mode has a component N/2 (it would alias), or for
 * a zero or non-finite spectrum.  Host only.
 */
qp_status qp_modes_from_spectrum(int n, int N, const double *spec, double rel_tol, int max_modes,
                                 int32_t *modes, double *coef, int *g);

/* ---- the compressed stiffness matrix of Alg. 1 (comparison path) ---- */

/*
 * The paper stores Q = A o W as triples (i, j, Q_ij) (Alg. 1 and the
 * compressed matrix-vector product of Sec. 4.2).  This build keeps them as a
 * comparison for the matrix-free product: D * g entries ordered mode-major
 * (row i's entry for the r-th coefficient mode, in the problem's mode order,
 * is element r*D + i; an entry whose value is zero keeps its slot), values
 * computed in FP64 from the integer indices.  The arrays are the caller's
 * device buffers (rows, cols: int32; vals: complex (re, im) doubles), each of
 * qp_coo_entries(p) elements; nothing is allocated.
 */
int64_t qp_coo_entries(const qp_problem *p);
qp_status qp_coo_build_d(qp_problem *p, int32_t *rows, int32_t *cols, double *vals);
/* y = Q u from the triples of qp_coo_build_d (FP64; u, y: D complex, device,
 * not overlapping: QP_EINVAL). */
qp_status qp_coo_matvec_d(qp_problem *p, const int32_t *cols, const double *vals, const double *u,
                          double *y);

/* ---- single steps of the path, device pointers (used by parity tests) ---- */

/* y = Q u in FP64 (eq. linear_system; y[C(0)] = 0, u[C(0)] ignored).  u and
 * y must not overlap (QP_EINVAL): every output reads the neighbours of u. */
qp_status qp_matvec_d(qp_problem *p, const double *u, double *y);
/* y = Q u in FP64 on Hermitian half storage (Sec. 2.3: the coefficients of a
 * real function satisfy u_{-k} = conj(u_k); the coefficient is real, so Q
 * keeps that symmetry).  Odd N and a scalar coefficient only (QP_EINVAL
 * otherwise).  u, y: device, (D+1)/2 complex doubles each.  Layout: position 0
 * holds k = 0 (ignored on input, 0 on output); then, for t = n, n-1, ..., 1,
 * the entries of C(k) order with zero digits on axes 1..t-1 and digit
 * a_t in [1, (N-1)/2], i.e. the index range [S_t, (N+1)/2 S_t) with
 * S_t = N^(n-t), index i at position i - (S_t - 1)/2.  Those are the k != 0
 * whose first nonzero component is positive; k's partner -k is implied.
 * Its algorithmic bytes (u read once, y written once) are half those of
 * qp_matvec_d.  On a problem created with the half_storage option this is
 * qp_matvec_d (the plane-tile product on the stored half, about 0.6x the
 * full product's time); on a full-storage problem it runs a plain kernel,
 * one thread per stored entry, which re-reads its neighbours from memory
 * and takes longer than the full product (for speed create the problem
 * with half_storage).  u and y must not overlap (QP_EINVAL); synchronous. */
qp_status qp_matvec_half_d(qp_problem *p, const double *u, double *y);
/* y = Q u with float data and arithmetic (the FP32-IR inner product); u and
 * y (D float complex each) must not overlap (QP_EINVAL). */
qp_status qp_matvec32_d(qp_problem *p, const float *u, float *y);
/* Kernel time of the last qp_matvec_d or qp_matvec32_d call on p, in ms:
 * with the profile option on, those calls launch their kernel with a HIP
 * event pair that the launch itself records (so the time excludes the
 * dispatch gap in front of the kernel); *ms = -1 when the last call was not
 * timed.  QP_EINVAL for a null argument. */
qp_status qp_last_product_ms(const qp_problem *p, double *ms);
/* The diagonal preconditioner (eq. precond; kind per the options), D doubles. */
qp_status qp_precond_d(qp_problem *p, double *M);
/* Corrector right-hand side F_k = i (P k)_j Ahat_k, D complex doubles. */
qp_status qp_corrector_rhs_d(qp_problem *p, int j, double *F);
/* Signed multi-index k = C^{-1}(i) of every entry: D x n int32 (Sec. 3.1.2). */
qp_status qp_multi_index_d(qp_problem *p, int32_t *k);
/* A* flux form from d correctors stored back to back (d*D complex, device);
 * Astar: host d*d row-major. */
qp_status qp_astar_d(qp_problem *p, const double *chi, double *Astar);
/* Minimum and maximum of A over the collocation grid T_N^n (host outputs). */
qp_status qp_coef_extrema(qp_problem *p, double *amin, double *amax);

/* Wait for all work queued on the problem's stream. */
qp_status qp_synchronize(qp_problem *p);

/* Static description of a status code. */
const char *qp_strerror(qp_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char *qp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QP_H */
