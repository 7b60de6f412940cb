/*
 * hkgeneo.h -- C ABI of the MI355X two-level overlapping Schwarz preconditioner with the
 * H_k-GenEO coarse space, and of the flexible GMRES solver built on it.
 *
 * Problem (paper Sec. 1, eq. (1.1); Sec. 2.1, eqs. (2.11)-(2.12)):
 *     -div(A grad u) - k^2 u = f in Omega,  u = 0 on the boundary,
 * discretised by conforming P1 / Q1 finite elements: B = A - k^2 S with A the stiffness and S
 * the consistent mass matrix.  The preconditioner (eq. (2.23)) is
 *     M^{-1} = Z B_0^{-1} Z^T + sum_D E_D W_D B_D^{-1} R_D,     B_D = R_D B E_D,  B_0 = Z^T B Z,
 * where the subdomains D are the blocks of an element partition extended by element layers
 * (Def. 2.8), R_D restricts to the internal dofs of D (Def. 2.12), W_D is the identity
 * (additive Schwarz, eq. (2.22)) or the partition-of-unity weights 1/mu (Def. 2.13), and the
 * columns of Z are E_i Xi_i p_l for the eigenvectors p_l of the local indefinite generalised
 * eigenproblem b_{D_i}(p, v) = lambda (Xi_i p, Xi_i v)_{1,k,D_i} (Def. 2.14) with the smallest
 * eigenvalues, chosen as in Def. 2.15.
 *
 * Conventions
 *   - All entry points return an int32 status: 0 = HKG_OK, < 0 an error, > 0 a warning.
 *   - Arrays passed to hkgeneo_setup are HOST arrays; they are copied and not retained.
 *   - Vectors passed to hkgeneo_apply / hkgeneo_gmres_solve are DEVICE arrays (HIP device
 *     pointers on the current device) of float64, column-major n_dof x nrhs with leading
 *     dimension ld >= n_dof, owned by the caller.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - A context is not thread safe: calls on one context must not overlap.
 *   - Dense device matrices are column-major.
 */
#ifndef HKGENEO_H
#define HKGENEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HKG_OK 0
#define HKG_EINVAL (-1)            /* bad sizes or ids; overlap leaving a dof with mu = 0; k < 0     */
#define HKG_ENOMEM (-2)            /* device allocation failed                                       */
#define HKG_EHIP (-3)              /* HIP runtime error (also surfaces errors of earlier async calls) */
#define HKG_ESINGULAR_LOCAL (-4)   /* zero pivot in a local Dirichlet matrix B_D (subdomain named by
                                      hkgeneo_last_error)                                            */
#define HKG_EEIG (-5)              /* local eigenproblem failed: B~_GG singular, C_II not SPD, or more
                                      eigenvectors needed than max_eig_per_sub (hkgeneo_last_error)  */
#define HKG_ESINGULAR_COARSE (-6)  /* zero pivot in the coarse matrix B_0                             */
#define HKG_ENOTCONV 1             /* solve returned without reaching rtol; see hkgeneo_rhs_info      */

/* element types */
#define HKG_P1 1                   /* linear simplices (triangles in 2D)       */
#define HKG_Q1 2                   /* bilinear / trilinear tensor-product cells */

/* eigenvector selection (Def. 2.15) */
#define HKG_EIG_THRESHOLD 0        /* keep lambda < tau                                             */
#define HKG_EIG_FIXED 1            /* keep nev per subdomain                                        */

/* local prolongation weights */
#define HKG_PROLONG_AS 0           /* W_D = I, additive Schwarz of eq. (2.22)                       */
#define HKG_PROLONG_POU 1          /* W_D = diag(1/mu) on dof(D) (Def. 2.13)                        */
#define HKG_COARSE_HK 0            /* H_k-GenEO coarse space (Def. 2.14, 2.15)                      */
#define HKG_COARSE_DELTA 1         /* Delta-GenEO: the same on the nearby SPD problem (k = 0)       */
#define HKG_KRYLOV_RIGHT 0         /* right-preconditioned flexible GMRES, Euclidean inner product  */
#define HKG_KRYLOV_LEFT_DK 1       /* GMRES on eq. (2.24) in the D_k inner product (Theorem 3.1)    */

typedef struct hkgeneo_ctx hkgeneo_ctx;

/*
 * The discrete problem.  Every pointer is a host pointer; all are read during hkgeneo_setup only.
 *   elem_vert [n_elem*npe]   vertex ids of each element (npe = 3 for 2D P1, 4 for 2D Q1, 8 for 3D Q1;
 *                            Q1 local node a = ax + 2 ay (+ 4 az))
 *   vert_dof  [n_vert]       dof id of each vertex, -1 on the Dirichlet boundary
 *   elem_K, elem_M [n_elem*npe*npe]  row-major element stiffness (coefficient folded in) and mass
 *   row_ptr [n_dof+1], col_idx [nnz]  CSR pattern shared by A and S, column ids sorted per row
 *   A_val, S_val [nnz]       stiffness and consistent mass values on that pattern
 *   elem_part [n_elem]       non-overlapping partition, ids in [0, n_sub)
 *   overlap [n_sub]          element layers added to each block (>= 1)
 *   k                        wavenumber (>= 0)
 *   fine_part [n_elem]       NULL, or a finer non-overlapping element partition (ids >= 0) for the
 *                            nested decomposition of Sec. 2.3: the elements of each overlapping coarse
 *                            subdomain are split by it into Q_i pieces (ordered by id), each expanded
 *                            by fine_overlap layers of Def. 2.8 restricted to the coarse subdomain (so
 *                            the pieces cover it); the local solves of eq. (2.22) run on these fine
 *                            subdomains, the coarse space (Def. 2.14, 2.15) on the coarse ones.
 *                            Pieces without an interior dof are dropped.  hkgeneo_gmres_solve and
 *                            hkgeneo_apply only (the batched engine, the server and
 *                            hkgeneo_apply_noalloc reject nested contexts with HKG_EINVAL).
 *   fine_overlap             layers of that expansion (>= 0; used when fine_part is set)
 */
typedef struct {
    int32_t dim;
    int32_t elem_type;
    int32_t n_vert;
    int32_t n_elem;
    int32_t n_dof;
    int32_t nnz;
    const int32_t *elem_vert;
    const int32_t *vert_dof;
    const double *elem_K;
    const double *elem_M;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *A_val;
    const double *S_val;
    const int32_t *elem_part;
    int32_t n_sub;
    const int32_t *overlap;
    double k;
    const int32_t *fine_part;
    int32_t fine_overlap;
} hkgeneo_problem;

/*
 * Method options.  hkgeneo_default_options fills the defaults listed here.
 *   eig_mode, tau, nev   selection of Def. 2.15 (default HKG_EIG_FIXED, tau 0, nev 10); the count
 *                        is raised to include every lambda <= 0 and to close a cluster
 *                        (lambda_{m+1} - lambda_m <= cluster_rtol max(1, |lambda_m|)).
 *   cluster_rtol         default 1e-8
 *   max_eig_per_sub      hard cap on m_i (default 64); exceeding it is HKG_EEIG
 *   local_prec           64: local inverses stored and applied in float64; 32: stored and applied in
 *                        float32 with float32 accumulation (coarse space, Arnoldi, residuals and the
 *                        outer FGMRES stay float64)
 *   local_factor_prec    must be 64 (default): B_D = P L U and B_D^{-1} are formed in float64 and, with
 *                        local_prec 32, rounded once to float32 storage.  32 (a float32 LU) is rejected
 *                        with HKG_EINVAL: near a local resonance its O(cond(B_D) eps_32) error costs
 *                        FGMRES iterations (36 against 28 at h = 1/32, k = 10)
 *   prolong              HKG_PROLONG_AS (default) or HKG_PROLONG_POU
 *   two_level            1 (default): add the coarse correction; 0: one-level only
 *   restart, max_iter, rtol   FGMRES(restart) stopping at ||f - B u|| <= rtol ||f||
 *                        (defaults 50, 1000, 1e-8)
 *   keep_workspace       0 (default): free the factorisation workspace (dense local blocks, Schur
 *                        complements, eigen work arrays) when setup/factor returns; 1: keep it for
 *                        the next hkgeneo_factor (no allocation on refactorisation)
 *   krylov               HKG_KRYLOV_RIGHT (default): right-preconditioned flexible GMRES in the
 *                        Euclidean inner product, stopping at ||f - B u|| <= rtol ||f||;
 *                        HKG_KRYLOV_LEFT_DK: GMRES(restart) on the left-preconditioned system
 *                        M^{-1} B u = M^{-1} f (eq. 2.24) in the inner product <x, y>_{D_k} = y^T D_k x,
 *                        D_k = A + k^2 S (Prop 2.11): the setting of Theorem 3.1.  It stops at
 *                        ||M^{-1}(f - B u)||_{D_k} <= rtol ||M^{-1} f||_{D_k}; one more sparse product
 *                        (with D_k) per iteration.  hkgeneo_gmres_solve only (the batched engine and
 *                        the server reject such contexts with HKG_EINVAL).
 *   coarse_op            HKG_COARSE_HK (default): the H_k-GenEO eigenproblem of Def. 2.14 (indefinite
 *                        B~, D~ the Gram matrix of (.,.)_{1,k}); HKG_COARSE_DELTA: Delta-GenEO, the
 *                        comparison coarse space of Sec. 1, read as the same eigenproblem built from
 *                        the nearby SPD problem (k = 0: B~ and D~ both the Neumann matrix of a(.,.));
 *                        the local solves and B_0 = Z^T B Z keep the indefinite B either way.
 */
typedef struct {
    int32_t eig_mode;
    double tau;
    int32_t nev;
    double cluster_rtol;
    int32_t max_eig_per_sub;
    int32_t local_prec;
    int32_t prolong;
    int32_t two_level;
    int32_t restart;
    int32_t max_iter;
    double rtol;
    int32_t keep_workspace;
    int32_t local_factor_prec;
    int32_t krylov;
    int32_t coarse_op;
} hkgeneo_options;

/* per right-hand side outcome of hkgeneo_gmres_solve (host array of nrhs entries) */
typedef struct {
    int32_t iters;          /* preconditioner applications                         */
    int32_t converged;      /* 1 if ||f - B u|| <= rtol ||f|| (checked in float64)  */
    double relres_est;      /* Arnoldi recurrence estimate |g_{j+1}| / ||f||         */
    double relres_true;     /* ||f - B u|| / ||f|| recomputed at the end             */
} hkgeneo_rhs_info;

/* summary of a context (host struct) */
typedef struct {
    int32_t n_dof;
    int32_t n_sub;
    int32_t lambda_overlap;   /* Lambda: max number of subdomains containing one element       */
    int32_t m0;               /* coarse dimension sum_i m_i                                    */
    int32_t sum_nI;           /* sum of |dof(D_i)|                                             */
    int32_t max_nI;
    int32_t max_nG;           /* max |ovdof(D_i) \ dof(D_i)|                                   */
    int32_t bad_sub;          /* -1 for a context that was set up (failures return no context)  */
    int64_t device_bytes;     /* device memory held by the context                             */
    double setup_ms;          /* wall time of hkgeneo_setup                                    */
    int64_t peak_device_bytes; /* high-water mark of device_bytes, setup/factor workspace included */
} hkgeneo_stats;

/* Fill `opt` with the defaults documented above. */
void hkgeneo_default_options(hkgeneo_options *opt);

/*
 * Build the preconditioner (Sec. 2.3-2.4): overlap extension, index sets and multiplicities on the
 * host; local Dirichlet factors, local eigenproblems, coarse basis and coarse factor on the device.
 * Synchronous: returns after the device work is done, so its status is final.
 * On success *out owns every device buffer; release it with hkgeneo_destroy.  On failure *out is NULL.
 */
int32_t hkgeneo_setup(const hkgeneo_problem *prob, const hkgeneo_options *opt, void *stream,
                      hkgeneo_ctx **out);

/*
 * Recompute every numeric part of the preconditioner (the local blocks, local eigenproblems, coarse
 * space, coarse and local factors) on the device from the inputs that hkgeneo_setup made resident;
 * the host partition and the index sets are reused.  Synchronous; statuses as for hkgeneo_setup.
 * Separates the numeric factorisation from the host analysis, so that it can be timed and repeated
 * with its inputs in device memory.
 */
int32_t hkgeneo_factor(hkgeneo_ctx *ctx, void *stream);

/*
 * z = M^{-1} r (eq. (2.23)) for nrhs columns.  r and z are device arrays n_dof x nrhs (ld >= n_dof),
 * must not alias.  Asynchronous on `stream`; HIP errors surface on the next synchronous call.
 * Errors: HKG_EINVAL for a NULL pointer, nrhs < 1 or ld < n_dof.
 */
int32_t hkgeneo_apply(hkgeneo_ctx *ctx, const double *r, double *z, int32_t nrhs, int32_t ld,
                      void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hkgeneo_apply without any allocation.  The same kernels
 * and result as hkgeneo_apply; the temporaries (local vectors, the coarse restriction Z^T r and the
 * partial sums of the coarse product: 8 nrhs (sum n_I + m0 (1 + ceil(m0 / 64))) bytes, each part
 * rounded up to 256 bytes) live in one fixed array of HKG_APPLY_NOALLOC_MAX_BYTES per GPU, which
 * the library holds from the first call on that GPU until the process ends; nothing in it needs to
 * start at zero.  Every call on a GPU uses that GPU's one array, so calls that overlap in time on
 * one GPU (different streams or host threads) race: order them on one stream.
 * Errors: as hkgeneo_apply; HKG_EINVAL also when the temporaries exceed HKG_APPLY_NOALLOC_MAX_BYTES.
 */
#define HKG_APPLY_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int32_t hkgeneo_apply_noalloc(hkgeneo_ctx *ctx, const double *r, double *z, int32_t nrhs, int32_t ld,
                              void *stream);

/*
 * Solve B u = f (Sec. 1: GMRES on the preconditioned system, analysed by the Elman theory of
 * Theorem 3.1) with M^{-1} = M^{-1}_{AS,2} of eq. (2.23) as preconditioner, starting from u = 0,
 * independently for each of the nrhs columns: right-preconditioned flexible GMRES(restart) in the
 * Euclidean inner product, or (options.krylov = HKG_KRYLOV_LEFT_DK) GMRES(restart) on eq. (2.24) in
 * the D_k inner product.  f, u are device arrays n_dof x nrhs (ld >= n_dof); `info` is a host array
 * of nrhs entries (may be NULL): iterations, convergence by the variant's own criterion, its
 * recurrence estimate, and the Euclidean true residual ||f - B u|| / ||f||.  Synchronous.
 * Returns HKG_OK if every column converged, HKG_ENOTCONV otherwise (u holds the last iterate).
 */
int32_t hkgeneo_gmres_solve(hkgeneo_ctx *ctx, const double *f, double *u, int32_t nrhs, int32_t ld,
                            hkgeneo_rhs_info *info, void *stream);

/*
 * Batched solves: several set-up problems stepped together.
 *
 * One FGMRES iteration (the preconditioner of eq. (2.23) and the CGS2 Arnoldi step) runs as one
 * launch per phase for every (problem, subdomain or row block, right-hand side) item of the live
 * set, whatever the sizes of the problems; the iteration is captured once as a HIP graph and
 * replayed.  The Arnoldi index and the state of every (problem, rhs) pair live on the device, and a
 * second captured graph (the restart phase: x update, true residual ||f - B u|| in FP64, stop or
 * start the next cycle) serves the pairs that reach the end of a cycle, so each pair restarts on
 * its own.  The launch shape of the local solves is chosen by timing the candidates when the live
 * set changes (cached per shape).  A problem's iterates are bitwise the same whichever other
 * problems share the live set and whichever launch shape is picked.  Stopping rule and results as
 * in hkgeneo_gmres_solve, with rtol and max_iter taken from each problem's options.
 *
 * Common rules: contexts must outlive every batch or server call that uses them and must not be
 * used by another call while one runs; every context must use the restart length of the batch or
 * server; hkgeneo_factor on a context is allowed between solves.  f and u are device arrays
 * n_dof x nrhs with leading dimension ld >= n_dof, u must not alias f.  Neither object is
 * thread-safe.  Each owns an internal HIP stream (default priority) and its Krylov workspace.
 */

/* A fixed set of nprob problems: ctxs[p] (host array of handles) with nrhs[p] right-hand sides.
 * Errors: HKG_EINVAL for NULL handles, nprob < 1, nrhs[p] outside 1..65535 or different restart
 * lengths; HKG_ENOMEM; HKG_EHIP.  On failure *out is NULL. */
typedef struct hkgeneo_batch hkgeneo_batch;
int32_t hkgeneo_batch_create(hkgeneo_ctx *const *ctxs, const int32_t *nrhs, int32_t nprob,
                             hkgeneo_batch **out);

/*
 * Solve every problem of the batch from u = 0.  f[p], u[p], ld[p]: host arrays of nprob device
 * pointers / leading dimensions.  The call waits for `stream` (the caller's) before reading f and
 * returns when every u[p] is final (synchronous).  info: host array of sum(nrhs) entries in problem
 * order (may be NULL).  Returns HKG_OK if every column converged, HKG_ENOTCONV otherwise;
 * HKG_EINVAL for a NULL pointer, ld[p] < n_dof or a subdomain too large for the batched local
 * solve (2 |dof(D)| + 2048 doubles of LDS must fit in 160 KiB).
 */
int32_t hkgeneo_batch_solve(hkgeneo_batch *b, const double *const *f, double *const *u, const int32_t *ld,
                            hkgeneo_rhs_info *info, void *stream);

/* Device bytes held by the batch itself (workspace and descriptor tables). */
int64_t hkgeneo_batch_bytes(const hkgeneo_batch *b);

/* Launch shape the autotuner chose for the batched local solves (waves per 64-row tile). */
int32_t hkgeneo_batch_local_waves(const hkgeneo_batch *b);

/* Measurement hook.  enable = 1 clears earlier records and, until disabled, launches the iterations
 * directly instead of replaying the graph (same kernels and launch shapes) with HIP events around
 * every batched local-solve launch on the batch's stream; 0 returns to graph replay.
 * hkgeneo_batch_profile_read sums the recorded durations (ms) and counts the launches. */
int32_t hkgeneo_batch_profile(hkgeneo_batch *b, int32_t enable);
int32_t hkgeneo_batch_profile_read(hkgeneo_batch *b, double *total_ms, int64_t *launches);

void hkgeneo_batch_destroy(hkgeneo_batch *b);

/*
 * Server: continuous batching of solve requests.  Requests are submitted at any time and queued;
 * at every check period (a few iterations) the server admits queued requests in arrival order
 * while a slot is free (at most max_requests live) and their Krylov workspace fits in
 * workspace_budget bytes, runs the restart phase if some pair needs it, replays the iteration
 * graph, and retires requests whose right-hand sides have all stopped.  Admission and retirement
 * happen only at iteration boundaries; the work of all live requests shares every launch.
 * max_nrhs bounds nrhs per request.
 * Errors: HKG_EINVAL for max_requests outside 1..65535, max_nrhs outside 1..65535, restart outside
 * 1..1024, workspace_budget <= 0.
 */
typedef struct hkgeneo_server hkgeneo_server;
typedef struct {
    int32_t queued, live, live_rhs, completed_waiting, local_waves, pad_;
    int64_t workspace_bytes;    /* Krylov workspace held, including buffers kept for reuse */
    int64_t device_bytes;       /* all device bytes held by the server */
    int64_t iterations;         /* iteration graph launches */
    int64_t restarts;           /* restart graph launches */
    int64_t captures;           /* graph captures (one pair per change of the live set) */
    int64_t admitted, retired;
} hkgeneo_server_stats;

int32_t hkgeneo_server_create(int64_t workspace_budget, int32_t max_requests, int32_t max_nrhs,
                              int32_t restart, hkgeneo_server **out);

/* Queue a request (asynchronous): solve ctx's system for nrhs columns of f into u, from u = 0;
 * `tag` is returned by hkgeneo_server_poll.  The server waits for `stream` (recorded now) before it
 * reads f.  f and u must stay valid until the request is polled.
 * Errors: HKG_EINVAL (NULL pointer, nrhs outside 1..max_nrhs, ld < n_dof, other restart, subdomain
 * too large for the batched local solve), HKG_ENOMEM if its workspace alone exceeds the budget. */
int32_t hkgeneo_server_submit(hkgeneo_server *s, hkgeneo_ctx *ctx, const double *f, double *u,
                              int32_t nrhs, int32_t ld, int64_t tag, void *stream);

/* Run up to `periods` check periods (returns early when nothing is live or queued).  *pending
 * (may be NULL) receives the number of requests live or queued afterwards. */
int32_t hkgeneo_server_pump(hkgeneo_server *s, int32_t periods, int32_t *pending);

/* Pop one finished request: returns its nrhs (> 0) and fills *tag, *status (HKG_OK or
 * HKG_ENOTCONV) and info[0..nrhs) (host, capacity cap; may be NULL); 0 if none is waiting;
 * HKG_EINVAL if cap is too small (the request stays queued).  Its u is final. */
int32_t hkgeneo_server_poll(hkgeneo_server *s, int64_t *tag, int32_t *status, hkgeneo_rhs_info *info,
                            int32_t cap);

int32_t hkgeneo_server_query(const hkgeneo_server *s, hkgeneo_server_stats *out);

/* Waits for the server's stream; queued and live requests are dropped (their u is undefined). */
void hkgeneo_server_destroy(hkgeneo_server *s);

/* w = B x for nrhs columns (device arrays, ld >= n_dof).  Asynchronous. */
int32_t hkgeneo_matvec(hkgeneo_ctx *ctx, const double *x, double *w, int32_t nrhs, int32_t ld,
                       void *stream);

/*
 * Measurement hook.  enable = 1 starts recording HIP events around every launch of the local-solve
 * kernel (gather + product with the local inverses, the kernel that dominates one application) on
 * the stream it is launched on, and clears earlier records; 0 stops recording.
 */
int32_t hkgeneo_profile(hkgeneo_ctx *ctx, int32_t enable);

/* Sum of the recorded local-solve kernel durations (ms) and the number of launches recorded;
 * waits for the recorded events. */
int32_t hkgeneo_profile_read(hkgeneo_ctx *ctx, double *total_ms, int64_t *launches);

/* Scalar summary of a context. */
int32_t hkgeneo_query(const hkgeneo_ctx *ctx, hkgeneo_stats *out);

/*
 * Per-subdomain sizes into host arrays of n_sub entries (any may be NULL):
 * nI = |dof(D_i)|, nG = |Gamma_i|, m = selected eigenvectors m_i.
 */
int32_t hkgeneo_query_subdomains(const hkgeneo_ctx *ctx, int32_t *nI, int32_t *nG, int32_t *m);

/*
 * First-level subdomains of a nested context (Sec. 2.3): their number, and per subdomain (arrays of
 * that length, each may be NULL) |dof(Omega_{i,j}^f)| and the coarse subdomain i that owns it;
 * *lambda_fine: Lambda of Sec. 2.4 counted over them.  A context without nesting reports its
 * coarse subdomains (each its own owner).  Call first with nI = owner = NULL to get the count.
 */
int32_t hkgeneo_query_fine(const hkgeneo_ctx *ctx, int32_t *n_fine, int32_t *nI, int32_t *owner,
                           int32_t *lambda_fine);

/*
 * Index sets of subdomain `sub` into host arrays: dof ids of dof(D) ascending (nI entries) and of
 * Gamma ascending (nG entries); either may be NULL.  mu (host, n_dof entries, may be NULL) receives
 * the multiplicities of Def. 2.13 when sub == 0.
 */
int32_t hkgeneo_query_index_sets(const hkgeneo_ctx *ctx, int32_t sub, int32_t *dof, int32_t *gamma,
                                 int32_t *mu);

/*
 * Eigen data of subdomain `sub` (host arrays): the count smallest eigenvalues of Def. 2.14
 * ascending (count <= m_i + 1 when m_i < nI, else m_i), and the coarse basis block Z_i = X_I P_i
 * (nI x m_i column-major), either may be NULL.
 */
int32_t hkgeneo_query_eigen(const hkgeneo_ctx *ctx, int32_t sub, double *lambda, int32_t count,
                            double *Z);

/* The coarse matrix B_0 = Z^T B Z (m0 x m0 column-major, host array). */
int32_t hkgeneo_query_coarse_matrix(const hkgeneo_ctx *ctx, double *B0);

/*
 * Host-only overlapping decomposition (no device work): Def. 2.8 applied overlap[i] times to each
 * block of elem_part, then dof(D_i) and Gamma_i = ovdof(D_i) \ dof(D_i) (Def. 2.12), the
 * multiplicities mu (Def. 2.13) and Lambda.  Only the element, vertex and partition fields of `prob`
 * are read.  Outputs are host arrays, each optional (NULL): nI, nG [n_sub]; dof, gamma the
 * concatenated ascending index sets (sum nI, sum nG entries; call once without them to size them);
 * mu [n_dof]; lambda_overlap one int.  Errors: HKG_EINVAL for bad ids or a dof internal to no
 * subdomain (overlap too small).
 */
int32_t hkgeneo_partition(const hkgeneo_problem *prob, int32_t *nI, int32_t *nG, int32_t *dof, int32_t *gamma,
                          int32_t *mu, int32_t *lambda_overlap);

/* Release every device buffer of the context (NULL is ignored). */
void hkgeneo_destroy(hkgeneo_ctx *ctx);

/* Static description of a status code. */
const char *hkgeneo_strerror(int32_t status);

/* Detail of the last failure on the calling thread (empty if none); valid until the next call. */
const char *hkgeneo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HKGENEO_H */
