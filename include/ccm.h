/*
 * ccm.h -- C ABI of libccm, an MI355X (gfx950) library for the convex
 * clustering model (CCM) of arXiv 2501.15964 ("PyClustrPath"), Section 1:
 *
 *     min_X  1/2 sum_i ||x_i - a_i||_2^2 + gamma sum_{i<j} w_ij ||x_i - x_j||_q
 *
 * over a sparse weight graph, solved along a gamma path (Section 1, last
 * paragraph) by SSNAL or ADMM (Section 1, Table 3), with the relative KKT
 * residual as stopping test and the relative duality gap of Section 4
 * reported beside it.
 *
 * Conventions that hold for every entry point:
 *  - Array arguments are DEVICE pointers (memory of the current HIP device)
 *    unless the name ends in _host.  Dense matrices are row-major FP64:
 *    A and X are n x d (row i = point i), U is m x d (row l = edge l).
 *  - The caller owns every buffer; the library never frees caller memory.
 *    Work space is device memory that the library caches per device: a call
 *    takes blocks from the cache (or allocates them), uses them in the order
 *    of `stream` and returns them to the cache before it returns, so later
 *    calls reuse them without allocating.  The cache holds at most half of
 *    the device's memory; ccm_release_workspace() frees it.  All work is
 *    enqueued on `stream`; calls that return host values synchronise that
 *    stream.
 *  - Edges: l = (src_l, dst_l) is an undirected edge with weight w_l.  On
 *    input any order and orientation is accepted; self-loops and zero
 *    weights are dropped and duplicate pairs are merged by adding their
 *    weights (exact for the model, since w||z|| + w'||z|| = (w+w')||z||).
 *    The library works on the canonical edge list (src < dst, sorted by
 *    (src, dst)); U_out rows follow that canonical order, which equals the
 *    input order whenever the input is already canonical (as the k-NN
 *    builder's output is).
 *  - q is 1.0, 2.0 or INFINITY.  The dual ball of edge l has radius
 *    r_l = gamma w_l in the dual norm q* (q = 1 <-> q* = inf, 2 <-> 2,
 *    inf <-> 1).
 *  - Errors: a non-zero ccm_status; ccm_last_error() returns a thread-local
 *    text.  Argument checks finish before anything is launched.
 *    Non-convergence is not an error: the per-gamma status says so and the
 *    last iterate is returned.
 *  - All reductions are deterministic (fixed order, no floating-point
 *    atomics): the same inputs give bit-identical outputs run to run.
 */
#ifndef CCM_H
#define CCM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ccm_status;
enum {
    CCM_OK = 0,
    CCM_E_INVALID = 1,      /* bad argument (sizes, indices, NaN, negative weight ...) */
    CCM_E_UNSUPPORTED = 2,  /* valid request outside what the library implements */
    CCM_E_HIP = 3,          /* a HIP runtime call failed */
    CCM_E_NOMEM = 4,        /* device allocation failed */
    CCM_E_CAPACITY = 5,     /* a caller buffer is too small (see *_cap arguments) */
    CCM_E_NOT_CONVERGED = 6 /* an iterative solve inside the call stopped before its
                               tolerance (outputs hold its last iterate) */
};

/* solver: SSNAL and ADMM (Section 1, Table 3), fast AMA (Table 3), and the
 * Halpern-Peaceman-Rachford method named as future work in the conclusion
 * (CCM_HPR: ADMM's splitting with the Peaceman-Rachford relaxation 2 inside
 * Halpern's anchored iteration, anchor restarts on the fixed-point residual) */
enum { CCM_SSNAL = 0, CCM_ADMM = 1, CCM_AMA = 2, CCM_HPR = 3 };
enum { CCM_CONVERGED = 0, CCM_MAX_ITER = 1, CCM_TIMEOUT = 2,
       CCM_NUMERICAL = 3 };                                   /* per-gamma status */

const char* ccm_status_string(ccm_status s);
const char* ccm_last_error(void);
const char* ccm_version(void);

/* Frees the work space the library caches (on every device used so far),
 * after the work that last used each block has finished.  Blocks in use by
 * a call running on another thread are kept.  CCM_E_HIP if a HIP call fails. */
ccm_status ccm_release_workspace(void);

/* ---------------------------------------------------------------------------
 * Options.  Pass NULL for the defaults below, or fill a struct obtained from
 * ccm_default_options().  Heuristic parameters change iteration counts, not
 * the unique solution X*.
 */
typedef struct {
    int32_t method;        /* CCM_SSNAL (default), CCM_ADMM, CCM_AMA or CCM_HPR */
    int32_t max_outer;     /* SSNAL outer (augmented Lagrangian) iterations per gamma. 300 */
    int32_t max_newton;    /* SSNAL Newton steps per outer iteration.  60 */
    int32_t cg_max_iter;   /* CG iterations per linear solve.  500 */
    int32_t max_iter;      /* ADMM / AMA / HPR iterations per gamma.  20000 */
    int32_t check_every;   /* ADMM / AMA / HPR: KKT test every this many iterations.  10 */
    int32_t cg_chunk;      /* CG iterations launched between host checks.  8 */
    int32_t profile;       /* 1: time every kernel class with HIP events (ccm_stats.kern_*);
                              2: time only the Newton/CG matvec class (less host work);
                              0: off */
    double sigma0;         /* initial penalty (SSNAL: of every gamma; ADMM: on a cold
                              start); <= 0: default 1 */
    double sigma_max;      /* SSNAL penalty cap.  1e4 */
    double tau;            /* ADMM multiplier step.  1.618 */
    double time_budget_s;  /* wall-clock budget for the whole path; <= 0: none */
    int32_t locality;      /* order in which the vertex kernels visit the points:
                              1: connected components one after another, each in
                              breadth-first levels from its smallest point (the
                              rows gathered at the same time are neighbours, so
                              the caches hold them); 0: the input order; -1
                              (default): 1 when n d >= 2^22, else 0.  Changes the
                              summation order only, never the data layout */
    int32_t window_chunk;  /* incidences per row group of a vertex-kernel window, 1 to
                              4096 (else CCM_E_INVALID); 0 (default): the tuned value for
                              the row width and q (a table the package's window tuner
                              writes); changes the summation order of split vertices, so
                              results depend on it (each value deterministic) */
    int32_t dual_scale;    /* SSNAL path continuation.  1: before each gamma after the
                              first, the rows of U on the boundary of the previous gamma's
                              dual balls (q = 1: the coordinates at +-r) are scaled by
                              gamma_t / gamma_{t-1}: the dual of an edge whose endpoints are
                              apart is gamma w_l times a direction that moves slowly along
                              the path.  0: (X, U) carried over unchanged.  -1 (default):
                              1 for q = 2, 0 otherwise (measured faster, resp. slower).
                              Other values: CCM_E_INVALID.  Only the starting point
                              changes, not the solution */
} ccm_options;

ccm_options ccm_default_options(void);

/* Kernel classes timed when ccm_options.profile = 1 (only CCM_K_MATVEC when 2). */
enum { CCM_K_EDGE = 0, CCM_K_SCATTER = 1, CCM_K_MATVEC = 2, CCM_K_CGUPDATE = 3,
       CCM_K_OTHER = 4, CCM_NK = 5 };

/* Per-gamma statistics. */
typedef struct {
    int32_t outer, newton, cg, linesearch;  /* iteration counts (ADMM/AMA: outer = iterations) */
    double seconds;                         /* wall time of this gamma (host clock) */
    double f_p, f_d;                        /* primal (CCM) value, dual value at Pi_C(U) */
    double sigma;                           /* penalty at exit */
    double kern_ms[CCM_NK];                 /* profile != 0: summed kernel time per class */
    int64_t kern_calls[CCM_NK];             /* profile != 0: launches per class */
    double matvec_bytes;                    /* profile != 0: algorithmic bytes of the timed
                                               Newton / CG matvec launches that did work
                                               (each launch: read V once, write the output
                                               once, the incidence entries with their vertex
                                               ids, and the Jacobian payload: per-incidence
                                               scalars, lane masks, rows of Pi of edges with
                                               P != I); 0 when profile = 0 */
    int64_t matvec_launches;                /* the number of those launches (= kern_calls of
                                               CCM_K_MATVEC; with profile = 2 one launch in
                                               four is timed; launches issued after CG
                                               convergence return at once and are counted
                                               in class CCM_K_OTHER) */
} ccm_stats;

/* ---------------------------------------------------------------------------
 * k-NN Gaussian weight graph (Section 2.2: the Data Processor computes the
 * weights w_ij from A; Section 1 only asks w_ij = w_ji >= 0).
 *
 * For every point i the k nearest other points j by squared Euclidean
 * distance, where d^2(i, j) is the FP64 sum of fl((a_ik - a_jk)^2) over
 * features in ascending order with every product and sum rounded separately
 * (so d^2 is bit-defined), ties broken by the smaller j.  The pairs are
 * union-symmetrised (i ~ j iff j in kNN(i) or i in kNN(j)) and weighted
 * w = exp(-phi d^2); phi > 0 is used as given, phi <= 0 selects
 * 1 / median of the n k directed neighbour distances (mean of the two middle
 * values when n k is even).  Edges whose weight underflows to 0 are dropped.
 *
 * A      : n x d FP64, device.  n >= 2, 1 <= d, 1 <= k <= min(n - 1, 32).
 * src,dst: int32[m_cap], w: double[m_cap] device outputs, canonical order
 *          (src < dst, sorted by (src, dst)).  m_cap >= n k always suffices.
 * m_out_host   : number of edges written.
 * phi_out_host : phi used (may be NULL).
 * Errors: CCM_E_INVALID (sizes, non-finite A), CCM_E_CAPACITY (m_cap too
 * small: *m_out_host then holds the needed size and nothing is written).
 * Synchronises `stream`.
 */
ccm_status ccm_build_knn_graph(const double* A, int64_t n, int64_t d, int32_t k, double phi,
                               int32_t* src, int32_t* dst, double* w, int64_t m_cap,
                               int64_t* m_out_host, double* phi_out_host, hipStream_t stream);

/* The same graph for quantised data given as integer codes: the points are
 * a_i = scale * K_i with K an n x d uint8 array (device), and
 * d^2(i, j) = (double)D_ij * scale * scale with D_ij = sum_k (K_ik - K_jk)^2
 * computed exactly in integer arithmetic (int8 matrix cores with int32
 * accumulation); ties broken by the smaller j.  1 <= d <= 2048 (a tile of
 * 64 candidate rows is held in LDS); CCM_E_INVALID otherwise.  Other
 * arguments, outputs and errors as for ccm_build_knn_graph.
 */
ccm_status ccm_build_knn_graph_u8(const uint8_t* K, int64_t n, int64_t d, double scale, int32_t k,
                                  double phi, int32_t* src, int32_t* dst, double* w,
                                  int64_t m_cap, int64_t* m_out_host, double* phi_out_host,
                                  hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Clustering path (Section 1: solve (CCM) for gamma_1 < ... < gamma_T; the
 * solutions are continuous in gamma, so each gamma is warm-started from the
 * previous one).
 *
 * A          : n x d FP64 (device).
 * src,dst,w  : m edges (device), see the conventions above.  w finite, >= 0.
 * gammas_host: n_gamma values, finite and >= 0, solved in the given order.
 * q          : 1.0, 2.0 or INFINITY.
 * tol        : stop when the relative KKT residual max(R_D, R_C, R_U) <= tol,
 *              R_D = ||X - A + B^T U|| / (1 + ||A||),
 *              R_C = ||Pi_C(BX + U) - U|| / (1 + ||BX|| + ||U||),
 *              R_U = ||U - Pi_C(U)|| / (1 + ||U||).
 * opts       : NULL for defaults.
 * Outputs (any output pointer may be NULL unless stated):
 *   X_out          : n_gamma x n x d (device), required.
 *   U_out          : n_gamma x m_canon x d (device) dual solutions; m_canon <= m.
 *   labels_out     : n_gamma x n int32 (device) cluster labels: points i, j
 *                    share a label iff they are joined by a chain of edges
 *                    with ||x_i - x_j||_2 <= 1e-5 (1 + S), S = max_i ||a_i - mean(a)||_2;
 *                    labels number clusters by their smallest point index.
 *   n_clusters_host: n_gamma int32.
 *   kkt_host       : n_gamma x 4 doubles: R_D, R_C, R_U, eta where
 *                    eta = |f_p - f_d| / (1 + |f_p| + |f_d|) (Section 4).
 *   status_host    : n_gamma int32 (CCM_CONVERGED, CCM_MAX_ITER, CCM_TIMEOUT,
 *                    CCM_NUMERICAL).
 *   stats_host     : n_gamma ccm_stats.
 * X_warm, U_warm : optional device warm start for the first gamma (n x d and
 *                  m_canon x d); NULL = cold start (X = A, U = 0).
 * Errors: CCM_E_INVALID, CCM_E_UNSUPPORTED (q), CCM_E_NOMEM, CCM_E_HIP.
 * Synchronises `stream`.
 */
ccm_status ccm_solve_path(const double* A, int64_t n, int64_t d,
                          const int32_t* src, const int32_t* dst, const double* w, int64_t m,
                          const double* gammas_host, int32_t n_gamma, double q, double tol,
                          const ccm_options* opts,
                          double* X_out, double* U_out, int32_t* labels_out,
                          int32_t* n_clusters_host, double* kkt_host, int32_t* status_host,
                          ccm_stats* stats_host,
                          const double* X_warm, const double* U_warm, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched paths: many independent (CCM) instances of uneven n, d and q, each
 * solved along the same gamma sequence to its own relative KKT <= tol (its
 * residuals normalised by its own norms).  Instances with equal (q, d) are
 * solved together as one block-diagonal problem, so every kernel launch
 * serves all of them; SSNAL only (opts->method is ignored).
 *
 * Instance i is described by inst_host[i]:
 *   n, d, m   : points, features, edges (n >= 1, 1 <= d <= 1024, m >= 0);
 *   a_offset  : element offset of its A (n x d, row-major) in A_all;
 *   e_offset  : offset of its m edges in src_all / dst_all / w_all; endpoints
 *               are local (0 .. n-1) and the edges canonical (src < dst,
 *               sorted by (src, dst), w > 0);
 *   x_offset  : element offset of its outputs in X_out_all: n_gamma
 *               consecutive n x d blocks, gamma-major;
 *   l_offset  : element offset in labels_all: n_gamma blocks of n labels
 *               (numbered within the instance as in ccm_solve_path);
 *   q         : 1.0, 2.0 or INFINITY.
 * Host outputs are indexed [i * n_gamma + t]: n_clusters_host, status_host,
 * and kkt_host (4 doubles each: R_D, R_C, R_U, eta).  labels_all, kkt_host,
 * n_clusters_host and status_host may be NULL.
 * Errors: CCM_E_INVALID (descriptor, edges), CCM_E_UNSUPPORTED (q, d).
 * Synchronises `stream`.
 */
typedef struct {
    int64_t n, d, m;
    int64_t a_offset, e_offset, x_offset, l_offset;
    double q;
} ccm_instance;

ccm_status ccm_solve_path_batched(const ccm_instance* inst_host, int32_t n_inst,
                                  const double* A_all, const int32_t* src_all,
                                  const int32_t* dst_all, const double* w_all,
                                  const double* gammas_host, int32_t n_gamma, double tol,
                                  const ccm_options* opts, double* X_out_all, int32_t* labels_all,
                                  int32_t* n_clusters_host, double* kkt_host,
                                  int32_t* status_host, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Vector-Jacobian product of the solution map X*(A, w, gamma) at one gamma,
 * q = 2 (implicit differentiation of the optimality conditions of (CCM),
 * Section 1, through the generalized Jacobian of the SSNAL subproblem in its
 * exact limit).  With the clusters c of a solution held fixed (every edge
 * with a positive fusion margin), the points of a cluster share one value
 * and the adjoint system in cluster space is
 *     (diag(|c|) (x) I + B_c^T H B_c) lambda = g,   g_c = sum_{i in c} dL/dx_i,
 *     H_l = gamma w_l (I - ghat ghat^T) / ||x_i - x_j||   (edges joining two clusters),
 * solved by preconditioned CG; then
 *     dL/da_i = lambda_{c(i)},
 *     dL/dlog w_l = -gamma w_l <lambda_{c(i)} - lambda_{c(j)}, ghat_l>  (0 inside a cluster),
 *     dL/dgamma = -sum_l w_l <lambda_{c(i)} - lambda_{c(j)}, ghat_l>.
 *
 * A, X, dL_dX, dL_dA : n x d (device).  X and labels must come from a tight
 *                      solve at this gamma (e.g. ccm_solve_path with tol 1e-10).
 * src, dst, w        : canonical edges (src < dst, sorted, w > 0), m of them.
 * labels             : int32[n] cluster labels in [0, K) (ccm_solve_path output).
 * dL_dlogw           : double[m] (device) or NULL;  dL_dgamma_host: double or NULL.
 * tol, max_iter      : CG stop at ||residual|| <= tol ||g|| or max_iter iterations.
 * iters_host         : CG iterations used (may be NULL).
 * Errors: CCM_E_UNSUPPORTED for q != 2; CCM_E_INVALID (sizes, non-canonical
 * edges, labels out of range); CCM_E_NOT_CONVERGED when the CG reached
 * max_iter or broke down (p.Hp <= 0) before ||residual|| <= tol ||g||: the
 * gradients are then written from its last iterate.  Synchronises `stream`.
 */
ccm_status ccm_path_vjp(const double* A, int64_t n, int64_t d, const int32_t* src,
                        const int32_t* dst, const double* w, int64_t m, double gamma, double q,
                        const double* X, const int32_t* labels, const double* dL_dX,
                        double* dL_dA, double* dL_dlogw, double* dL_dgamma_host, double tol,
                        int32_t max_iter, int32_t* iters_host, hipStream_t stream);

/* w_l = exp(log_w_l) for l < m (device arrays): the edge weights of a model
 * parameterised by log weights (as the autograd wrapper of the binding is),
 * computed in the library.  Errors: CCM_E_INVALID (m < 0). */
ccm_status ccm_weights_from_log(const double* log_w, int64_t m, double* w, hipStream_t stream);

/* Number of canonical edges the library derives from (src, dst, w); the
 * row count of each U_out block.  Synchronises `stream`. */
ccm_status ccm_canonical_edge_count(const int32_t* src, const int32_t* dst, const double* w,
                                    int64_t m, int64_t n, int64_t* m_canon_host,
                                    hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Edge operators on their own (the steps every path solver iterates; Section
 * 1 notes that additions and matrix-vector products dominate the cost).
 * Edges must be canonical here (src < dst, sorted, w > 0); m >= 0.
 *
 * ccm_op_gather   : Y = B X, (BX)_l = x_src - x_dst.                Y: m x d.
 * ccm_op_project  : Pi_l = projection of Y_l onto {||u||_{q*} <= gamma w_l}.
 * ccm_op_prox     : Z_l = prox of gamma w_l ||.||_q at Y_l = Y_l - Pi_l (Moreau).
 * ccm_op_scatter  : out = B^T Z, out_i = sum_{l: src_l=i} z_l - sum_{l: dst_l=i} z_l.
 * ccm_op_hess_matvec : out = V + sigma B^T P B V with P an element of the
 *                  generalized Jacobian of Pi_C at Y = U + sigma B X (the SSNAL
 *                  Newton matrix); on a ball boundary the identity branch.
 *                  `repeats` >= 1 applies the same matvec that many times
 *                  (for timing); *ms_host (may be NULL) receives the average
 *                  duration of one matvec launch measured with HIP events.
 * ccm_kkt         : residuals of an arbitrary pair (X, U): out_host[0..6] =
 *                  R_D, R_C, R_U, eta, f_p, f_d, max(R_D,R_C,R_U).
 * ccm_labels      : cluster labels of X as for ccm_solve_path (S from A).
 * Synchronous variants (those with _host outputs) synchronise `stream`.
 */
ccm_status ccm_op_gather(const double* X, int64_t n, int64_t d, const int32_t* src,
                         const int32_t* dst, int64_t m, double* Y, hipStream_t stream);
ccm_status ccm_op_project(const double* Y, int64_t m, int64_t d, const double* w, double gamma,
                          double q, double* Pi, hipStream_t stream);
ccm_status ccm_op_prox(const double* Y, int64_t m, int64_t d, const double* w, double gamma,
                       double q, double* Z, hipStream_t stream);
ccm_status ccm_op_scatter(const double* Z, int64_t m, int64_t d, const int32_t* src,
                          const int32_t* dst, int64_t n, double* out, hipStream_t stream);
ccm_status ccm_op_hess_matvec(const double* X, const double* U, int64_t n, int64_t d,
                              const int32_t* src, const int32_t* dst, const double* w, int64_t m,
                              double gamma, double sigma, double q, const double* V, double* out,
                              int32_t repeats, double* ms_host, hipStream_t stream);
ccm_status ccm_kkt(const double* A, const double* X, const double* U, int64_t n, int64_t d,
                   const int32_t* src, const int32_t* dst, const double* w, int64_t m,
                   double gamma, double q, double* out_host, hipStream_t stream);
ccm_status ccm_labels(const double* A, const double* X, int64_t n, int64_t d,
                      const int32_t* src, const int32_t* dst, int64_t m, int32_t* labels,
                      int32_t* n_clusters_host, hipStream_t stream);

/* ccm_labels for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same labels and count as ccm_labels, but every temporary (spread partials,
 * fused-edge flags, union-find parents, scan buffers) lives in one fixed
 * 32 MiB device array that the library holds on each device it runs on until
 * the process ends; the call allocates and frees nothing.  Capacity: the
 * buffers need about 4 m + 8 n bytes plus 1 KiB per feature, so for example
 * n = 1e6, m = 4e6, d <= 1024 fits; larger problems return CCM_E_CAPACITY
 * before anything is launched (also when n > 2^22 or m > 2^23).  All calls on
 * one device share the array and it keeps the last call's contents (every
 * buffer is written before it is read): calls that overlap on one device,
 * on any streams or threads, race and must be serialised by the caller.
 * The caller passes inputs and outputs as for ccm_labels.  Synchronises
 * `stream` (to return n_clusters_host). */
ccm_status ccm_labels_noalloc(const double* A, const double* X, int64_t n, int64_t d,
                              const int32_t* src, const int32_t* dst, int64_t m, int32_t* labels,
                              int32_t* n_clusters_host, hipStream_t stream);

/* Plain device copy of `bytes` bytes with the library's streaming kernel
 * (calibration of achievable HBM bandwidth).  *ms_host: average duration of
 * one launch over `repeats` launches, from HIP events. */
ccm_status ccm_stream_copy(const void* src, void* dst, int64_t bytes, int32_t repeats,
                           double* ms_host, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CCM_H */
