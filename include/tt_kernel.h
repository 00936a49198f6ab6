/*
 * tt_kernel.h -- C ABI of the MI355X (gfx950) implementation of the
 * parametric Chebyshev / tensor-train kernel low-rank method ("PTTK") of
 * Khan & Saibaba, "Parametric kernel low-rank approximations using tensor
 * train decomposition" (arXiv 2406.06344).
 *
 * The method approximates the parametric kernel matrix
 *     K(X, Y; theta)[i, j] = kappa(x_i, y_j; theta)          (Section 1)
 * with rows indexed by the N_s source points x_i and columns by the N_t
 * target points y_j, in the form K ~ S H(theta) T^T (the low-rank form of
 * Section 1).  In this library S is called U (N_s x r_s), T is called V
 * (N_t x r_t) and H(theta) is called M(theta) (r_s x r_t).
 *
 * Conventions shared by every entry point
 *  - Every call returns tt_status: 0 = OK, > 0 = warning (result usable),
 *    < 0 = error (outputs untouched or partially written; the handle, if any,
 *    stays valid).  Nothing is thrown across the ABI.  tt_kernel_last_error()
 *    returns a thread-local message for the last non-OK status.
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every pointer it
 *    passes and keeps it valid for the duration of the call (and, for
 *    asynchronous calls, until the work on `stream` has completed).
 *  - `stream` is a hipStream_t (NULL = the null stream).  All device work of
 *    a call is enqueued on it; calls return without synchronising unless the
 *    comment says otherwise.
 *  - Floating-point buffers named "dtype" hold float (TTK_FP32) or double
 *    (TTK_FP64) according to tt_kernel_params.dtype.  Kernel-entry
 *    evaluation feeding the cross approximation, its pivot selection, the
 *    QR/LU/SVD of the small cores and the core orthogonalisation always run
 *    in double precision on the device.
 *  - Points are passed structure-of-arrays: coordinate j of point p at
 *    X[j * n + p].
 *  - Matrices are column-major unless stated; "ld" arguments are leading
 *    dimensions in elements.
 *  - Working memory the library allocates (device and pinned host) is not
 *    returned to HIP when a call or a handle releases it: it goes to a pool
 *    of the calling thread and device, at most 1 GiB per kind, and later
 *    allocations on that thread take it from there.  A block is reused only
 *    after a device synchronisation, so work still queued on any stream can
 *    never see it change.  An allocation that fails first frees the pool's
 *    idle blocks and retries.
 */
#ifndef TT_KERNEL_H
#define TT_KERNEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tt_kernel* tt_kernel_t;

typedef enum {
  TTK_OK = 0,
  TTK_WARN_NOT_CONVERGED = 1,   /* cross stopped by a cap with sampled error > tol */
  TTK_ERR_ARG = -1,             /* invalid argument (sizes, pointers, ranges)     */
  TTK_ERR_HIP = -2,             /* a HIP runtime call failed                      */
  TTK_ERR_OOM = -3,             /* device or host allocation failed               */
  TTK_ERR_SINGULAR_CROSS = -4,  /* an intersection matrix of the cross is singular */
  TTK_ERR_UNSUPPORTED = -5      /* combination not implemented                    */
} tt_status;

/* Kernel functions of Table 1 (r = ||x - y||_2), plus two test kernels.
 * Parameter vector theta, in this order:                                     */
typedef enum {
  TTK_SE = 1,           /* exp(-(r/l)^2)                         theta = (l)     */
  TTK_EXPONENTIAL = 2,  /* exp(-r/l)                             theta = (l)     */
  TTK_MATERN32 = 3,     /* (1 + a) e^-a,  a = sqrt(3) r / l      theta = (l)     */
  TTK_MATERN52 = 4,     /* (1 + a + a^2/3) e^-a, a = sqrt(5) r/l theta = (l)     */
  TTK_MATERN_NU = 5,    /* Matern with fixed nu = kernel_const   theta = (l)     */
  TTK_MATERN = 6,       /* 2^(1-nu)/Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / l,
                           kappa(0) = 1                          theta = (l, nu) */
  TTK_MULTIQUADRIC = 7, /* sqrt(1 + (r/l)^2)                     theta = (l)     */
  TTK_TPS = 8,          /* (r/l)^2 log((r/l)^2), 0 at r = 0      theta = (l)     */
  TTK_LAPLACE3D = 9,    /* 1/r                                   no theta        */
  TTK_LAPLACE2D = 10,   /* -log r                                no theta        */
  TTK_BIHARMONIC = 11,  /* r^-2                                  no theta        */
  TTK_THINPLATE = 12,   /* r^2 log r                             no theta        */
  TTK_TEST_POLY = 13,   /* (1 + theta x.y)^3 (test only)         theta = (t)     */
  TTK_TEST_SEP = 14     /* exp(sum x) theta exp(-sum y) (test)   theta = (t)     */
} tt_kernel_kind;

typedef enum { TTK_FP64 = 0, TTK_FP32 = 1 } tt_dtype;

/* Build parameters (inputs of the offline stage, Algorithm 2). */
typedef struct {
  int d;                 /* spatial dimension, 1..3                                  */
  int d_theta;           /* parameter dimension, 0..2: the kind's parameter count, or
                            0 with theta_fixed (non-parametric TTK)                 */
  int n_spatial;         /* Chebyshev nodes per spatial dimension, 2..32             */
  int n_param;           /* Chebyshev nodes per parameter dimension, 2..32           */
  int kind;              /* tt_kernel_kind                                           */
  double kernel_const;   /* nu for TTK_MATERN_NU, unused otherwise                   */
  double box_s[6];       /* source box [alpha_1, beta_1, ..., alpha_d, beta_d]       */
  double box_t[6];       /* target box, same layout                                  */
  double box_theta[4];   /* parameter box [alpha_1, beta_1, alpha_2, beta_2]         */
  double tol;            /* tolerance of the cross (sampled relative Chebyshev-norm
                            error) and of the rounding of its cores                  */
  int max_rank;          /* cap on every TT rank of the cross (<= 256)               */
  int max_sweeps;        /* cap on cross sweeps                                      */
  int init_card;         /* 1 or 2: cardinality of the initial index sets (App. B)   */
  int init_max_it;       /* iterations of the index initialisation (App. B uses 10)  */
  int n_test;            /* multi-indices of the sampled stopping test (0 = default
                            max(1000, 20 D n))                                       */
  uint64_t seed;         /* key of every random draw of the cross                    */
  int dtype;             /* tt_dtype of U, V, M and the apply                        */
  int symmetric_psd;     /* 1 = PTTK-Global-1 (Algorithm 4), X = Y and box_t = box_s,
                            and the build also computes the thin QR [U V] = Q R      */
  double theta_fixed[2]; /* d_theta = 0 for a kind that has parameters: the
                            non-parametric TTK method (Section 4.1, H = I) for the
                            kernel at theta = theta_fixed (e.g. l = 1, or (l, nu)
                            for TTK_MATERN); every value must be positive.
                            Ignored when d_theta equals the kind's parameter count */
} tt_kernel_params;

typedef struct {
  int D;                       /* 2 d + d_theta                                      */
  int r_s, r_t;                /* columns of U and V (ranks r_d and r_{d+d_theta})   */
  int ranks[9];                /* ranks r_0..r_D of the rounded cores                */
  int cross_ranks[9];          /* ranks of the cross before rounding                 */
  int64_t kernel_evals;        /* kernel evaluations made on the device by the build */
  int sweeps;                  /* cross sweeps made                                  */
  int n_decisions;             /* update-cross steps logged                          */
  double sampled_error;        /* final sampled relative Chebyshev-norm error        */
  double init_max_cond;        /* max condition number of the chosen initial sets    */
  double min_margin;           /* smallest relative top-2 margin of a pivot decision */
  double t_cross_ms, t_round_ms, t_factor_ms;   /* build phase timings             */
  int64_t n_src, n_tgt;
  int dtype;
} tt_kernel_info;

/* One decision of the update cross step (Algorithm 5), for parity checks. */
typedef struct {
  int sweep, k;              /* sweep (0-based) and super-core k (1..D-1)             */
  int rank_before;           /* |I^{<=k}| before the step                             */
  int64_t sample_pos;        /* chosen sample, linear position row * cols + col        */
  int bit;                   /* random bit: 1 = row search, 0 = column search          */
  int pivot_row, pivot_col;  /* final pivot position in the super-core unfolding       */
  int added;                 /* 1 if (row, col) was appended to (I^{<=k}, I^{>k})      */
  double sample_max, sample_margin, pivot_abs, search_margin, tau;
} tt_kernel_decision;

/* Offline stage (Algorithm 2 with a rounding step on the small cores):
 *  1. Chebyshev grid of every dimension (Section 2.4),
 *  2. TT greedy-cross on f_kappa(x, theta, y) over the grid (Algorithms 5-7,
 *     interpolation formula of Appendix A), kernel entries evaluated on the
 *     device in double precision,
 *  3. TT-Round (Algorithm 1) of the cross cores at tol, orthogonalisation so
 *     that source cores are left- and target cores right-orthonormal, and the
 *     change of the spatial cores to the Chebyshev coefficient basis,
 *  4. Phase 3 (Algorithm 2): U = S and V = T by contracting each point's
 *     Chebyshev values through the spatial cores.
 * X: device, dtype, SoA d x n_src, points inside box_s.  Y: device, dtype,
 * SoA d x n_tgt, inside box_t.  Points outside their box are an error of the
 * caller (the result is then an extrapolation).  Synchronises `stream`.
 * On success *out receives a new handle owning U, V, the cores and the
 * cross record; TTK_WARN_NOT_CONVERGED also returns a usable handle. */
tt_status tt_kernel_build_offline(const tt_kernel_params* p,
                                  const void* X, int64_t n_src,
                                  const void* Y, int64_t n_tgt,
                                  void* stream, tt_kernel_t* out);

/* Same as tt_kernel_build_offline but skips steps 2-3: the nodal TT cores
 * G_1..G_D (Section 2.3) are given on the host in double precision,
 * concatenated, core k stored as G_k[a, i, b] at a + i r_{k-1} + b r_{k-1} n_k
 * (the little-endian layout of Section 2.2); ranks[0..D] with r_0 = r_D = 1.
 * They must already be gauge-fixed as the caller wants them.  Used to restore
 * a stored offline stage and to test Phase 3 on given cores. */
tt_status tt_kernel_build_from_cores(const tt_kernel_params* p, const int* ranks,
                                     const double* cores,
                                     const void* X, int64_t n_src,
                                     const void* Y, int64_t n_tgt,
                                     void* stream, tt_kernel_t* out);

/* Phase 3 alone (Algorithm 2, Phase 3) for other points of the same boxes:
 * side 0 gives rows of U for n points in box_s, side 1 rows of V for n points
 * in box_t (the offline stage does not depend on the points beyond their
 * boxes; Section 4.1 notes the case of points that move inside fixed boxes).
 * P: device, dtype, SoA d x n.  out: device, dtype, n x r row-major
 * (r = r_s or r_t).  One kernel launch on `stream`. */
tt_status tt_kernel_factor_rows(tt_kernel_t h, int side, const void* P, int64_t n, void* out,
                                void* stream);

/* Online stage (Algorithm 3): M(theta_b) = H_1(theta_b1) ... H_dt(theta_bdt)
 * with H_j = G_{d+j} x_2 q^p_j(theta_bj), for b = 0..B-1.
 * theta: device, dtype, B x d_theta row-major.  M_out: device, dtype,
 * B x r_s x r_t, matrix b column-major at M_out + b r_s r_t.  dM_out: NULL or
 * device, dtype, B x d_theta x r_s x r_t: dM(theta_b)/dtheta_j, obtained by
 * replacing q^p_j with its derivative (the differentiated Chebyshev series).
 * theta outside box_theta extrapolates.  For d_theta = 0, M = I. */
tt_status tt_kernel_online_core(tt_kernel_t h, const void* theta, int B,
                                void* M_out, void* dM_out, void* stream);

/* Apply: y_b = U M(theta_b) V^T x_b for b = 0..B-1 (the low-rank form of
 * Section 1, used as a matrix in outer loops).  X: device, dtype, n_tgt x B
 * column-major with leading dimension ldx >= n_tgt.  Y: device, dtype, n_src x B,
 * ldy >= n_src.  W_save: NULL or device, dtype, r_t x B (column-major):
 * receives W = V^T X for a later backward call.  B = 1 runs the plain
 * two-pass form; B > 1 the batched form (one pass over V and U for all b). */
tt_status tt_kernel_apply(tt_kernel_t h, const void* theta, int B,
                          const void* X, int64_t ldx, void* Y, int64_t ldy,
                          void* W_save, void* stream);

/* The batched apply of tt_kernel_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation).  Same arguments, kernels and result; the working
 * memory (M(theta_b), W, Z, the partial sums of the reduction over points and
 * the online-core workspace) is carved from a fixed scratch array of 64 MiB
 * that the library holds on every device it runs on until the process ends;
 * its address is looked up on the first call on a device.  Nothing is
 * allocated, by the library or through any other library.  A call whose
 * working memory exceeds the scratch returns TTK_ERR_ARG (naming the bytes
 * needed) before launching anything: roughly B * (r_s r_t * sizeof(dtype)
 * + 2 * (r_d r_m + r_m r_t) * 8) bytes plus the partial sums, so at ranks
 * near 75 a call takes a few hundred thetas; split larger batches.  All calls
 * on one device share the scratch: calls that overlap in time on one device
 * (on different streams or host threads) race and must not be issued. */
tt_status tt_kernel_apply_noalloc(tt_kernel_t h, const void* theta, int B,
                                  const void* X, int64_t ldx, void* Y, int64_t ldy,
                                  void* W_save, void* stream);

/* Projection onto the factor basis, the first contraction of the apply and
 * of its backward pass (T^T x and S^T g in the low-rank form of Section 1):
 * W = U^T X (side 0, X: n_src x B) or W = V^T X (side 1, X: n_tgt x B).
 * X: device, dtype, column-major, ldx >= the side's point count.  W: device,
 * dtype, r x B column-major (r = r_s or r_t).  Sums over points are formed
 * per point chunk and added in a fixed order (deterministic). */
tt_status tt_kernel_project(tt_kernel_t h, int side, const void* X, int64_t ldx, int B, void* W, void* stream);

/* Plain per-theta apply for all b: B independent two-pass applies (reads V and
 * U once per theta).  The reference point for the batched form. */
tt_status tt_kernel_apply_plain(tt_kernel_t h, const void* theta, int B,
                                const void* X, int64_t ldx, void* Y, int64_t ldy,
                                void* stream);

/* Backward of L = sum_b <g_b, y_b> for y_b as in tt_kernel_apply:
 *   dX[:, b]      = V M(theta_b)^T U^T g_b
 *   dtheta[b, j]  = (U^T g_b)^T dM(theta_b)/dtheta_j (V^T x_b)
 * G: device, dtype, n_src x B (ldg).  X: as in apply (used only when W_saved
 * is NULL).  W_saved: NULL or the W_save of the forward call.  dX: NULL or
 * device n_tgt x B (lddx).  dtheta: NULL or device, dtype, B x d_theta
 * row-major.  Exact derivatives of the approximation (not of kappa). */
tt_status tt_kernel_apply_backward(tt_kernel_t h, const void* theta, int B,
                                   const void* X, int64_t ldx, const void* W_saved,
                                   const void* G, int64_t ldg,
                                   void* dX, int64_t lddx, void* dtheta, void* stream);

/* PTTK-Global-1, online part (Algorithm 4, Section 3.5), for a handle built
 * with symmetric_psd = 1 (the build computed [U V] = Q R, Q: N x k with
 * orthonormal columns, R: k x k upper triangular, k = r_s + r_t, by blocked
 * Householder QR in double precision).  For each theta_b:
 *   Hhat_b = [[0, M_b / 2], [M_b^T / 2, 0]]  (M_b = M(theta_b), Algorithm 3),
 *   R Hhat_b R^T = U_b Lambda_b U_b^T,  W_b = U_b max(Lambda_b, 0) U_b^T,
 * so that Q W_b Q^T is the nearest (in the Frobenius norm) positive
 * semidefinite matrix to the symmetric part of U M_b V^T restricted to the
 * range of Q.  Computed in double precision (one-sided Jacobi SVD of the
 * symmetric k x k matrix: |.| of a symmetric matrix is V Sigma V^T).
 * theta: device, dtype, B x d_theta row-major.  W_out: device, dtype,
 * B x k x k, matrix b column-major at W_out + b k k. */
tt_status tt_kernel_global_online(tt_kernel_t h, const void* theta, int B, void* W_out, void* stream);

/* Global-1 apply y_b = Q W_b Q^T x_b (N x N, symmetric PSD).  Exactly one of
 * theta (device, B x d_theta: W is formed as in tt_kernel_global_online) and
 * W (device, dtype, B x k x k from tt_kernel_global_online) is non-NULL.
 * X, Y: device, dtype, N x B column-major, ldx, ldy >= N. */
tt_status tt_kernel_global_apply(tt_kernel_t h, const void* theta, const void* W, int B,
                                 const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream);

/* Phase 4 of Algorithm 2: TT-Round (Algorithm 1, tolerance eps) of the TT
 * [T^(1)(S), G_{d+1}, ..., G_{d+d_theta}, T^(3)(T^T)] whose outer cores hold
 * the factor matrices S = U and T = V of the points.  With S = Q_S R_S and
 * T = Q_T R_T (tall-skinny QR, float64), rounding that TT is rounding the
 * small TT [R_S, G_{d+1}, ..., R_T^T] and multiplying Q_S and Q_T back in,
 * since Q_S and Q_T have orthonormal columns; the handle then holds the
 * rounded U (N_s x r_s'), V (N_t x r_t') and parameter cores, and every
 * online call and apply uses them.  The spatial cores no longer describe U
 * and V afterwards: tt_kernel_factor_rows, tt_kernel_get_cores and
 * tt_kernel_get_coeff_cores return TTK_ERR_UNSUPPORTED.  Synchronises
 * `stream`.  TTK_ERR_ARG: eps <= 0 or a Global-1 handle;
 * TTK_ERR_UNSUPPORTED: r_s or r_t above 128, or fewer points than columns. */
tt_status tt_kernel_phase4_round(tt_kernel_t h, double eps, void* stream);

/* PTTK-Global-2: Algorithm 4 with Compress = true, for one theta.  The
 * positive eigenpairs of R Hhat R^T (Hhat as for Global-1), in decreasing
 * order of eigenvalue, are kept up to the smallest r_c whose discarded tail
 * sqrt(sum_{i > r_c} lambda_i^2) is at most eps ||R Hhat R^T||_F (the
 * Frobenius norm of the symmetric part of S H(theta) T^T, Q being
 * orthonormal); then Z = Q Uhat (the O(N r^2) product of the Compress
 * branch), so that K(X, X; theta) ~ Z diag(lambda) Z^T.
 * theta: device, dtype, d_theta values (NULL if d_theta = 0).  Z_out:
 * device, dtype, N x r_c row-major with leading dimension ldz >= r_s + r_t
 * (the caller sizes it for the largest r_c, r_s + r_t).  lam_out: device,
 * dtype, r_s + r_t values (the first r_c written).  *rc: host, r_c (0 if no
 * eigenvalue is positive).  Synchronises `stream` (r_c is decided on the
 * host).  TTK_ERR_ARG: not a Global handle, eps <= 0, a NULL output or
 * ldz < r_s + r_t. */
tt_status tt_kernel_global2_online(tt_kernel_t h, const void* theta, double eps, void* Z_out, int64_t ldz,
                                   void* lam_out, int* rc, void* stream);

/* Global-2 apply y_b = Z diag(lam) Z^T x_b for the (Z, lam, r_c) of
 * tt_kernel_global2_online (one theta) and B right-hand sides.  Z: device,
 * dtype, N x rc row-major (ldz >= rc); lam: device, dtype, rc.  X, Y:
 * device, dtype, N x B column-major (ldx, ldy >= N).  rc = 0 gives Y = 0. */
tt_status tt_kernel_global2_apply(tt_kernel_t h, const void* Z, int64_t ldz, const void* lam, int rc, int B,
                                  const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream);

/* Global-1 factors: *k = r_s + r_t (k may be NULL); Q_out: NULL or device,
 * dtype, N x k row-major; R_out: NULL or host FP64 k x k column-major
 * (synchronises `stream` when given). */
tt_status tt_kernel_global_factors(tt_kernel_t h, int* k, void* Q_out, double* R_out, void* stream);

/* ------------------------------------------------------------------------
 * Interaction lists: many source/target box pairs at once (Section 1 names
 * the low-rank blocks of FMM / H-matrix forms as the use case).
 *
 * Pairs whose grid tensors coincide share one TT: every kernel of Table 1
 * depends on x and y only through r = ||x - y||_2, so a common translation,
 * reflection of an axis or permutation of the axes of both boxes leaves the
 * tensor unchanged up to reversing / permuting node indices.  A pair is
 * mapped to its canonical frame (axes sorted by (source side, target side,
 * |centre offset|), offsets made non-negative, source box at [0, side]);
 * pairs with equal canonical boxes form one class and one cross / rounding
 * is run per class.  The two test kernels get one class per pair.  Phase 3
 * then runs for the points of every pair, through its class cores with its
 * own axis order and orientation, in ONE persistent launch over a work list
 * of (pair, 64-point tile) items.
 */
typedef struct tt_kernel_batch* tt_kernel_batch_t;

typedef struct {
  double box_s[6];          /* source box [alpha_1, beta_1, ..., alpha_d, beta_d]    */
  double box_t[6];          /* target box, same layout                               */
  int64_t src_off, n_src;   /* sources of the pair: points src_off .. src_off+n_src-1 of X */
  int64_t tgt_off, n_tgt;   /* targets: points tgt_off .. tgt_off+n_tgt-1 of Y       */
} tt_kernel_pair;

typedef struct {
  int num_pairs, num_classes;
  int64_t kernel_evals;     /* device kernel evaluations of all class builds          */
  int64_t factor_rows;      /* sum over pairs of n_src + n_tgt                        */
  double t_cross_ms, t_round_ms, t_factor_ms;
  int factor_grid;          /* workgroups of the persistent Phase 3 launch (0 = one
                               per tile, or one launch per pair in double precision) */
  int reduce_rows;          /* rows per work item of the tall reductions (last apply) */
  int graph;                /* 1 if applies replay a captured HIP graph               */
} tt_kernel_batch_info;

/* Build a batch: p gives the kernel, the grid sizes, the tolerance and dtype
 * (its box_s / box_t are ignored).  pairs: host array of num_pairs >= 1.
 * X: device, dtype, SoA d x n_x (all source points), Y: device, dtype,
 * SoA d x n_y; each pair's points must lie in its boxes.  Synchronises
 * `stream`.  The Phase 3 launch shape (workgroups of the persistent launch)
 * is chosen by timing candidates on the device unless set by
 * tt_kernel_batch_configure before a refactor. */
tt_status tt_kernel_batch_build(const tt_kernel_params* p, const tt_kernel_pair* pairs, int num_pairs,
                                const void* X, int64_t n_x, const void* Y, int64_t n_y,
                                void* stream, tt_kernel_batch_t* out);

/* Overrides of the autotuned choices (0 = choose by timing): use_graph (1 =
 * capture the apply once per argument set and replay it, 0 = launch
 * directly), factor_grid (workgroups of the persistent Phase 3 launch, -1 =
 * one per tile), reduce_rows (rows per item of the tall reductions). */
tt_status tt_kernel_batch_configure(tt_kernel_batch_t b, int use_graph, int factor_grid, int reduce_rows);

/* Phase 3 again for new points with the same pair layout (same offsets and
 * counts, same boxes): one persistent launch on `stream`. */
tt_status tt_kernel_batch_factor(tt_kernel_batch_t b, const void* X, const void* Y, void* stream);

/* info: host.  class_of_pair: NULL or host int[num_pairs].  class_ranks:
 * NULL or host int[num_classes * 9] (ranks r_0..r_D of each class). */
tt_status tt_kernel_batch_get_info(tt_kernel_batch_t b, tt_kernel_batch_info* info, int* class_of_pair,
                                   int* class_ranks);

/* Borrowed handle of class c (owned by the batch: do not destroy).  It has
 * no points (n_src = n_tgt = 0); its cores, online core and cross record are
 * those of the class, in the canonical frame. */
tt_status tt_kernel_batch_get_class(tt_kernel_batch_t b, int c, tt_kernel_t* h);

/* Rows of U (n_src x r_s) and V (n_tgt x r_t) of one pair, row-major dtype,
 * into device buffers (either may be NULL). */
tt_status tt_kernel_batch_get_factors(tt_kernel_batch_t b, int pair, void* U_out, void* V_out, void* stream);

/* Apply over the list, for b = 0..B-1:
 *   Y[:, b] = sum_p E_p U_p M_c(p)(theta_b) V_p^T F_p^T X[:, b]
 * (E_p, F_p scatter / gather the pair's source / target rows; rows covered by
 * no pair are set to 0), and when G is not NULL the backward pass of
 * L = sum_b <g_b, y_b>:
 *   dX[:, b] = sum_p F_p V_p M_c^T U_p^T E_p^T G[:, b]   (dX may be NULL)
 *   dtheta[b, j] = sum_p (U_p^T g_pb)^T dM_c/dtheta_j (V_p^T x_pb)   (may be NULL)
 * theta: device, dtype, B x d_theta.  X: n_y x B (ldx), Y: n_x x B (ldy),
 * G: n_x x B (ldg), dX: n_y x B (lddx), dtheta: B x d_theta; all device,
 * dtype, column-major.  Every tall contraction is one launch over a work list
 * of (pair, row chunk, theta tile) items; the whole sequence is captured as a
 * HIP graph on the first call with a given argument set and replayed on
 * later calls with the same arguments.  Calls on one batch must not overlap. */
tt_status tt_kernel_batch_apply(tt_kernel_batch_t b, const void* theta, int B, const void* X, int64_t ldx,
                                void* Y, int64_t ldy, const void* G, int64_t ldg, void* dX, int64_t lddx,
                                void* dtheta, void* stream);

tt_status tt_kernel_batch_destroy(tt_kernel_batch_t b);

/* ------------------------------------------------------------------------
 * A parametric hierarchical matrix for K(X, X; theta) (Section 1: the
 * admissible blocks of fast multipole and hierarchical-matrix methods are the
 * separated boxes the method targets; the Conclusions name hierarchical
 * parametric approximations).  The root box (box_s of the parameters) is
 * refined uniformly to the leaf level L, the smallest level with at most
 * leaf_points points per leaf on average (L d <= 30).  At every level k >= 2
 * a cell's far blocks are its interaction list: the cells whose parents are
 * neighbours of its parent (or the parent itself) but which are not its own
 * neighbours (max_j |i_j - i'_j| >= 2).  Every far block is a pair of the
 * pair batch above (one TT per geometry class, Phase 3 for all pairs in one
 * launch, the apply as one captured graph); the blocks between neighbouring
 * leaves (a leaf with itself included) are summed directly on the device in
 * double precision.  Points are sorted by the Morton code of their leaf, so
 * every cell is one contiguous range of the sorted points.  Kernels that are
 * unbounded at r = 0 (Laplace 2-D/3-D, biharmonic, thin-plate) leave the
 * self terms i = j out. */
typedef struct tt_kernel_hmat* tt_kernel_hmat_t;

typedef struct {
  int levels;               /* leaf level L                                           */
  int num_classes;          /* TT builds (geometry classes) of the far blocks          */
  int64_t leaves, nonempty_leaves;
  int64_t far_pairs;        /* far blocks (interaction-list pairs over all levels)     */
  int64_t near_pairs;       /* (leaf, neighbouring leaf) blocks summed directly        */
  int64_t kernel_evals;     /* device kernel evaluations of the class builds           */
  double t_tree_ms, t_build_ms;
} tt_kernel_hmat_info;

/* p: kernel, grid sizes, tolerance, dtype; box_s = the root box (box_t is
 * ignored).  X: device, dtype, SoA d x N, inside the root box.  Synchronises
 * `stream`.  TTK_ERR_ARG: no points, leaf_points < 1, an empty root box or a
 * parameter error of the pair batch.  TTK_WARN_NOT_CONVERGED: the cross of at
 * least one geometry class stopped above tol; *out is set and usable. */
tt_status tt_kernel_hmat_build(const tt_kernel_params* p, const void* X, int64_t N, int leaf_points, void* stream,
                               tt_kernel_hmat_t* out);

/* Y[:, b] = H(theta_b) X[:, b] for b = 0..B-1: theta device, dtype,
 * B x d_theta; X, Y device, dtype, N x B column-major (ldx, ldy >= N), in the
 * order of the points given to the build. */
tt_status tt_kernel_hmat_apply(tt_kernel_hmat_t h, const void* theta, int B, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, void* stream);

tt_status tt_kernel_hmat_get_info(tt_kernel_hmat_t h, tt_kernel_hmat_info* info);

/* Host outputs, each NULL or sized from the info: far, 7 ints per far block
 * (level, source cell i_0 i_1 i_2, target cell i_0 i_1 i_2, unused
 * coordinates 0); near, 6 ints per near block (the two leaves); perm, N ints
 * (sorted position -> index of the point as given). */
tt_status tt_kernel_hmat_get_lists(tt_kernel_hmat_t h, int32_t* far, int32_t* near, int32_t* perm);

/* The pair batch of the far blocks (owned by the hierarchical matrix; NULL
 * when there is no far block). */
tt_status tt_kernel_hmat_get_batch(tt_kernel_hmat_t h, tt_kernel_batch_t* b);

tt_status tt_kernel_hmat_destroy(tt_kernel_hmat_t h);

/* f_kappa at P grid multi-indices (Section 2.4, entries of the grid tensor),
 * in double precision on the device.  idx: device int32, P x D row-major,
 * 0-based node indices in the (x, theta, y) order.  out: device double, P. */
tt_status tt_kernel_eval_entries(const tt_kernel_params* p, const int32_t* idx, int64_t P,
                                 double* out, void* stream);

/* Dense kernel block K(X, Y; theta)[i, j] (rows = sources, Section 1) in
 * precision `dtype` of p.  X: device SoA d x nx, Y: device SoA d x ny, theta:
 * host, d_theta values.  K: device, column-major nx x ny (ldk >= nx). */
tt_status tt_kernel_eval_dense(const tt_kernel_params* p, const void* X, int64_t nx,
                               const void* Y, int64_t ny, const double* theta,
                               void* K, int64_t ldk, void* stream);

/* Query.  Synchronous, host memory. */
tt_status tt_kernel_get_info(tt_kernel_t h, tt_kernel_info* info);

/* Copy U (n_src x r_s) and V (n_tgt x r_t), row-major dtype, into device
 * buffers (either may be NULL). */
tt_status tt_kernel_get_factors(tt_kernel_t h, void* U_out, void* V_out, void* stream);

/* Rounded, gauge-fixed nodal cores G_1..G_D in double precision, host, in
 * the layout of tt_kernel_build_from_cores; `capacity` doubles available. */
tt_status tt_kernel_get_cores(tt_kernel_t h, double* cores, int64_t capacity);

/* Coefficient-basis cores: the rounded cores after the change of basis of
 * mode 2 that turns the nodal (Lagrange) interpolant of Section 2.4 into a
 * sum of Chebyshev polynomials, Ghat_k[:, j, :] = sum_i C[j, i] G_k[:, i, :]
 * with C[j, i] = (c_j / n) T_j(zeta_i), c_0 = 1, c_j = 2 (regrouping the
 * basis polynomials of Lemma 1).  These are the cores Phase 3 and the online
 * stage contract.  Host, double precision, in the layout of
 * tt_kernel_get_cores; spatial cores of a TTK_FP32 handle are the float32
 * copies Phase 3 reads, widened.  Synchronous; `capacity` doubles available. */
tt_status tt_kernel_get_coeff_cores(tt_kernel_t h, double* cores, int64_t capacity);

/* Cross record: index sets I^{<=k} (k = 1..D-1) and I^{>k} as host int32
 * arrays.  left: capacity sum_k r_k k, rows of I^{<=k} concatenated for
 * k = 1..D-1, each row k indices.  right: same for I^{>k}, rows of D - k
 * indices.  decisions: up to max_decisions entries.  Any pointer may be NULL. */
tt_status tt_kernel_get_cross(tt_kernel_t h, int32_t* left, int32_t* right,
                              tt_kernel_decision* decisions, int max_decisions);

tt_status tt_kernel_destroy(tt_kernel_t h);

const char* tt_kernel_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_KERNEL_H */
