/*
 * feast.h -- C ABI of the MI355X (gfx950) oblique-projection FEAST path.
 *
 * The method (Yin, Chan, Yeung, arXiv:1404.1768) finds the eigenpairs of a
 * regular pencil  A x = lambda B x  (A, B complex n x n, non-Hermitian) whose
 * eigenvalues lie strictly inside a circle |z - gamma| < rho (Section 1).
 * Every iteration filters a block with a quadrature of the spectral projector
 * (eq. 8-4), which needs one shifted solve (z_j B - A) Y_j = B U_1 per node
 * (eq. 4-4), and extracts eigenpairs by oblique projection onto span(U) with
 * the test space B span(U) (eqs. 6-3-12 .. 7-10, Theorem 3.2); Algorithm 5
 * (GFEAST) iterates this with its three stopping rules.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex data are interleaved double complex {re, im} (feast_z), the
 *    memory layout of torch.complex128 / numpy.complex128.  The mixed form
 *    keeps its factors internally in complex64; no call takes complex64.
 *  - Matrices are ROW-MAJOR ("C order"): element (i, j) of an r x c matrix
 *    with leading dimension ld (ld >= c) is at index i*ld + j.
 *  - Pointers named dX are device pointers (HIP device memory on the current
 *    device); pointers named hX are host pointers.  The caller owns every
 *    buffer it passes; the library keeps no pointer after a call returns.
 *  - Cached factors: a plan (or batch) keeps the LU factors of its shifted
 *    matrices and reuses them on a later call only if A and B have the same
 *    content as when they were factored (Section 4.3 reuses the factors of
 *    the same shifted matrices).  Each call that may reuse them reads A and B
 *    once for a 64-bit content fingerprint (a position-keyed hash of every
 *    entry's bits; any single-entry change is always detected, several
 *    changes are missed with probability about 2^-64), so a different pencil
 *    placed at the same address, or A or B changed in place, is refactored.
 *    The fingerprint costs one read of A and B and a host wait for two words.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All device work of a plan is enqueued on its stream; entry points that
 *    return host data synchronise that stream before returning.
 *  - A plan is not re-entrant: one call at a time per plan.
 *  - Return value: FEAST_OK (0) on success, a positive status for a result
 *    that is returned with a warning, a negative code for a failure.  No C++
 *    exception crosses this interface.  Argument checks happen on the host
 *    before any device work, so they can be exercised without a GPU.
 */
#ifndef FEAST_MI355X_H
#define FEAST_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } feast_z;

typedef struct feast_plan feast_plan;

enum feast_status {
  FEAST_OK = 0,
  FEAST_SINGULAR = 1,          /* an exact zero pivot at some node (node/column in feast_last_error) */
  FEAST_REFINE_STAGNATED = 2,  /* mixed form: refinement did not reach its target at some node */
  FEAST_EINVAL = -1,           /* bad size, leading dimension, null pointer, contour or option */
  FEAST_EDEVICE = -2,          /* HIP runtime error */
  FEAST_ENOMEM = -3,           /* device or host allocation failed */
  FEAST_ENUMERIC = -4,         /* host reduced eigensolver or QR broke down */
  FEAST_ESCRATCH = -5          /* the request needs more than feast_zgetrs_batched_noalloc's
                                  fixed scratch memory */
};

enum feast_rule { FEAST_TRAPEZOID = 0, FEAST_GAUSS_LEGENDRE = 1 };
enum feast_prec { FEAST_FP64 = 0, FEAST_MIXED = 1 };

/* The circle Gamma = {|z - center| = radius} and its quadrature (eq. 8-4).
 * FEAST_TRAPEZOID: z_j = center + radius*exp(i*pi*(2j-1)/N), w_j = (z_j-center)/N.
 * FEAST_GAUSS_LEGENDRE: z_j = center + radius*exp(i*(1+t_j)*pi),
 *                       w_j = omega_j*(z_j-center)/2 with (t_j, omega_j) the
 *                       N-point Gauss-Legendre rule on [-1, 1]. */
typedef struct {
  feast_z center;
  double radius;       /* > 0 */
  int32_t nodes;       /* N >= 1 (N <= 1024) */
  int32_t rule;        /* enum feast_rule */
} feast_contour;

/* Options of Algorithm 5 and of the implementation. */
typedef struct {
  double eps;          /* convergence tolerance on e(k) = max r_i (default 1e-10) */
  double eta;          /* selection tolerance separating true from spurious pairs (default 1e-3) */
  int32_t max_iter;    /* iteration cap (default 20) */
  int32_t prec;        /* enum feast_prec (default FEAST_FP64) */
  double refine_tol;   /* mixed form: per-node normwise backward-error target of the
                          final filter (default 4*2^-53) */
  int32_t max_sweeps;  /* mixed form: refinement sweeps per filter at most (default 6) */
  int32_t nb;          /* LU panel width: 64 or 128, 0 = automatic (128) */
  int32_t profile;     /* 1: time the LU trailing-update GEMM launches with HIP events on
                          the plan's stream (reported in feast_info); default 0 */
  int32_t lookahead;   /* 1: factor the next panel on a second stream while the rest of the
                          trailing matrix is updated by persistent workgroups that leave
                          ahead_cus compute units free for it; 0: panels and updates in
                          sequence (default 0: at n = 4000 the overlap gains 1-2 % of the
                          factorisation, the persistent update being slower per flop) */
  int32_t update_tile; /* LU trailing-update tile: 0 = 64 x 64, 1 = 128 x 64 (default 0) */
  int32_t batch_update; /* batched form's trailing-update loop: 0 = from the tuned table
                           (with nb = 0 for the panel width too), 1 = four real products per
                           complex step, 2 = three products, operand-pipelined, 3 = four
                           products, operand-pipelined (default 0) */
  int32_t ahead_cus;   /* look-ahead: compute units left to the panel factorisation, 8 to 128
                          (0 = 32) */
  int32_t ahead_rows;  /* look-ahead: only steps whose trailing block has at most this many
                          rows look ahead, the others run in sequence (0 = 2048) */
} feast_opts;

/* Fill *o with the defaults listed above. */
void feast_opts_default(feast_opts *o);

/* Quadrature nodes and weights of eq. (8-4) (host only).  hz, hw: N entries each.
 * Returns FEAST_EINVAL for a null pointer or an invalid contour. */
int feast_nodes(const feast_contour *c, feast_z *hz, feast_z *hw);

/* Create a plan for order n and subspace size m (1 <= m <= n).  The plan owns
 * the device workspace and, after the first filter, the LU factors of every
 * shifted matrix z_j B - A (N n^2 complex entries: complex128 for FEAST_FP64,
 * complex64 for FEAST_MIXED), reused by every later filter as Section 4.3
 * allows.  *plan is set to NULL on failure. */
int feast_plan_create(feast_plan **plan, int64_t n, int64_t m, const feast_contour *c,
                      const feast_opts *o, void *stream);

/* Release the plan and all memory it owns.  NULL is accepted. */
int feast_plan_destroy(feast_plan *plan);

/* Drop the cached factors: the next call factors again whatever the
 * fingerprints say (a caller that wants to time the factorisation).  The
 * host ordering feast_solve_csr keeps for a sparsity pattern is not a factor
 * and stays (it is made again only for other patterns). */
int feast_plan_invalidate(feast_plan *plan);

/* The filter of eq. (8-4) applied to a block (Algorithm 5, filter step):
 *   U = sum_j w_j (z_j B - A)^{-1} B V,   V, U: n x m.
 * The first call (or the first after feast_plan_invalidate, or with a pencil
 * whose content differs from the cached one) factors every z_j B - A with
 * partial pivoting and caches the factors.
 * FEAST_MIXED factors in complex64 and refines every node solution in FP64
 * (residual B V - (z_j B - A) Y_j, correction with the complex64 factors,
 * FP64 update) until the backward-error target or max_sweeps.
 * dU must not overlap dA, dB or dV.  Returns FEAST_SINGULAR for an exact zero
 * pivot (the solution then holds non-finite values). */
int feast_filter(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                 int64_t ldb, const feast_z *dV, int64_t ldv, feast_z *dU, int64_t ldu);

/* Oblique projection (Algorithm 5: its QR steps and the reduced pencil; eqs. 6-3-13, 7-10):
 *   U = U_1 R_1 (QR),  B U_1 = U_2 R_2 (QR),
 *   At = U_2^* A U_1,  Bt = U_2^* B U_1   (m x m, written to host memory).
 * In: dU (n x m).  Out: dU overwritten by the orthonormal U_1; dAU1 = A U_1 and
 * dBU1 = B U_1 (n x m each, kept for the residuals and the next filter);
 * hAt, hBt (m x m, row-major, leading dimension m).  Synchronises the stream.
 * Returns FEAST_ENUMERIC if U is numerically rank deficient beyond what the
 * shifted Cholesky QR can repair. */
int feast_project(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                  int64_t ldb, feast_z *dU, int64_t ldu, feast_z *dAU1, int64_t ldau,
                  feast_z *dBU1, int64_t ldbu, feast_z *hAt, feast_z *hBt);

/* Bandwidth-bound kernels timed with opts.profile = 1 (feast_info.hbm[class]). */
enum feast_kclass {
  FEAST_K_SHIFT = 0,     /* z_j B - A for all nodes: reads A, B, writes N shifted matrices */
  FEAST_K_WSUM = 1,      /* U = sum_j w_j Y_j: reads N node blocks, writes U */
  FEAST_K_GATHER = 2,    /* row permutation of the right-hand sides for every node */
  FEAST_K_Z2C = 3,       /* complex128 -> complex64 right-hand sides (mixed form) */
  FEAST_K_C2Z = 4,       /* complex64 solutions -> complex128 (set or add; mixed form) */
  FEAST_K_FINGERPRINT = 5, /* content fingerprints of A and B (factor reuse check) */
  FEAST_K_CLASSES = 6
};
/* launches, summed event time and algorithmic HBM bytes (every operand byte
   read once and every result byte written once) of one kernel class */
typedef struct {
  int32_t launches;
  double ms;
  double bytes;
} feast_kprof;

/* Per-run record of Algorithm 5 (optional output of feast_solve). */
#define FEAST_MAX_HISTORY 64
typedef struct {
  int32_t iters;                       /* k at which the run stopped */
  int32_t filters;                     /* filter applications (the first is Search's) */
  int32_t count[FEAST_MAX_HISTORY];    /* c(k), k = 1..iters */
  double err[FEAST_MAX_HISTORY];       /* e(k) (+inf when c(k) = 0) */
  int32_t sweeps[FEAST_MAX_HISTORY];   /* mixed form: refinement sweeps of each filter */
  double t_factor_ms, t_filter_ms, t_project_ms, t_host_eig_ms, t_ritz_ms, t_total_ms;
  /* with opts.profile = 1: the trailing-update GEMMs A22 -= L21 U12 of the last
     factorisation -- number of launches, summed event time, and algorithmic
     flops (8 (n-k)^2 kb per matrix and step, complex multiply-add = 8 flops) */
  int32_t lu_gemm_launches;
  double lu_gemm_ms;
  double lu_gemm_flops;
  /* with opts.profile = 1: the bandwidth-bound kernels of this call, per class */
  feast_kprof hbm[FEAST_K_CLASSES];
  /* mixed form: ||d_1||_F / ||Y_0||_F of each filter's first FP64 correction
     (about the forward error of the complex64 solves, u32 cond(z_j B - A);
     0 for a filter without corrections) */
  double contraction[FEAST_MAX_HISTORY];
  /* feast_solve_csr: lower and upper bandwidth of the reordered pencil */
  int32_t band_kl, band_ku;
  /* mixed form: the filter (1-based count, as in sweeps[]) after which the
     solve switched to FP64 factors because that filter's contraction would
     need more than max_sweeps corrections (or was not finite); 0: no switch */
  int32_t fp64_fallback;
} feast_info;

/* GFEAST (Algorithm 5) with the subspace size fixed to m and a caller-supplied
 * start block V in place of Search (the Search call becomes one filter
 * application of V followed by QR):
 *   outputs: *s_found selected eigenpairs; hLambda[0..s_found) their eigenvalues
 *   (host, capacity m); dX columns 0..s_found-1 their eigenvectors (device,
 *   n x m, unit 2-norm, largest-modulus entry real positive); hRes[0..s_found)
 *   their residuals r_i of eq. (5-1) (host, capacity m, may be NULL);
 *   *err = Err; *flag = 1 (converged), 0 (no improvement, previous iterate
 *   returned), -1 (iteration cap reached); info (may be NULL) the per-iteration record.
 * Selection: |lambda - center| < radius and r_i < eta; when nothing is
 * selected e(k) = +inf and the two count-based stops are skipped.  Mixed plans apply
 * fixed FP64 refinement sweeps per filter (the accuracy is judged by e(k)):
 * none on the first filter, one on later filters; once an iteration with a
 * settled count misses eps without at least halving e(k), every later filter
 * refines each node until its normwise backward error reaches refine_tol (at
 * most max_sweeps; a filter already launched is refined further from its
 * node solutions).  In the mixed form the no-improvement stop (flag 0) is
 * taken only once that verified refinement is on: an earlier rise of e(k)
 * switches it on and the iteration continues (the rise can come from the
 * complex64 solves rather than from the subspace).  When a refined filter's
 * contraction rho = ||d_1|| / ||Y_0|| is not finite, or so slow that
 * rho^(s+1) <= eps / 10 needs s > max_sweeps corrections, the solve refactors
 * every node in FP64, repeats that filter and finishes in FP64
 * (info->fp64_fallback); the plan is left unfactored in its mixed precision.
 * Synchronises the stream. */
int feast_solve(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                int64_t ldb, const feast_z *dV, int64_t ldv, feast_z *hLambda,
                feast_z *dX, int64_t ldx, double *hRes, int32_t *s_found, double *err,
                int32_t *flag, feast_info *info);

/* ---------------------------------------------------------------------------
 * Sparse pencils (the problems of Table 1 are sparse): A and B in compressed
 * sparse row form, factored as band matrices
 * ------------------------------------------------------------------------- */

/* An n x n sparse matrix in CSR form, every array on the device: row i's
 * entries are col[rowptr[i] .. rowptr[i+1]) with values val[...] (complex128).
 * Columns within a row in any order, each at most once; rowptr[0] = 0 and
 * rowptr[n] = nnz < 2^31. */
typedef struct feast_csr {
  int64_t n;
  int64_t nnz;
  const int32_t *rowptr;  /* n + 1 entries */
  const int32_t *col;     /* nnz entries, 0 <= col < n */
  const feast_z *val;     /* nnz entries */
} feast_csr;

/* GFEAST (Algorithm 5) as feast_solve, for a pencil given in CSR form.  The
 * shifted systems of eq. (4-4) are the same; their storage and factorisation
 * differ: the host orders the rows and columns of the union pattern of A and B
 * (from its pattern only) by reverse Cuthill-McKee, or keeps the natural order
 * where that is at least as narrow, and every node's z_j B - A
 * in that order is factored on the device as a band matrix with partial
 * pivoting (row interchanges within the kl subdiagonals, U widened to kl + ku
 * superdiagonals); the filter's node solves are band triangular solves, and
 * B V, A U_1, B U_1 are sparse x dense products.  Eigenvalues, residuals and
 * eigenvectors (in the caller's row order) are those of the dense pencil.
 * Outputs and stopping rules as feast_solve; info->band_kl/band_ku report the
 * bandwidths and info->t_factor_ms includes the host's symbolic work (pattern
 * copies, ordering).  The ordering is kept in the plan: a later call whose A
 * and B have the same patterns (rowptr and col equal entry by entry) reuses
 * it and skips that work; the values are gathered and the band factors
 * recomputed on every call.
 * Errors: FEAST_EINVAL for a mixed plan (band factors are FP64 only), a
 * malformed pattern (message names the fault), or kl + ku > 63 after
 * reordering (the band kernels keep a column's or a right-hand side's window
 * in registers; such a pencil is factored densely by feast_solve);
 * FEAST_SINGULAR for an exact zero pivot.
 * Synchronises the stream. */
int feast_solve_csr(feast_plan *plan, const feast_csr *A, const feast_csr *B,
                    const feast_z *dV, int64_t ldv, feast_z *hLambda, feast_z *dX,
                    int64_t ldx, double *hRes, int32_t *s_found, double *err,
                    int32_t *flag, feast_info *info);

/* Host only: the ordering feast_solve_csr uses, for one pattern (host arrays
 * rowptr[n + 1], col[rowptr[n]]): reverse Cuthill-McKee of the symmetrised
 * pattern (diagonal ignored), or the natural order where that is at least as
 * narrow; hperm[new] = old (n entries, caller-allocated) and the lower and
 * upper bandwidth of the pattern in that order.  FEAST_EINVAL for a malformed
 * pattern.  No device work. */
int feast_csr_order(int64_t n, const int32_t *hrowptr, const int32_t *hcol, int32_t *hperm,
                    int64_t *kl, int64_t *ku);

/* ---------------------------------------------------------------------------
 * Block_CIRR (Algorithm 1, Section 2): the paper's comparison method, on the
 * plan's cached factors
 * ------------------------------------------------------------------------- */

typedef struct feast_cirr_info {
  int64_t t;    /* columns of the moment block, h g */
  double ms;    /* wall time of the call */
} feast_cirr_info;

/* Algorithm 1 with the plan's contour and quadrature:
 *   moments: R_i = sum_j w_j mu_j^i (z_j B - A)^{-1} Y, i = 0..g-1, with the
 *           shifted, scaled powers mu_j = (z_j - center)/radius (the same span
 *           as z_j^i for i < g, better scaled) -- the quadrature of F_i Y of
 *           eq. (2-2-21);
 *   basis: an orthonormal basis U of span[R_0 .. R_{g-1}] (shifted Cholesky
 *           QR3; Rayleigh-Ritz depends on the span only, so this gives the
 *           eigenvalues of the SVD's left factor);
 *   reduced pencil: eigenpairs of (U^* A U, U^* B U) on the host (QZ);
 *   Ritz pairs: x_i = U y_i; selected: |lambda - center| < radius and
 *           r_i < eta (eq. 5-1), as in Algorithm 5's selection.
 * dY: device, n x h (leading dimension ldy >= h), the random block; h g <= m.
 * Outputs as feast_solve: hLambda/hRes (host, capacity m), dX (device n x m,
 * leading dimension ldx >= m), *s_found.  Mixed plans refine the node
 * solutions once in FP64.  There is no outer iteration: accuracy follows
 * the quadrature (outside eigenvalues leak in at 1/(1 + mu^N)).  Synchronises
 * the stream. */
int feast_cirr(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
               int64_t ldb, const feast_z *dY, int64_t ldy, int32_t h, int32_t g,
               feast_z *hLambda, feast_z *dX, int64_t ldx, double *hRes, int32_t *s_found,
               feast_cirr_info *info);

/* ---------------------------------------------------------------------------
 * Irregular contours (Section 4.3): eigenpairs inside a closed curve Gamma are
 * found by solving inside a circle that encloses Gamma and keeping those
 * inside Gamma.  Gamma is a closed polygon given by its vertices (host
 * array, either orientation, no repeated closing vertex).  Host only.
 * ------------------------------------------------------------------------- */

/* The smallest circle enclosing the nv >= 1 vertices (it encloses the
 * polygon), radius enlarged by the factor (1 + margin), margin >= 0: a margin
 * keeps eigenvalues near the vertices away from the circle, where the filter
 * value falls to 1/2.  FEAST_EINVAL for bad arguments or non-finite vertices. */
int feast_enclosing_circle(int32_t nv, const feast_z *vertices, double margin, feast_z *center,
                           double *radius);

/* inside[i] = 1 if lambda[i] lies inside the polygon (even-odd rule; a point on
 * an edge may be reported either way), else 0, for i < k.  nv >= 3. */
int feast_region_select(int32_t nv, const feast_z *vertices, int64_t k, const feast_z *lambda,
                        int32_t *inside);

/* ---------------------------------------------------------------------------
 * Search (Algorithm 4, Section 4.1): bounds the unknown count s of eigenvalues
 * inside the contour from above by t
 * ------------------------------------------------------------------------- */

typedef struct feast_search_info {
  int64_t t;        /* numerical rank of the last block: the upper bound of s */
  int64_t s0;       /* trace estimate ceil(Re trace(Y_0^* U) / p) */
  int64_t used;     /* columns of the random pool consumed */
  int32_t rounds;   /* rank-revealing tests performed */
  int32_t filters;  /* filter applications */
  double ms;        /* wall time of the call */
} feast_search_info;

/* Algorithm 4 on the plan's cached factors (factored first if needed):
 *   first sample: U = Q_N Y_0 for the first p columns Y_0 of the pool dY;
 *   trace estimate: s_0 = ceil(Re trace(Y_0^* U) / p),
 *     s_dagger = min(max(p, s_0), m);
 *   widening: U gets s_dagger - p more filtered columns from the pool, in order;
 *   rank test: rank-revealing step, t = numerical rank; if t < s_dagger stop, else U = U_1, p = t, s_dagger = min(ceil(alpha t), m) and repeat.
 * dY: device, n x ycols (leading dimension ldy >= ycols), entries N(0,1) drawn
 * by the caller (the paper's Y is real: pass zero imaginary parts); columns are
 * consumed left to right.  The numerical rank counts |R_jj| >= tau |R_00| of
 * the column-pivoted triangular factor (the paper names rank-revealing QR but
 * no threshold; tau = 1e-3 separates the filter's inside values near 1 from
 * outside values 1/(1 + mu^N)).  The rank-revealing step is the diagonally
 * pivoted Cholesky of the Gram matrix U^* U, which has the pivots and |R_jj|
 * of the column-pivoted QR of U; decisions at tau >> sqrt(eps) are unaffected
 * by squaring the condition number.
 * Output: dU1 (device, n x t, leading dimension ldu >= m) an orthonormal basis
 * of the t leading pivot columns (the first t columns of the QR's Q), and
 * *info.  The plan's m caps s_dagger: FEAST_EINVAL (with a message) when the
 * block is still of full rank at m columns, or when the pool runs out.
 * Mixed plans do not refine Search's filters.  Synchronises the stream. */
int feast_search(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                 int64_t ldb, const feast_z *dY, int64_t ldy, int64_t ycols, int32_t p,
                 double alpha, double tau, feast_z *dU1, int64_t ldu, feast_search_info *info);

/* Change the plan's subspace size to m (1 <= m <= n), keeping the cached
 * factors (they do not depend on m); workspaces grow as needed.  Used to run
 * Algorithm 5 with Search's t. */
int feast_plan_set_m(feast_plan *plan, int64_t m);

/* Algorithm 5 after its Search call, from Search's basis: dU1 (device, n x m,
 * leading dimension ldu >= m, orthonormal, already filtered) is Search's U_1; the
 * outputs are those of feast_solve (info->filters counts this call's filters
 * only). */
int feast_solve_from(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                     int64_t ldb, const feast_z *dU1, int64_t ldu, feast_z *hLambda,
                     feast_z *dX, int64_t ldx, double *hRes, int32_t *s_found, double *err,
                     int32_t *flag, feast_info *info);

/* ---------------------------------------------------------------------------
 * Adjoint form (derivatives of the eigenvalues found by feast_solve)
 * ------------------------------------------------------------------------- */

/* Left eigenvectors y_i (y_i^* A = lambda_i y_i^* B) of the s right eigenvectors
 * X (device, n x s) found inside the contour, from the adjoint of the filter of
 * eq. (8-4) on the plan's cached factors:
 *   W <- sum_j conj(w_j) (z_j B - A)^{-*} B^* W,  W_0 = X,   `sweeps` times.
 * That operator maps every left eigenvector y_k to conj(f(lambda_k)) y_k, so
 * each sweep damps the components outside the contour by the filter values
 * there (without the B^* the sweeps stall at about max|f| outside times the
 * departure of B from the identity).  Then Y = W (W^* B X)^{-*}, so that
 * Y^* B X = I (y_i^* B x_i = 1).
 * The (z_j B - A)^* solves reuse the forward factors: U^* first, then L^*, then
 * the transposed row permutation.  FP64 plans only.  dY: n x s (device).
 * Synchronises the stream. */
int feast_left_eigvecs(feast_plan *plan, const feast_z *dA, int64_t lda, const feast_z *dB,
                       int64_t ldb, const feast_z *dX, int64_t ldx, int64_t s, int32_t sweeps,
                       feast_z *dY, int64_t ldy);

/* Gradients of a real loss L of the eigenvalues lambda_i (first-order
 * perturbation: d lambda_i = y_i^* (dA - lambda_i dB) x_i with y_i^* B x_i = 1).
 * hG[i] = dL/d conj(lambda_i) in PyTorch's convention (for L = sum |lambda_i|^2,
 * hG[i] = 2 lambda_i).  Outputs (device, n x n, overwritten):
 *   dGA = sum_i hG[i] y_i x_i^*,   dGB = -sum_i hG[i] conj(lambda_i) y_i x_i^*.
 * Synchronises the stream. */
int feast_eig_grad(feast_plan *plan, const feast_z *dX, int64_t ldx, const feast_z *dY,
                   int64_t ldy, int64_t s, const feast_z *hLam, const feast_z *hG, feast_z *dGA,
                   int64_t ldga, feast_z *dGB, int64_t ldgb);

/* Message describing the last failure of this plan ("" if none). */
const char *feast_last_error(const feast_plan *plan);

/* ---------------------------------------------------------------------------
 * Batched form: many independent pencils of uneven order in lockstep
 * ------------------------------------------------------------------------- */

/* A batch of `count` independent pencils (A_p, B_p), p = 0..count-1, of orders
 * n[p] with subspace sizes m[p] and contours c[p] (every contour with the same
 * number of nodes N).  All count*N shifted matrices z_pj B_p - A_p are
 * factored together: each pencil is padded with an identity block to a
 * multiple of 64, the pencils are ordered by size so that the ones still
 * active at a panel step are a prefix, and every panel step, triangular solve
 * and trailing update is one grouped launch over all active pencils (the LU
 * factors are cached as in feast_filter, Section 4.3).  The device work of a
 * factorisation and of a filter is captured once in a HIP graph and replayed.
 * All pointer arguments of the batch calls below are HOST arrays of `count`
 * entries (device pointers or host buffers as stated), in the caller's order.
 * Options as for a plan.  The grouped LU's panel width (64 or 128) and its
 * trailing-update loop come from a table written by the project's autotuner
 * (timings of every candidate per order bucket and precision on an MI355X),
 * looked up with the order that splits the batch's LU work (sum of n_p^3) in
 * half; opts.nb = 64 or 128 and opts.batch_update = 1..3 override it.
 * The batch owns its device memory (factors, node solutions, workspaces) and a
 * page-locked host buffer of 2 sum_p m[p]^2 complex entries through which the
 * reduced pencils reach the host; feast_batch_destroy frees all of it.
 * Limits: 1 <= count <= 4096, 1 <= m[p] <= n[p] <= 16384. */
typedef struct feast_batch feast_batch;

typedef struct {
  int32_t iters;        /* largest iteration count over the pencils */
  int32_t filters;      /* grouped filters applied */
  int32_t graph_launches; /* HIP graph replays (factorisations + filters) */
  double t_factor_ms, t_filter_ms, t_project_ms, t_host_eig_ms, t_total_ms;
} feast_batch_info;

int feast_batch_create(feast_batch **batch, int32_t count, const int64_t *n, const int64_t *m,
                       const feast_contour *c, const feast_opts *o, void *stream);
int feast_batch_destroy(feast_batch *batch);
/* Drop the cached factors (the next call factors again). */
int feast_batch_invalidate(feast_batch *batch);
const char *feast_batch_last_error(const feast_batch *batch);

/* U_p = sum_j w_pj (z_pj B_p - A_p)^{-1} B_p V_p for every pencil (eqs. 8-4,
 * 4-4).  dA, dB: n x n, dV, dU: n x m (device, row-major, leading dimensions
 * in lda, ldb, ldv, ldu).  Mixed plans apply `sweeps` FP64 refinement
 * corrections per node (0 = the complex64 solve alone).  FEAST_SINGULAR when
 * an exact zero pivot occurs (pencil and node in feast_batch_last_error). */
int feast_batch_filter(feast_batch *batch, const feast_z *const *dA, const int64_t *lda,
                       const feast_z *const *dB, const int64_t *ldb, const feast_z *const *dV,
                       const int64_t *ldv, feast_z *const *dU, const int64_t *ldu,
                       int32_t sweeps);

/* Algorithm 5 for every pencil, as feast_solve, with the filters of all
 * pencils still iterating run as one grouped filter (pencils that have
 * stopped keep their result).  Per pencil p: hLambda[p] (host, >= m[p]
 * entries), dX[p] (device n x m, leading dimension ldx[p]), hRes[p] (host,
 * >= m[p], may be NULL as a whole array), s_found[p], err[p], flag[p],
 * iters[p] (host arrays of count entries).  Mixed plans refine with one
 * grouped sweep count: none on the first filter, one correction per node
 * afterwards, one more whenever a refined iteration of some pencil misses eps
 * without at least halving e(k) (at most max_sweeps); a rise of some pencil's
 * e(k) while the count is below max_sweeps also adds a sweep instead of
 * stopping that pencil with flag 0.  The second filter is
 * launched before the first iteration's host eigensolves (a pencil that stops
 * there has had it computed for nothing).
 * info may be NULL. */
int feast_batch_solve(feast_batch *batch, const feast_z *const *dA, const int64_t *lda,
                      const feast_z *const *dB, const int64_t *ldb, const feast_z *const *dV,
                      const int64_t *ldv, feast_z *const *hLambda, feast_z *const *dX,
                      const int64_t *ldx, double *const *hRes, int32_t *s_found, double *err,
                      int32_t *flag, int32_t *iters, feast_batch_info *info);

/* ---------------------------------------------------------------------------
 * Host-side pieces of Algorithm 5 (no device needed)
 * ------------------------------------------------------------------------- */

/* All eigenpairs of the t x t pencil At y = lambda Bt y (Algorithm 5, reduced eigenproblem;
 * the paper solves it with an xGGEV-type solver): complex QZ.  Inputs are
 * row-major with leading dimensions lda, ldb and are not modified.  Outputs:
 * halpha, hbeta (t each; lambda_i = alpha_i/beta_i, beta_i = 0 for an infinite
 * eigenvalue) and the right eigenvectors as the COLUMNS of hY (t x t,
 * row-major, leading dimension ldy, each of unit 2-norm).  Returns
 * FEAST_ENUMERIC if the QZ iteration does not converge. */
int feast_reduced_eig(int64_t t, const feast_z *hAt, int64_t lda, const feast_z *hBt,
                      int64_t ldb, feast_z *halpha, feast_z *hbeta, feast_z *hY, int64_t ldy);

/* Stopping rules of Algorithm 5 after iteration k.  Returns 1 (converged:
 * c(k) = c(k-1) and e(k) < eps), 0 (no improvement: c(k) = c(k-1) and
 * e(k) > e(k-1)), -1 (iteration cap: k = max_iter) or 2 (continue).  The two
 * count-based rules are skipped when c_k = 0; convergence is tested first. */
int feast_stop_rule(int32_t k, int32_t c_k, double e_k, int32_t c_prev, double e_prev,
                    double eps, int32_t max_iter);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points (the building blocks of the filter), batched over
 * `batch` independent problems with element strides between them.
 * ------------------------------------------------------------------------- */

/* In-place LU with partial pivoting of `batch` n x n row-major matrices:
 * P_b M_b = L_b U_b (L unit lower).  dPiv[b*n + i] is the 0-based row swapped
 * with row i at step i (LAPACK order).  dInfo[b] = 0, or 1 + the first column
 * with an exact zero pivot.  nb = panel width (64 or 128, 0 = automatic).  Synchronous
 * on `stream`.  The pivot test uses |re| + |im|, ties to the lowest row. */
int feast_zgetrf_batched(int64_t n, int32_t batch, feast_z *dM, int64_t ldm, int64_t strideM,
                         int32_t *dPiv, int32_t *dInfo, int32_t nb, void *stream);

/* Solve M_b X_b = R_b (trans = 0) or M_b^* X_b = R_b (trans = 2) in place in
 * dX (n x nrhs per problem) with the factors of feast_zgetrf_batched. */
int feast_zgetrs_batched(int64_t n, int64_t nrhs, int32_t batch, const feast_z *dLU,
                         int64_t ldm, int64_t strideM, const int32_t *dPiv, feast_z *dX,
                         int64_t ldx, int64_t strideX, int32_t trans, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the solves
 * of feast_zgetrs_batched (same arguments, same kernels, same results) with
 * every temporary (inverted 64 x 64 diagonal blocks of L and U, the row
 * permutation, a staging block: 2 batch ceil(n/64) 64^2 complex128 +
 * batch n int32 + batch n nrhs complex128 entries, each piece rounded up to
 * 256 bytes) in a fixed 64 MiB device array that the library holds on every
 * GPU it runs on until the process ends.  No device memory is allocated or
 * freed, and the call does not wait: the work is enqueued on `stream` and the
 * call returns (synchronise the stream, or capture it).  Requests needing
 * more than 64 MiB return FEAST_ESCRATCH before any device work.  Every call
 * on one GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other threads) race; calls ordered on one stream do not.  Nothing
 * in the array needs clearing between calls (every piece is written before
 * it is read). */
int feast_zgetrs_batched_noalloc(int64_t n, int64_t nrhs, int32_t batch, const feast_z *dLU,
                                 int64_t ldm, int64_t strideM, const int32_t *dPiv, feast_z *dX,
                                 int64_t ldx, int64_t strideX, int32_t trans, void *stream);

/* C_b = alpha op(A_b) B_b + beta C_b with op(A) = A (transA = 0, A is M x K)
 * or op(A) = A^* (transA = 2, A stored K x M); B is K x N, C is M x N.  The
 * FP64 MFMA complex GEMM used by every dense step of the path. */
int feast_zgemm_batched(int32_t transA, int64_t M, int64_t N, int64_t K, feast_z alpha,
                        const feast_z *dA, int64_t lda, int64_t strideA, const feast_z *dB,
                        int64_t ldb, int64_t strideB, feast_z beta, feast_z *dC, int64_t ldc,
                        int64_t strideC, int32_t batch, void *stream);

/* Library version (major*10000 + minor*100 + patch). */
int feast_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FEAST_MI355X_H */
