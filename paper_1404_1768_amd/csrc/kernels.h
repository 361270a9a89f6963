// Host-side launchers of the device kernels (all asynchronous on `s`).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.h"

namespace feast {

template <typename T> struct GemmArgs {
  int64_t M, N, K;
  const T *A;
  int64_t lda, sA;
  const T *B;
  int64_t ldb, sB;
  T *C;
  int64_t ldc, sC;
  z64 alpha, beta;
  int32_t batch;
  int32_t splits;
  int64_t kchunk;
  T *work;
  int64_t tile0;  // grouped launches: first linear tile of this problem
  // shifted-operand products only (left null otherwise): op(A_b) is
  // shift[b] A2 - A, and the accumulators start from C0 (+ b sC0) instead of C
  const T *A2;
  const z64 *shift;
  const T *C0;
  int64_t ldc0, sC0;
};

// Residuals of shifted systems in one launch: for b < batch,
//   C_b = R_b - (shift[b] A2 - A) Y_b
// with A, A2 (M x K, leading dimension lda, shared by all b), Y_b = Y + b sY
// (K x N, ldy), R_b = R + b sR (M x N, ldr) and C_b = C + b sC (ldc); shift
// is a device array of `batch` complex values.  The shifted matrix is formed
// tile by tile while it is staged, so the product costs one GEMM per b.
void zgemm_shift_residual(hipStream_t s, int64_t M, int64_t N, int64_t K, const z64 *A,
                          const z64 *A2, int64_t lda, const z64 *shift, const z64 *Y, int64_t ldy,
                          int64_t sY, const z64 *R, int64_t ldr, int64_t sR, z64 *C, int64_t ldc,
                          int64_t sC, int32_t batch);

// GEMM_UPDATE / GEMM_UPDATE_TALL: the 64 x 64 / 128 x 64 configurations under
// kernel names of their own (the LU trailing update); GEMM_SOLVE: C -= A B
// (no transpose) on the update's 64 x 64 tile under a third name (the
// triangular solves), other products as GEMM_SQUARE.
enum { GEMM_SQUARE = 0, GEMM_TALL = 1, GEMM_UPDATE = 3, GEMM_UPDATE_TALL = 4, GEMM_SOLVE = 5 };

// C_b = alpha op(A_b) B_b + beta C_b; transA 0: A is M x K; 2: A stored K x M, op = ^*.
// `work` (optional, work_elems entries) enables split-K for small outputs.
// GEMM_TALL uses 128-row tiles (needed for in-place products with M <= 128).
void zgemm(hipStream_t s, int transA, int64_t M, int64_t N, int64_t K, z64 alpha, const z64 *A,
           int64_t lda, int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 beta, z64 *C,
           int64_t ldc, int64_t sC, int32_t batch, z64 *work = nullptr, int64_t work_elems = 0,
           int cfg = GEMM_SQUARE);
void cgemm(hipStream_t s, int transA, int64_t M, int64_t N, int64_t K, z64 alpha, const c64 *A,
           int64_t lda, int64_t sA, const c64 *B, int64_t ldb, int64_t sB, z64 beta, c64 *C,
           int64_t ldc, int64_t sC, int32_t batch, c64 *work = nullptr, int64_t work_elems = 0,
           int cfg = GEMM_SQUARE);

// The LU trailing update C_b -= A_b B_b (row-major, batch strided, the tile of
// GEMM_UPDATE) on `wgs` persistent workgroups (rounded down to a multiple of
// 8, at least 8, at most what the tiles need), each of which takes a whole
// compute unit: the units beyond `wgs` stay free for work on other streams.
void zupdate_persistent(hipStream_t s, int64_t M, int64_t N, int64_t K, const z64 *A, int64_t lda,
                        int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 *C, int64_t ldc,
                        int64_t sC, int32_t batch, int wgs);
void cupdate_persistent(hipStream_t s, int64_t M, int64_t N, int64_t K, const c64 *A, int64_t lda,
                        int64_t sA, const c64 *B, int64_t ldb, int64_t sB, c64 *C, int64_t ldc,
                        int64_t sC, int32_t batch, int wgs);

// Grouped product: `count` independent problems (each a uniform batch, 64 x 64
// tiles, no split-K) in one launch.  gemm_group_tiles fills tile0 (and splits,
// kchunk) of a host table and returns the total tile count; the launch reads
// the table from device memory.  sub: every problem is C -= A B (alpha = -1,
// beta = 1); ta: 0 or 2 (2 only with sub = false).
//   variant (sub = true, ta = 0 only): GROUP_PLAIN (four real products per
//   complex step, unpipelined, BK = 16); GROUP_UPDATE_M3: the three-product,
//   operand-pipelined loop (BK = 8); GROUP_UPDATE_PIPE: four products on the
//   operand-pipelined loop.
enum { GROUP_PLAIN = 0, GROUP_UPDATE_M3 = 1, GROUP_UPDATE_PIPE = 2 };
template <typename T> int64_t gemm_group_tiles(GemmArgs<T> *tab, int count);
template <typename T>
void gemm_group(hipStream_t s, int ta, bool sub, const GemmArgs<T> *dtab, int count,
                int64_t total_tiles, int variant = GROUP_PLAIN);

// ---- LU building blocks (k_lu.hip); T = z64 or c64 --------------------------
//
// Every launcher below runs over a uniform batch (M + b * stride, order n) or,
// with grp != nullptr, over a grouped one (GrpMat, common.h): n is then the
// largest order (the stride of the flat pivot/info arrays) and each matrix
// reads its own order; matrices too small for the requested columns skip the
// launch.

// Factor columns [c0, c0+w) (rows [c0, n)) of each matrix with partial pivoting,
// swapping rows over the panel columns [pk0, pk0+pkb) as well.  Returns false
// if w is larger than the register-resident leaf supports for n - c0 rows.
template <typename T>
bool leaf_lu(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
             int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info,
             const GrpMat *grp = nullptr, int nodes = 1);
// Largest leaf width for `rows` remaining rows.
template <typename T> int leaf_max_width(int64_t rows);

// Whole LU with partial pivoting of `count` small matrices (grouped table,
// order n_b <= lu_small_max_order<T>(): 128 for complex64, 64 for complex128),
// each held in LDS by one workgroup of a persistent grid.  Pivots to
// ipiv + b pstride, info[b] as leaf_lu.
template <typename T> int lu_small_max_order();
template <typename T>
void lu_small(hipStream_t s, const GrpMat *grp, int nodes, int count, int64_t pstride,
              int32_t *ipiv, int32_t *info);

// Rows [r0, r0+kb) swapped with ipiv[r0..r0+kb) over columns [0, clo) and [chi, n).
template <typename T>
void laswp_outside(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                   int64_t r0, int kb, int64_t clo, int64_t chi, const int32_t *ipiv,
                   const GrpMat *grp = nullptr, int nodes = 1);

// X <- L11^{-1} X for the unit-lower L11 = M[c0:c0+w1, c0:c0+w1] and
// X = M[c0:c0+w1, c0+w1:c0+w1+w2] (w1, w2 <= 64).
template <typename T>
void trsm_small(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t c0,
                int w1, int w2);

// Both halves of one panel recursion step (w1, w2 <= panel_update_max_width()):
// X = L11^{-1} X as in trsm_small (one workgroup per matrix), then
// M[c0+w1:n, c0+w1:c0+w1+w2] -= M[c0+w1:n, c0:c0+w1] X (64-row chunks).
template <typename T>
void panel_update(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                  int64_t c0, int w1, int w2, const GrpMat *grp = nullptr, int nodes = 1);
int panel_update_max_width();

// Inverses of the diagonal blocks of the unit-lower L (lower=true) or of the
// upper U (lower=false) factor: block I covers rows/cols [I*nb, min(n,(I+1)*nb)).
// out[b][I] is an nb x nb row-major block (ld nb).  Blocks [blk0, blk1).
template <typename T>
void diag_block_inverse(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch,
                        int64_t n, int nb, int64_t blk0, int64_t blk1, bool lower, T *out,
                        int64_t out_stride, const GrpMat *grp = nullptr, int nodes = 1);

// Inverted 128-row diagonal blocks (row-major 128 x 128, istride2 apart per
// matrix) built from the inverted 64-row blocks of diag_block_inverse (nb = 64,
// istride apart) and the factor's off-diagonal 64 x 64 blocks.
template <typename T>
void inverse_pairs(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                   const T *inv64, int64_t istride, T *inv128, int64_t istride2, bool lower);

// perm[b][i] = original row at position i of P_b (from LAPACK-order ipiv).
void perm_from_ipiv(hipStream_t s, const int32_t *ipiv, int32_t *perm, int64_t n, int32_t batch,
                    const GrpMat *grp = nullptr, int nodes = 1);

// info[b] = min(info[b]) helper is inside leaf_lu; zero the array:
void fill_i32(hipStream_t s, int32_t *p, int64_t count, int32_t v);

// ---- grouped small-matrix kernels of the batched orthonormalisation ----------
// (k_misc.hip).  Entry b of each GrpMat array is one pencil's matrix: base,
// leading dimension ld, order n; `count` entries, one workgroup row each.

// G_b += shift_rel[b] * trace(G_b) * I (shift_rel: device array).
void add_shift_grp(hipStream_t s, const GrpMat *g, int count, const double *shift_rel);
// Zero the strict lower triangle (or all) of every n_b x n_b matrix (tmax = max n_b).
void zero_lower_grp(hipStream_t s, const GrpMat *g, int count, int64_t tmax, bool all);
// dst_b = src_b for src_b.n rows and dst_b.stride columns (max_elems = max rows*cols).
void copy_grp(hipStream_t s, const GrpMat *src, const GrpMat *dst, int count, int64_t max_elems);
// Cholesky of the diagonal 64 x 64 block at (J0, J0) of every matrix of a group
// and the inverse of its factor (k_chol_inv per matrix): R into the block, R^{-1}
// (upper triangle only) to Dinv + b * dstride + (J0 / 64) * 4096 (leading dimension 64).
void chol_inv_grp(hipStream_t s, const GrpMat *g, int count, int64_t J0, int32_t *flag,
                  int flag_stride, z64 *Dinv, int64_t dstride);
// Sum of split-K partials (k_sum_splits_grp): max_elems >= rows x cols of every dst.
void sum_splits_grp(hipStream_t s, const GrpMat *dst, const GrpMat *src, int count,
                    int64_t max_elems);
// Diagonal blocks I of Dinv + b * dstride (64 x 64 each) into X_b.
void put_diag_grp(hipStream_t s, const GrpMat *g, int count, int64_t nblk_max, const z64 *Dinv,
                  int64_t dstride);

// ---- element-wise and reduction kernels (k_misc.hip) ------------------------

// M_j = z_j B - A for every node j (out: N matrices n x n, ld ldm, stride sM).
void shift_assemble_z(hipStream_t s, const z64 *A, int64_t lda, const z64 *B, int64_t ldb,
                      const z64 *z, int32_t N, int64_t n, z64 *M, int64_t ldm, int64_t sM);
void shift_assemble_c(hipStream_t s, const z64 *A, int64_t lda, const z64 *B, int64_t ldb,
                      const z64 *z, int32_t N, int64_t n, c64 *M, int64_t ldm, int64_t sM);

// Y_b[i, :] = R_b[perm_b[i], :] for rows i < n, with R_b = R + b sR (sR = 0:
// one shared R) and perm_b = perm + b pstride (pstride 0: n).
template <typename T>
void gather_rows(hipStream_t s, const T *R, int64_t ldr, int64_t sR, const int32_t *perm,
                 int64_t n, int64_t m, int32_t batch, T *Y, int64_t ldy, int64_t sY,
                 int64_t pstride = 0);
// Ones on the diagonal of rows [n0, n) of `batch` matrices.
template <typename T>
void pad_diag(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n0,
              int64_t n);
// Y[perm_b[i], :] = X_b[i, :]  (scatter, used by the ^* solve).
template <typename T>
void scatter_rows(hipStream_t s, const T *X, int64_t ldx, int64_t sX, const int32_t *perm,
                  int64_t n, int64_t m, int32_t batch, T *Y, int64_t ldy, int64_t sY);

// U = sum_j w_j Y_j (fixed summation order; w on the device).
void weighted_sum(hipStream_t s, const z64 *Y, int64_t ldy, int64_t sY, const z64 *w,
                  int32_t N, int64_t n, int64_t m, z64 *U, int64_t ldu);

// Copy / convert blocks.  The conversions between complex128 and complex64
// optionally scale by a power of two: z_to_c writes X 2^-e, c_to_z and
// add_c_to_z read X 2^e, with e the binary exponent of sqrt(nrm2[0] / cnt)
// (nrm2 on the device: the squared Frobenius norm of the right-hand side,
// cnt its number of entries; nrm2 = nullptr: no scaling).
void copy_block_z(hipStream_t s, const z64 *X, int64_t ldx, int64_t n, int64_t m, z64 *Y,
                  int64_t ldy);
void z_to_c(hipStream_t s, const z64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
            int32_t batch, c64 *Y, int64_t ldy, int64_t sY, const double *nrm2 = nullptr,
            double cnt = 1.0);
// Y = X (complex64 -> complex128), per batch.
void c_to_z(hipStream_t s, const c64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
            int32_t batch, z64 *Y, int64_t ldy, int64_t sY, const double *nrm2 = nullptr,
            double cnt = 1.0);
// Refinement residual of all nodes in the n x (N m) layout:
// T1[:, j m + c] <- R[:, c] - z_j T2[:, j m + c] + T1[:, j m + c]   (T1 = A Y, T2 = B Y)
// for the used columns c < used (default m) of every node block.
void shift_residual(hipStream_t s, const z64 *R, int64_t ldr, z64 *T1, const z64 *T2,
                    int64_t ldt, const z64 *z, int32_t N, int64_t n, int64_t m,
                    int64_t used = -1);
// Y += X (complex64 correction into FP64 solution), per batch.
void add_c_to_z(hipStream_t s, const c64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
                int32_t batch, z64 *Y, int64_t ldy, int64_t sY, const double *nrm2 = nullptr,
                double cnt = 1.0);

// Residual norms of Ritz pairs: for every column i of the n x t blocks AX, BX:
// out[3i+0] = ||AX_i - lam_i BX_i||^2, out[3i+1] = ||AX_i||^2, out[3i+2] = ||BX_i||^2.
// part: workspace of ceil(n/64) * 3t doubles.
void ritz_norms(hipStream_t s, const z64 *AX, const z64 *BX, int64_t ld, int64_t n, int64_t t,
                const z64 *lam, double *part, double *out);

// Per-column squared norms of an n x t block into out[t]; part: ceil(n/64)*t doubles.
void col_norms2(hipStream_t s, const z64 *X, int64_t ld, int64_t n, int64_t t, double *part,
                double *out);

// Frobenius-norm-squared per batch: out[b] = sum |X_b|^2 (n x m blocks);
// part: workspace of max(64 * batch, 1024) doubles.
void fro2_batched(hipStream_t s, const z64 *X, int64_t ld, int64_t sX, int64_t n, int64_t m,
                  int32_t batch, double *part, double *out);
// out[0] = sum |X|^2 of one complex64 n x m block (accumulated in FP64);
// part: workspace of 1024 doubles.
void fro2_c(hipStream_t s, const c64 *X, int64_t ld, int64_t n, int64_t m, double *part,
            double *out);

// Content fingerprints of `count` n_b x n_b complex128 matrices (entry b of
// the device table tab, or a0 / a1 by value when tab is null and count <= 2)
// into out[b] (device, zeroed here first); nmax bounds every n_b.  Reading
// every entry once, it lets a cache of factors check that a matrix is unchanged.
void fingerprint(hipStream_t s, const GrpMat *tab, int count, GrpMat a0, GrpMat a1,
                 int64_t nmax, uint64_t *out);

// Blocked pieces: diagonal += shift_rel * trace; Cholesky of one jb x jb (<= 64)
// diagonal block inside a matrix of leading dimension ld, R written over it
// (strict lower part zeroed) and R^{-1} (jb x jb) to Rinv with leading
// dimension ldi (flag[0] = 1 + the first non-positive pivot column, numbered
// from col0); zero the strict lower triangle (or everything) of a t x t matrix.
void add_diag_shift(hipStream_t s, z64 *G, int64_t t, double shift_rel);
void chol_inv_block(hipStream_t s, z64 *G, int64_t ld, int jb, int col0, int32_t *flag, z64 *Rinv,
                    int64_t ldi);
void zero_lower(hipStream_t s, z64 *X, int64_t t, bool all);

// Gather columns idx[0..k) of the n x t block X into Y (n x k) and normalise each
// to unit 2-norm with its largest-modulus entry real positive.
void gather_normalize_cols(hipStream_t s, const z64 *X, int64_t ldx, int64_t n,
                           const int32_t *idx, int64_t k, z64 *Y, int64_t ldy, double *part);

// Adjoint helpers: broadcast an n x c block to the N node slots of an n x (N c)
// block; Y = X^* (rows x cols -> cols x rows); X[:, c] *= d[c]; t x t identity.
void bcast_cols(hipStream_t s, const z64 *X, int64_t ldx, int64_t n, int64_t c, int32_t N, z64 *Y,
                int64_t ldy);
void conj_transpose(hipStream_t s, const z64 *X, int64_t ldx, int64_t rows, int64_t cols, z64 *Y,
                    int64_t ldy);
void scale_cols(hipStream_t s, z64 *X, int64_t ldx, int64_t n, int64_t c, const z64 *d);
void identity(hipStream_t s, z64 *X, int64_t t);

// Sparse pencils in band form (k_band.hip).  A and B are values va, vb on one
// CSR pattern (rp, ci) whose entries lie within kl subdiagonals and ku
// superdiagonals; M_j = z_j B - A.
// Band LU with partial pivoting of every node (one workgroup each): Lf holds
// node j's multipliers of column k at (j n + k) kl + i - 1 (rows k + i), Uf
// its row k of U at (j n + k)(kl + ku + 1) + t (column k + t), Dinv the
// reciprocal of U's diagonal entry k at j n + k, piv the row exchanged with k,
// info the first zero-pivot column + 1 (0: none).
void band_lu(hipStream_t s, const int32_t *rp, const int32_t *ci, const z64 *va, const z64 *vb,
             const z64 *z, int32_t N, int64_t n, int kl, int ku, z64 *Lf, z64 *Uf, z64 *Dinv,
             int32_t *piv, int32_t *info);
// Y_j = M_j^{-1} R (R: n x m, ldr; node j's solution at Y + j sY, leading
// dimension ldy) with the band factors above.
void band_solve(hipStream_t s, const z64 *Lf, const z64 *Uf, const z64 *Dinv, const int32_t *piv,
                int32_t N, int64_t n, int kl, int ku, const z64 *R, int64_t ldr, int64_t m,
                z64 *Y, int64_t ldy, int64_t sY);
// YA = A X, YB = B X on the shared pattern (a null output is skipped).
void csr_spmm(hipStream_t s, const int32_t *rp, const int32_t *ci, const z64 *va, const z64 *vb,
              int64_t n, const z64 *X, int64_t ldx, int64_t m, z64 *YA, int64_t ldya, z64 *YB,
              int64_t ldyb);
// dst[e] = src[map[e]], zero where map[e] < 0.
void gather_vals(hipStream_t s, const int32_t *map, const z64 *src, int64_t cnt, z64 *dst);

}  // namespace feast
