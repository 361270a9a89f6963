// Bandwidth- and latency-bound kernels of the path: shifted-matrix assembly,
// pivot gathers, the weighted node sum, column norms for the Ritz residuals,
// and the small t x t kernels of the orthonormalisation.
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

// Row-wise element kernels: a workgroup of 256 threads is 4 waves, each wave
// one row; a wave's 64 lanes step through a slice of kRowSlice columns of its
// row, so consecutive lanes touch consecutive elements (coalesced 16-byte
// accesses for complex128) and no index is divided.  Grid: x = column slices,
// y = groups of 4 rows (rows strided by 4 gridDim.y beyond 65535 groups),
// z = batch.
constexpr int kRowSlice = 512;

inline dim3 rowwise_grid(int64_t rows, int64_t cols, int32_t batch) {
  const int64_t gy = std::min<int64_t>((rows + 3) / 4, 65535);
  return dim3(static_cast<unsigned>(std::max<int64_t>((cols + kRowSlice - 1) / kRowSlice, 1)),
              static_cast<unsigned>(std::max<int64_t>(gy, 1)),
              static_cast<unsigned>(std::max<int32_t>(batch, 1)));
}

#define ROWWISE_FOR(rows, cols, row, col)                                             \
  for (int64_t row = blockIdx.y * 4ll + (threadIdx.x >> 6); row < (rows);             \
       row += 4ll * gridDim.y)                                                         \
    for (int64_t col = blockIdx.x * static_cast<int64_t>(kRowSlice) + (threadIdx.x & 63), \
                 col##_end = std::min<int64_t>((blockIdx.x + 1ll) * kRowSlice, (cols));  \
         col < col##_end; col += 64)

// M_j = z_j B - A for all N nodes: A and B are read once, each element is
// written N times (the write of the N shifted matrices bounds this kernel).
template <typename T>
__global__ __launch_bounds__(256) void k_shift(const z64 *__restrict__ A, int64_t lda,
                                               const z64 *__restrict__ B, int64_t ldb,
                                               const z64 *__restrict__ z, int32_t N, int64_t n,
                                               T *__restrict__ M, int64_t ldm, int64_t sM) {
  const int64_t col = blockIdx.x * 256ll + threadIdx.x;
  const int64_t row = blockIdx.y;
  if (col >= n) return;
  const z64 a = A[row * lda + col], b = B[row * ldb + col];
  for (int j = 0; j < N; ++j) {
    const z64 zj = z[j];
    T v;
    v.x = static_cast<decltype(v.x)>(zj.x * b.x - zj.y * b.y - a.x);
    v.y = static_cast<decltype(v.y)>(zj.x * b.y + zj.y * b.x - a.y);
    M[j * sM + row * ldm + col] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const T *__restrict__ R, int64_t ldr,
                                                     int64_t sR, const int32_t *__restrict__ perm,
                                                     int64_t pstride, int64_t n, int64_t m,
                                                     T *__restrict__ Y, int64_t ldy, int64_t sY) {
  const int b = blockIdx.z;
  ROWWISE_FOR(n, m, row, c) {
    const int64_t src = perm[b * pstride + row];
    Y[b * sY + row * ldy + c] = R[b * sR + src * ldr + c];
  }
}

// T1 = R - z_j T2 + T1 on the used columns c < used of every node block j
// (node blocks m columns apart; R is shared, n x used).
__global__ __launch_bounds__(256) void k_shift_residual(const z64 *__restrict__ R, int64_t ldr,
                                                        z64 *__restrict__ T1,
                                                        const z64 *__restrict__ T2, int64_t ldt,
                                                        const z64 *__restrict__ z, int64_t n,
                                                        int64_t m, int64_t used, int32_t N) {
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  const int64_t cols = static_cast<int64_t>(N) * used;
  if (idx >= n * cols) return;
  const int64_t row = idx / cols, k = idx % cols;
  const int64_t j = k / used, c = k % used, col = j * m + c;
  const z64 zj = z[j], r = R[row * ldr + c], t2 = T2[row * ldt + col];
  z64 &t1 = T1[row * ldt + col];
  t1.x = r.x - (zj.x * t2.x - zj.y * t2.y) + t1.x;
  t1.y = r.y - (zj.x * t2.y + zj.y * t2.x) + t1.y;
}

// Power-of-two scaling of the complex64 solves in the mixed form: blocks are
// converted to complex64 as X 2^-e and back as Y 2^e, with e the binary
// exponent of the root mean square sqrt(nrm2[0] / cnt) of the right-hand side
// (e = 0 without nrm2, or for a zero or non-finite norm).  Multiplying by a
// power of two is exact in FP64 and leaves the complex64 rounding unchanged,
// but keeps right-hand sides and refinement residuals of badly scaled pencils
// inside complex64's exponent range (residuals shrink to about 1e-16 of the
// right-hand side, below complex64's smallest normal number for a right-hand
// side near 1e-25).
__device__ inline int solve_scale_exp(const double *nrm2, double cnt) {
  if (!nrm2) return 0;
  const double rms = sqrt(nrm2[0] / cnt);
  if (!(rms > 0.0) || !isfinite(rms)) return 0;
  return ilogb(rms);
}

__global__ __launch_bounds__(256) void k_c_to_z(const c64 *__restrict__ X, int64_t ldx, int64_t sX,
                                                int64_t n, int64_t m, z64 *__restrict__ Y,
                                                int64_t ldy, int64_t sY,
                                                const double *__restrict__ nrm2, double cnt) {
  const int b = blockIdx.z;
  const int e = solve_scale_exp(nrm2, cnt);
  ROWWISE_FOR(n, m, row, col) {
    const c64 v = X[b * sX + row * ldx + col];
    Y[b * sY + row * ldy + col] =
        make_double2(ldexp(static_cast<double>(v.x), e), ldexp(static_cast<double>(v.y), e));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_rows(const T *__restrict__ X, int64_t ldx,
                                                      int64_t sX, const int32_t *__restrict__ perm,
                                                      int64_t n, int64_t m, T *__restrict__ Y,
                                                      int64_t ldy, int64_t sY) {
  const int b = blockIdx.z;
  ROWWISE_FOR(n, m, row, c) {
    const int64_t dst = perm[b * n + row];
    Y[b * sY + dst * ldy + c] = X[b * sX + row * ldx + c];
  }
}

__global__ __launch_bounds__(256) void k_weighted_sum(const z64 *__restrict__ Y, int64_t ldy,
                                                      int64_t sY, const z64 *__restrict__ w,
                                                      int32_t N, int64_t n, int64_t m,
                                                      z64 *__restrict__ U, int64_t ldu) {
  ROWWISE_FOR(n, m, row, col) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < N; ++j) {
      const z64 y = Y[j * sY + row * ldy + col];
      const z64 wj = w[j];
      sr += wj.x * y.x - wj.y * y.y;
      si += wj.x * y.y + wj.y * y.x;
    }
    U[row * ldu + col] = make_double2(sr, si);
  }
}

__global__ __launch_bounds__(256) void k_copy_block(const z64 *__restrict__ X, int64_t ldx,
                                                    int64_t n, int64_t m, z64 *__restrict__ Y,
                                                    int64_t ldy) {
  ROWWISE_FOR(n, m, row, col) Y[row * ldy + col] = X[row * ldx + col];
}

__global__ __launch_bounds__(256) void k_z_to_c(const z64 *__restrict__ X, int64_t ldx, int64_t sX,
                                                int64_t n, int64_t m, c64 *__restrict__ Y,
                                                int64_t ldy, int64_t sY,
                                                const double *__restrict__ nrm2, double cnt) {
  const int b = blockIdx.z;
  const int e = solve_scale_exp(nrm2, cnt);
  ROWWISE_FOR(n, m, row, col) {
    const z64 v = X[b * sX + row * ldx + col];
    Y[b * sY + row * ldy + col] =
        make_float2(static_cast<float>(ldexp(v.x, -e)), static_cast<float>(ldexp(v.y, -e)));
  }
}

__global__ __launch_bounds__(256) void k_add_c_to_z(const c64 *__restrict__ X, int64_t ldx,
                                                    int64_t sX, int64_t n, int64_t m,
                                                    z64 *__restrict__ Y, int64_t ldy, int64_t sY,
                                                    const double *__restrict__ nrm2, double cnt) {
  const int b = blockIdx.z;
  const int e = solve_scale_exp(nrm2, cnt);
  ROWWISE_FOR(n, m, row, col) {
    const c64 v = X[b * sX + row * ldx + col];
    z64 &y = Y[b * sY + row * ldy + col];
    y.x += ldexp(static_cast<double>(v.x), e);
    y.y += ldexp(static_cast<double>(v.y), e);
  }
}

// Partial column sums over a chunk of 64 rows: one thread per column.
__global__ __launch_bounds__(256) void k_ritz_part(const z64 *__restrict__ AX,
                                                   const z64 *__restrict__ BX, int64_t ld,
                                                   int64_t n, int64_t t,
                                                   const z64 *__restrict__ lam,
                                                   double *__restrict__ part) {
  const int64_t chunk = blockIdx.x;
  const int64_t r0 = chunk * 64;
  const int64_t r1 = (r0 + 64 < n) ? r0 + 64 : n;
  for (int64_t c = threadIdx.x; c < t; c += 256) {
    const z64 l = lam[c];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const z64 ax = AX[r * ld + c], bx = BX[r * ld + c];
      const double dr = ax.x - (l.x * bx.x - l.y * bx.y);
      const double di = ax.y - (l.x * bx.y + l.y * bx.x);
      s0 += dr * dr + di * di;
      s1 += ax.x * ax.x + ax.y * ax.y;
      s2 += bx.x * bx.x + bx.y * bx.y;
    }
    part[(chunk * t + c) * 3 + 0] = s0;
    part[(chunk * t + c) * 3 + 1] = s1;
    part[(chunk * t + c) * 3 + 2] = s2;
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int64_t chunks,
                                                   int64_t width, double *__restrict__ out) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= width) return;
  double s = 0.0;
  for (int64_t k = 0; k < chunks; ++k) s += part[k * width + i];
  out[i] = s;
}

// out[b] = sum_k part[b * len + k], one thread per b (fixed order).
__global__ __launch_bounds__(256) void k_sum_rows(const double *__restrict__ part, int64_t len,
                                                  int64_t count, double *__restrict__ out) {
  const int64_t b = blockIdx.x * 256ll + threadIdx.x;
  if (b >= count) return;
  double acc = 0.0;
  for (int64_t k = 0; k < len; ++k) acc += part[b * len + k];
  out[b] = acc;
}

__global__ __launch_bounds__(256) void k_col_part(const z64 *__restrict__ X, int64_t ld, int64_t n,
                                                  int64_t t, double *__restrict__ part) {
  const int64_t chunk = blockIdx.x;
  const int64_t r0 = chunk * 64;
  const int64_t r1 = (r0 + 64 < n) ? r0 + 64 : n;
  for (int64_t c = threadIdx.x; c < t; c += 256) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const z64 x = X[r * ld + c];
      s += x.x * x.x + x.y * x.y;
    }
    part[chunk * t + c] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fro_part(const T *__restrict__ X, int64_t ld, int64_t sX,
                                                  int64_t n, int64_t m, double *__restrict__ part) {
  // part[b * gridDim.x + blockIdx.x]
  __shared__ double red[256];
  const int b = blockIdx.y;
  double s = 0.0;
  const int64_t total = n * m;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < total; i += 256ll * gridDim.x) {
    const int64_t row = i / m, col = i % m;
    const T x = X[b * sX + row * ld + col];
    s += static_cast<double>(x.x) * x.x + static_cast<double>(x.y) * x.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = red[0];
}

// Content fingerprint of n x n complex128 matrices: the wrapping 64-bit sum,
// over every entry (i, j), of a bijective mix of the entry's bits keyed by its
// position i n + j.  A change of any one entry always changes the sum (each
// term is a bijection of the entry's bits), a change of several entries is
// missed with probability about 2^-64, and the sum does not depend on the
// order in which workgroups add their parts.  Matrix b is tab[b] when tab is
// given, else a0 (b = 0) or a1 (b = 1); out[b] must be zero on entry.
// (each term: xor with the position key, multiply by an odd constant, fold the
// high half down -- three bijections of the 64-bit word)
__device__ inline uint64_t fp_mix(uint64_t x) {
  x *= 0x81dadef4bc2dd44dull;
  return x ^ (x >> 32);
}

__global__ __launch_bounds__(256) void k_fingerprint(const GrpMat *__restrict__ tab, GrpMat a0,
                                                     GrpMat a1, unsigned long long *__restrict__ out) {
  const int b = blockIdx.z;
  const GrpMat e = tab ? tab[b] : (b == 0 ? a0 : a1);
  const z64 *X = static_cast<const z64 *>(e.base);
  const int64_t n = e.n;
  uint64_t h = 0;
  ROWWISE_FOR(n, n, row, col) {
    const z64 v = X[row * e.ld + col];
    const uint64_t key = static_cast<uint64_t>(row * n + col) * 0x9e3779b97f4a7c15ull;
    h += fp_mix(static_cast<uint64_t>(__double_as_longlong(v.x)) ^ key);
    h += fp_mix(static_cast<uint64_t>(__double_as_longlong(v.y)) ^ ~key);
  }
  // wave sums, then one atomic per workgroup (integer sums are order-free)
  __shared__ uint64_t part[4];
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(out + b, static_cast<unsigned long long>(part[0] + part[1] + part[2] + part[3]));
}

// A += shift_rel * trace(A) on the diagonal (t x t, one workgroup).
__global__ __launch_bounds__(256) void k_add_shift(z64 *__restrict__ G, int64_t t, double shift_rel) {
  __shared__ double red[256];
  double tr = 0.0;
  for (int64_t i = threadIdx.x; i < t; i += 256) tr += G[i * t + i].x;
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double sh = shift_rel * red[0];
  for (int64_t i = threadIdx.x; i < t; i += 256) G[i * t + i].x += sh;
}

// Cholesky of one jb x jb (jb <= 64) Hermitian diagonal block and the inverse
// of its factor, by one workgroup of S*S threads (S = 32: 1024 threads).  The
// upper triangle of the block is read; R (upper) is written over it with the
// strict lower part zeroed, and R^{-1} (jb x jb, upper) to Rinv (leading
// dimension ldi).  Thread (ti, tj) holds the E*E entries (ti + S a, tj + S b),
// a, b < E = 64/S, in registers; wave wv holds the rows ti in
// [RW wv, RW (wv + 1)), RW = 64/S.  Cholesky step k subtracts
// conj(G_ki) G_kj / G_kk from every entry with k < i <= j (row k is read-only
// during the step); the inverse runs the same way from the bottom,
// X_i. = B_i. / R_ii and B_r. -= R_ri X_i. for r < i with B = I to start.
// Each step passes one finished row through LDS (double-buffered; its owners
// write all E of their row blocks and readers take block i / S, because
// choosing a register block by i would move the array to scratch memory), so
// it needs one barrier, and skips the blocks whose entries it cannot change.
// flag[0] = 1 + col0 + k for the first non-positive pivot k (a unit pivot is
// used in its place so the kernel finishes).
template <int S>
__device__ __forceinline__ void chol_inv_body(z64 *__restrict__ G, int64_t ld, int jb, int col0,
                                              int32_t *__restrict__ flag,
                                              z64 *__restrict__ Rinv, int64_t ldi) {
  constexpr int E = 64 / S, RW = 64 / S;
  __shared__ z64 row[2][E][64];
  __shared__ z64 Rs[64][65];
  __shared__ double dg[64];
  const int tid = threadIdx.x, ti = tid / S, tj = tid % S;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  z64 v[E][E];
#pragma unroll
  for (int a = 0; a < E; ++a)
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = ti + S * a, j = tj + S * b;
      v[a][b] = (i <= j && j < jb) ? G[i * ld + j] : make_double2(0.0, 0.0);
    }
  if (ti == 0)
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
      for (int b = 0; b < E; ++b) row[0][a][tj + S * b] = v[a][b];
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    const z64 *rk = row[k & 1][k / S];
    double d = rk[k].x;
    if (!(d > 0.0)) {
      if (tid == 0 && flag[0] == 0) flag[0] = col0 + k + 1;
      d = 1.0;
    }
    if (tid == 0) dg[k] = d;
    // all LDS reads of the step first, then branch-free updates (masked rows
    // and columns take a zero update), so the reads overlap
    z64 ri[E], rj[E];
#pragma unroll
    for (int a = 0; a < E; ++a) ri[a] = rk[ti + S * a];
#pragma unroll
    for (int b = 0; b < E; ++b) rj[b] = rk[tj + S * b];
    const double rd = 1.0 / d;
#pragma unroll
    for (int a = 0; a < E; ++a) {
      if (S * a + RW * wv + RW - 1 <= k) continue;  // the wave's rows of this block are done
      const int i = ti + S * a;
      const bool on = i > k && i < jb;
      const double qr = on ? ri[a].x * rd : 0.0, qi = on ? -ri[a].y * rd : 0.0;  // conj(G_ki)/G_kk
#pragma unroll
      for (int b = a; b < E; ++b) {  // columns j >= i only
        const int j = tj + S * b;
        const bool up = j >= i && j < jb;
        const double dx = qr * rj[b].x - qi * rj[b].y, dy = qr * rj[b].y + qi * rj[b].x;
        v[a][b].x -= up ? dx : 0.0;
        v[a][b].y -= up ? dy : 0.0;
      }
    }
    const int nk = k + 1;
    if (nk < jb && ti == nk % S)  // the owners of row k + 1 publish it
#pragma unroll
      for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) row[nk & 1][a][tj + S * b] = v[a][b];
    __syncthreads();
  }
  // R_ij = G_ij / sqrt(d_i) for i <= j (row i stops changing after step i - 1)
#pragma unroll
  for (int a = 0; a < E; ++a) {
    const int i = ti + S * a;
    const double sq = (i < jb) ? sqrt(dg[i]) : 1.0, sc = 1.0 / sq;
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int j = tj + S * b;
      z64 r = (i <= j && j < jb) ? make_double2(v[a][b].x * sc, v[a][b].y * sc)
                                 : make_double2(0.0, 0.0);
      if (i == j && i < jb) r = make_double2(sq, 0.0);
      Rs[i][j] = r;
      if (i < jb && j < jb) G[i * ld + j] = r;
      v[a][b] = make_double2(i == j && i < jb ? 1.0 : 0.0, 0.0);
    }
  }
  __syncthreads();
  // X = R^{-1}, from the bottom: at step i the owners scale row i by 1/R_ii
  // (a factor per row block, not a select on v) and publish it
  for (int i = jb - 1; i >= 0; --i) {
    const double rii = 1.0 / Rs[i][i].x;
#pragma unroll
    for (int a = 0; a < E; ++a) {
      const double f = (ti + S * a == i) ? rii : 1.0;
#pragma unroll
      for (int b = 0; b < E; ++b) {
        v[a][b].x *= f;
        v[a][b].y *= f;
      }
    }
    if (i == 0) break;
    if (ti == i % S)
#pragma unroll
      for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) row[i & 1][a][tj + S * b] = v[a][b];
    __syncthreads();
    const z64 *xi = row[i & 1][i / S];
    z64 qa[E], xb[E];
#pragma unroll
    for (int a = 0; a < E; ++a) qa[a] = Rs[ti + S * a][i];
#pragma unroll
    for (int b = 0; b < E; ++b) xb[b] = xi[tj + S * b];
#pragma unroll
    for (int a = 0; a < E; ++a) {
      if (S * a + RW * wv >= i) continue;  // none of the wave's rows of this block is above i
      const int r = ti + S * a;
      const bool on = r < i;
      const double qr = on ? qa[a].x : 0.0, qi = on ? qa[a].y : 0.0;
#pragma unroll
      for (int b = a; b < E; ++b) {  // X_rj = 0 for j < r
        if (S * b + S - 1 < i) continue;
        const int j = tj + S * b;
        const bool up = j >= i && j < jb;
        const double dx = qr * xb[b].x - qi * xb[b].y, dy = qr * xb[b].y + qi * xb[b].x;
        v[a][b].x -= up ? dx : 0.0;
        v[a][b].y -= up ? dy : 0.0;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < E; ++a)
#pragma unroll
    for (int b = 0; b < E; ++b) {
      const int i = ti + S * a, j = tj + S * b;
      if (i < jb && j < jb) Rinv[i * ldi + j] = (i <= j) ? v[a][b] : make_double2(0.0, 0.0);
    }
}

template <int S>
__global__ __launch_bounds__(S * S) void k_chol_inv(z64 *__restrict__ G, int64_t ld, int jb,
                                                    int col0, int32_t *__restrict__ flag,
                                                    z64 *__restrict__ Rinv, int64_t ldi) {
  chol_inv_body<S>(G, ld, jb, col0, flag, Rinv, ldi);
}

// The same over a group: matrix b = blockIdx.x of g, its diagonal block at
// (J0, J0) (skipped when J0 is past its order); the inverse of the factor to
// Dinv + b * dstride + (J0 / 64) * 4096 (leading dimension 64), a breakdown
// to flag[b * flag_stride].
template <int S>
__global__ __launch_bounds__(S * S) void k_chol_inv_grp(const GrpMat *__restrict__ g, int64_t J0,
                                                        int32_t *__restrict__ flag,
                                                        int flag_stride, z64 *__restrict__ Dinv,
                                                        int64_t dstride) {
  const GrpMat e = g[blockIdx.x];
  if (J0 >= e.n) return;
  const int jb = static_cast<int>(e.n - J0 < 64 ? e.n - J0 : 64);
  chol_inv_body<S>(static_cast<z64 *>(e.base) + J0 * e.ld + J0, e.ld, jb, static_cast<int>(J0),
                   flag + blockIdx.x * flag_stride, Dinv + blockIdx.x * dstride + (J0 / 64) * 4096,
                   64);
}

// Strict lower triangle of a t x t matrix set to zero; optionally the whole matrix.
__global__ __launch_bounds__(256) void k_zero_lower(z64 *__restrict__ X, int64_t t, int all) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= t * t) return;
  const int64_t i = e / t, j = e % t;
  if (all || j < i) X[e] = make_double2(0.0, 0.0);
}

// Column gather + normalisation: block per selected column.
__global__ __launch_bounds__(256) void k_gather_norm(const z64 *__restrict__ X, int64_t ldx,
                                                     int64_t n, const int32_t *__restrict__ idx,
                                                     z64 *__restrict__ Y, int64_t ldy) {
  __shared__ double s_n[256];
  __shared__ double s_m[256];
  __shared__ int64_t s_i[256];
  const int64_t k = blockIdx.x;
  const int64_t c = idx[k];
  double nr = 0.0, mx = -1.0;
  int64_t mi = 0;
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const z64 v = X[r * ldx + c];
    const double a2 = v.x * v.x + v.y * v.y;
    nr += a2;
    if (a2 > mx) {
      mx = a2;
      mi = r;
    }
  }
  s_n[threadIdx.x] = nr;
  s_m[threadIdx.x] = mx;
  s_i[threadIdx.x] = mi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s_n[threadIdx.x] += s_n[threadIdx.x + o];
      const double om = s_m[threadIdx.x + o];
      const int64_t oi = s_i[threadIdx.x + o];
      if (om > s_m[threadIdx.x] || (om == s_m[threadIdx.x] && oi < s_i[threadIdx.x])) {
        s_m[threadIdx.x] = om;
        s_i[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double nrm = sqrt(s_n[0]);
  const z64 piv = X[s_i[0] * ldx + c];
  const double pa = sqrt(piv.x * piv.x + piv.y * piv.y);
  // scale = conj(piv)/(|piv| * nrm)
  z64 sc = make_double2(1.0 / nrm, 0.0);
  if (pa > 0.0) sc = make_double2(piv.x / (pa * nrm), -piv.y / (pa * nrm));
  for (int64_t r = threadIdx.x; r < n; r += 256) {
    const z64 v = X[r * ldx + c];
    Y[r * ldy + k] = make_double2(v.x * sc.x - v.y * sc.y, v.x * sc.y + v.y * sc.x);
  }
}

// Y[:, j*s + c] = X[:, c] for every node j (broadcast of one block to N slots).
__global__ __launch_bounds__(256) void k_bcast_cols(const z64 *__restrict__ X, int64_t ldx,
                                                    int64_t n, int64_t s, int32_t N,
                                                    z64 *__restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  if (idx >= n * s * N) return;
  const int64_t row = idx / (s * N), col = idx % (s * N);
  Y[row * ldy + col] = X[row * ldx + col % s];
}

// Y (cols x rows) = X^* for the rows x cols block X.
__global__ __launch_bounds__(256) void k_conj_transpose(const z64 *__restrict__ X, int64_t ldx,
                                                        int64_t rows, int64_t cols,
                                                        z64 *__restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx / cols, j = idx % cols;
  const z64 v = X[i * ldx + j];
  Y[j * ldy + i] = make_double2(v.x, -v.y);
}

// X[:, c] *= d[c]
__global__ __launch_bounds__(256) void k_scale_cols(z64 *__restrict__ X, int64_t ldx, int64_t n,
                                                    int64_t s, const z64 *__restrict__ d) {
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  if (idx >= n * s) return;
  const int64_t i = idx / s, c = idx % s;
  const z64 v = X[i * ldx + c], f = d[c];
  X[i * ldx + c] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
}

// Identity of order t (row-major, ld t).
__global__ __launch_bounds__(256) void k_identity(z64 *__restrict__ X, int64_t t) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= t * t) return;
  X[e] = make_double2((e / t == e % t) ? 1.0 : 0.0, 0.0);
}


// ---- grouped forms over the pencils of a batch (GrpMat descriptors, one
// matrix per entry: base, leading dimension ld, order n; entries are
// matrices of the pencils in a list) ----

// G_b += shift_rel[b] * trace(G_b) * I (t = n_b).
__global__ __launch_bounds__(256) void k_add_shift_grp(const GrpMat *__restrict__ g,
                                                       const double *__restrict__ shift_rel) {
  __shared__ double red[256];
  const GrpMat e = g[blockIdx.x];
  z64 *G = static_cast<z64 *>(e.base);
  const int64_t t = e.n, ld = e.ld;
  double tr = 0.0;
  for (int64_t i = threadIdx.x; i < t; i += 256) tr += G[i * ld + i].x;
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double sh = shift_rel[blockIdx.x] * red[0];
  for (int64_t i = threadIdx.x; i < t; i += 256) G[i * ld + i].x += sh;
}

// Zero the strict lower triangle (all = 0) or everything (all = 1) of the
// n_b x n_b matrix b.
__global__ __launch_bounds__(256) void k_zero_lower_grp(const GrpMat *__restrict__ g, int all) {
  const GrpMat e = g[blockIdx.y];
  const int64_t q = blockIdx.x * 256ll + threadIdx.x;
  if (q >= e.n * e.n) return;
  const int64_t i = q / e.n, j = q % e.n;
  if (all || j < i) static_cast<z64 *>(e.base)[i * e.ld + j] = make_double2(0.0, 0.0);
}

// Y_b = X_b for rows x cols blocks: src[b] (ld, n = rows), dst[b] (ld), cols[b]
// columns taken from dst[b].stride (unused as a stride here).
__global__ __launch_bounds__(256) void k_copy_grp(const GrpMat *__restrict__ src,
                                                  const GrpMat *__restrict__ dst) {
  const GrpMat a = src[blockIdx.y], c = dst[blockIdx.y];
  const int64_t rows = a.n, cols = c.stride;
  const int64_t q = blockIdx.x * 256ll + threadIdx.x;
  if (q >= rows * cols) return;
  const int64_t i = q / cols, j = q % cols;
  static_cast<z64 *>(c.base)[i * c.ld + j] = static_cast<const z64 *>(a.base)[i * a.ld + j];
}

// Split-K partials summed in a fixed order: for matrix b, dst[b] = {C, ldc,
// cols, rows} and src[b] = {W, -, S, -} with the S partials (rows x cols each,
// dense) back to back at W; C = W_0 + ... + W_{S-1}.
__global__ __launch_bounds__(256) void k_sum_splits_grp(const GrpMat *__restrict__ dst,
                                                        const GrpMat *__restrict__ src) {
  const GrpMat c = dst[blockIdx.y], w = src[blockIdx.y];
  const int64_t rows = c.n, cols = c.stride, per = rows * cols;
  const int64_t q = blockIdx.x * 256ll + threadIdx.x;
  if (q >= per) return;
  const z64 *W = static_cast<const z64 *>(w.base);
  double sr = 0.0, si = 0.0;
  for (int64_t s = 0; s < w.stride; ++s) {
    const z64 v = W[s * per + q];
    sr += v.x;
    si += v.y;
  }
  static_cast<z64 *>(c.base)[(q / cols) * c.ld + q % cols] = make_double2(sr, si);
}

// Diagonal blocks of the inverted factor into X_b: block I of Dinv (64 x 64,
// matrix b at Dinv + b * dstride) to X_b[I*64 : , I*64 : ] (rb = min(64, n_b - I*64)).
__global__ __launch_bounds__(256) void k_put_diag_grp(const GrpMat *__restrict__ g,
                                                      const z64 *__restrict__ Dinv,
                                                      int64_t dstride) {
  const GrpMat e = g[blockIdx.y];
  const int64_t I = blockIdx.x;
  const int64_t r0 = I * 64;
  if (r0 >= e.n) return;
  const int rb = static_cast<int>(e.n - r0 < 64 ? e.n - r0 : 64);
  const z64 *D = Dinv + blockIdx.y * dstride + I * 4096;
  z64 *X = static_cast<z64 *>(e.base) + r0 * e.ld + r0;
  for (int q = threadIdx.x; q < rb * rb; q += 256) {
    const int i = q / rb, j = q % rb;
    X[i * e.ld + j] = D[i * 64 + j];
  }
}
}  // namespace

void bcast_cols(hipStream_t s, const z64 *X, int64_t ldx, int64_t n, int64_t c, int32_t N, z64 *Y,
                int64_t ldy) {
  const int64_t tot = n * c * N;
  hipLaunchKernelGGL(k_bcast_cols, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s,
                     X, ldx, n, c, N, Y, ldy);
}

void conj_transpose(hipStream_t s, const z64 *X, int64_t ldx, int64_t rows, int64_t cols, z64 *Y,
                    int64_t ldy) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(k_conj_transpose, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0,
                     s, X, ldx, rows, cols, Y, ldy);
}

void scale_cols(hipStream_t s, z64 *X, int64_t ldx, int64_t n, int64_t c, const z64 *d) {
  const int64_t tot = n * c;
  hipLaunchKernelGGL(k_scale_cols, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0, s,
                     X, ldx, n, c, d);
}

void identity(hipStream_t s, z64 *X, int64_t t) {
  hipLaunchKernelGGL(k_identity, dim3(static_cast<unsigned>((t * t + 255) / 256)), dim3(256), 0, s,
                     X, t);
}

void shift_assemble_z(hipStream_t s, const z64 *A, int64_t lda, const z64 *B, int64_t ldb,
                      const z64 *z, int32_t N, int64_t n, z64 *M, int64_t ldm, int64_t sM) {
  hipLaunchKernelGGL((k_shift<z64>), dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n)),
                     dim3(256), 0, s, A, lda, B, ldb, z, N, n, M, ldm, sM);
}
void shift_assemble_c(hipStream_t s, const z64 *A, int64_t lda, const z64 *B, int64_t ldb,
                      const z64 *z, int32_t N, int64_t n, c64 *M, int64_t ldm, int64_t sM) {
  hipLaunchKernelGGL((k_shift<c64>), dim3(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n)),
                     dim3(256), 0, s, A, lda, B, ldb, z, N, n, M, ldm, sM);
}

template <typename T>
void gather_rows(hipStream_t s, const T *R, int64_t ldr, int64_t sR, const int32_t *perm,
                 int64_t n, int64_t m, int32_t batch, T *Y, int64_t ldy, int64_t sY,
                 int64_t pstride) {
  if (batch <= 0 || n <= 0 || m <= 0) return;
  hipLaunchKernelGGL((k_gather_rows<T>), rowwise_grid(n, m, batch), dim3(256), 0, s, R,
                     ldr, sR, perm, pstride > 0 ? pstride : n, n, m, Y, ldy, sY);
}
template void gather_rows<z64>(hipStream_t, const z64 *, int64_t, int64_t, const int32_t *,
                               int64_t, int64_t, int32_t, z64 *, int64_t, int64_t, int64_t);
template void gather_rows<c64>(hipStream_t, const c64 *, int64_t, int64_t, const int32_t *,
                               int64_t, int64_t, int32_t, c64 *, int64_t, int64_t, int64_t);

// Ones on the diagonal of rows [n0, n) of `batch` matrices (the identity block
// that pads a pencil's shifted matrices to a multiple of the panel width).
template <typename T>
__global__ __launch_bounds__(256) void k_pad_diag(T *__restrict__ M, int64_t ld, int64_t stride,
                                                  int64_t n0, int64_t n) {
  const int64_t i = n0 + blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  T one;
  one.x = 1;
  one.y = 0;
  M[blockIdx.y * stride + i * ld + i] = one;
}

template <typename T>
void pad_diag(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n0,
              int64_t n) {
  if (n <= n0 || batch <= 0) return;
  hipLaunchKernelGGL((k_pad_diag<T>), dim3(static_cast<unsigned>((n - n0 + 255) / 256), batch),
                     dim3(256), 0, s, M, ld, stride, n0, n);
}
template void pad_diag<z64>(hipStream_t, z64 *, int64_t, int64_t, int32_t, int64_t, int64_t);
template void pad_diag<c64>(hipStream_t, c64 *, int64_t, int64_t, int32_t, int64_t, int64_t);

void shift_residual(hipStream_t s, const z64 *R, int64_t ldr, z64 *T1, const z64 *T2, int64_t ldt,
                    const z64 *z, int32_t N, int64_t n, int64_t m, int64_t used) {
  if (used < 0) used = m;
  const int64_t tot = n * static_cast<int64_t>(N) * used;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_shift_residual, dim3(static_cast<unsigned>((tot + 255) / 256)), dim3(256), 0,
                     s, R, ldr, T1, T2, ldt, z, n, m, used, N);
}

void c_to_z(hipStream_t s, const c64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
            int32_t batch, z64 *Y, int64_t ldy, int64_t sY, const double *nrm2, double cnt) {
  const int64_t tot = n * m;
  if (tot <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(k_c_to_z, rowwise_grid(n, m, batch), dim3(256), 0, s, X, ldx, sX, n, m, Y,
                     ldy, sY, nrm2, cnt);
}

template <typename T>
void scatter_rows(hipStream_t s, const T *X, int64_t ldx, int64_t sX, const int32_t *perm,
                  int64_t n, int64_t m, int32_t batch, T *Y, int64_t ldy, int64_t sY) {
  if (batch <= 0 || n <= 0 || m <= 0) return;
  hipLaunchKernelGGL((k_scatter_rows<T>), rowwise_grid(n, m, batch), dim3(256), 0, s, X,
                     ldx, sX, perm, n, m, Y, ldy, sY);
}
template void scatter_rows<z64>(hipStream_t, const z64 *, int64_t, int64_t, const int32_t *,
                                int64_t, int64_t, int32_t, z64 *, int64_t, int64_t);

void weighted_sum(hipStream_t s, const z64 *Y, int64_t ldy, int64_t sY, const z64 *w, int32_t N,
                  int64_t n, int64_t m, z64 *U, int64_t ldu) {
  const int64_t tot = n * m;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_weighted_sum, rowwise_grid(n, m, 1), dim3(256), 0, s,
                     Y, ldy, sY, w, N, n, m, U, ldu);
}

void copy_block_z(hipStream_t s, const z64 *X, int64_t ldx, int64_t n, int64_t m, z64 *Y,
                  int64_t ldy) {
  const int64_t tot = n * m;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_copy_block, rowwise_grid(n, m, 1), dim3(256), 0, s,
                     X, ldx, n, m, Y, ldy);
}

void z_to_c(hipStream_t s, const z64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
            int32_t batch, c64 *Y, int64_t ldy, int64_t sY, const double *nrm2, double cnt) {
  const int64_t tot = n * m;
  if (tot <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(k_z_to_c, rowwise_grid(n, m, batch), dim3(256), 0, s, X, ldx, sX, n, m, Y,
                     ldy, sY, nrm2, cnt);
}

void add_c_to_z(hipStream_t s, const c64 *X, int64_t ldx, int64_t sX, int64_t n, int64_t m,
                int32_t batch, z64 *Y, int64_t ldy, int64_t sY, const double *nrm2, double cnt) {
  const int64_t tot = n * m;
  if (tot <= 0 || batch <= 0) return;
  hipLaunchKernelGGL(k_add_c_to_z, rowwise_grid(n, m, batch), dim3(256), 0, s, X, ldx, sX, n, m,
                     Y, ldy, sY, nrm2, cnt);
}

void ritz_norms(hipStream_t s, const z64 *AX, const z64 *BX, int64_t ld, int64_t n, int64_t t,
                const z64 *lam, double *part, double *out) {
  const int64_t chunks = (n + 63) / 64;
  hipLaunchKernelGGL(k_ritz_part, dim3(static_cast<unsigned>(chunks)), dim3(256), 0, s, AX, BX, ld,
                     n, t, lam, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(static_cast<unsigned>((3 * t + 255) / 256)), dim3(256), 0, s,
                     part, chunks, 3 * t, out);
}

void col_norms2(hipStream_t s, const z64 *X, int64_t ld, int64_t n, int64_t t, double *part,
                double *out) {
  const int64_t chunks = (n + 63) / 64;
  hipLaunchKernelGGL(k_col_part, dim3(static_cast<unsigned>(chunks)), dim3(256), 0, s, X, ld, n, t,
                     part);
  hipLaunchKernelGGL(k_sum_parts, dim3(static_cast<unsigned>((t + 255) / 256)), dim3(256), 0, s,
                     part, chunks, t, out);
}

void fro2_batched(hipStream_t s, const z64 *X, int64_t ld, int64_t sX, int64_t n, int64_t m,
                  int32_t batch, double *part, double *out) {
  const int blocks = (batch == 1 && n * m > (1 << 22)) ? 1024 : 64;
  hipLaunchKernelGGL((k_fro_part<z64>), dim3(blocks, batch), dim3(256), 0, s, X, ld, sX, n, m,
                     part);
  hipLaunchKernelGGL(k_sum_rows, dim3(static_cast<unsigned>((batch + 255) / 256)), dim3(256), 0, s,
                     part, static_cast<int64_t>(blocks), static_cast<int64_t>(batch), out);
}

void fro2_c(hipStream_t s, const c64 *X, int64_t ld, int64_t n, int64_t m, double *part,
            double *out) {
  const int blocks = n * m > (1 << 22) ? 1024 : 64;
  hipLaunchKernelGGL((k_fro_part<c64>), dim3(blocks, 1), dim3(256), 0, s, X, ld, 0, n, m, part);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, part, static_cast<int64_t>(blocks),
                     static_cast<int64_t>(1), out);
}

void fingerprint(hipStream_t s, const GrpMat *tab, int count, GrpMat a0, GrpMat a1,
                 int64_t nmax, uint64_t *out) {
  if (count <= 0) return;
  fill_i32(s, reinterpret_cast<int32_t *>(out), 2ll * count, 0);
  if (nmax <= 0) return;
  // about 2048 workgroups over all matrices (each wave strides over rows), so
  // the per-workgroup atomics stay few
  dim3 g = rowwise_grid(nmax, nmax, count);
  const int64_t want = std::max<int64_t>(1, 2048 / (static_cast<int64_t>(g.x) * count));
  g.y = static_cast<unsigned>(std::min<int64_t>(g.y, want));
  hipLaunchKernelGGL(k_fingerprint, g, dim3(256), 0, s, tab, a0, a1,
                     reinterpret_cast<unsigned long long *>(out));
}

void add_diag_shift(hipStream_t s, z64 *G, int64_t t, double shift_rel) {
  hipLaunchKernelGGL(k_add_shift, dim3(1), dim3(256), 0, s, G, t, shift_rel);
}

void chol_inv_block(hipStream_t s, z64 *G, int64_t ld, int jb, int col0, int32_t *flag, z64 *Rinv,
                    int64_t ldi) {
  hipLaunchKernelGGL((k_chol_inv<32>), dim3(1), dim3(1024), 0, s, G, ld, jb, col0, flag, Rinv, ldi);
}

void zero_lower(hipStream_t s, z64 *X, int64_t t, bool all) {
  hipLaunchKernelGGL(k_zero_lower, dim3(static_cast<unsigned>((t * t + 255) / 256)), dim3(256), 0,
                     s, X, t, all ? 1 : 0);
}

void gather_normalize_cols(hipStream_t s, const z64 *X, int64_t ldx, int64_t n, const int32_t *idx,
                           int64_t k, z64 *Y, int64_t ldy, double *part) {
  (void)part;
  if (k <= 0) return;
  hipLaunchKernelGGL(k_gather_norm, dim3(static_cast<unsigned>(k)), dim3(256), 0, s, X, ldx, n, idx,
                     Y, ldy);
}

}  // namespace feast

namespace feast {

void add_shift_grp(hipStream_t s, const GrpMat *g, int count, const double *shift_rel) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_add_shift_grp, dim3(count), dim3(256), 0, s, g, shift_rel);
}

void chol_inv_grp(hipStream_t s, const GrpMat *g, int count, int64_t J0, int32_t *flag,
                  int flag_stride, z64 *Dinv, int64_t dstride) {
  if (count <= 0) return;
  hipLaunchKernelGGL((k_chol_inv_grp<32>), dim3(count), dim3(1024), 0, s, g, J0, flag, flag_stride,
                     Dinv, dstride);
}

void zero_lower_grp(hipStream_t s, const GrpMat *g, int count, int64_t tmax, bool all) {
  if (count <= 0 || tmax <= 0) return;
  hipLaunchKernelGGL(k_zero_lower_grp, dim3(static_cast<unsigned>((tmax * tmax + 255) / 256), count),
                     dim3(256), 0, s, g, all ? 1 : 0);
}

void copy_grp(hipStream_t s, const GrpMat *src, const GrpMat *dst, int count, int64_t max_elems) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(k_copy_grp, dim3(static_cast<unsigned>((max_elems + 255) / 256), count),
                     dim3(256), 0, s, src, dst);
}

void sum_splits_grp(hipStream_t s, const GrpMat *dst, const GrpMat *src, int count,
                    int64_t max_elems) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(k_sum_splits_grp, dim3(static_cast<unsigned>((max_elems + 255) / 256), count),
                     dim3(256), 0, s, dst, src);
}

void put_diag_grp(hipStream_t s, const GrpMat *g, int count, int64_t nblk_max, const z64 *Dinv,
                  int64_t dstride) {
  if (count <= 0 || nblk_max <= 0) return;
  hipLaunchKernelGGL(k_put_diag_grp, dim3(static_cast<unsigned>(nblk_max), count), dim3(256), 0, s,
                     g, Dinv, dstride);
}

}  // namespace feast
