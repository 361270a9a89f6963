// Blocked LU with partial pivoting of the shifted matrices z_j B - A (the
// shifted systems of eq. 4-4, factored once and reused, Section 4.3).
// Row-major storage: a row swap moves contiguous memory, and a panel row is a
// contiguous run of the panel width.
//
// Kernels here are the latency-bound parts of the factorisation; the flops of
// the trailing and panel updates run in the MFMA GEMM (k_gemm.hip).
#include <climits>

#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

template <typename T> __device__ inline T czero() {
  T z;
  z.x = 0;
  z.y = 0;
  return z;
}

// One workgroup of 1024 threads per matrix holds the leaf columns [c0, c0+w)
// of rows [c0, n) in registers (thread t owns rows c0 + t + 1024 q) and
// factors them column by column: |re|+|im| argmax over the column (wave64
// shuffles, then every thread reduces the 16 wave results from LDS; ties go to
// the lowest row), exchange of the pivot row with the diagonal row, scaling and
// the rank-1 update of the remaining leaf columns -- two barriers per column.
// The leaf's row swaps are then applied to the other columns of the enclosing
// panel [pk0, pk0+pkb) as one gather: the composed permutation of the at most
// 2w rows involved is read in full before any of it is written.
template <typename T, int RPT, int IB>
__global__ __launch_bounds__(1024) void k_leaf(T *__restrict__ Mall, int64_t ld_in, int64_t stride,
                                               int64_t n_in, int64_t c0, int w, int64_t pk0,
                                               int pkb, int32_t *__restrict__ ipiv_all,
                                               int32_t *__restrict__ info_all,
                                               const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  const int b = blockIdx.x;
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, b);
  T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  if (c0 + w > n) return;  // (grouped: this matrix is already factored)
  int32_t *ipiv = ipiv_all + b * n_in;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double s_val[2][16];
  __shared__ int s_idx[2][16];
  __shared__ int s_pivs[IB];
  __shared__ T s_prow[IB];
  __shared__ T s_crow[IB];
  __shared__ int s_key[2 * IB], s_src[2 * IB];
  __shared__ int s_nkey;
  int info_local = 0;

  T a[RPT][IB];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = c0 + tid + 1024 * q;
#pragma unroll
    for (int c = 0; c < IB; ++c) a[q][c] = (r < n && c < w) ? M[r * ld + c0 + c] : czero<T>();
  }

#pragma unroll
  for (int c = 0; c < IB; ++c) {
    if (c >= w) break;
    const int64_t rc = c0 + c;
    const int par = c & 1;
    double best = -1.0;
    int bidx = INT_MAX;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t r = c0 + tid + 1024 * q;
      if (r >= rc && r < n) {
        const double v = Tr::abs1(a[q][c]);
        if (v > best) {
          best = v;
          bidx = static_cast<int>(r);
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bidx, off, 64);
      if (ov > best || (ov == best && oi < bidx)) {
        best = ov;
        bidx = oi;
      }
    }
    if (lane == 0) {
      s_val[par][wave] = best;
      s_idx[par][wave] = bidx;
    }
    __syncthreads();
    double bv = s_val[par][0];
    int bi = s_idx[par][0];
#pragma unroll
    for (int k = 1; k < 16; ++k) {
      const double v = s_val[par][k];
      const int i = s_idx[par][k];
      if (v > bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
      }
    }
    if (bi == INT_MAX) {  // no comparable entry (NaN column): keep the diagonal row
      bi = static_cast<int>(rc);
      bv = 0.0;
    }
    if (bv == 0.0 && info_local == 0) info_local = static_cast<int>(rc) + 1;
    const int64_t p = bi;
    if (tid == 0) {
      s_pivs[c] = bi;
      ipiv[rc] = bi;
    }
    const int64_t prel = p - c0;
    const int ptid = static_cast<int>(prel & 1023), pq = static_cast<int>(prel >> 10);
    if (tid == ptid) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == pq)
#pragma unroll
          for (int k = 0; k < IB; ++k) s_prow[k] = a[q][k];
    }
    if (tid == c) {
#pragma unroll
      for (int k = 0; k < IB; ++k) s_crow[k] = a[0][k];
    }
    __syncthreads();
    if (tid == c) {
#pragma unroll
      for (int k = 0; k < IB; ++k) a[0][k] = s_prow[k];
    }
    if (tid == ptid && p != rc) {
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == pq)
#pragma unroll
          for (int k = 0; k < IB; ++k) a[q][k] = s_crow[k];
    }
    const T piv = s_prow[c];
    const bool zero = (piv.x == 0 && piv.y == 0);
    const T inv = zero ? czero<T>() : Tr::recip(piv);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int64_t r = c0 + tid + 1024 * q;
      if (r > rc && r < n) {
        const T l = Tr::mul(a[q][c], inv);
        a[q][c] = l;
#pragma unroll
        for (int k = c + 1; k < IB; ++k) a[q][k] = Tr::fms(a[q][k], l, s_prow[k]);
      }
    }
  }

#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = c0 + tid + 1024 * q;
    if (r < n)
#pragma unroll
      for (int c = 0; c < IB; ++c)
        if (c < w) M[r * ld + c0 + c] = a[q][c];
  }
  // composed permutation of the rows touched by the leaf's swaps
  if (tid == 0) {
    int nk = 0;
    for (int c = 0; c < w; ++c) {
      const int r1 = static_cast<int>(c0) + c, r2 = s_pivs[c];
      int i1 = -1, i2 = -1;
      for (int k = 0; k < nk; ++k) {
        if (s_key[k] == r1) i1 = k;
        if (s_key[k] == r2) i2 = k;
      }
      if (i1 < 0) {
        s_key[nk] = r1;
        s_src[nk] = r1;
        i1 = nk++;
      }
      if (i2 < 0) {
        s_key[nk] = r2;
        s_src[nk] = r2;
        i2 = nk++;
      }
      const int t = s_src[i1];
      s_src[i1] = s_src[i2];
      s_src[i2] = t;
    }
    s_nkey = nk;
  }
  __syncthreads();
  const int nk = s_nkey;
  const int ncol = pkb;  // panel columns; the leaf's own columns are skipped
  T v[2];
  int64_t dst[2], col[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + 1024 * h;
    dst[h] = -1;
    if (e < ncol * nk) {
      const int k = e / ncol;
      col[h] = pk0 + e % ncol;
      if ((col[h] < c0 || col[h] >= c0 + w) && s_key[k] != s_src[k]) {
        v[h] = M[static_cast<int64_t>(s_src[k]) * ld + col[h]];
        dst[h] = s_key[k];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (dst[h] >= 0) M[dst[h] * ld + col[h]] = v[h];
  if (tid == 0 && info_local != 0 && info_all[b] == 0) info_all[b] = info_local;
}

template <typename T>
__global__ __launch_bounds__(256) void k_laswp_outside(T *__restrict__ Mall, int64_t ld_in,
                                                       int64_t stride, int64_t n_in, int64_t r0,
                                                       int kb, int64_t clo, int64_t chi,
                                                       const int32_t *__restrict__ ipiv_all,
                                                       const GrpMat *__restrict__ grp, int nodes) {
  const int b = blockIdx.y;
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, b);
  T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  if (r0 + kb > n) return;
  const int32_t *ipiv = ipiv_all + b * n_in;
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  const int64_t ncols = clo + (n - chi);
  if (t >= ncols) return;
  const int64_t col = (t < clo) ? t : chi + (t - clo);
  for (int i = 0; i < kb; ++i) {
    const int64_t r = r0 + i, p = ipiv[r];
    if (p != r) {
      const T x = M[r * ld + col];
      M[r * ld + col] = M[p * ld + col];
      M[p * ld + col] = x;
    }
  }
}

// X = L11^{-1} X with L11 unit lower (w1 x w1), X (w1 x w2), both inside the
// matrix; one workgroup per matrix, one thread per column of X.
template <typename T>
__global__ __launch_bounds__(64) void k_trsm_small(T *__restrict__ Mall, int64_t ld,
                                                   int64_t stride, int64_t c0, int w1, int w2) {
  using Tr = cplx_traits<T>;
  __shared__ T sL[64][65];
  __shared__ T sX[64][65];
  T *M = Mall + blockIdx.x * stride;
  const int tid = threadIdx.x;
  for (int i = 0; i < w1; ++i) {
    if (tid < w1) sL[i][tid] = M[(c0 + i) * ld + c0 + tid];
    if (tid < w2) sX[i][tid] = M[(c0 + i) * ld + c0 + w1 + tid];
  }
  __syncthreads();
  if (tid < w2) {
    for (int i = 1; i < w1; ++i) {
      T x = sX[i][tid];
      for (int k = 0; k < i; ++k) x = Tr::fms(x, sL[i][k], sX[k][tid]);
      sX[i][tid] = x;
    }
    for (int i = 1; i < w1; ++i) M[(c0 + i) * ld + c0 + w1 + tid] = sX[i][tid];
  }
}

// One recursion step of the panel factorisation in a single launch, for
// w1, w2 <= 32:
//   X = L11^{-1} X      for X = M[c0:c0+w1, c0+w1:c0+w1+w2], L11 unit lower (w1 x w1),
//   C -= L21 X          for C = M[c0+w1:n, c0+w1:c0+w1+w2], L21 = M[c0+w1:n, c0:c0+w1].
// write_x = false: every workgroup solves the small triangular system in LDS
// (eight lanes per column share each inner product) and updates 64 rows of C
// from an LDS copy of its L21 rows, 8 outputs per thread; X in the matrix is
// left as it was, because workgroups that start later still read it.
// write_x = true (one workgroup per matrix, launched afterwards): solve again
// and store X.  The update is a rank-w1 product with w1 <= 32: it is bound by
// the traffic of C, so it runs on the VALU.
constexpr int kPU = 32;
template <typename T>
__global__ __launch_bounds__(256) void k_panel_update(T *__restrict__ Mall, int64_t ld_in,
                                                      int64_t stride, int64_t n_in, int64_t c0,
                                                      int w1, int w2, bool write_x,
                                                      const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  __shared__ T sL[64][kPU + 1];
  __shared__ T sX[kPU][kPU + 1];
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, blockIdx.y);
  T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  if (c0 + w1 + w2 > n) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < w1 * w1; e += 256) {
    const int i = e / w1, k = e % w1;
    sL[i][k] = M[(c0 + i) * ld + c0 + k];
  }
  for (int e = tid; e < w1 * w2; e += 256) {
    const int i = e / w2, j = e % w2;
    sX[i][j] = M[(c0 + i) * ld + c0 + w1 + j];
  }
  __syncthreads();
  {
    // forward substitution: column j = tid / 8, lanes q = tid % 8 split the sum
    const int j = tid >> 3, q = tid & 7;
    for (int i = 1; i < w1; ++i) {
      T part = Tr::make(0.0, 0.0);
      if (j < w2)
        for (int k = q; k < i; k += 8) part = Tr::fms(part, sL[i][k], sX[k][j]);
#pragma unroll
      for (int off = 1; off < 8; off <<= 1) {
        part.x += __shfl_xor(part.x, off);
        part.y += __shfl_xor(part.y, off);
      }
      if (q == 0 && j < w2) {
        T x = sX[i][j];
        x.x += part.x;
        x.y += part.y;
        sX[i][j] = x;
      }
      // the eight lanes of a column are in one wavefront: order its LDS accesses
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
  __syncthreads();
  if (write_x) {
    for (int e = tid; e < w1 * w2; e += 256) {
      const int i = e / w2, j = e % w2;
      if (i > 0) M[(c0 + i) * ld + c0 + w1 + j] = sX[i][j];
    }
    return;
  }
  const int64_t r0 = c0 + w1 + static_cast<int64_t>(blockIdx.x) * 64;
  const int rows = static_cast<int>((n - r0 < 64) ? n - r0 : 64);
  if (rows <= 0) return;
  // L21 rows of this chunk into LDS (sL is free after the solve)
  for (int e = tid; e < rows * w1; e += 256) {
    const int i = e / w1, k = e % w1;
    sL[i][k] = M[(r0 + i) * ld + c0 + k];
  }
  __syncthreads();
  const int ti = tid >> 4, tj = tid & 15;
  T acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      acc[a][b] = (i < rows && j < w2) ? M[(r0 + i) * ld + c0 + w1 + j] : Tr::make(0.0, 0.0);
    }
  for (int k = 0; k < w1; ++k) {
    T l[4], x[2];
#pragma unroll
    for (int a = 0; a < 4; ++a) l[a] = sL[ti + 16 * a][k];
#pragma unroll
    for (int b = 0; b < 2; ++b) x[b] = sX[k][tj + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = Tr::fms(acc[a][b], l[a], x[b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      if (i < rows && j < w2) M[(r0 + i) * ld + c0 + w1 + j] = acc[a][b];
    }
}

// Inverse of one diagonal block (lower unit or upper non-unit), one thread per column.
template <typename T>
__global__ __launch_bounds__(64) void k_diag_inv(const T *__restrict__ Mall, int64_t ld_in,
                                                 int64_t stride, int64_t n_in, int nb, int64_t blk0,
                                                 bool lower, T *__restrict__ out,
                                                 int64_t out_stride,
                                                 const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  __shared__ T sD[64][65];
  __shared__ T sX[64][65];
  const int64_t I = blk0 + blockIdx.x;
  const int b = blockIdx.y;
  const MatRef<const T> mr = mat_of<const T>(grp, nodes, Mall, ld_in, stride, n_in, b);
  const T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  const int64_t r0 = I * nb;
  const int rb = static_cast<int>((n - r0 < nb) ? n - r0 : nb);
  const int tid = threadIdx.x;
  for (int i = 0; i < rb; ++i)
    if (tid < rb) sD[i][tid] = M[(r0 + i) * ld + r0 + tid];
  __syncthreads();
  const int j = tid;
  if (j < rb) {
    if (lower) {
      for (int i = 0; i < j; ++i) sX[i][j] = czero<T>();
      sX[j][j] = Tr::make(1.0, 0.0);
      for (int i = j + 1; i < rb; ++i) {
        T x = czero<T>();
        for (int k = j; k < i; ++k) x = Tr::fms(x, sD[i][k], sX[k][j]);
        sX[i][j] = x;
      }
    } else {
      for (int i = j + 1; i < rb; ++i) sX[i][j] = czero<T>();
      sX[j][j] = Tr::recip(sD[j][j]);
      for (int i = j - 1; i >= 0; --i) {
        T x = czero<T>();
        for (int k = i + 1; k <= j; ++k) x = Tr::fms(x, sD[i][k], sX[k][j]);
        sX[i][j] = Tr::mul(x, Tr::recip(sD[i][i]));
      }
    }
  }
  __syncthreads();
  T *o = out + b * out_stride + I * static_cast<int64_t>(nb) * nb;
  for (int i = 0; i < nb; ++i)
    if (tid < nb) o[i * nb + tid] = (i < rb && tid < rb) ? sX[i][tid] : czero<T>();
}

// n: order (pivot vectors of the batch are n_stride apart; grouped batches read
// each matrix's order from grp)
__global__ __launch_bounds__(256) void k_perm(const int32_t *__restrict__ ipiv_all,
                                              int32_t *__restrict__ perm_all, int64_t n_stride,
                                              const GrpMat *__restrict__ grp, int nodes) {
  extern __shared__ int32_t sp[];
  const int b = blockIdx.x;
  const int64_t n = grp ? grp[b / nodes].n : n_stride;
  const int32_t *ipiv = ipiv_all + b * n_stride;
  int32_t *perm = perm_all + b * n_stride;
  for (int64_t i = threadIdx.x; i < n; i += 256) sp[i] = static_cast<int32_t>(i);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int64_t i = 0; i < n; ++i) {
      const int32_t p = ipiv[i];
      const int32_t x = sp[i];
      sp[i] = sp[p];
      sp[p] = x;
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += 256) perm[i] = sp[i];
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename T, int RPT, int IB>
void launch_leaf(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                 int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info,
                 const GrpMat *grp, int nodes) {
  hipLaunchKernelGGL((k_leaf<T, RPT, IB>), dim3(batch), dim3(1024), 0, s, M, ld, stride, n, c0, w,
                     pk0, pkb, ipiv, info, grp, nodes);
}

}  // namespace

template <> int leaf_max_width<z64>(int64_t rows) {
  if (rows <= 2048) return 8;
  if (rows <= 4096) return 4;
  if (rows <= 8192) return 2;
  if (rows <= 16384) return 1;
  return 0;
}
template <> int leaf_max_width<c64>(int64_t rows) {
  if (rows <= 4096) return 8;
  if (rows <= 8192) return 4;
  if (rows <= 16384) return 2;
  return 0;
}

template <>
bool leaf_lu<z64>(hipStream_t s, z64 *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                  int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info,
                  const GrpMat *grp, int nodes) {
  const int64_t rows = n - c0;
  if (w < 1 || w > leaf_max_width<z64>(rows) || pkb > 1024) return false;
  if (rows <= 1024)
    launch_leaf<z64, 1, 8>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 2048)
    launch_leaf<z64, 2, 8>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 4096)
    launch_leaf<z64, 4, 4>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 8192)
    launch_leaf<z64, 8, 2>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else
    launch_leaf<z64, 16, 1>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  return true;
}

template <>
bool leaf_lu<c64>(hipStream_t s, c64 *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                  int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info,
                  const GrpMat *grp, int nodes) {
  const int64_t rows = n - c0;
  if (w < 1 || w > leaf_max_width<c64>(rows) || pkb > 1024) return false;
  if (rows <= 1024)
    launch_leaf<c64, 1, 8>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 2048)
    launch_leaf<c64, 2, 8>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 4096)
    launch_leaf<c64, 4, 8>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 8192)
    launch_leaf<c64, 8, 4>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else
    launch_leaf<c64, 16, 2>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  return true;
}

template <typename T>
void laswp_outside(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                   int64_t r0, int kb, int64_t clo, int64_t chi, const int32_t *ipiv,
                   const GrpMat *grp, int nodes) {
  const int64_t ncols = clo + (n - chi);
  if (ncols <= 0 || kb <= 0) return;
  hipLaunchKernelGGL((k_laswp_outside<T>), dim3(static_cast<unsigned>((ncols + 255) / 256), batch),
                     dim3(256), 0, s, M, ld, stride, n, r0, kb, clo, chi, ipiv, grp, nodes);
}
template void laswp_outside<z64>(hipStream_t, z64 *, int64_t, int64_t, int32_t, int64_t, int64_t,
                                 int, int64_t, int64_t, const int32_t *, const GrpMat *, int);
template void laswp_outside<c64>(hipStream_t, c64 *, int64_t, int64_t, int32_t, int64_t, int64_t,
                                 int, int64_t, int64_t, const int32_t *, const GrpMat *, int);

template <typename T>
void trsm_small(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t c0,
                int w1, int w2) {
  if (w1 <= 1 || w2 <= 0) return;
  hipLaunchKernelGGL((k_trsm_small<T>), dim3(batch), dim3(64), 0, s, M, ld, stride, c0, w1, w2);
}
template void trsm_small<z64>(hipStream_t, z64 *, int64_t, int64_t, int32_t, int64_t, int, int);
template void trsm_small<c64>(hipStream_t, c64 *, int64_t, int64_t, int32_t, int64_t, int, int);

template <typename T>
void panel_update(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                  int64_t c0, int w1, int w2, const GrpMat *grp, int nodes) {
  if (w1 <= 0 || w2 <= 0 || w1 > kPU || w2 > kPU) return;
  const int64_t rows = n - c0 - w1;
  const unsigned chunks = static_cast<unsigned>(rows > 0 ? (rows + 63) / 64 : 1);
  if (rows > 0)
    hipLaunchKernelGGL((k_panel_update<T>), dim3(chunks, batch), dim3(256), 0, s, M, ld, stride, n,
                       c0, w1, w2, false, grp, nodes);
  hipLaunchKernelGGL((k_panel_update<T>), dim3(1, batch), dim3(256), 0, s, M, ld, stride, n, c0, w1,
                     w2, true, grp, nodes);
}
template void panel_update<z64>(hipStream_t, z64 *, int64_t, int64_t, int32_t, int64_t, int64_t,
                                int, int, const GrpMat *, int);
template void panel_update<c64>(hipStream_t, c64 *, int64_t, int64_t, int32_t, int64_t, int64_t,
                                int, int, const GrpMat *, int);
int panel_update_max_width() { return kPU; }

template <typename T>
void diag_block_inverse(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch,
                        int64_t n, int nb, int64_t blk0, int64_t blk1, bool lower, T *out,
                        int64_t out_stride, const GrpMat *grp, int nodes) {
  if (blk1 <= blk0) return;
  hipLaunchKernelGGL((k_diag_inv<T>), dim3(static_cast<unsigned>(blk1 - blk0), batch), dim3(64),
                     0, s, M, ld, stride, n, nb, blk0, lower, out, out_stride, grp, nodes);
}
template void diag_block_inverse<z64>(hipStream_t, const z64 *, int64_t, int64_t, int32_t,
                                      int64_t, int, int64_t, int64_t, bool, z64 *, int64_t,
                                      const GrpMat *, int);
template void diag_block_inverse<c64>(hipStream_t, const c64 *, int64_t, int64_t, int32_t,
                                      int64_t, int, int64_t, int64_t, bool, c64 *, int64_t,
                                      const GrpMat *, int);

void perm_from_ipiv(hipStream_t s, const int32_t *ipiv, int32_t *perm, int64_t n, int32_t batch,
                    const GrpMat *grp, int nodes) {
  hipLaunchKernelGGL(k_perm, dim3(batch), dim3(256), static_cast<unsigned>(n * sizeof(int32_t)), s,
                     ipiv, perm, n, grp, nodes);
}

void fill_i32(hipStream_t s, int32_t *p, int64_t count, int32_t v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s,
                     p, count, v);
}

}  // namespace feast
