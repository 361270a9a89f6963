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

// 32-bit lane exchange through DPP (VALU, no LDS round trip); lanes that the
// pattern gives no source read 0, the identity of the unsigned maxima below.
template <int CTRL> __device__ inline uint32_t dpp32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ inline uint64_t dpp64(uint64_t v) {
  return (static_cast<uint64_t>(dpp32<CTRL>(static_cast<uint32_t>(v >> 32))) << 32) |
         dpp32<CTRL>(static_cast<uint32_t>(v));
}
// Maximum of an unsigned key over the 64 lanes of a wavefront, returned
// uniformly: swaps inside quads, rotations inside rows of 16, then the
// broadcasts of lane 15 and lane 31 that leave the full maximum in lane 63.
__device__ inline uint64_t wave_max_u64(uint64_t k) {
  uint64_t o;
  o = dpp64<0xb1>(k);  // quad_perm [1,0,3,2]
  k = o > k ? o : k;
  o = dpp64<0x4e>(k);  // quad_perm [2,3,0,1]
  k = o > k ? o : k;
  o = dpp64<0x124>(k);  // row_ror:4
  k = o > k ? o : k;
  o = dpp64<0x128>(k);  // row_ror:8
  k = o > k ? o : k;
  o = dpp64<0x142>(k);  // row_bcast:15
  k = o > k ? o : k;
  o = dpp64<0x143>(k);  // row_bcast:31
  k = o > k ? o : k;
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(k), 63);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(k >> 32), 63);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Maximum over each row of 16 lanes, left in every lane of the row.
__device__ inline uint64_t row16_max_u64(uint64_t k) {
  uint64_t o;
  o = dpp64<0xb1>(k);
  k = o > k ? o : k;
  o = dpp64<0x4e>(k);
  k = o > k ? o : k;
  o = dpp64<0x124>(k);
  k = o > k ? o : k;
  o = dpp64<0x128>(k);
  k = o > k ? o : k;
  return k;
}
__device__ inline uint64_t uniform_u64(uint64_t k) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(k));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(k >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Pivot keys: |re| + |im| of a candidate as an unsigned integer that orders
// like the value (IEEE bits of a non-negative number, plus one so that 0 marks
// "no candidate"; NaN is no candidate).  complex64 packs the row index into
// the low half (complemented, so the lowest row wins a tie) and needs one
// reduction; complex128 breaks ties in a second reduction over the row index.
template <typename T> struct PivKey;
template <> struct PivKey<c64> {
  static constexpr bool kPacked = true;
  __device__ static uint64_t key(c64 a, int row) {
    const float v = fabsf(a.x) + fabsf(a.y);
    if (!(v >= 0.0f)) return 0;
    return (static_cast<uint64_t>(__float_as_uint(v)) << 32) | (0xFFFFFFFFu - static_cast<uint32_t>(row));
  }
};
template <> struct PivKey<z64> {
  static constexpr bool kPacked = false;
  __device__ static uint64_t key(z64 a, int) {
    const double v = fabs(a.x) + fabs(a.y);
    if (!(v >= 0.0)) return 0;
    return static_cast<uint64_t>(__double_as_longlong(v)) + 1;
  }
};

// Rows of the leaf staged through LDS in blocks of at most NT rows, so that
// global loads and stores walk along rows (IB consecutive lanes per row)
// instead of one row per lane.
template <typename T, int NT, int IB> struct LeafStage {
  static constexpr int kRows = (NT * (IB + 1) * static_cast<int>(sizeof(T)) <= 81920) ? NT : NT / 2;
};

// One workgroup of NT threads per matrix holds the leaf columns [c0, c0+w)
// of rows [c0, n) in registers (thread t owns rows c0 + t + NT q) and factors
// them column by column with partial pivoting (largest |re|+|im|, lowest row
// on ties; Section 4.3 reuses these factors for every filter).
// Per column: each wavefront reduces its pivot key with DPP, the winning lane
// posts its key and whole row to LDS, the owner of the diagonal row posts
// that row, and after one barrier every thread picks the winner among the
// posts, exchanges the two rows and applies the rank-1 update.  Posts are
// double-buffered by column parity, so one barrier per column suffices.
// The per-column selection work is repeated by every wavefront, so fewer,
// fuller wavefronts (NT < 1024, more rows per thread) shorten a column.
template <typename T, int NT, int RPT, int IB>
__global__ __launch_bounds__(NT) void k_leaf(T *__restrict__ Mall, int64_t ld_in, int64_t stride,
                                             int64_t n_in, int64_t c0, int w, int64_t pk0,
                                             int pkb, int32_t *__restrict__ ipiv_all,
                                             int32_t *__restrict__ info_all,
                                             const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  using PK = PivKey<T>;
  constexpr int SR = LeafStage<T, NT, IB>::kRows;
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "at most 16 wavefronts");
  const int b = blockIdx.x;
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, b);
  T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  if (c0 + w > n) return;  // (grouped: this matrix is already factored)
  int32_t *ipiv = ipiv_all + b * n_in;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ T stg[SR][IB + 1];
  __shared__ uint64_t s_key[2][16];
  __shared__ uint32_t s_row[2][16];
  __shared__ T s_post[2][16][IB];
  __shared__ T s_crow[2][IB];
  __shared__ int s_pivs[IB];
  int info_local = 0;
  // rows of this thread relative to c0: tid + NT q (32-bit: rows < 2^31)
  const int nrel = static_cast<int>(n - c0);

  T a[RPT][IB];
#pragma unroll
  for (int q = 0; q < RPT; ++q)
#pragma unroll
    for (int h = 0; h < NT / SR; ++h) {
      const int64_t base = c0 + NT * q + SR * h;
      const T *Mb = M + base * ld + c0;
      const int lim = static_cast<int>(n - base < SR ? n - base : SR);  // rows of this block
      if (lim <= 0) {  // the block lies below the matrix (uniform): nothing to read
        if (tid >= SR * h && tid < SR * (h + 1))
#pragma unroll
          for (int c = 0; c < IB; ++c) a[q][c] = czero<T>();
        continue;
      }
      // addresses clamped into the block's rows (lim >= 1), so all loads issue
      // before the first wait
      T t[SR * IB / NT];
#pragma unroll
      for (int k = 0; k < SR * IB / NT; ++k) {
        const int e = tid + NT * k, i = e / IB, c = e % IB;
        t[k] = Mb[(i < lim ? i : 0) * static_cast<int>(ld) + (c < w ? c : 0)];
      }
#pragma unroll
      for (int k = 0; k < SR * IB / NT; ++k) {
        const int e = tid + NT * k, i = e / IB, c = e % IB;
        stg[i][c] = (i < lim && c < w) ? t[k] : czero<T>();
      }
      __syncthreads();
      if (tid >= SR * h && tid < SR * (h + 1))
#pragma unroll
        for (int c = 0; c < IB; ++c) a[q][c] = stg[tid - SR * h][c];
      __syncthreads();
    }

#pragma unroll
  for (int c = 0; c < IB; ++c) {
    if (c >= w) break;
    const int64_t rc = c0 + c;
    const int par = c & 1;
    // this thread's best candidate (relative rows c .. nrel-1)
    uint64_t best = 0;
    int bq = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      const uint64_t k = (r >= c && r < nrel) ? PK::key(a[q][c], static_cast<int>(c0) + r) : 0;
      if (k > best) {  // strict: the lowest row of this thread wins a tie
        best = k;
        bq = q;
      }
    }
    const int myrow = static_cast<int>(c0) + tid + NT * bq;
    const uint64_t wbest = wave_max_u64(best);
    bool mine = best == wbest && wbest != 0;
    if constexpr (!PK::kPacked) {
      // ties in value: the lowest row among the lanes holding the maximum
      const uint64_t ik = mine ? 0xFFFFFFFFull - static_cast<uint32_t>(myrow) : 0;
      const uint64_t wi = wave_max_u64(ik);
      mine = mine && ik == wi;
    }
    if (mine) {
      s_key[par][wave] = wbest;
      s_row[par][wave] = static_cast<uint32_t>(myrow);
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (q == bq)
#pragma unroll
          for (int k = 0; k < IB; ++k) s_post[par][wave][k] = a[q][k];
    }
    if (wbest == 0 && lane == 0) s_key[par][wave] = 0;  // no candidate in this wavefront
    if (tid == c)
#pragma unroll
      for (int k = 0; k < IB; ++k) s_crow[par][k] = a[0][k];
    __syncthreads();
    // the winner among the posts: lane v of every row of 16 reads post v
    const int pv = lane & 15;
    const uint64_t pk = pv < NW ? s_key[par][pv] : 0;
    const uint32_t prw = pv < NW ? s_row[par][pv] : 0xFFFFFFFFu;
    const uint64_t gk = uniform_u64(row16_max_u64(pk));
    uint32_t grow = 0xFFFFFFFFu - static_cast<uint32_t>(gk);
    if constexpr (!PK::kPacked) {  // ties in value: the lowest row
      const uint64_t rk = (pk == gk && gk != 0) ? 0xFFFFFFFFull - prw : 0;
      grow = 0xFFFFFFFFu - static_cast<uint32_t>(uniform_u64(row16_max_u64(rk)));
    }
    const uint64_t hit = __builtin_amdgcn_ballot_w64(gk != 0 && pk == gk && prw == grow);
    const int gw = hit ? static_cast<int>(__builtin_ctzll(hit) & 15) : -1;
    int64_t p = rc;
    T prow[IB];
    if (gw >= 0) {
      p = grow;
#pragma unroll
      for (int k = 0; k < IB; ++k) prow[k] = s_post[par][gw][k];
    } else {  // no comparable entry (NaN column): keep the diagonal row
#pragma unroll
      for (int k = 0; k < IB; ++k) prow[k] = s_crow[par][k];
    }
    const T piv = prow[c];
    const bool zero = (piv.x == 0 && piv.y == 0);
    if ((zero || gw < 0) && info_local == 0) info_local = static_cast<int>(rc) + 1;
    if (tid == 0) s_pivs[c] = static_cast<int>(p);
    if (p != rc) {
      const int prel = static_cast<int>(p - c0);
      const int ptid = prel % NT, pq = prel / NT;
      if (tid == c)
#pragma unroll
        for (int k = 0; k < IB; ++k) a[0][k] = prow[k];
      if (tid == ptid)
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == pq)
#pragma unroll
            for (int k = 0; k < IB; ++k) a[q][k] = s_crow[par][k];
    }
    const T inv = zero ? czero<T>() : Tr::recip(piv);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + NT * q;
      if (r > c && r < nrel) {
        const T l = Tr::mul(a[q][c], inv);
        a[q][c] = l;
#pragma unroll
        for (int k = c + 1; k < IB; ++k) a[q][k] = Tr::fms(a[q][k], l, prow[k]);
      }
    }
  }

  // leaf columns back through LDS (row-contiguous stores), then the pivots
#pragma unroll
  for (int q = 0; q < RPT; ++q)
#pragma unroll
    for (int h = 0; h < NT / SR; ++h) {
      const int64_t base = c0 + NT * q + SR * h;
      __syncthreads();
      if (tid >= SR * h && tid < SR * (h + 1))
#pragma unroll
        for (int c = 0; c < IB; ++c) stg[tid - SR * h][c] = a[q][c];
      __syncthreads();
      T *Mb = M + base * ld + c0;
      const int lim = static_cast<int>(n - base < SR ? n - base : SR);
#pragma unroll
      for (int k = 0; k < SR * IB / NT; ++k) {
        const int e = tid + NT * k, i = e / IB, c = e % IB;
        if (i < lim && c < w) Mb[i * static_cast<int>(ld) + c] = stg[i][c];
      }
    }
  if (tid < w) ipiv[c0 + tid] = s_pivs[tid];
  // The leaf's swaps (c0 + c <-> s_pivs[c], in order) applied to the other
  // columns of the panel as one gather.  Destinations: the w leaf rows and
  // each distinct pivot row below them; each thread finds the source of its
  // destination by walking the swaps backwards, and all sources are read
  // before any destination is written.
  int pv_[IB];
#pragma unroll
  for (int c = 0; c < IB; ++c) pv_[c] = c < w ? s_pivs[c] : -1;
  // panel columns (clipped to the matrix: in a grouped launch a wide panel can
  // extend past a smaller matrix's last column); the leaf's own columns are skipped
  const int ncol = static_cast<int>(pk0 + pkb <= n ? pkb : n - pk0);
  constexpr int H = 2048 / NT;  // 2 w pkb <= 2048 elements
  T v[H];
  int64_t dst[H], col[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const int e = tid + NT * h;
    v[h] = czero<T>();
    col[h] = 0;
    dst[h] = -1;
    const int k = e / ncol;
    if (k < 2 * w) {
      int key = -1;
      if (k < w) {
        key = static_cast<int>(c0) + k;
      } else {
        const int j = k - w;
        int pj = -1;
#pragma unroll
        for (int c = 0; c < IB; ++c)
          if (c == j) pj = pv_[c];
        bool first = pj >= c0 + w;
#pragma unroll
        for (int c = 0; c < IB; ++c)
          if (c < j && pv_[c] == pj) first = false;
        if (first) key = pj;
      }
      if (key >= 0) {
        int src = key;
#pragma unroll
        for (int c = IB - 1; c >= 0; --c)
          if (c < w) {
            const int top = static_cast<int>(c0) + c;
            if (src == top) src = pv_[c];
            else if (src == pv_[c]) src = top;
          }
        col[h] = pk0 + e % ncol;
        if ((col[h] < c0 || col[h] >= c0 + w) && src != key) {
          v[h] = M[static_cast<int64_t>(src) * ld + col[h]];
          dst[h] = key;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < H; ++h)
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
  // (grouped: a panel wider than what is left of a smaller matrix is clipped
  // to its last row and column; a matrix already factored has nothing to swap)
  const int kbe = static_cast<int>(r0 + kb <= n ? kb : n - r0);
  if (kbe <= 0) return;
  const int64_t chie = chi < n ? chi : n;
  const int32_t *ipiv = ipiv_all + b * n_in;
  const int64_t t = blockIdx.x * 256ll + threadIdx.x;
  const int64_t ncols = clo + (n - chie);
  if (t >= ncols) return;
  const int64_t col = (t < clo) ? t : chie + (t - clo);
  for (int i = 0; i < kbe; ++i) {
    const int64_t r = r0 + i, p = ipiv[r];
    if (p != r) {
      const T x = M[r * ld + col];
      M[r * ld + col] = M[p * ld + col];
      M[p * ld + col] = x;
    }
  }
}

// X = L11^{-1} X with L11 unit lower (w1 x w1), X (w1 x w2), w1, w2 <= 64, both
// inside the matrix; one workgroup of 256 threads per matrix, X in registers
// (the layout of k_diag_inv), forward substitution with one barrier per row.
template <typename T>
__global__ __launch_bounds__(256) void k_trsm_small(T *__restrict__ Mall, int64_t ld,
                                                    int64_t stride, int64_t c0, int w1, int w2) {
  using Tr = cplx_traits<T>;
  __shared__ T sL[64][65];
  __shared__ T rowb[2][4][64];
  T *M = Mall + blockIdx.x * stride;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    sL[i][j] = (i < w1 && j < w1) ? M[(c0 + i) * ld + c0 + j] : czero<T>();
  }
  T x[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = ti + 16 * a, j = tj + 16 * c;
      x[a][c] = (i < w1 && j < w2) ? M[(c0 + i) * ld + c0 + w1 + j] : czero<T>();
    }
  for (int i = 0; i + 1 < w1; ++i) {
    if (ti == (i & 15))  // the owners of row i publish it (all four row blocks)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) rowb[i & 1][a][tj + 16 * c] = x[a][c];
    __syncthreads();
    T la[4], xb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) la[a] = sL[ti + 16 * a][i];
#pragma unroll
    for (int c = 0; c < 4; ++c) xb[c] = rowb[i & 1][i >> 4][tj + 16 * c];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (16 * a + 4 * wv + 3 <= i) continue;
      const T l = (ti + 16 * a > i) ? la[a] : czero<T>();  // rows r > i only
#pragma unroll
      for (int c = 0; c < 4; ++c) x[a][c] = Tr::fms(x[a][c], l, xb[c]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = ti + 16 * a, j = tj + 16 * c;
      if (i >= 1 && i < w1 && j < w2) M[(c0 + i) * ld + c0 + w1 + j] = x[a][c];
    }
}

// One recursion step of the panel factorisation for w1, w2 <= 32:
//   X = L11^{-1} X      for X = M[c0:c0+w1, c0+w1:c0+w1+w2], L11 unit lower (w1 x w1),
//   C -= L21 X          for C = M[c0+w1:n, c0+w1:c0+w1+w2], L21 = M[c0+w1:n, c0:c0+w1].
// The update is a rank-w1 product with w1 <= 32: it is bound by the traffic of
// C, so it runs on the VALU.
constexpr int kPU = 32;
// The small triangular solve of one matrix by one workgroup: L11 and X staged
// in LDS, forward substitution with eight lanes per column sharing each inner
// product, rows 1.. of the solved X stored back.
template <typename T>
__device__ void panel_solve_body(T *__restrict__ M, int64_t ld, int64_t c0, int w1, int w2,
                                 T (*sL)[kPU + 1], T (*sX)[kPU + 1]) {
  using Tr = cplx_traits<T>;
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
  for (int e = tid; e < w1 * w2; e += 256) {
    const int i = e / w2, j = e % w2;
    if (i > 0) M[(c0 + i) * ld + c0 + w1 + j] = sX[i][j];
  }
}

// The panel update in two launches: the small triangular solve once per
// matrix (k_panel_solve: X = L11^{-1} X written back), then the rank-w1 update
// of the rows below by every 64-row chunk (k_panel_rank, reading the solved X).
// (Fusing both into one launch makes every chunk repeat the solve, a chain of
// up to 31 dependent LDS steps that then dominates the launch: measured slower.)
template <typename T>
__global__ __launch_bounds__(256) void k_panel_solve(T *__restrict__ Mall, int64_t ld_in,
                                                     int64_t stride, int64_t n_in, int64_t c0,
                                                     int w1, int w2,
                                                     const GrpMat *__restrict__ grp, int nodes) {
  __shared__ T sL[64][kPU + 1];
  __shared__ T sX[kPU][kPU + 1];
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, blockIdx.x);
  if (c0 + w1 + w2 > mr.n) return;
  panel_solve_body<T>(mr.M, mr.ld, c0, w1, w2, sL, sX);
}

template <typename T>
__global__ __launch_bounds__(256) void k_panel_rank(T *__restrict__ Mall, int64_t ld_in,
                                                    int64_t stride, int64_t n_in, int64_t c0,
                                                    int w1, int w2,
                                                    const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  __shared__ T sL[64][kPU + 1];
  __shared__ T sX[kPU][kPU + 1];
  const MatRef<T> mr = mat_of<T>(grp, nodes, Mall, ld_in, stride, n_in, blockIdx.y);
  T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  if (c0 + w1 + w2 > n) return;
  const int64_t r0 = c0 + w1 + static_cast<int64_t>(blockIdx.x) * 64;
  if (r0 >= n) return;  // (a chunk beyond a smaller matrix of a grouped launch)
  const int rows = static_cast<int>((n - r0 < 64) ? n - r0 : 64);
  const int tid = threadIdx.x;
  for (int e = tid; e < w1 * w2; e += 256) {
    const int i = e / w2, j = e % w2;
    sX[i][j] = M[(c0 + i) * ld + c0 + w1 + j];
  }
  for (int e = tid; e < rows * w1; e += 256) {
    const int i = e / w1, k = e % w1;
    sL[i][k] = M[(r0 + i) * ld + c0 + k];
  }
  const int ti = tid >> 4, tj = tid & 15;
  T acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      acc[a][b] = (i < rows && j < w2) ? M[(r0 + i) * ld + c0 + w1 + j] : Tr::make(0.0, 0.0);
    }
  __syncthreads();
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

// LU with partial pivoting (largest |re| + |im|, lowest row on ties, as the
// leaves) of small matrices held whole in LDS: a persistent grid whose
// workgroups take matrices b = blockIdx.x, blockIdx.x + gridDim.x, ... of a
// grouped table (order n_b <= NP), each factored column by column -- pivot
// search over the column, row exchange, multipliers, rank-1 update of the
// trailing block -- with the rows and columns spread over the 256 threads.
// Pivots (LAPACK order) to ipiv_all + b pstride, info_all[b] = 1 + the first
// column with an exact zero pivot (or 0).
template <typename T, int NP>
__global__ __launch_bounds__(256) void k_lu_small(const GrpMat *__restrict__ grp, int nodes,
                                                  int count, int64_t pstride,
                                                  int32_t *__restrict__ ipiv_all,
                                                  int32_t *__restrict__ info_all) {
  using Tr = cplx_traits<T>;
  using PK = PivKey<T>;
  static_assert(NP <= 256, "one row per thread in the pivot search");
  __shared__ T sM[NP][NP + 1];
  __shared__ T sl[NP];
  __shared__ uint64_t s_key[4];
  __shared__ int s_piv[NP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b = blockIdx.x; b < count; b += gridDim.x) {
    const MatRef<T> mr = mat_of<T>(grp, nodes, static_cast<T *>(nullptr), 0, 0, 0, b);
    T *M = mr.M;
    const int64_t ld = mr.ld;
    const int n = static_cast<int>(mr.n);
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e - i * n;
      sM[i][j] = M[i * ld + j];
    }
    __syncthreads();
    int info = 0;
    for (int c = 0; c < n; ++c) {
      // pivot search: thread t looks at row c + t
      const int r = c + tid;
      uint64_t k = (r < n) ? PK::key(sM[r][c], r) : 0;
      uint64_t wk = wave_max_u64(k);
      if (lane == 0) s_key[wave] = wk;
      __syncthreads();
      uint64_t best = s_key[0];
      for (int w = 1; w < 4; ++w) best = s_key[w] > best ? s_key[w] : best;
      int p = c;
      if constexpr (PK::kPacked) {
        if (best != 0) p = static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(best));
      } else if (best != 0) {
        // ties in value: the lowest row among the candidates holding the maximum
        __syncthreads();
        const uint64_t ik = (k == best && k != 0) ? 0xFFFFFFFFull - static_cast<uint32_t>(r) : 0;
        wk = wave_max_u64(ik);
        if (lane == 0) s_key[wave] = wk;
        __syncthreads();
        uint64_t bi = s_key[0];
        for (int w = 1; w < 4; ++w) bi = s_key[w] > bi ? s_key[w] : bi;
        p = static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(bi));
      }
      if (best == 0 && info == 0) info = c + 1;  // (no comparable entry: keep the diagonal row)
      if (tid == 0) s_piv[c] = p;
      // exchange rows c and p
      if (p != c)
        for (int j = tid; j < n; j += 256) {
          const T x = sM[c][j];
          sM[c][j] = sM[p][j];
          sM[p][j] = x;
        }
      __syncthreads();
      const T piv = sM[c][c];
      const bool zero = piv.x == 0 && piv.y == 0;
      if (zero && info == 0) info = c + 1;
      const T inv = zero ? czero<T>() : Tr::recip(piv);
      if (r > c && r < n) {
        const T l = Tr::mul(sM[r][c], inv);
        sl[r] = l;
        sM[r][c] = l;
      }
      __syncthreads();
      // rank-1 update of the trailing block: thread (tr, tc) = (tid / 16, tid % 16)
      for (int i = c + 1 + (tid >> 4); i < n; i += 16) {
        const T l = sl[i];
        for (int j = c + 1 + (tid & 15); j < n; j += 16) sM[i][j] = Tr::fms(sM[i][j], l, sM[c][j]);
      }
      __syncthreads();
    }
    for (int e = tid; e < n * n; e += 256) {
      const int i = e / n, j = e - i * n;
      M[i * ld + j] = sM[i][j];
    }
    for (int i = tid; i < n; i += 256) ipiv_all[b * pstride + i] = s_piv[i];
    if (tid == 0) info_all[b] = info;
    __syncthreads();  // (sM, s_piv reused by the next matrix)
  }
}

// Register layout shared by the 64 x 64 triangular kernels below: 256 threads,
// thread (ti, tj) = (tid / 16, tid % 16) holds the 16 entries (ti + 16a,
// tj + 16c), a, c < 4, and wave wv = tid / 64 holds rows ti in [4 wv, 4 wv + 4)
// of every 16-row block.  A substitution step publishes one finished row
// through double-buffered LDS rows, so it needs one barrier, and skips the
// 16 x 16 blocks whose entries it cannot change (a wave-uniform test).  The
// owners of row i write all four of their rows and readers take block i / 16:
// choosing the register block by i would put the array in scratch memory.

// Inverse of one nb x nb diagonal block (nb = 64; lower unit or upper
// non-unit) of each matrix, X = D^{-1} with X = I to start:
//   lower: forward, row i of X is final at step i; rows r > i take
//          X_r. -= D_ri X_i.;
//   upper: backward, X_i. = X_i. / D_ii at step i; rows r < i take
//          X_r. -= D_ri X_i..
// Written zero padded to 64 x 64 at out + b out_stride + I 64^2.
template <typename T>
__global__ __launch_bounds__(256) void k_diag_inv(const T *__restrict__ Mall, int64_t ld_in,
                                                  int64_t stride, int64_t n_in, int nb, int64_t blk0,
                                                  bool lower, T *__restrict__ out,
                                                  int64_t out_stride,
                                                  const GrpMat *__restrict__ grp, int nodes) {
  using Tr = cplx_traits<T>;
  __shared__ T sD[64][65];
  __shared__ T rowb[2][4][64];
  const int64_t I = blk0 + blockIdx.x;
  const int b = blockIdx.y;
  const MatRef<const T> mr = mat_of<const T>(grp, nodes, Mall, ld_in, stride, n_in, b);
  const T *M = mr.M;
  const int64_t ld = mr.ld, n = mr.n;
  const int64_t r0 = I * nb;
  const int rb = static_cast<int>((n - r0 < nb) ? n - r0 : nb);
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    sD[i][j] = (i < rb && j < rb) ? M[(r0 + i) * ld + r0 + j] : czero<T>();
  }
  T x[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      x[a][c] = (ti + 16 * a == tj + 16 * c && ti + 16 * a < rb) ? Tr::make(1.0, 0.0) : czero<T>();
  __syncthreads();
  if (lower) {
    for (int i = 0; i + 1 < rb; ++i) {
      if (ti == (i & 15))  // the owners of row i publish it (all four row blocks)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 4; ++c) rowb[i & 1][a][tj + 16 * c] = x[a][c];
      __syncthreads();
      T la[4], xb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) la[a] = sD[ti + 16 * a][i];
#pragma unroll
      for (int c = 0; c < 4; ++c) xb[c] = rowb[i & 1][i >> 4][tj + 16 * c];
      // masked operands (rows r > i, columns j <= i) instead of masked results:
      // a select on the register array would move it to scratch memory
#pragma unroll
      for (int c = 0; c < 4; ++c) xb[c] = (tj + 16 * c <= i) ? xb[c] : czero<T>();
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (16 * a + 4 * wv + 3 <= i) continue;
        const T l = (ti + 16 * a > i) ? la[a] : czero<T>();
#pragma unroll
        for (int c = 0; c <= a; ++c) {  // X_rj = 0 for j > r
          if (16 * c > i) continue;
          x[a][c] = Tr::fms(x[a][c], l, xb[c]);
        }
      }
    }
  } else {
    for (int i = rb - 1; i >= 0; --i) {
      {  // the owners of row i scale and publish it (selects keep x in registers)
        const T di = Tr::recip(sD[i][i]);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const T f = (ti + 16 * a == i) ? di : Tr::make(1.0, 0.0);
#pragma unroll
          for (int c = 0; c < 4; ++c) x[a][c] = Tr::mul(x[a][c], f);
        }
        if (ti == (i & 15))
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) rowb[i & 1][a][tj + 16 * c] = x[a][c];
      }
      __syncthreads();
      if (i == 0) break;
      T ua[4], xb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) ua[a] = sD[ti + 16 * a][i];
#pragma unroll
      for (int c = 0; c < 4; ++c) xb[c] = rowb[i & 1][i >> 4][tj + 16 * c];
#pragma unroll
      for (int c = 0; c < 4; ++c) xb[c] = (tj + 16 * c >= i) ? xb[c] : czero<T>();
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (16 * a + 4 * wv >= i) continue;
        const T u = (ti + 16 * a < i) ? ua[a] : czero<T>();  // rows r < i only
#pragma unroll
        for (int c = a; c < 4; ++c) {  // X_rj = 0 for j < r
          if (16 * c + 15 < i) continue;
          x[a][c] = Tr::fms(x[a][c], u, xb[c]);
        }
      }
    }
  }
  T *o = out + b * out_stride + I * static_cast<int64_t>(nb) * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) o[(ti + 16 * a) * nb + tj + 16 * c] = x[a][c];
}

// Inverse of a 128-row diagonal block of a triangular factor from the inverses
// I1, I2 of its two 64-row halves (zero padded past the order) and the
// off-diagonal 64 x 64 block C of the factor:
//   lower (unit):  [L11 0; C L22]^{-1} = [I1 0; -I2 C I1  I2]
//   upper:         [U11 C; 0 U22]^{-1} = [I1  -I1 C I2; 0 I2]
// One workgroup per (block, matrix); the two 64 x 64 x 64 products run from
// LDS, 16 outputs per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_inv_pair(const T *__restrict__ F, int64_t ld,
                                                  int64_t fstride, int64_t n,
                                                  const T *__restrict__ inv64, int64_t istride,
                                                  T *__restrict__ inv128, int64_t istride2,
                                                  bool lower) {
  using Tr = cplx_traits<T>;
  __shared__ T sA[64][65];
  __shared__ T sB[64][65];
  const int64_t B = blockIdx.x, b = blockIdx.y;
  const int64_t r0 = 128 * B;
  const int h2 = static_cast<int>((n - r0 - 64 < 64) ? n - r0 - 64 : 64);  // rows of the second half
  const T *M = F + b * fstride;
  const T *I1 = inv64 + b * istride + (2 * B) * 4096;
  const T *I2 = I1 + 4096;
  T *out = inv128 + b * istride2 + B * 16384;
  const int tid = threadIdx.x;
  // the two diagonal halves (the second one absent when h2 <= 0)
  for (int e = tid; e < 128 * 128; e += 256) {
    const int i = e >> 7, j = e & 127;
    T v = czero<T>();
    if (i < 64 && j < 64) v = I1[i * 64 + j];
    else if (i >= 64 && j >= 64 && h2 > 0) v = I2[(i - 64) * 64 + (j - 64)];
    out[e] = v;
  }
  if (h2 <= 0) return;
  // first product: lower T = C I1 (C = rows [r0+64, r0+64+h2) x cols [r0, r0+64)),
  //                upper T = I1 C (C = rows [r0, r0+64) x cols [r0+64, r0+64+h2))
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e >> 6, j = e & 63;
    if (lower) {
      sA[i][j] = (i < h2) ? M[(r0 + 64 + i) * ld + r0 + j] : czero<T>();
      sB[i][j] = I1[i * 64 + j];
    } else {
      sA[i][j] = I1[i * 64 + j];
      sB[i][j] = (j < h2) ? M[(r0 + i) * ld + r0 + 64 + j] : czero<T>();
    }
  }
  __syncthreads();
  T acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e >> 6, j = e & 63;
    T x = czero<T>();
    for (int l = 0; l < 64; ++l) x = Tr::fms(x, sA[i][l], sB[l][j]);  // accumulates -(A B)
    acc[q] = x;
  }
  __syncthreads();
  // second product with the negated first one: lower X = I2 (-C I1), upper X = (-I1 C) I2
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e >> 6, j = e & 63;
    if (lower) {
      sB[i][j] = acc[q];
      sA[i][j] = I2[i * 64 + j];
    } else {
      sA[i][j] = acc[q];
      sB[i][j] = I2[i * 64 + j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e >> 6, j = e & 63;
    T x = czero<T>();
    for (int l = 0; l < 64; ++l) x = Tr::fms(x, sA[i][l], sB[l][j]);
    // x = -(sA sB): negate back to the product of the (already negated) factors
    x.x = -x.x;
    x.y = -x.y;
    if (lower) out[(64 + i) * 128 + j] = x;
    else out[i * 128 + 64 + j] = x;
  }
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

template <typename T, int RPT, int IB, int NT = 1024>
void launch_leaf(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                 int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info,
                 const GrpMat *grp, int nodes) {
  hipLaunchKernelGGL((k_leaf<T, NT, RPT, IB>), dim3(batch), dim3(NT), 0, s, M, ld, stride, n, c0, w,
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
  if (w < 1 || w > leaf_max_width<z64>(rows) || 2 * w * pkb > 2048) return false;
  // (complex128 leaves of up to 2048 rows run a little faster with 512 threads)
  if (rows <= 1024)
    launch_leaf<z64, 2, 8, 512>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
  else if (rows <= 2048)
    launch_leaf<z64, 4, 8, 512>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info, grp, nodes);
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
  if (w < 1 || w > leaf_max_width<c64>(rows) || 2 * w * pkb > 2048) return false;
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
  // (n: the largest order of a grouped launch; every matrix has at most this many columns)
  const int64_t ncols = clo + (n > chi ? n - chi : 0);
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
  hipLaunchKernelGGL((k_trsm_small<T>), dim3(batch), dim3(256), 0, s, M, ld, stride, c0, w1, w2);
}
template void trsm_small<z64>(hipStream_t, z64 *, int64_t, int64_t, int32_t, int64_t, int, int);
template void trsm_small<c64>(hipStream_t, c64 *, int64_t, int64_t, int32_t, int64_t, int, int);

template <> int lu_small_max_order<z64>() { return 64; }
template <> int lu_small_max_order<c64>() { return 128; }

template <typename T>
void lu_small(hipStream_t s, const GrpMat *grp, int nodes, int count, int64_t pstride,
              int32_t *ipiv, int32_t *info) {
  if (count <= 0) return;
  // persistent: at most four workgroups per compute unit, each looping over matrices
  const unsigned grid = static_cast<unsigned>(std::min(count, 1024));
  hipLaunchKernelGGL((k_lu_small<T, (sizeof(T) == 16 ? 64 : 128)>), dim3(grid), dim3(256), 0, s,
                     grp, nodes, count, pstride, ipiv, info);
}
template void lu_small<z64>(hipStream_t, const GrpMat *, int, int, int64_t, int32_t *, int32_t *);
template void lu_small<c64>(hipStream_t, const GrpMat *, int, int, int64_t, int32_t *, int32_t *);

template <typename T>
void panel_update(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                  int64_t c0, int w1, int w2, const GrpMat *grp, int nodes) {
  if (w1 <= 0 || w2 <= 0 || w1 > kPU || w2 > kPU || batch <= 0) return;
  const int64_t rows = n - c0 - w1;
  hipLaunchKernelGGL((k_panel_solve<T>), dim3(batch), dim3(256), 0, s, M, ld, stride, n, c0, w1, w2,
                     grp, nodes);
  if (rows > 0)
    hipLaunchKernelGGL((k_panel_rank<T>), dim3(static_cast<unsigned>((rows + 63) / 64), batch),
                       dim3(256), 0, s, M, ld, stride, n, c0, w1, w2, grp, nodes);
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
  hipLaunchKernelGGL((k_diag_inv<T>), dim3(static_cast<unsigned>(blk1 - blk0), batch), dim3(256),
                     0, s, M, ld, stride, n, nb, blk0, lower, out, out_stride, grp, nodes);
}
template void diag_block_inverse<z64>(hipStream_t, const z64 *, int64_t, int64_t, int32_t,
                                      int64_t, int, int64_t, int64_t, bool, z64 *, int64_t,
                                      const GrpMat *, int);
template void diag_block_inverse<c64>(hipStream_t, const c64 *, int64_t, int64_t, int32_t,
                                      int64_t, int, int64_t, int64_t, bool, c64 *, int64_t,
                                      const GrpMat *, int);

template <typename T>
void inverse_pairs(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                   const T *inv64, int64_t istride, T *inv128, int64_t istride2, bool lower) {
  const int64_t nb2 = (n + 127) / 128;
  if (nb2 <= 0 || batch <= 0) return;
  hipLaunchKernelGGL((k_inv_pair<T>), dim3(static_cast<unsigned>(nb2), batch), dim3(256), 0, s, M,
                     ld, stride, n, inv64, istride, inv128, istride2, lower);
}
template void inverse_pairs<z64>(hipStream_t, const z64 *, int64_t, int64_t, int32_t, int64_t,
                                 const z64 *, int64_t, z64 *, int64_t, bool);
template void inverse_pairs<c64>(hipStream_t, const c64 *, int64_t, int64_t, int32_t, int64_t,
                                 const c64 *, int64_t, c64 *, int64_t, bool);

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
