// Sparse pencils in band form on gfx950: the shifted matrices z_j B - A of a
// pencil whose non-zeros (after a bandwidth-reducing reordering) lie within kl
// subdiagonals and ku superdiagonals.  A and B arrive as values on one shared
// (union) CSR pattern; the node factorisations are band LU factorisations with
// partial pivoting, the node solves band triangular solves, and the products
// A X, B X of the projection CSR x dense products.  (The shifted systems of
// eq. 4-4 are the same; only their storage and factorisation differ from the
// dense path.)
//
// Band LU (row interchanges as in LAPACK's band factorisation): at column k
// the pivot is the largest |re| + |im| among rows k .. k + kl (lowest row on
// ties), the two rows are exchanged on the active columns only, and U gains up
// to kl superdiagonals from the exchanges, so its rows hold WC = kl + ku + 1
// entries.  The multipliers of column k are kept in the order of the
// exchanges, so the forward solve applies exchange k and then column k's
// multipliers, k = 0, 1, ...
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

// Partners for a wave-wide all-reduce without the LDS crossbar: DPP within
// rows of 16 lanes (exchange within pairs, within quads, mirrored within
// eight and within sixteen; each step pairs lanes whose groups already agree),
// then v_permlane16_swap / v_permlane32_swap across rows and halves, which
// hand every lane both members of its pair in the same order.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(u), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, static_cast<uint64_t>(static_cast<uint32_t>(lo)) |
                                        (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32));
}
template <bool ROWS16>
__device__ inline void swap_pair(double v, double &a, double &b) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const unsigned u0 = static_cast<unsigned>(u), u1 = static_cast<unsigned>(u >> 32);
  const auto x = ROWS16 ? __builtin_amdgcn_permlane16_swap(u0, u0, false, false)
                        : __builtin_amdgcn_permlane32_swap(u0, u0, false, false);
  const auto y = ROWS16 ? __builtin_amdgcn_permlane16_swap(u1, u1, false, false)
                        : __builtin_amdgcn_permlane32_swap(u1, u1, false, false);
  a = __builtin_bit_cast(double, static_cast<uint64_t>(x[0]) | (static_cast<uint64_t>(y[0]) << 32));
  b = __builtin_bit_cast(double, static_cast<uint64_t>(x[1]) | (static_cast<uint64_t>(y[1]) << 32));
}
template <bool ROWS16>
__device__ inline void swap_pair(int v, int &a, int &b) {
  const unsigned u = static_cast<unsigned>(v);
  const auto x = ROWS16 ? __builtin_amdgcn_permlane16_swap(u, u, false, false)
                        : __builtin_amdgcn_permlane32_swap(u, u, false, false);
  a = static_cast<int>(x[0]);
  b = static_cast<int>(x[1]);
}

// v of lane l (l wave-uniform) in every lane, through scalar registers
__device__ inline double lane_at(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(u), l);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), l);
  return __builtin_bit_cast(double, static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32));
}

// (key, idx) of the lane with the largest key, the lowest index on ties, in
// every lane of the wavefront (all 64 lanes active)
__device__ inline void wave_argmax(double &key, int &idx) {
  auto take = [&](double ok, int oi) {
    if (ok > key || (ok == key && oi < idx)) {
      key = ok;
      idx = oi;
    }
  };
  // partners: lane ^ 1, lane ^ 2, 7 - lane mod 8, 15 - lane mod 16
  take(dpp_f64<0xB1>(key), __builtin_amdgcn_mov_dpp(idx, 0xB1, 0xF, 0xF, false));
  take(dpp_f64<0x4E>(key), __builtin_amdgcn_mov_dpp(idx, 0x4E, 0xF, 0xF, false));
  take(dpp_f64<0x141>(key), __builtin_amdgcn_mov_dpp(idx, 0x141, 0xF, 0xF, false));
  take(dpp_f64<0x140>(key), __builtin_amdgcn_mov_dpp(idx, 0x140, 0xF, 0xF, false));
  double k0, k1;
  int i0, i1;
  swap_pair<true>(key, k0, k1);  // rows 2r and 2r + 1
  swap_pair<true>(idx, i0, i1);
  key = k0;
  idx = i0;
  take(k1, i1);
  swap_pair<false>(key, k0, k1);  // the two halves
  swap_pair<false>(idx, i0, i1);
  key = k0;
  idx = i0;
  take(k1, i1);
}

constexpr int kBandCH = 32;  // rows staged per chunk (LU: CSR rows; solves: factor and block rows)

// a - b c as four fused multiply-adds (the shared zfms rounds b c first and
// costs six instructions; the band kernels' steps run at one wavefront's
// instruction rate)
__device__ inline z64 band_fms(z64 a, z64 b, z64 c) {
  return zmake(fma(b.y, c.y, fma(-b.x, c.x, a.x)), fma(-b.y, c.x, fma(-b.x, c.y, a.y)));
}

// 1 / (x + i y) with one division: scaled first by the power of two 2^-e that
// puts the larger of |x|, |y| in [1/2, 1) (exact), so the squared modulus lies
// in [1/4, 2] and neither overflows nor underflows; then conj / |.|^2, scaled
// back.  (The shared zrecip, Smith's method, takes two divisions; here the
// reciprocal is on the pivot's critical path.)  x + i y != 0.
__device__ inline z64 band_recip(double x, double y) {
  int e;
  (void)frexp(fmax(fabs(x), fabs(y)), &e);
  const double a = ldexp(x, -e), b = ldexp(y, -e);
  const double d = 1.0 / fma(a, a, b * b);
  return zmake(ldexp(a * d, -e), ldexp(-b * d, -e));
}

// One workgroup (256 threads) per node j.  Thread t < WC owns window column
// slot t for the whole factorisation and keeps that column's rows k .. k + kl
// in registers (w[i] = row k + i; W >= kl + 1 is the compile-time bound); slot
// t holds column k + ((t - k) mod WC).  Every kBandCH columns the workgroup
// stages the next kBandCH incoming rows (row k + kl + 1 enters at column k) as
// dense band rows of z_j B - A in LDS, every load issued before the first
// wait.  The owners (WC <= 64) are lanes of wave 0, which does every column's
// work; the other waves only stage.  Per column k, one wavefront barrier:
//   before it, the owner of column k posts that column to LDS and wave 0 finds
//   the pivot (largest |re| + |im|, lowest row on ties) and the multipliers;
//   after it, every owner exchanges rows k and k + p of its column, writes its
//   entry of U's row k, applies the multipliers, moves its rows up by one and
//   takes the staged row's entry as row k + kl + 1 (the owner of column k
//   starts column k + WC, zero above the new row).
// The multipliers are double-buffered by the parity of k.
template <int W>
__global__ __launch_bounds__(256) void k_band_lu(const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci,
                                                 const z64 *__restrict__ va,
                                                 const z64 *__restrict__ vb,
                                                 const z64 *__restrict__ zn, int64_t n, int kl,
                                                 int ku, z64 *__restrict__ Lf,
                                                 z64 *__restrict__ Uf, z64 *__restrict__ Dinv,
                                                 int32_t *__restrict__ piv,
                                                 int32_t *__restrict__ info) {
  const int KR = kl + 1, WC = kl + ku + 1;
  // one block, so that the per-column arrays sit at the low LDS addresses
  // (immediate offsets) whatever the allocator's order
  struct Lds {
    z64 sl[2][64];  // multipliers of column k (index 1 .. kl), by the parity of k
    z64 colbuf[64];
    int32_t srp[kBandCH + 1];
    int info;
    // the staged rows of two chunks (row q of a chunk at SR[b][q WC + c -
    // (row - kl)], c its column); the first window's rows 0 .. kl pass
    // through SR[0] kBandCH at a time
    z64 SR[2][kBandCH * 64];
  };
  __shared__ Lds sm;
  auto &sl = sm.sl;
  auto &colbuf = sm.colbuf;
  auto &srp = sm.srp;
  auto &s_info = sm.info;
  z64 *SR = sm.SR[0];
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const z64 z = zn[j];
  z64 *L = Lf + static_cast<int64_t>(j) * n * kl;
  z64 *U = Uf + static_cast<int64_t>(j) * n * WC;
  z64 *Di = Dinv + static_cast<int64_t>(j) * n;
  int32_t *pv = piv + static_cast<int64_t>(j) * n;

  // stage rows r0 .. r0 + cnt - 1 (all < n) into SR (row q at SR[q WC + c - (r0 + q - kl)])
  auto stage = [&](int64_t r0, int cnt) {
    for (int e = tid; e < cnt * WC; e += 256) SR[e] = zmake(0.0, 0.0);
    if (tid <= cnt) srp[tid] = rp[r0 + tid];
    __syncthreads();
    const int e0 = srp[0], e1 = srp[cnt];
    // (at most kBandCH rows of at most 64 entries: 8 per thread, loaded 4 at a time)
    for (int h = 0; h < 2; ++h) {
      int32_t c4[4];
      z64 a4[4], b4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + tid + 256 * (4 * h + q);
        const int ee = e < e1 ? e : e0;
        c4[q] = ci[ee];
        a4[q] = va[ee];
        b4[q] = vb[ee];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + tid + 256 * (4 * h + q);
        if (e < e1) {
          int row = 0;  // the chunk row holding entry e
          while (row + 1 < cnt && srp[row + 1] <= e) ++row;
          const z64 b = b4[q], a = a4[q];
          SR[row * WC + c4[q] - (r0 + row - kl)] =
              zmake(z.x * b.x - z.y * b.y - a.x, z.x * b.y + z.y * b.x - a.y);
        }
      }
    }
    __syncthreads();
  };

  // waves 1-3 (192 threads, 6 per row): rows r0 .. r0 + cnt - 1 (< n) into
  // SR[b] while wave 0 factors; each thread owns the slots c = sub mod 6 of
  // its row, zeroes them and writes the row's entries that fall there, so no
  // barrier orders the staging threads among themselves
  static_assert(192 / 6 >= kBandCH, "a staging row per 6 threads");
  auto stage_bg = [&](int b, int64_t r0, int cnt) {
    const int t = tid - 64, row = t / 6, sub = t - 6 * row;
    if (row >= cnt) return;
    z64 *dst = sm.SR[b] + row * WC;
    for (int c = sub; c < WC; c += 6) dst[c] = zmake(0.0, 0.0);
    const int64_t r = r0 + row;
    const int64_t base = r - kl;  // the column of slot 0
    for (int e = rp[r], e1 = rp[r + 1]; e < e1; ++e) {
      const int c = static_cast<int>(ci[e] - base);
      if (c % 6 == sub) {
        const z64 bv = vb[e], av = va[e];
        dst[c] = zmake(z.x * bv.x - z.y * bv.y - av.x, z.x * bv.y + z.y * bv.x - av.y);
      }
    }
  };
  // the rows entering during the chunk of columns k0 .. k0 + kBandCH - 1
  auto chunk_rows = [&](int64_t k0, int64_t *r0) {
    const int ch = static_cast<int>(n - k0 < kBandCH ? n - k0 : kBandCH);
    *r0 = k0 + KR;
    return *r0 < n ? static_cast<int>(n - *r0 < ch ? n - *r0 : ch) : 0;
  };

  if (tid == 0) s_info = 0;
  const bool owner = tid < WC;
  z64 w[W];
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = zmake(0.0, 0.0);
  const int r1 = static_cast<int>(KR < n ? KR : n);  // the first window's rows
  for (int h = 0; h < r1; h += kBandCH) {
    const int cnt = r1 - h < kBandCH ? r1 - h : kBandCH;
    __syncthreads();  // the previous rows are read
    stage(h, cnt);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      // window row i, column tid: SR index (i - h) WC + tid - (i - kl)
      const int c = tid - i + kl;
      if (owner && i >= h && i < h + cnt && c >= 0 && c < WC) w[i] = SR[(i - h) * WC + c];
    }
  }

  __syncthreads();  // the first window is read: SR[0] takes chunk 0's rows
  if (tid >= 64) {
    int64_t r0;
    const int cnt = chunk_rows(0, &r0);
    stage_bg(0, r0, cnt);
  }
  int ck = 0;  // slot of column k
  for (int64_t k0 = 0, c = 0; k0 < n; k0 += kBandCH, ++c) {
    const int ch = static_cast<int>(n - k0 < kBandCH ? n - k0 : kBandCH);
    int64_t r0;
    const int cnt = chunk_rows(k0, &r0);  // incoming rows of this chunk's columns
    const z64 *SRc = sm.SR[c & 1];
    __syncthreads();  // this chunk's rows are staged; the other buffer is free
    if (tid >= 64) {  // the next chunk's rows, while wave 0 factors this one's
      if (k0 + kBandCH < n) {
        int64_t r0n;
        const int cntn = chunk_rows(k0 + kBandCH, &r0n);
        stage_bg(static_cast<int>((c + 1) & 1), r0n, cntn);
      }
      continue;
    }
    for (int kk = 0; kk < ch; ++kk) {
      const int64_t k = k0 + kk;
      const int par = static_cast<int>(k & 1);
      {
        if (tid == ck) {
#pragma unroll
          for (int i = 0; i < W; ++i) colbuf[i] = w[i];  // (rows past k + kl are not read)
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const int i = lane;
        const bool valid = i < KR && k + i < n;
        const z64 v = valid ? colbuf[i] : zmake(0.0, 0.0);
        const double a1 = zabs1(v);
        double key = valid ? (a1 == a1 ? a1 : -1.0) : -2.0;
        int idx = valid ? i : 1 << 30;
        wave_argmax(key, idx);
        key = lane_at(key, 0);  // (every lane holds it: a scalar from here on)
        const int p = __builtin_amdgcn_readfirstlane(idx < KR ? idx : 0);
        const double ux = lane_at(v.x, p), uy = lane_at(v.y, p);
        const double v0x = lane_at(v.x, 0), v0y = lane_at(v.y, 0);
        const bool zero = !(key > 0.0);
        const z64 inv = zero ? zmake(0.0, 0.0) : band_recip(ux, uy);
        if (i >= 1 && i < W) {  // zero past row k + kl and past row n - 1
          const z64 src = (i == p) ? zmake(v0x, v0y) : v;
          const z64 l = valid ? zmul(src, inv) : zmake(0.0, 0.0);
          sl[par][i] = l;
          if (i < KR) L[k * kl + (i - 1)] = l;
        }
        if (lane == 0) {
          pv[k] = static_cast<int32_t>(k + p);
          Di[k] = inv;
          if (zero && s_info == 0) s_info = static_cast<int>(k) + 1;
        }
        // every owner is a lane of this wavefront: a wavefront barrier makes
        // the multipliers visible
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (owner) {
          int jo = tid - ck;  // this column's offset from column k
          if (jo < 0) jo += WC;
          // exchange rows k and k + p (row k's slot is dead after the step):
          // one uniform branch per slot, the empty asm keeping each arm a
          // branch rather than a select of four registers per slot
          z64 rpv = w[0];
          if (p != 0) {
#pragma unroll
            for (int i = 1; i < W; ++i)
              if (i == p) {
                asm volatile("" ::: "memory");
                rpv = w[i];
                w[i] = w[0];
              }
          }
          U[k * WC + jo] = (k + jo < n) ? rpv : zmake(0.0, 0.0);
          // the incoming row k + KR at this slot's next column (k + jo, or
          // k + WC for the slot of column k): staged index WC - 1 or jo - 1
          const z64 nv = (kk < cnt) ? SRc[kk * WC + (jo == 0 ? WC - 1 : jo - 1)] : zmake(0.0, 0.0);
          // the multipliers (zero past row k + kl: no bound per row) in groups
          // of G, all in flight before the group's first product
          const z64 *lk = sl[par];
          constexpr int G = W <= 24 ? W - 1 : 8;
#pragma unroll
          for (int g = 1; g < W; g += G) {
            z64 lr[G];
#pragma unroll
            for (int t = 0; t < G; ++t)
              if (g + t < W) lr[t] = lk[g + t];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < G; ++t)
              if (g + t < W) w[g + t] = band_fms(w[g + t], lr[t], rpv);
          }
          // rows move up one slot; the slot of column k (leaving) starts column
          // k + WC with zeros above the incoming row: one multiply by 1 or 0
          // per entry does both (the window's entries are finite).  The widest
          // window has no registers for the products: it zeroes, then moves.
          if constexpr (W <= 48) {
            const double keep = jo == 0 ? 0.0 : 1.0;
#pragma unroll
            for (int i = 0; i + 1 < W; ++i) w[i] = zmake(w[i + 1].x * keep, w[i + 1].y * keep);
          } else {
            if (jo == 0) {
              asm volatile("" ::: "memory");
#pragma unroll
              for (int i = 0; i < W; ++i) w[i] = zmake(0.0, 0.0);
            }
#pragma unroll
            for (int i = 0; i + 1 < W; ++i) w[i] = w[i + 1];
          }
          w[W - 1] = zmake(0.0, 0.0);
#pragma unroll
          for (int i = 0; i < W; ++i)
            if (i == KR - 1) {
              asm volatile("" ::: "memory");
              w[i] = nv;
            }
        }
      }
      if (++ck == WC) ck = 0;
    }
  }
  __syncthreads();
  if (tid == 0) info[j] = s_info;
}

// The node solves Y_j = M_j^{-1} R with M_j's band factors (node j =
// blockIdx.x), as two kernels so that each holds one window in registers:
//   k_band_fwd: exchanges and unit-lower multipliers, two lanes per
//     right-hand side (32 columns of R per blockIdx.y): lanes l and l + 32
//     keep rows k .. k + WF / 2 - 1 and the WF / 2 rows after them of column
//     l (WF >= kl + 1; rows past k + kl wait unchanged) and write row k of
//     the result to Y_j;
//   k_band_bwd: U, four lanes per right-hand side (16 columns per
//     blockIdx.y): lanes l, l + 16, l + 32, l + 48 keep the solved rows
//     k + 1 .. k + WB / 4 of column l and the three runs of WB / 4 rows after
//     them (WB >= kl + ku); each sums its quarter of row k's products, the
//     quarters add, and lane l overwrites row k of Y_j with the solution
//     (times the stored pivot reciprocal).
// Factor rows and block rows are staged kBandCH at a time through LDS (loads
// issued 16 at a time before they are written), so each step reads only LDS
// and registers.
struct BandStage {
  // dst[q P + c] = src[q S + off + c] for lo <= c < lim, zero for the other
  // c < P (rows q < cnt; cnt P <= kBandCH * 64), 16 loads in flight per lane.
  // The zeros pad every factor row to the register window, so a step needs no
  // per-entry bound.
  template <int P>
  __device__ __forceinline__ static void padded(z64 *dst, const z64 *src, int S, int off,
                                                int lo, int lim, int cnt, int lane) {
    for (int h = 0; h < 2; ++h) {
      z64 t[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * (16 * h + q), row = e / P, c = e - row * P;
        t[q] = (row < cnt && c >= lo && c < lim) ? src[row * S + off + c] : zmake(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * (16 * h + q);
        if (e < cnt * P) dst[e] = t[q];
      }
    }
  }
  // rows[q][lane] = M[(r0 + q) ldm + cc] for q < cnt (rows >= lim read as zero)
  __device__ __forceinline__ static void rows(z64 (*dst)[64], const z64 *M, int64_t ldm,
                                              int64_t r0, int cnt, int64_t lim, int64_t cc,
                                              int lane) {
    for (int h = 0; h < 2; ++h) {
      z64 t[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t r = r0 + 16 * h + q;
        t[q] = (16 * h + q < cnt && r < lim) ? M[r * ldm + cc] : zmake(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) dst[16 * h + q][lane] = t[q];
    }
  }
};

// Windows shift once per block of kBandU rows rather than at every row: within
// a block, step r addresses the window kBandU entries further along (forward)
// or back (backward), so the entries stay put and one block move of the
// window follows the block.
constexpr int kBandU = 4;
static_assert(kBandCH % kBandU == 0, "chunks hold whole blocks");

// One row of the forward solve at block step r.  Lanes l and l + 32 share a
// column: slot r + s holds row k + s in the near half (lanes below 32) and row
// k + H + s in the far half, s < H.  Rows k and k + p (p wave-uniform) are
// exchanged inside the near half, or across the halves through
// v_permlane32_swap when p >= H: one uniform branch per slot, the empty asm
// keeping each arm a branch rather than a select of four registers per slot.
// Row k (near slot r, multiplier 0) is y; every slot s takes
// f[s] y off (f: the half's H multipliers, loaded before the first product,
// at most G in flight); then the far half's first row moves to the near
// half's slot r + H and row k + 2H enters the far half there.
template <int H, int r, int N>
__device__ inline z64 band_fwd_row(z64 (&w)[N], const z64 *f, int p, z64 nv, int half) {
  static_assert(r + H < N, "window inside the buffer");
  if (p != 0) {
    if (p < H) {
#pragma unroll
      for (int i = 1; i < H; ++i)
        if (i == p) {
          asm volatile("" ::: "memory");
          if (half == 0) {
            const z64 t = w[r + i];
            w[r + i] = w[r];
            w[r] = t;
          }
        }
    } else {
      const int q = p - H;  // row k + p is far slot r + q
      z64 x = w[r];         // the near half sends row k, the far half row k + p
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (i == q) {
          asm volatile("" ::: "memory");
          if (half) x = w[r + i];
        }
      z64 xn, xf;
      swap_pair<false>(x.x, xn.x, xf.x);
      swap_pair<false>(x.y, xn.y, xf.y);
      if (half == 0) w[r] = xf;
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (i == q) {
          asm volatile("" ::: "memory");
          if (half) w[r + i] = xn;
        }
    }
  }
  z64 y, yf;
  swap_pair<false>(w[r].x, y.x, yf.x);
  swap_pair<false>(w[r].y, y.y, yf.y);
  constexpr int G = H <= 24 ? H : H / 2;
#pragma unroll
  for (int g = 0; g < H; g += G) {
    z64 fr[G];
#pragma unroll
    for (int t = 0; t < G; ++t) fr[t] = f[g + t];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < G; ++t) w[r + g + t] = band_fms(w[r + g + t], fr[t], y);
  }
  z64 un, uf;  // the halves' slot r after the update: far's is row k + H
  swap_pair<false>(w[r].x, un.x, uf.x);
  swap_pair<false>(w[r].y, un.y, uf.y);
  w[r + H] = half ? nv : uf;
  return y;
}

template <int WF>
__global__ __launch_bounds__(128) void k_band_fwd(const z64 *__restrict__ Lf,
                                                  const int32_t *__restrict__ piv, int64_t n,
                                                  int kl, const z64 *__restrict__ R, int64_t ldr,
                                                  int64_t m, z64 *__restrict__ Y, int64_t ldy,
                                                  int64_t sY) {
  constexpr int UF = kBandU, H = WF / 2;
  static_assert(WF % 2 == 0, "two halves of the window");
  // two chunks' staging (wave 1 fills one while wave 0 solves from the other)
  __shared__ z64 fac[2][kBandCH * WF];  // per row: 0, then the kl multipliers, zero-padded
  __shared__ z64 rows[2][kBandCH][64];  // the rows of R entering the window (both halves load them)
  __shared__ int32_t s_piv[2][kBandCH];
  const int j = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63, half = lane >> 5;
  const int64_t col = static_cast<int64_t>(blockIdx.y) * 32 + (lane & 31);
  const bool act = col < m;
  // idle lanes (col >= m, in the last block only) duplicate column m - 1 of
  // their own wavefront, so they may store: same values, same instruction
  const int64_t cc = act ? col : m - 1;
  const z64 *L = Lf + static_cast<int64_t>(j) * n * kl;
  const int32_t *pv = piv + static_cast<int64_t>(j) * n;
  z64 *Yj = Y + static_cast<int64_t>(j) * sY;
  // wave 1: the chunk of rows k0 .. k0 + kBandCH - 1 into buffer b
  auto stage = [&](int b, int64_t k0) {
    const int ch = static_cast<int>(n - k0 < kBandCH ? n - k0 : kBandCH);
    BandStage::padded<WF>(fac[b], L + k0 * kl, kl, -1, 1, kl + 1, ch, lane);
    if (lane < ch) s_piv[b][lane] = pv[k0 + lane] - static_cast<int32_t>(k0 + lane);
    BandStage::rows(rows[b], R, ldr, k0 + WF, ch, n, cc, lane);
  };
  z64 w[H + UF];
#pragma unroll
  for (int i = 0; i < H + UF; ++i) {
    const int64_t row = static_cast<int64_t>(half) * H + i;
    w[i] = (i < H && row < n) ? R[row * ldr + cc] : zmake(0.0, 0.0);
  }
  if (wv == 1) stage(0, 0);
  for (int64_t k0 = 0, c = 0; k0 < n; k0 += kBandCH, ++c) {
    const int ch = static_cast<int>(n - k0 < kBandCH ? n - k0 : kBandCH);
    const int b = static_cast<int>(c & 1);
    __syncthreads();  // this chunk is staged; the other buffer is free
    if (wv == 1) {
      if (k0 + kBandCH < n) stage(b ^ 1, k0 + kBandCH);
      continue;
    }
    for (int kb = 0; kb < ch; kb += UF) {
      const z64 *f = fac[b] + kb * WF + half * H;
      // unconditional stores (no divergent branch in the row; both halves
      // store the same y)
      z64 *yk = Yj + (k0 + kb) * ldy + cc;
      // the last chunk may end inside a block (ch - kb < UF)
      const int nb = __builtin_amdgcn_readfirstlane(ch - kb);
      // the block's exchanges, read together (kb + UF <= kBandCH: in bounds)
      int pb[UF];
#pragma unroll
      for (int r = 0; r < UF; ++r) pb[r] = s_piv[b][kb + r];
#define FEAST_FWD_STEP(r)                                                                   \
  if (r < nb) {                                                                             \
    const int p = __builtin_amdgcn_readfirstlane(pb[r]);                                    \
    const z64 y = band_fwd_row<H, r>(w, f + r * WF, p, rows[b][kb + r][lane], half);        \
    yk[r * ldy] = y;                                                                        \
  }
      FEAST_FWD_STEP(0) FEAST_FWD_STEP(1) FEAST_FWD_STEP(2) FEAST_FWD_STEP(3)
#undef FEAST_FWD_STEP
#pragma unroll
      for (int i = 0; i < H; ++i) w[i] = w[i + UF];
    }
  }
}

// Across the four quarters of a wavefront (lanes l, l + 16, l + 32, l + 48 for
// l < 16): the sum of v over the four, added in the same order in every lane,
// and the value of the previous quarter (quarter 0 gets its own back).
__device__ inline double quarter_sum(double v) {
  double a, b, c, d;
  swap_pair<false>(v, a, b);  // quarters 0 + 2 and 1 + 3
  swap_pair<true>(a + b, c, d);
  return c + d;
}
__device__ inline double quarter_prev(double v, int qt) {
  double e, o, lo, hi;
  swap_pair<true>(v, e, o);                   // even and odd quarter's of each pair
  swap_pair<false>(qt == 0 ? o : v, lo, hi);  // quarter 2 gets quarter 0's: quarter 1's value
  return (qt & 1) ? e : (qt == 2 ? lo : v);
}

template <int WB>
__global__ __launch_bounds__(128) void k_band_bwd(const z64 *__restrict__ Uf,
                                                  const z64 *__restrict__ Dinv, int64_t n, int kl,
                                                  int ku, int64_t m, z64 *__restrict__ Y,
                                                  int64_t ldy, int64_t sY) {
  constexpr int UB = kBandU, Q = WB / 4;
  static_assert(WB % 4 == 0 && Q >= UB, "a quarter's block rows come from the quarter before");
  const int WC = kl + ku + 1, WU = kl + ku;
  // two chunks' staging (wave 1 fills one while wave 0 solves from the other)
  __shared__ z64 fac[2][kBandCH * WB];  // rows of U past the diagonal (WU each, zero-padded)
  __shared__ z64 rows[2][kBandCH][64];  // the forward results of those rows (all quarters)
  __shared__ z64 dinv[2][kBandCH];
  const int j = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63, qt = lane >> 4;
  const int64_t col = static_cast<int64_t>(blockIdx.y) * 16 + (lane & 15);
  const bool act = col < m;
  const int64_t cc = act ? col : m - 1;
  const z64 *U = Uf + static_cast<int64_t>(j) * n * WC;
  const z64 *Di = Dinv + static_cast<int64_t>(j) * n;
  z64 *Yj = Y + static_cast<int64_t>(j) * sY;
  // Lanes l, l + 16, l + 32, l + 48 share column l: quarter q sums the terms
  // t = qQ + 1 .. (q + 1)Q of row k.  Step r of a block (rows descending):
  // b[UB - 1 - r + t] = solved row k + qQ + t, t = 1 .. Q; rows past n - 1
  // stay zero (and U's entries there are stored zero).
  // wave 1: the chunk of rows k1 - kBandCH .. k1 - 1 (from 0) into buffer bf;
  // its rows of Y hold forward results until wave 0 reaches them
  auto stage = [&](int bf, int64_t k1) {
    const int ch = static_cast<int>(k1 < kBandCH ? k1 : kBandCH);
    const int64_t kb0 = k1 - ch;
    BandStage::padded<WB>(fac[bf], U + kb0 * WC, WC, 1, 0, WU, ch, lane);
    if (lane < ch) dinv[bf][lane] = Di[kb0 + lane];
    BandStage::rows(rows[bf], Yj, ldy, kb0, ch, n, cc, lane);
  };
  z64 b[Q + UB];
#pragma unroll
  for (int i = 0; i < Q + UB; ++i) b[i] = zmake(0.0, 0.0);
  if (wv == 1) stage(0, n);
  for (int64_t k1 = n, c = 0; k1 > 0; k1 -= kBandCH, ++c) {
    const int ch = static_cast<int>(k1 < kBandCH ? k1 : kBandCH);
    const int64_t kb0 = k1 - ch;  // rows kb0 .. k1 - 1
    const int bf = static_cast<int>(c & 1);
    __syncthreads();  // this chunk is staged; the other buffer is free
    if (wv == 1) {
      if (kb0 > 0) stage(bf ^ 1, kb0);
      continue;
    }
    for (int q = 0; q < ch; q += UB) {
      // a quarter's first UB slots are the previous quarter's last UB
      // (quarter 0's own are rewritten by this block's rows before it reads
      // them)
#pragma unroll
      for (int i = 0; i < UB; ++i)
        b[i] = zmake(quarter_prev(b[Q + i].x, qt), quarter_prev(b[Q + i].y, qt));
      // the last chunk may end inside a block
      const int nb = __builtin_amdgcn_readfirstlane(ch - q);
#pragma unroll
      for (int r = 0; r < UB; ++r) {
        if (r < nb) {
          const int kk = ch - 1 - (q + r);
          const z64 *f = fac[bf] + kk * WB + qt * Q;
          z64 s2[2] = {qt == 0 ? rows[bf][kk][lane] : zmake(0.0, 0.0), zmake(0.0, 0.0)};
          // the quarter's factor loads all in flight before its first product
          z64 fr[Q];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int t = 0; t < Q; ++t) fr[t] = f[t];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int t = 1; t <= Q; ++t)
            s2[t & 1] = band_fms(s2[t & 1], fr[t - 1], b[UB - 1 - r + t]);
          const z64 sq = zadd(s2[0], s2[1]);
          const z64 y = zmul(zmake(quarter_sum(sq.x), quarter_sum(sq.y)), dinv[bf][kk]);
          if (qt == 0) {
            if (act) Yj[(kb0 + kk) * ldy + col] = y;
            b[UB - 1 - r] = y;
          }
        }
      }
#pragma unroll
      for (int i = Q - 1; i >= 0; --i) b[i + UB] = b[i];
    }
  }
}

// YA = A X and YB = B X (either may be null) on the union pattern: one
// wavefront per row, lanes over the columns.
__global__ __launch_bounds__(256) void k_csr_spmm(const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci,
                                                  const z64 *__restrict__ va,
                                                  const z64 *__restrict__ vb, int64_t n,
                                                  const z64 *__restrict__ X, int64_t ldx,
                                                  int64_t m, z64 *__restrict__ YA, int64_t ldya,
                                                  z64 *__restrict__ YB, int64_t ldyb) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const int e0 = rp[row], e1 = rp[row + 1];
  for (int64_t c0 = 0; c0 < m; c0 += 64) {
    const int64_t col = c0 + lane;
    if (col >= m) break;
    z64 sa = zmake(0.0, 0.0), sb = zmake(0.0, 0.0);
    for (int e = e0; e < e1; ++e) {
      const z64 x = X[static_cast<int64_t>(ci[e]) * ldx + col];
      if (YA) {
        const z64 a = va[e];
        sa = zadd(sa, zmul(a, x));
      }
      if (YB) {
        const z64 b = vb[e];
        sb = zadd(sb, zmul(b, x));
      }
    }
    if (YA) YA[row * ldya + col] = sa;
    if (YB) YB[row * ldyb + col] = sb;
  }
}

// dst[e] = src[map[e]] (or zero where map[e] < 0)
__global__ __launch_bounds__(256) void k_gather_vals(const int32_t *__restrict__ map,
                                                     const z64 *__restrict__ src, int64_t cnt,
                                                     z64 *__restrict__ dst) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= cnt) return;
  const int32_t s = map[e];
  dst[e] = s >= 0 ? src[s] : zmake(0.0, 0.0);
}

}  // namespace

namespace {
// register window classes of the band kernels
int band_class(int w) { return w <= 16 ? 16 : w <= 24 ? 24 : w <= 32 ? 32 : w <= 48 ? 48 : 64; }

#define FEAST_BAND_DISPATCH(cls, KERNEL, ...)                                   \
  switch (cls) {                                                               \
    case 16: hipLaunchKernelGGL((KERNEL<16>), __VA_ARGS__); break;             \
    case 24: hipLaunchKernelGGL((KERNEL<24>), __VA_ARGS__); break;             \
    case 32: hipLaunchKernelGGL((KERNEL<32>), __VA_ARGS__); break;             \
    case 48: hipLaunchKernelGGL((KERNEL<48>), __VA_ARGS__); break;             \
    default: hipLaunchKernelGGL((KERNEL<64>), __VA_ARGS__); break;             \
  }
}  // namespace

// (kl + ku <= 63: kl + 1 <= 64 rows in the registers of a column owner, and at
// most 64 owners, all in the first wavefront)
void band_lu(hipStream_t s, const int32_t *rp, const int32_t *ci, const z64 *va, const z64 *vb,
             const z64 *z, int32_t N, int64_t n, int kl, int ku, z64 *Lf, z64 *Uf, z64 *Dinv,
             int32_t *piv, int32_t *info) {
  if (N <= 0 || n <= 0) return;
  FEAST_BAND_DISPATCH(band_class(kl + 1), k_band_lu, dim3(N), dim3(256), 0, s, rp, ci, va, vb, z,
                      n, kl, ku, Lf, Uf, Dinv, piv, info)
}

void band_solve(hipStream_t s, const z64 *Lf, const z64 *Uf, const z64 *Dinv, const int32_t *piv,
                int32_t N, int64_t n, int kl, int ku, const z64 *R, int64_t ldr, int64_t m,
                z64 *Y, int64_t ldy, int64_t sY) {
  if (N <= 0 || n <= 0 || m <= 0) return;
  // forward: 32 columns per wavefront (two lanes each); backward: 16 (four)
  const dim3 gf(N, static_cast<unsigned>((m + 31) / 32));
  const dim3 gb(N, static_cast<unsigned>((m + 15) / 16));
  // (a second wavefront per block stages the next chunk)
  FEAST_BAND_DISPATCH(band_class(kl + 1), k_band_fwd, gf, dim3(128), 0, s, Lf, piv, n, kl, R,
                      ldr, m, Y, ldy, sY)
  FEAST_BAND_DISPATCH(band_class(kl + ku), k_band_bwd, gb, dim3(128), 0, s, Uf, Dinv, n, kl, ku,
                      m, Y, ldy, sY)
}

void csr_spmm(hipStream_t s, const int32_t *rp, const int32_t *ci, const z64 *va, const z64 *vb,
              int64_t n, const z64 *X, int64_t ldx, int64_t m, z64 *YA, int64_t ldya, z64 *YB,
              int64_t ldyb) {
  if (n <= 0 || m <= 0) return;
  hipLaunchKernelGGL(k_csr_spmm, dim3(static_cast<unsigned>((n + 3) / 4)), dim3(256), 0, s, rp, ci,
                     va, vb, n, X, ldx, m, YA, ldya, YB, ldyb);
}

void gather_vals(hipStream_t s, const int32_t *map, const z64 *src, int64_t cnt, z64 *dst) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_gather_vals, dim3(static_cast<unsigned>((cnt + 255) / 256)), dim3(256), 0, s,
                     map, src, cnt, dst);
}

}  // namespace feast
