// Batched complex GEMM on the gfx950 matrix cores.
//
//   C_b = alpha * op(A_b) * B_b + beta * C_b        (row-major, interleaved complex)
//
// FP64 (z64): every complex 16x16x4 tile product is four real
// v_mfma_f64_16x16x4_f64 products (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br),
// i.e. 8 real flops per complex multiply-add, the count the roofline uses.
// FP32 (c64): the same structure on v_mfma_f32_16x16x4_f32.
//
// Tiles: BM x BN outputs per 256-thread workgroup (4 waves in a 2x2 grid, each
// wave owning a (BM/2) x (BN/2) block of 16x16 MFMA tiles), K in steps of 16
// complex.  Operands are staged through LDS as separate real/imaginary planes
// stored k-major, so that each MFMA operand fragment is 16 consecutive LDS
// words per k row; the next K step is prefetched into registers while the
// current one is multiplied (two LDS buffers, one barrier per step).
//
// Lane layouts (measured on gfx950):
//   A operand (16x4): lane l holds A[l%16][l/16]; B operand (4x16): B[l/16][l%16]
//   f64 result: lane l, element r holds D[4r + l/16][l%16]
//   f32 result: lane l, element r holds D[4(l/16) + r][l%16]
//
// A launch covers batch x splits x tiles workgroups mapped XCD-contiguously.
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

template <typename T> struct mfma_ops;

template <> struct mfma_ops<z64> {
  using real = double;
  using acc_t = dx4;
  __device__ static acc_t mma(real a, real b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of element r of the 16x16 result held by `lane`
  __device__ static int out_row(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <> struct mfma_ops<c64> {
  using real = float;
  using acc_t = fx4;
  __device__ static acc_t mma(real a, real b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int out_row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T> __device__ inline T ld_cplx(const T *p) { return *p; }

// SUB = true computes C -= op(A) B exactly: the accumulators start from C (loaded
// before the K loop, so its latency overlaps the first operand loads) and the
// MFMAs use -A; the epilogue is then a plain store.  SUB = false is the general
// C = alpha op(A) B + beta C with the C read in the epilogue.
// One output tile: `lin` indexes the tiles x batch x splits of problem d.
//
// SHF (with SUB, TA = 0): the A operand is shift[b] A2 - A, formed from the two
// staged tiles in registers before they are written to LDS, and the
// accumulators start from C0 rather than C (C = C0 - (shift A2 - A) B).
//
// NG > 1: the workgroup is NG groups of 256 threads, each with LDS planes of
// its own, working on NG tiles at once.  A group's four wavefronts meet at a
// barrier of their own (an LDS counter, gcount, that each wavefront raises by
// one per barrier and waits on until it reaches *gphase), so the groups do
// not run in lockstep: while one waits for its operands another computes.
// A group with no tile of its own passes own = false with any valid lin: it
// stages operands but issues no MFMAs or stores.
constexpr int kFoldK = 128;  // three-product form: K steps between folds of T1 (power of 2)

template <typename T, int BM, int BN, int TA, bool SUB, int BK, bool M3, bool SHF = false,
          bool PIPE = true, int NG = 1>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T> &d, int64_t lin, bool own = true,
                                          uint32_t *gcount = nullptr, uint32_t *gphase = nullptr) {
  static_assert(!SHF || (SUB && TA == 0), "shifted operand: C0 - (s A2 - A) B only");
  using Ops = mfma_ops<T>;
  using real = typename Ops::real;
  using acc_t = typename Ops::acc_t;
  static_assert(BK == 8 || BK == 16, "BK");
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  // LDS row pitch (32 banks of 4 bytes).  FP64 planes: a read of 16
  // consecutive doubles covers the 32 banks; an odd pitch keeps the 16 rows of
  // an A store apart.  complex64 planes: pitch BM + 2 (reads of rows k and k+1
  // then share banks 2-way; an XOR swizzle removing that measured no faster
  // and costs registers).
  constexpr bool F32 = sizeof(real) == 4;
  constexpr int PA = F32 ? BM + 2 : BM + 1, PB = F32 ? BN + 2 : BN + 1;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  __shared__ real gAr[NG][2][BK][PA], gAi[NG][2][BK][PA], gBr[NG][2][BK][PB], gBi[NG][2][BK][PB];
  // (NG > 1 runs in a loop over tiles: the thread index passes through an
  // empty asm statement so that the addresses derived from it are formed
  // again in each round instead of being held in registers across the loop)
  int tx = static_cast<int>(threadIdx.x);
  if constexpr (NG > 1) asm volatile("" : "+v"(tx));
  const int gsel = NG > 1 ? __builtin_amdgcn_readfirstlane(tx >> 8) : 0;  // wave-uniform
  auto &sAr = gAr[gsel];
  auto &sAi = gAi[gsel];
  auto &sBr = gBr[gsel];
  auto &sBi = gBi[gsel];
  // M3: the three-multiplication complex product
  //   T1 = (Ar + Ai) Br,  P = -Ai (Br + Bi),  Q = Ar (Bi - Br),
  //   Re(AB) = T1 + P,    Im(AB) = T1 + Q
  // (3 real MFMAs per complex step instead of 4; its normwise rounding bound is
  // about twice the usual one).
  // The operand sums are formed once, when a tile is staged in LDS: plane
  // sAs = Ar + Ai, sBs = Br + Bi, and sBi holds Bi - Br.
  __shared__ real gAs[NG][2][M3 ? BK : 1][M3 ? PA : 1], gBs[NG][2][M3 ? BK : 1][M3 ? PB : 1];
  auto &sAs = gAs[gsel];
  auto &sBs = gBs[gsel];

  const int64_t tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  const int64_t tiles = tm * tn;
  const int64_t total = tiles * d.batch * d.splits;
  if (lin >= total) return;
  const int64_t tile = lin % tiles;
  lin /= tiles;
  const int64_t bidx = lin % d.batch;
  const int64_t split = lin / d.batch;
  // tiles in groups of up to 8 tile rows, column by column inside a group:
  // consecutive workgroups share the A row panels of the group (kept in L2)
  // and read each B column panel once per group instead of once per tile row
  constexpr int64_t G = 8;
  const int64_t grp = tile / (G * tn);
  const int64_t gr0 = grp * G;
  const int64_t grows = (tm - gr0 < G) ? tm - gr0 : G;
  const int64_t gt = tile - grp * G * tn;
  const int64_t m0 = (gr0 + gt % grows) * BM, n0 = (gt / grows) * BN;
  const int64_t kbeg = split * d.kchunk;
  const int64_t kend = (kbeg + d.kchunk < d.K) ? kbeg + d.kchunk : d.K;

  const T *A = d.A + bidx * d.sA;
  const T *B = d.B + bidx * d.sB;
  const T *A2 = SHF ? d.A2 + bidx * d.sA : nullptr;
  real zr = 0, zi = 0;
  if constexpr (SHF) {
    zr = static_cast<real>(d.shift[bidx].x);
    zi = static_cast<real>(d.shift[bidx].y);
  }

  const int tid = NG > 1 ? (tx & 255) : tx;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // barrier of the threads that share this tile's LDS planes
  auto tile_sync = [&]() {
    if constexpr (NG == 1) {
      __syncthreads();
    } else {
      *gphase += 4;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) __hip_atomic_fetch_add(gcount, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      while (__hip_atomic_load(gcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < *gphase)
        __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
  };
  // a wavefront whose whole output block lies outside C (ragged last tile)
  // stages operands and meets the barriers but issues no MFMAs
  const bool live = own && (m0 + wm * WM < d.M) && (n0 + wn * WN < d.N);

  T ra[NA], rb[NB];
  T ra2[SHF ? NA : 1];

  auto gload = [&](int64_t k0) {
    if (TA == 0) {
      // A is M x K row-major: BK lanes read one row's BK consecutive elements
      const int kk = tid % BK, rr = tid / BK;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int64_t r = m0 + rr + (256 / BK) * i, k = k0 + kk;
        ra[i] = (r < d.M && k < kend) ? A[r * d.lda + k] : T{};
        if constexpr (SHF) ra2[i] = (r < d.M && k < kend) ? A2[r * d.lda + k] : T{};
      }
    } else {
      // A stored K x M row-major; op(A) = A^*
      const int rr = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int64_t r = m0 + rr + 64 * (i % (BM / 64)), k = k0 + kk + 4 * (i / (BM / 64));
        ra[i] = (r < d.M && k < kend) ? A[k * d.lda + r] : T{};
      }
    }
    const int cc = tid & 63, kk = tid >> 6;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int64_t c = n0 + cc + 64 * (i % (BN / 64)), k = k0 + kk + 4 * (i / (BN / 64));
      rb[i] = (c < d.N && k < kend) ? B[k * d.ldb + c] : T{};
    }
  };
  auto sstore = [&](int buf) {
    if (TA == 0) {
      const int kk = tid % BK, rr = tid / BK;
      if constexpr (SHF) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          const real ex = zr * ra2[i].x - zi * ra2[i].y - ra[i].x;
          const real ey = zr * ra2[i].y + zi * ra2[i].x - ra[i].y;
          ra[i].x = ex;
          ra[i].y = ey;
        }
      }
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        sAr[buf][kk][rr + (256 / BK) * i] = ra[i].x;
        sAi[buf][kk][rr + (256 / BK) * i] = ra[i].y;
        if constexpr (M3) sAs[buf][kk][rr + (256 / BK) * i] = ra[i].x + ra[i].y;
      }
    } else {
      const int rr = tid & 63, kk = tid >> 6;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int r = rr + 64 * (i % (BM / 64)), k = kk + 4 * (i / (BM / 64));
        sAr[buf][k][r] = ra[i].x;
        sAi[buf][k][r] = -ra[i].y;
        if constexpr (M3) sAs[buf][k][r] = ra[i].x - ra[i].y;
      }
    }
    const int cc = tid & 63, kk = tid >> 6;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int c = cc + 64 * (i % (BN / 64)), k = kk + 4 * (i / (BN / 64));
      sBr[buf][k][c] = rb[i].x;
      if constexpr (M3) {
        sBi[buf][k][c] = rb[i].y - rb[i].x;
        sBs[buf][k][c] = rb[i].x + rb[i].y;
      } else {
        sBi[buf][k][c] = rb[i].y;
      }
    }
  };

  acc_t cr[FM][FN], ci[FM][FN];
  acc_t t1[M3 ? FM : 1][M3 ? FN : 1];
  if constexpr (M3) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) t1[a][b][r] = 0;
  }
  T *C = d.C + bidx * d.sC;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[a][b][r] = 0;
        ci[a][b][r] = 0;
        if (SUB) {
          // every lane loads (element (0, 0) stands in outside C) and the
          // bound selects the value afterwards: a load under a branch would be
          // waited for inside it, one memory round trip per element
          const int64_t row = m0 + wm * WM + a * 16 + Ops::out_row(lane, r);
          const int64_t col = n0 + wn * WN + b * 16 + (lane & 15);
          const bool in = row < d.M && col < d.N;
          const int64_t rr = in ? row : 0, cc = in ? col : 0;
          const T o = SHF ? d.C0[bidx * d.sC0 + rr * d.ldc0 + cc] : C[rr * d.ldc + cc];
          cr[a][b][r] = in ? o.x : real(0);
          ci[a][b][r] = in ? o.y : real(0);
        }
      }

  const int nk = static_cast<int>((kend - kbeg + BK - 1) / BK);
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
    tile_sync();
  }
  const int col16 = lane & 15, krow = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kbeg + static_cast<int64_t>(kt + 1) * BK);
    if constexpr (M3) {
      if (live) {
        // cr accumulates P, ci accumulates Q, t1 accumulates T1 (A negated for
        // C -= A B).  The operands of k-step kk + 1 are read from LDS while the
        // MFMAs of step kk issue (two MFMAs per LDS read), so the read latency
        // hides behind the matrix cores instead of stalling them.
        real as[2][FM], ai[2][FM], ar[2][FM], br[2][FN], bs[2][FN], bd[2][FN];
        auto ops = [&](int kk, int o) {
          const int kr = kk * 4 + krow;
#pragma unroll
          for (int a = 0; a < FM; ++a) {
            const int c = wm * WM + a * 16 + col16;
            as[o][a] = SUB ? -sAs[buf][kr][c] : sAs[buf][kr][c];
            ai[o][a] = SUB ? sAi[buf][kr][c] : -sAi[buf][kr][c];  // -Ai for P
            ar[o][a] = SUB ? -sAr[buf][kr][c] : sAr[buf][kr][c];
          }
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            const int c = wn * WN + b * 16 + col16;
            br[o][b] = sBr[buf][kr][c];
            bs[o][b] = sBs[buf][kr][c];
            bd[o][b] = sBi[buf][kr][c];
          }
        };
        ops(0, 0);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
          const int o = kk & 1;
          if (kk + 1 < BK / 4) ops(kk + 1, o ^ 1);
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) t1[a][b] = Ops::mma(as[o][a], br[o][b], t1[a][b]);
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) cr[a][b] = Ops::mma(ai[o][a], bs[o][b], cr[a][b]);
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) ci[a][b] = Ops::mma(ar[o][a], bd[o][b], ci[a][b]);
          if (kk + 1 < BK / 4) {
            // interleave: 3 FM FN MFMAs with the next step's 3 (FM + FN) LDS reads
#pragma unroll
            for (int g = 0; g < 3 * (FM + FN); ++g) {
              __builtin_amdgcn_sched_group_barrier(0x008, (3 * FM * FN) / (3 * (FM + FN)), 0);
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
          }
        }
        // T1 folded into both parts every kFoldK steps of K: the shared term
        // then never sums more than kFoldK products before it meets P and Q,
        // whatever the launch's K (long K ranges otherwise let T1 and P grow
        // far beyond their difference, and the complex64 factors lose digits)
        if (((kt + 1) & (kFoldK / BK - 1)) == 0 && kt + 1 < nk) {  // (the last fold is the epilogue's)
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                cr[a][b][r] += t1[a][b][r];
                ci[a][b][r] += t1[a][b][r];
                t1[a][b][r] = 0;
              }
        }
      }
    } else if (live && !PIPE) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int kr = kk * 4 + krow;
        real ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) {
          ar[a] = sAr[buf][kr][wm * WM + a * 16 + col16];
          ai[a] = sAi[buf][kr][wm * WM + a * 16 + col16];
          if (SUB) {  // accumulate (-A) B
            ar[a] = -ar[a];
            ai[a] = -ai[a];
          }
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          br[b] = sBr[buf][kr][wn * WN + b * 16 + col16];
          bi[b] = sBi[buf][kr][wn * WN + b * 16 + col16];
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            cr[a][b] = Ops::mma(ar[a], br[b], cr[a][b]);
            ci[a][b] = Ops::mma(ar[a], bi[b], ci[a][b]);
          }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            cr[a][b] = Ops::mma(-ai[a], bi[b], cr[a][b]);
            ci[a][b] = Ops::mma(ai[a], br[b], ci[a][b]);
          }
      }
    } else if (live) {
      // four real products per complex step, the next step's operands read
      // while the current MFMAs issue (as above)
      real ar[2][FM], ai[2][FM], br[2][FN], bi[2][FN];
      auto ops = [&](int kk, int o) {
        const int kr = kk * 4 + krow;
#pragma unroll
        for (int a = 0; a < FM; ++a) {
          ar[o][a] = sAr[buf][kr][wm * WM + a * 16 + col16];
          ai[o][a] = sAi[buf][kr][wm * WM + a * 16 + col16];
          if (SUB) {  // accumulate (-A) B:  Cr += (-Ar) Br - (-Ai) Bi, Ci += (-Ar) Bi + (-Ai) Br
            ar[o][a] = -ar[o][a];
            ai[o][a] = -ai[o][a];
          }
        }
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          br[o][b] = sBr[buf][kr][wn * WN + b * 16 + col16];
          bi[o][b] = sBi[buf][kr][wn * WN + b * 16 + col16];
        }
      };
      ops(0, 0);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int o = kk & 1;
        if (kk + 1 < BK / 4) ops(kk + 1, o ^ 1);
        // two sweeps over all tiles: an accumulator is reused only after every
        // other accumulator of the wave has been issued once
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            cr[a][b] = Ops::mma(ar[o][a], br[o][b], cr[a][b]);
            ci[a][b] = Ops::mma(ar[o][a], bi[o][b], ci[a][b]);
          }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) {
            cr[a][b] = Ops::mma(-ai[o][a], bi[o][b], cr[a][b]);
            ci[a][b] = Ops::mma(ai[o][a], br[o][b], ci[a][b]);
          }
        if (kk + 1 < BK / 4) {
          // interleave: 4 FM FN MFMAs with the next step's 2 (FM + FN) LDS reads
#pragma unroll
          for (int g = 0; g < 2 * (FM + FN); ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, (4 * FM * FN) / (2 * (FM + FN)), 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
          }
        }
      }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    tile_sync();
  }

  if constexpr (M3) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cr[a][b][r] += t1[a][b][r];
          ci[a][b][r] += t1[a][b][r];
        }
  }
  // epilogue
  const real alr = static_cast<real>(d.alpha.x), ali = static_cast<real>(d.alpha.y);
  const real ber = static_cast<real>(d.beta.x), bei = static_cast<real>(d.beta.y);
  const bool use_beta = (ber != 0 || bei != 0);
  T *W = (d.splits > 1) ? d.work + (split * d.batch + bidx) * d.M * d.N : nullptr;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * WM + a * 16 + Ops::out_row(lane, r);
        const int64_t col = n0 + wn * WN + b * 16 + col16;
        if (own && row < d.M && col < d.N) {
          const real xr = cr[a][b][r], xi = ci[a][b][r];
          T v;
          if (SUB) {
            v.x = xr;
            v.y = xi;
            C[row * d.ldc + col] = v;
            continue;
          }
          v.x = alr * xr - ali * xi;
          v.y = alr * xi + ali * xr;
          if (W) {
            W[row * d.N + col] = v;
          } else {
            if (use_beta) {
              const T o = C[row * d.ldc + col];
              v.x += ber * o.x - bei * o.y;
              v.y += ber * o.y + bei * o.x;
            }
            C[row * d.ldc + col] = v;
          }
        }
      }
}

// UPD only renames the instance used for the LU trailing update (same code), so
// that kernel traces time that update on its own.
// Complex products take three real MFMAs per step (M3) in the single-problem
// complex64 kernels and in the FP64 trailing update (where the extra LDS plane
// and accumulators still allow two workgroups per compute unit at BK = 8).
// Other FP64 products and the plain grouped kernels keep four (the grouped
// trailing update has a three-product form of its own, k_gemm_grp_upd).
template <typename T> constexpr bool kM3 = sizeof(T) == 8;

// Waves per SIMD the register allocation must leave room for (512 registers a
// lane are shared by the waves of a SIMD): the complex64 64 x 64 tile fits
// three workgroups per compute unit in LDS at BK = 16 and at 168 registers
// (at BK = 8, the trailing update, it takes 121 registers and runs four); the
// complex128 64 x 64 tiles and the complex64 128 x 64 tiles fit two at 256
// (left to themselves they take over 300, one wave per SIMD).  None of them
// spills; the complex128 128 x 64 tile would.
template <typename T, int BM>
constexpr int kWaves = BM != 64 ? (sizeof(T) == 8 ? 2 : 1) : (sizeof(T) == 8 ? 3 : 2);

template <typename T, int BM, int BN, int TA, bool SUB, int BK, bool UPD = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<T, BM>)))
void k_gemm(const GemmArgs<T> d, int64_t grid_total) {
  gemm_tile<T, BM, BN, TA, SUB, BK, kM3<T> || UPD>(d, xcd_remap(blockIdx.x, grid_total));
}

// C -= A B of the triangular solves (GEMM_SOLVE): the trailing update's tile
// (three real products per complex step, BK = 8) under a name of its own, so
// kernel traces and counters time the update alone.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<T, 64>)))
void k_gemm_solve(const GemmArgs<T> d, int64_t grid_total) {
  gemm_tile<T, 64, 64, 0, true, 8, true>(d, xcd_remap(blockIdx.x, grid_total));
}

// The LU trailing update C -= A B (the tile above) on a fixed number of
// persistent workgroups, each filling one compute unit on its own: NG tile
// groups of 256 threads (four wavefronts a SIMD in complex64, two in
// complex128, as the one-tile launch reaches), about 99 KB of LDS, so that no
// second workgroup of any kernel fits beside it.  The compute units left over
// stay free for the next panel's factorisation on another stream.
// Workgroup w runs on XCD w mod 8; XCD x works through the tile range
// [x per, (x + 1) per) in rounds, NG consecutive tiles a workgroup per round.
// At n = 4000, K = 128 on 224 of the 256 units it reaches 0.56 (complex64)
// and 0.55 (complex128) of peak, against 0.78 and 0.81 for the one-tile
// launch on the whole chip (0.47 and 0.52 with one workgroup barrier for all
// groups, which keeps them in lockstep).
template <typename T> constexpr int kPersistGroups = sizeof(T) == 8 ? 4 : 2;

template <typename T>
__global__ __launch_bounds__(256 * kPersistGroups<T>)
__attribute__((amdgpu_waves_per_eu(kPersistGroups<T>)))
void k_gemm_upd_pers(const GemmArgs<T> d, int64_t total, int64_t per, int rounds) {
  constexpr int NG = kPersistGroups<T>;
  const int64_t x = blockIdx.x & 7, j = blockIdx.x >> 3, p8 = gridDim.x >> 3;
  const int g = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 8));  // wave-uniform
  __shared__ uint32_t gcount[NG];
  if (threadIdx.x < NG) gcount[threadIdx.x] = 0;
  __syncthreads();
  uint32_t phase = 0;  // barriers this wavefront's group has passed, times 4
  for (int i = 0; i < rounds; ++i) {
    const int64_t lin = x * per + (i * p8 + j) * NG + g;
    const bool own = lin < total;
    gemm_tile<T, 64, 64, 0, true, 8, true, false, true, NG>(d, own ? lin : total - 1, own,
                                                              &gcount[g], &phase);
  }
}

// C_b = C0_b - (shift[b] A2 - A) B_b (FP64: three-product form at BK = 8, as the
// trailing update).
template <typename T, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<T, 64>)))
void k_gemm_shift(const GemmArgs<T> d, int64_t grid_total) {
  gemm_tile<T, 64, 64, 0, true, BK, true, true>(d, xcd_remap(blockIdx.x, grid_total));
}

// A group of independent problems in one launch: tab[e].tile0 is the first
// linear tile of problem e (increasing); a workgroup finds its problem by
// bisection over the table.
// (the grouped tiles keep the unpipelined four-product loop: the complex64 one
// then fits four workgroups per compute unit, 128 registers a lane; the
// complex128 one takes the two-wave budget of the single-problem tile)
template <typename T>
__device__ inline int find_problem(const GemmArgs<T> *__restrict__ tab, int count, int64_t lin) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].tile0 <= lin) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int BM, int BN, int TA, bool SUB, int BK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 16 ? 2 : 1)))
void k_gemm_grp(const GemmArgs<T> *__restrict__ tab, int count, int64_t grid_total) {
  const int64_t lin = xcd_remap(blockIdx.x, grid_total);
  const GemmArgs<T> d = tab[find_problem(tab, count, lin)];
  gemm_tile<T, BM, BN, TA, SUB, BK, false, false, false>(d, lin - d.tile0);
}

// The grouped LU trailing update C -= A B with the single-problem update's
// loop: three real products per complex step, next operands read from LDS
// while the MFMAs issue, BK = 8 (complex128 in the two-wave register budget,
// complex64 at four workgroups per compute unit).  The batched form picks it
// (or a four-product loop) per precision and order from its tuned table.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<T, 64>)))
void k_gemm_grp_upd(const GemmArgs<T> *__restrict__ tab, int count, int64_t grid_total) {
  const int64_t lin = xcd_remap(blockIdx.x, grid_total);
  const GemmArgs<T> d = tab[find_problem(tab, count, lin)];
  gemm_tile<T, 64, 64, 0, true, 8, true, false, true>(d, lin - d.tile0);
}

// The grouped update C -= A B with four real products per complex step and
// the operand-pipelined loop (BK = 16, the single-problem tiles' register
// budget): the candidate between the plain grouped loop and the
// three-product one for either precision.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWaves<T, 64>)))
void k_gemm_grp_pipe(const GemmArgs<T> *__restrict__ tab, int count, int64_t grid_total) {
  const int64_t lin = xcd_remap(blockIdx.x, grid_total);
  const GemmArgs<T> d = tab[find_problem(tab, count, lin)];
  gemm_tile<T, 64, 64, 0, true, 16, false, false, true>(d, lin - d.tile0);
}

// Deterministic reduction of split-K partials: C = sum_s W_s + beta C.
template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(const GemmArgs<T> d) {
  const int64_t per = d.M * d.N;
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  if (idx >= per * d.batch) return;
  const int64_t b = idx / per, e = idx % per;
  const int64_t row = e / d.N, col = e % d.N;
  double sr = 0.0, si = 0.0;
  for (int s = 0; s < d.splits; ++s) {
    const T v = d.work[(s * d.batch + b) * per + e];
    sr += v.x;
    si += v.y;
  }
  T *C = d.C + b * d.sC + row * d.ldc + col;
  if (d.beta.x != 0.0 || d.beta.y != 0.0) {
    const T o = *C;
    sr += d.beta.x * o.x - d.beta.y * o.y;
    si += d.beta.x * o.y + d.beta.y * o.x;
  }
  T v;
  v.x = static_cast<decltype(v.x)>(sr);
  v.y = static_cast<decltype(v.y)>(si);
  *C = v;
}

template <typename T, int BM, int BN, int BK = 16>
void launch_cfg(hipStream_t s, const GemmArgs<T> &d, int ta, bool update = false) {
  const int64_t tiles = ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
  const int64_t total = tiles * d.batch * d.splits;
  const int64_t padded = (total + 7) / 8 * 8;
  const dim3 grid(static_cast<unsigned>(padded));
  // C -= op(A) B is recognised from alpha = -1, beta = 1 without split-K
  const bool sub = d.splits == 1 && d.alpha.x == -1.0 && d.alpha.y == 0.0 && d.beta.x == 1.0 &&
                   d.beta.y == 0.0;
  if (ta == 0) {
    // (BK = 8: two workgroups per compute unit in FP64, four in complex64; the
    // 128-row tiles take this instance for every C -= A B, which at BK = 16
    // would spill in complex64)
    if (sub && (update || BM > 64))
      hipLaunchKernelGGL((k_gemm<T, BM, BN, 0, true, 8, true>), grid, dim3(256), 0, s, d, padded);
    else if (sub) {
      if constexpr (BM == 64)
        hipLaunchKernelGGL((k_gemm<T, BM, BN, 0, true, BK>), grid, dim3(256), 0, s, d, padded);
    }
    else
      hipLaunchKernelGGL((k_gemm<T, BM, BN, 0, false, BK>), grid, dim3(256), 0, s, d, padded);
  } else {
    if (sub)
      hipLaunchKernelGGL((k_gemm<T, BM, BN, 2, true, BK>), grid, dim3(256), 0, s, d, padded);
    else
      hipLaunchKernelGGL((k_gemm<T, BM, BN, 2, false, BK>), grid, dim3(256), 0, s, d, padded);
  }
}

template <typename T>
void gemm_impl(hipStream_t s, GemmArgs<T> d, int ta, int cfg, int64_t work_elems) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  if (d.K <= 0) {
    // C = beta C: a GEMM with an empty K range does exactly that.
    d.K = 0;
  }
  d.splits = 1;
  d.kchunk = d.K > 0 ? d.K : 1;
  // (a 128 x 128 complex64 tile measured slower than 64 x 64 in the LU update,
  // and the FP64 one needs more than the 512 registers of a lane: not used)
  const int BM = (cfg == GEMM_TALL || cfg == GEMM_UPDATE_TALL) ? 128 : 64;
  const int64_t tiles = ((d.M + BM - 1) / BM) * ((d.N + 63) / 64);
  // Split K when the output is too small to fill the chip (aiming at about
  // three workgroups per compute unit, each K chunk at least 64 long: the
  // Gram products of an n x m block, m <= 160, are otherwise a few long
  // workgroups).
  if (d.work && d.K >= 512 && tiles * d.batch < 512) {
    int64_t sp = (768 + tiles * d.batch - 1) / (tiles * d.batch);
    sp = std::min<int64_t>(sp, d.K / 64);
    while (sp > 1 && sp * d.batch * d.M * d.N > work_elems) --sp;
    if (sp > 1) {
      d.splits = static_cast<int32_t>(sp);
      d.kchunk = ((d.K + sp - 1) / sp + 15) / 16 * 16;
      d.splits = static_cast<int32_t>((d.K + d.kchunk - 1) / d.kchunk);
    }
  }
  const bool sub = d.splits == 1 && d.alpha.x == -1.0 && d.alpha.y == 0.0 && d.beta.x == 1.0 &&
                   d.beta.y == 0.0;
  if (cfg == GEMM_SOLVE && ta == 0 && sub) {
    const int64_t tiles2 = ((d.M + 63) / 64) * ((d.N + 63) / 64) * d.batch;
    const int64_t padded = (tiles2 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_gemm_solve<T>), dim3(static_cast<unsigned>(padded)), dim3(256), 0, s, d,
                       padded);
  } else if (cfg == GEMM_TALL || cfg == GEMM_UPDATE_TALL) {
    launch_cfg<T, 128, 64>(s, d, ta, cfg == GEMM_UPDATE_TALL);
  } else {
    launch_cfg<T, 64, 64>(s, d, ta, cfg == GEMM_UPDATE);
  }
  if (d.splits > 1) {
    const int64_t n = d.M * d.N * d.batch;
    hipLaunchKernelGGL((k_splitk_reduce<T>), dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256),
                       0, s, d);
  }
}

}  // namespace

template <typename T>
int64_t gemm_group_tiles(GemmArgs<T> *tab, int count) {
  int64_t t = 0;
  for (int e = 0; e < count; ++e) {
    tab[e].splits = 1;
    tab[e].kchunk = tab[e].K > 0 ? tab[e].K : 1;
    tab[e].tile0 = t;
    t += ((tab[e].M + 63) / 64) * ((tab[e].N + 63) / 64) * tab[e].batch;
  }
  return t;
}
template int64_t gemm_group_tiles<z64>(GemmArgs<z64> *, int);
template int64_t gemm_group_tiles<c64>(GemmArgs<c64> *, int);

template <typename T>
void gemm_group(hipStream_t s, int ta, bool sub, const GemmArgs<T> *dtab, int count,
                int64_t total_tiles, int variant) {
  if (count <= 0 || total_tiles <= 0) return;
  const int64_t padded = (total_tiles + 7) / 8 * 8;
  const dim3 grid(static_cast<unsigned>(padded));
  if (ta == 0) {
    if (sub && variant == GROUP_UPDATE_M3)
      hipLaunchKernelGGL((k_gemm_grp_upd<T>), grid, dim3(256), 0, s, dtab, count, padded);
    else if (sub && variant == GROUP_UPDATE_PIPE)
      hipLaunchKernelGGL((k_gemm_grp_pipe<T>), grid, dim3(256), 0, s, dtab, count, padded);
    else if (sub)
      hipLaunchKernelGGL((k_gemm_grp<T, 64, 64, 0, true, 16>), grid, dim3(256), 0, s, dtab, count,
                         padded);
    else
      hipLaunchKernelGGL((k_gemm_grp<T, 64, 64, 0, false, 16>), grid, dim3(256), 0, s, dtab, count,
                         padded);
  } else {
    hipLaunchKernelGGL((k_gemm_grp<T, 64, 64, 2, false, 16>), grid, dim3(256), 0, s, dtab, count,
                       padded);
  }
}
template void gemm_group<z64>(hipStream_t, int, bool, const GemmArgs<z64> *, int, int64_t, int);
template void gemm_group<c64>(hipStream_t, int, bool, const GemmArgs<c64> *, int, int64_t, int);

void zgemm_shift_residual(hipStream_t s, int64_t M, int64_t N, int64_t K, const z64 *A,
                          const z64 *A2, int64_t lda, const z64 *shift, const z64 *Y, int64_t ldy,
                          int64_t sY, const z64 *R, int64_t ldr, int64_t sR, z64 *C, int64_t ldc,
                          int64_t sC, int32_t batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  GemmArgs<z64> d{M, N, K, A, lda, 0, Y, ldy, sY, C, ldc, sC, make_double2(-1.0, 0.0),
                  make_double2(1.0, 0.0), batch, 1, K > 0 ? K : 1, nullptr, 0, A2, shift, R, ldr, sR};
  const int64_t total = ((M + 63) / 64) * ((N + 63) / 64) * batch;
  const int64_t padded = (total + 7) / 8 * 8;
  hipLaunchKernelGGL((k_gemm_shift<z64, 8>), dim3(static_cast<unsigned>(padded)), dim3(256), 0, s, d,
                     padded);
}

template <typename T>
void update_persistent(hipStream_t s, GemmArgs<T> d, int wgs) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0 || d.K <= 0) return;
  constexpr int NG = kPersistGroups<T>;
  d.splits = 1;
  d.kchunk = d.K;
  const int64_t total = ((d.M + 63) / 64) * ((d.N + 63) / 64) * d.batch;
  // multiples of 8 (one share per XCD), no more than the tiles need
  int64_t p = std::max<int64_t>(8, wgs / 8 * 8);
  p = std::min<int64_t>(p, (total + 8 * NG - 1) / (8 * NG) * 8);
  const int64_t rounds = (total + p * NG - 1) / (p * NG);
  const int64_t per = rounds * (p / 8) * NG;
  hipLaunchKernelGGL((k_gemm_upd_pers<T>), dim3(static_cast<unsigned>(p)), dim3(256 * NG), 0, s, d,
                     total, per, static_cast<int>(rounds));
}

void zupdate_persistent(hipStream_t s, int64_t M, int64_t N, int64_t K, const z64 *A, int64_t lda,
                        int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 *C, int64_t ldc,
                        int64_t sC, int32_t batch, int wgs) {
  GemmArgs<z64> d{M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, make_double2(-1.0, 0.0),
                  make_double2(1.0, 0.0), batch, 1, K, nullptr, 0};
  update_persistent<z64>(s, d, wgs);
}

void cupdate_persistent(hipStream_t s, int64_t M, int64_t N, int64_t K, const c64 *A, int64_t lda,
                        int64_t sA, const c64 *B, int64_t ldb, int64_t sB, c64 *C, int64_t ldc,
                        int64_t sC, int32_t batch, int wgs) {
  GemmArgs<c64> d{M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, make_double2(-1.0, 0.0),
                  make_double2(1.0, 0.0), batch, 1, K, nullptr, 0};
  update_persistent<c64>(s, d, wgs);
}

void zgemm(hipStream_t s, int transA, int64_t M, int64_t N, int64_t K, z64 alpha, const z64 *A,
           int64_t lda, int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 beta, z64 *C,
           int64_t ldc, int64_t sC, int32_t batch, z64 *work, int64_t work_elems, int cfg) {
  GemmArgs<z64> d{M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, batch, 1, K, work, 0};
  gemm_impl<z64>(s, d, transA, cfg, work_elems);
}

void cgemm(hipStream_t s, int transA, int64_t M, int64_t N, int64_t K, z64 alpha, const c64 *A,
           int64_t lda, int64_t sA, const c64 *B, int64_t ldb, int64_t sB, z64 beta, c64 *C,
           int64_t ldc, int64_t sC, int32_t batch, c64 *work, int64_t work_elems, int cfg) {
  GemmArgs<c64> d{M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, batch, 1, K, work, 0};
  gemm_impl<c64>(s, d, transA, cfg, work_elems);
}

}  // namespace feast
