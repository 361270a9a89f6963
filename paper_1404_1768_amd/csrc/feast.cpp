// Plan, drivers and C ABI of the gfx950 oblique-projection FEAST path.
//
//   feast_filter  : U = sum_j w_j (z_j B - A)^{-1} B V        (eqs. 8-4, 4-4)
//   feast_project : U = U_1 R_1, B U_1 = U_2 R_2, At = U_2^* A U_1, Bt = U_2^* B U_1
//                   (Algorithm 5's QR steps and reduced pencil; eqs. 6-3-13, 7-10)
//   feast_solve   : Algorithm 5 with the subspace size fixed
//
// Device layout.  Every matrix is row-major.  The plan caches, per node j,
// the LU factors of M_j = z_j B - A (N blocks of n x n, complex128 or
// complex64), the pivots, the permutation they define, and the inverses of
// the nb x nb diagonal blocks of L_j and U_j, which turn the blocked
// triangular solves into MFMA GEMMs.  The N node solutions live side by side
// in one n x (N m) block (node j in columns [j m, (j+1) m)), so that the FP64
// refinement residual of all nodes is one GEMM [A; B] * [Y_1 ... Y_N].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "host_eig.h"
#include "host_sparse.h"
#include "plan.h"

using namespace feast_drv;

namespace {

// ---------------------------------------------------------------------------
// Blocked right-looking LU of `batch` matrices (row-major, partial pivoting).
// Panels of width nb are factored recursively (left half, small TRSM, GEMM
// update of the right half, right half) down to register-resident leaves;
// then the panel's swaps reach the columns outside it, U12 = L11^{-1} A12 is
// an in-place MFMA product with the inverted diagonal block, and the trailing
// update A22 -= L21 U12 is one batched MFMA GEMM over all matrices.
// ---------------------------------------------------------------------------
template <typename T>
void panel_rec(hipStream_t s, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
               int64_t c0, int w, int64_t pk0, int pkb, int32_t *ipiv, int32_t *info) {
  const int ib = feast::leaf_max_width<T>(n - c0);
  if (w <= ib) {
    if (!feast::leaf_lu<T>(s, M, ld, stride, batch, n, c0, w, pk0, pkb, ipiv, info))
      throw HipError{hipErrorInvalidValue, "leaf_lu"};
    return;
  }
  const int w1 = w / 2, w2 = w - w1;
  panel_rec<T>(s, M, ld, stride, batch, n, c0, w1, pk0, pkb, ipiv, info);
  if (w2 <= feast::panel_update_max_width()) {
    feast::panel_update<T>(s, M, ld, stride, batch, n, c0, w1, w2);
    panel_rec<T>(s, M, ld, stride, batch, n, c0 + w1, w2, pk0, pkb, ipiv, info);
    return;
  }
  feast::trsm_small<T>(s, M, ld, stride, batch, c0, w1, w2);
  if (c0 + w1 < n)
    gemm_t<T>(s, 0, n - c0 - w1, w2, w1, zc(-1.0), M + (c0 + w1) * ld + c0, ld, stride,
              M + c0 * ld + c0 + w1, ld, stride, zc(1.0), M + (c0 + w1) * ld + c0 + w1, ld, stride,
              batch);
  panel_rec<T>(s, M, ld, stride, batch, n, c0 + w1, w2, pk0, pkb, ipiv, info);
}

struct LuProf {
  std::vector<hipEvent_t> *ev = nullptr;  // pairs around trailing-update launches
  int used = 0;
  double flops = 0.0;
};

// Tile of the solves' off-diagonal products X -= L X: complex128 takes the
// trailing update's tile (three real products per complex step, BK = 8; 2.6 ms
// less per FP64 solve at n = 4000), complex64's own tile already uses three
// products and measured no faster on the update's.
template <typename T> constexpr int kSolveCfg = sizeof(T) == 16 ? feast::GEMM_SOLVE : feast::GEMM_SQUARE;

// Diagonal blocks of the triangular factors are inverted in blocks of kIB rows;
// this is also the leaf size of the recursive triangular solves.
constexpr int kIB = 64;

// Panels per trailing update of the LU (the update's K is their total width):
// at n = 4000, three for complex128 (factor 128.3 -> 126.8 ms against two)
// and two for complex64 (three: 72.7 -> 73.1 ms, the narrow updates of the
// third panel cost more than the wider update saves).
template <typename T> constexpr int kGroup = sizeof(T) == 16 ? 3 : 2;

// X <- L^{-1} X for the unit-lower L = M[r0:r1, r0:r1] (r0 a multiple of kIB)
// and X = rows [r0, r1) of the block with columns starting at Xc (leading
// dimension ldx, batch stride sX): recursive halving, leaves are in-place MFMA
// products with the inverted kIB x kIB diagonal blocks.
//   lb: rows of the inverted diagonal blocks (64, or 128 with leaf products on
//   128-row tiles, which keep the in-place product within one workgroup).
template <typename T>
void trsm_lower_rec(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch,
                    const T *Linv, int64_t istride, int64_t r0, int64_t r1, T *X, int64_t ldx,
                    int64_t sX, int64_t ncols, int ta, int lb = kIB) {
  if (r1 - r0 <= lb) {
    gemm_t<T>(s, ta, r1 - r0, ncols, r1 - r0, zc(1.0), Linv + (r0 / lb) * lb * lb, lb, istride,
              X + r0 * ldx, ldx, sX, zc(0.0), X + r0 * ldx, ldx, sX, batch, nullptr, 0,
              lb > 64 ? feast::GEMM_TALL : feast::GEMM_SQUARE);
    return;
  }
  const int64_t half = ((r1 - r0 + 2 * lb - 1) / (2 * lb)) * lb;
  const int64_t mid = r0 + half;
  trsm_lower_rec<T>(s, M, ld, stride, batch, Linv, istride, r0, mid, X, ldx, sX, ncols, ta, lb);
  if (ta == 0)  // X[mid:r1] -= L[mid:r1, r0:mid] X[r0:mid]
    gemm_t<T>(s, 0, r1 - mid, ncols, mid - r0, zc(-1.0), M + mid * ld + r0, ld, stride,
              X + r0 * ldx, ldx, sX, zc(1.0), X + mid * ldx, ldx, sX, batch, nullptr, 0,
              kSolveCfg<T>);
  else  // lower factor given as (U^*): rows [mid, r1) of U^* are columns of U rows [r0, mid)
    gemm_t<T>(s, 2, r1 - mid, ncols, mid - r0, zc(-1.0), M + r0 * ld + mid, ld, stride,
              X + r0 * ldx, ldx, sX, zc(1.0), X + mid * ldx, ldx, sX, batch);
  trsm_lower_rec<T>(s, M, ld, stride, batch, Linv, istride, mid, r1, X, ldx, sX, ncols, ta, lb);
}

// X <- U^{-1} X for the upper U = M[r0:r1, r0:r1] (ta = 0), or X <- L^{-*} X
// with L^* unit upper (ta = 2, Linv holding the inverted blocks of L).
template <typename T>
void trsm_upper_rec(hipStream_t s, const T *M, int64_t ld, int64_t stride, int32_t batch,
                    const T *Inv, int64_t istride, int64_t r0, int64_t r1, T *X, int64_t ldx,
                    int64_t sX, int64_t ncols, int ta, int lb = kIB) {
  if (r1 - r0 <= lb) {
    gemm_t<T>(s, ta, r1 - r0, ncols, r1 - r0, zc(1.0), Inv + (r0 / lb) * lb * lb, lb, istride,
              X + r0 * ldx, ldx, sX, zc(0.0), X + r0 * ldx, ldx, sX, batch, nullptr, 0,
              lb > 64 ? feast::GEMM_TALL : feast::GEMM_SQUARE);
    return;
  }
  const int64_t half = ((r1 - r0 + 2 * lb - 1) / (2 * lb)) * lb;
  const int64_t mid = r0 + half;
  trsm_upper_rec<T>(s, M, ld, stride, batch, Inv, istride, mid, r1, X, ldx, sX, ncols, ta, lb);
  if (ta == 0)  // X[r0:mid] -= U[r0:mid, mid:r1] X[mid:r1]
    gemm_t<T>(s, 0, mid - r0, ncols, r1 - mid, zc(-1.0), M + r0 * ld + mid, ld, stride,
              X + mid * ldx, ldx, sX, zc(1.0), X + r0 * ldx, ldx, sX, batch, nullptr, 0,
              kSolveCfg<T>);
  else  // rows [r0, mid) of L^* are columns of L rows [mid, r1)
    gemm_t<T>(s, 2, mid - r0, ncols, r1 - mid, zc(-1.0), M + mid * ld + r0, ld, stride,
              X + mid * ldx, ldx, sX, zc(1.0), X + r0 * ldx, ldx, sX, batch);
  trsm_upper_rec<T>(s, M, ld, stride, batch, Inv, istride, r0, mid, X, ldx, sX, ncols, ta, lb);
}

// Streams and events of the look-ahead factorisation.
struct LuStreams {
  hipStream_t main = nullptr, side = nullptr;
  hipEvent_t cols_ready = nullptr, panel_done = nullptr;
  int update_cfg = feast::GEMM_UPDATE;  // tile of the trailing update
  int upd_wgs = 0;                      // look-ahead: persistent workgroups of the rest's update
  int64_t ahead_rows = 0;               // look-ahead: most trailing rows of a look-ahead step
};

template <typename T>
void update_persistent_t(hipStream_t s, int64_t M, int64_t N, int64_t K, const T *A, const T *B,
                         T *C, int64_t ld, int64_t stride, int32_t batch, int wgs);
template <>
void update_persistent_t<z64>(hipStream_t s, int64_t M, int64_t N, int64_t K, const z64 *A,
                              const z64 *B, z64 *C, int64_t ld, int64_t stride, int32_t batch,
                              int wgs) {
  feast::zupdate_persistent(s, M, N, K, A, ld, stride, B, ld, stride, C, ld, stride, batch, wgs);
}
template <>
void update_persistent_t<c64>(hipStream_t s, int64_t M, int64_t N, int64_t K, const c64 *A,
                              const c64 *B, c64 *C, int64_t ld, int64_t stride, int32_t batch,
                              int wgs) {
  feast::cupdate_persistent(s, M, N, K, A, ld, stride, B, ld, stride, C, ld, stride, batch, wgs);
}

template <typename T>
void lu_batched(const LuStreams &st, T *M, int64_t ld, int64_t stride, int32_t batch, int64_t n,
                int nb, int32_t *ipiv, int32_t *info, T *Linv, T *Uinv, int64_t istride,
                LuProf *prof = nullptr) {
  hipStream_t s = st.main;
  const bool ahead = st.side != nullptr;
  feast::fill_i32(s, info, batch, 0);
  // wgs > 0: the update on that many persistent workgroups (the look-ahead's)
  auto timed_gemm = [&](int64_t rows, int64_t cols, int64_t kb, const T *Ap, const T *Bp, T *Cp,
                        int wgs = 0) {
    const bool timed = prof && prof->ev && prof->used + 2 <= static_cast<int>(prof->ev->size());
    if (timed) HIPCHK(hipEventRecord((*prof->ev)[prof->used], s));
    if (wgs > 0)
      update_persistent_t<T>(s, rows, cols, kb, Ap, Bp, Cp, ld, stride, batch, wgs);
    else
      gemm_t<T>(s, 0, rows, cols, kb, zc(-1.0), Ap, ld, stride, Bp, ld, stride, zc(1.0), Cp, ld,
                stride, batch, nullptr, 0, st.update_cfg);
    if (timed) {
      HIPCHK(hipEventRecord((*prof->ev)[prof->used + 1], s));
      prof->used += 2;
      prof->flops += 8.0 * static_cast<double>(rows) * cols * kb * batch;
    }
  };
  // first panel
  panel_rec<T>(s, M, ld, stride, batch, n, 0, static_cast<int>(std::min<int64_t>(nb, n)), 0,
               static_cast<int>(std::min<int64_t>(nb, n)), ipiv, info);
  for (int64_t k0 = 0; k0 < n; k0 += nb) {
    const int kb = static_cast<int>(std::min<int64_t>(nb, n - k0));
    const int64_t k1 = k0 + kb, rest = n - k1;
    // the panel [k0, k1) is factored (on `s`, or on the side stream joined below)
    feast::laswp_outside<T>(s, M, ld, stride, batch, n, k0, kb, k0, k1, ipiv);
    feast::diag_block_inverse<T>(s, M, ld, stride, batch, n, kIB, k0 / kIB,
                                 (k1 + kIB - 1) / kIB, true, Linv, istride);
    if (rest <= 0) break;
    // U12 = L11^{-1} A12
    trsm_lower_rec<T>(s, M, ld, stride, batch, Linv, istride, k0, k1, M + k1, ld, stride, rest, 0);
    const int kb1 = static_cast<int>(std::min<int64_t>(nb, rest));
    if (ahead && rest > kb1 && rest <= st.ahead_rows) {
      // look-ahead: update the next panel's columns (whole chip), then factor
      // that panel on the side stream while the rest of the trailing matrix is
      // updated here by persistent workgroups that leave compute units to it
      // (only once the trailing block is short enough that the panel's
      // latency-bound kernels take a good part of a step)
      timed_gemm(rest, kb1, kb, M + k1 * ld + k0, M + k0 * ld + k1, M + k1 * ld + k1);
      HIPCHK(hipEventRecord(st.cols_ready, s));
      HIPCHK(hipStreamWaitEvent(st.side, st.cols_ready, 0));
      panel_rec<T>(st.side, M, ld, stride, batch, n, k1, kb1, k1, kb1, ipiv, info);
      HIPCHK(hipEventRecord(st.panel_done, st.side));
      timed_gemm(rest, rest - kb1, kb, M + k1 * ld + k0, M + k0 * ld + k1 + kb1,
                 M + k1 * ld + k1 + kb1, st.upd_wgs);
      HIPCHK(hipStreamWaitEvent(s, st.panel_done, 0));
    } else if (k1 + kb1 < n) {
      // up to kGroup<T> panels per trailing update (K = their total width): each
      // further panel's columns get the group's earlier panels' update, that
      // panel is factored and its exchanges applied outside it (including to
      // the group's L21 columns and to the columns still waiting for the
      // group's update: exchanging rows of both commutes with the update), its
      // rows get the same update, then its U12; one update with all the
      // group's panels covers the rest.  Same flops as one step per panel; the
      // trailing block is read and written once per group.
      int64_t kg = k1;  // end of the group's factored panels
      for (int g = 1; g < kGroup<T> && kg + nb < n; ++g) {
        const int64_t ks = kg, ke = kg + nb;
        timed_gemm(n - ks, static_cast<int>(nb), ks - k0, M + ks * ld + k0, M + k0 * ld + ks,
                   M + ks * ld + ks);
        panel_rec<T>(s, M, ld, stride, batch, n, ks, nb, ks, nb, ipiv, info);
        feast::laswp_outside<T>(s, M, ld, stride, batch, n, ks, nb, ks, ke, ipiv);
        feast::diag_block_inverse<T>(s, M, ld, stride, batch, n, kIB, ks / kIB,
                                     (ke + kIB - 1) / kIB, true, Linv, istride);
        timed_gemm(nb, n - ke, ks - k0, M + ks * ld + k0, M + k0 * ld + ke, M + ks * ld + ke);
        trsm_lower_rec<T>(s, M, ld, stride, batch, Linv, istride, ks, ke, M + ke, ld, stride,
                          n - ke, 0);
        kg = ke;
      }
      timed_gemm(n - kg, n - kg, kg - k0, M + kg * ld + k0, M + k0 * ld + kg, M + kg * ld + kg);
      const int kbn = static_cast<int>(std::min<int64_t>(nb, n - kg));
      panel_rec<T>(s, M, ld, stride, batch, n, kg, kbn, kg, kbn, ipiv, info);
      k0 = kg - nb;  // (the loop's step moves on to the panel at kg)
    } else {
      timed_gemm(rest, rest, kb, M + k1 * ld + k0, M + k0 * ld + k1, M + k1 * ld + k1);
      panel_rec<T>(s, M, ld, stride, batch, n, k1, kb1, k1, kb1, ipiv, info);
    }
  }
  const int64_t nblk = (n + kIB - 1) / kIB;
  feast::diag_block_inverse<T>(s, M, ld, stride, batch, n, kIB, 0, nblk, false, Uinv, istride);
}

// Triangular solves with the cached factors, in place on Y (per node: n x m,
// leading dimension ldy, node stride sY):
//   trans = 0: Y <- U^{-1} L^{-1} Y   (after the row permutation)
//   trans = 2: Y <- L^{-*} U^{-*} Y   (before the inverse permutation)
template <typename T>
void trsolve(hipStream_t s, const T *F, int64_t ld, int64_t fstride, int32_t batch, int64_t n,
             const T *Linv, const T *Uinv, int64_t istride, T *Y, int64_t m, int64_t ldy,
             int64_t sY, int trans, int lb = kIB) {
  if (trans == 0) {
    trsm_lower_rec<T>(s, F, ld, fstride, batch, Linv, istride, 0, n, Y, ldy, sY, m, 0, lb);
    trsm_upper_rec<T>(s, F, ld, fstride, batch, Uinv, istride, 0, n, Y, ldy, sY, m, 0, lb);
  } else {
    trsm_lower_rec<T>(s, F, ld, fstride, batch, Uinv, istride, 0, n, Y, ldy, sY, m, 2, lb);
    trsm_upper_rec<T>(s, F, ld, fstride, batch, Linv, istride, 0, n, Y, ldy, sY, m, 2, lb);
  }
}

// The plan's solves: leaves on its inverted 128 x 128 diagonal blocks.
template <typename T>
void plan_trsolve(feast_plan *p, hipStream_t s, T *Y, int64_t m, int64_t ldy, int64_t sY,
                  int trans) {
  trsolve<T>(s, p->F.as<T>(), p->n, p->fstride(), p->N, p->n, p->Linv2.as<T>(), p->Uinv2.as<T>(),
             p->istride2(), Y, m, ldy, sY, trans, 128);
}

// ---------------------------------------------------------------------------
// Plan helpers
// ---------------------------------------------------------------------------

// Fingerprints of A and B (n x n) into p->fp[0], p->fp[1] on the plan's stream.
void launch_fingerprints(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb) {
  p->fp.alloc(2 * sizeof(uint64_t));
  const feast::GrpMat a{const_cast<z64 *>(A), lda, 0, p->n}, b{const_cast<z64 *>(B), ldb, 0, p->n};
  ktimed(p, FEAST_K_FINGERPRINT, 32.0 * p->n * p->n,
         [&]() { feast::fingerprint(p->s, nullptr, 2, a, b, p->n, p->fp.as<uint64_t>()); });
}

int factor(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb) {
  const int64_t n = p->n;
  const int N = p->N;
  hipStream_t s = p->s;
  const size_t esz = p->mixed() ? sizeof(c64) : sizeof(z64);
  p->factored = false;
  p->F.alloc(esz * N * n * n);
  p->piv.alloc(sizeof(int32_t) * N * n);
  p->perm.alloc(sizeof(int32_t) * N * n);
  p->info.alloc(sizeof(int32_t) * N);
  p->Linv.alloc(esz * N * p->istride());
  p->Uinv.alloc(esz * N * p->istride());
  p->Linv2.alloc(esz * N * p->istride2());
  p->Uinv2.alloc(esz * N * p->istride2());
  LuProf prof;
  if (p->o.profile) {
    const size_t need = 4 * static_cast<size_t>((n + p->nb - 1) / p->nb);
    while (p->ev.size() < need) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      p->ev.push_back(e);
    }
    prof.ev = &p->ev;
  }
  hipStream_t sl = s;
  const int ahead_cus = p->o.ahead_cus ? p->o.ahead_cus : 32;
  const LuStreams lst{sl, p->o.lookahead ? p->side : nullptr, p->ev_cols, p->ev_panel,
                      p->o.update_tile ? feast::GEMM_UPDATE_TALL : feast::GEMM_UPDATE,
                      std::max(8, p->cus - ahead_cus),
                      p->o.ahead_rows ? p->o.ahead_rows : 2048};
  if (p->mixed()) {
    ktimed(p, FEAST_K_SHIFT, (32.0 + 8.0 * N) * n * n, [&]() {
      feast::shift_assemble_c(sl, A, lda, B, ldb, p->dz.as<z64>(), N, n, p->F.as<c64>(), n, n * n);
    });
    lu_batched<c64>(lst, p->F.as<c64>(), n, n * n, N, n, p->nb, p->piv.as<int32_t>(),
                    p->info.as<int32_t>(), p->Linv.as<c64>(), p->Uinv.as<c64>(), p->istride(),
                    &prof);
    for (const bool lower : {true, false})
      feast::inverse_pairs<c64>(sl, p->F.as<c64>(), n, n * n, N, n,
                                (lower ? p->Linv : p->Uinv).as<c64>(), p->istride(),
                                (lower ? p->Linv2 : p->Uinv2).as<c64>(), p->istride2(), lower);
  } else {
    ktimed(p, FEAST_K_SHIFT, (32.0 + 16.0 * N) * n * n, [&]() {
      feast::shift_assemble_z(sl, A, lda, B, ldb, p->dz.as<z64>(), N, n, p->F.as<z64>(), n, n * n);
    });
    lu_batched<z64>(lst, p->F.as<z64>(), n, n * n, N, n, p->nb, p->piv.as<int32_t>(),
                    p->info.as<int32_t>(), p->Linv.as<z64>(), p->Uinv.as<z64>(), p->istride(),
                    &prof);
    for (const bool lower : {true, false})
      feast::inverse_pairs<z64>(sl, p->F.as<z64>(), n, n * n, N, n,
                                (lower ? p->Linv : p->Uinv).as<z64>(), p->istride(),
                                (lower ? p->Linv2 : p->Uinv2).as<z64>(), p->istride2(), lower);
  }
  feast::perm_from_ipiv(s, p->piv.as<int32_t>(), p->perm.as<int32_t>(), n, N);
  double *nrm = p->nrm.as<double>();
  feast::fro2_batched(s, A, lda, 0, n, n, 1, p->part.as<double>(), nrm);
  feast::fro2_batched(s, B, ldb, 0, n, n, 1, p->part.as<double>(), nrm + 1);
  launch_fingerprints(p, A, lda, B, ldb);
  std::vector<int32_t> hinfo(N);
  double h2[2];
  uint64_t hfp[2];
  HIPCHK(hipMemcpyAsync(hinfo.data(), p->info.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(h2, nrm, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hfp, p->fp.p, sizeof(hfp), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  p->normA = std::sqrt(h2[0]);
  p->normB = std::sqrt(h2[1]);
  p->prof_launches = prof.used / 2;
  p->prof_flops = prof.flops;
  p->prof_ms = 0.0;
  for (int i = 0; i + 1 < prof.used; i += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
    p->prof_ms += ms;
  }
  p->factored = true;
  p->fpA = hfp[0];
  p->fpB = hfp[1];
  for (int j = 0; j < N; ++j)
    if (hinfo[j] != 0) {
      char buf[200];
      std::snprintf(buf, sizeof buf, "exact zero pivot at node %d (z = %.17g%+.17gi), column %d", j,
                    p->hz[j].real(), p->hz[j].imag(), hinfo[j] - 1);
      p->err = buf;
      return FEAST_SINGULAR;
    }
  return FEAST_OK;
}

// Reuse the cached factors only for the pencil they were computed from
// (Section 4.3: the factors of the same shifted matrices): one read of A and B
// for their fingerprints and a wait for the two words.
int ensure_factored(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb) {
  if (p->sp.on) return FEAST_OK;  // (a sparse call's band factors are made on entry)
  if (p->factored && p->checked) return FEAST_OK;
  if (p->factored) {
    launch_fingerprints(p, A, lda, B, ldb);
    uint64_t hfp[2];
    HIPCHK(hipMemcpyAsync(hfp, p->fp.p, sizeof(hfp), hipMemcpyDeviceToHost, p->s));
    HIPCHK(hipStreamSynchronize(p->s));
    if (hfp[0] == p->fpA && hfp[1] == p->fpB) {
      p->checked = true;
      return FEAST_OK;
    }
  }
  const int st = factor(p, A, lda, B, ldb);
  p->checked = p->factored;
  return st;
}

// FP64 form: Y_j = (z_j B - A)^{-1} R for all nodes (Y: n x N m, node j at columns j m).
// (cols: right-hand sides actually used, at most m; node j's block keeps its
// place at column j m of Y)
void solve_nodes_z(feast_plan *p, const z64 *R, int64_t ldr, int64_t cols) {
  const int64_t n = p->n, m = p->m, ldY = p->ldY();
  z64 *Y = p->Y.as<z64>();
  ktimed(p, FEAST_K_GATHER, 16.0 * n * cols * (1 + p->N), [&]() {
    feast::gather_rows<z64>(p->s, R, ldr, 0, p->perm.as<int32_t>(), n, cols, p->N, Y, ldY, m);
  });
  plan_trsolve<z64>(p, p->s, Y, cols, ldY, m, 0);
}

// Mixed form: complex64 LU solves; FP64 residual r_j = R - (z_j B - A) Y_j of
// all nodes (one launch, z_j B - A formed per staged tile); the complex64 correction
// d_j = (LU32_j)^{-1} r_j and the FP64 update Y_j += d_j.
//   target > 0 : sweep until every node's normwise backward error
//                ||r_j||_F / ((|z_j| ||B||_F + ||A||_F) ||Y_j||_F + ||R||_F) <= target
//                (at most max_sweeps corrections; each test costs one residual);
//   target <= 0: exactly `sweeps` corrections with no final residual (the caller
//                judges the accuracy, as Algorithm 5 does through eq. 5-1).
//   resume     : Y already holds this right-hand side's node solutions (a
//                filter that ran with fewer corrections): refine them further.
void solve_nodes_mixed(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb,
                       const z64 *R, int64_t ldr, double target, int sweeps, int64_t cols,
                       bool resume = false) {
  const int64_t n = p->n, m = cols, ldY = p->ldY(), sY = p->m;
  const int N = p->N;
  hipStream_t s = p->s;
  z64 *Y = p->Y.as<z64>();
  c64 *Yc = p->Yc.as<c64>();
  z64 *T1 = p->T1.as<z64>(), *T2 = p->T2.as<z64>();
  const c64 *F = p->F.as<c64>();
  const int32_t *perm = p->perm.as<int32_t>();
  double *part = p->part.as<double>(), *nrm = p->nrm.as<double>();
  // ||R||_F^2 sets the power-of-two scale of every complex64 solve below
  double *rn = p->rn.as<double>();
  const double rcnt = static_cast<double>(n) * m;
  feast::fro2_batched(s, R, ldr, 0, n, m, 1, rn + 8, rn);
  if (!resume) {  // complex64 solve of P_j R
    ktimed(p, FEAST_K_GATHER, 16.0 * n * m * (1 + N),
           [&]() { feast::gather_rows<z64>(s, R, ldr, 0, perm, n, m, N, T1, ldY, sY); });
    ktimed(p, FEAST_K_Z2C, 24.0 * n * ldY,
           [&]() { feast::z_to_c(s, T1, ldY, 0, n, ldY, 1, Yc, ldY, 0, rn, rcnt); });
    plan_trsolve<c64>(p, s, Yc, m, ldY, sY, 0);
    ktimed(p, FEAST_K_C2Z, 24.0 * n * ldY,
           [&]() { feast::c_to_z(s, Yc, ldY, 0, n, ldY, 1, Y, ldY, 0, rn, rcnt); });
  }
  p->last_sweeps = 0;
  p->last_be = -1.0;
  p->stagnated = false;
  const bool verify = target > 0.0;
  const int max_corr = verify ? p->o.max_sweeps : sweeps;
  if (!verify && sweeps <= 0) return;
  if (verify) feast::fro2_batched(s, R, ldr, 0, n, m, 1, part, nrm + 2 * N);
  std::vector<double> hn(2 * N + 1);
  double prev_worst = INFINITY;
  for (int sweep = 0; sweep <= max_corr; ++sweep) {
    if (!verify && sweep == max_corr) break;
    if (lda == ldb) {  // r_j = R - (z_j B - A) Y_j, shifted matrices formed tile by tile
      feast::zgemm_shift_residual(s, n, m, n, A, B, lda, p->dz.as<z64>(), Y, ldY, sY, R, ldr, 0, T1,
                                  ldY, sY, N);
    } else {
      gemm_t<z64>(s, 0, n, ldY, n, zc(1.0), A, lda, 0, Y, ldY, 0, zc(0.0), T1, ldY, 0, 1);
      gemm_t<z64>(s, 0, n, ldY, n, zc(1.0), B, ldb, 0, Y, ldY, 0, zc(0.0), T2, ldY, 0, 1);
      feast::shift_residual(s, R, ldr, T1, T2, ldY, p->dz.as<z64>(), N, n, sY, m);
    }
    if (verify) {
      feast::fro2_batched(s, T1, ldY, sY, n, m, N, part, nrm);
      feast::fro2_batched(s, Y, ldY, sY, n, m, N, part, nrm + N);
      HIPCHK(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * (2 * N + 1), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const double nR = std::sqrt(hn[2 * N]);
      double worst = 0.0;
      for (int j = 0; j < N; ++j) {
        const double mj = std::abs(p->hz[j]) * p->normB + p->normA;
        const double be = std::sqrt(hn[j]) / (mj * std::sqrt(hn[N + j]) + nR);
        worst = std::max(worst, be);
      }
      p->last_be = worst;
      if (worst <= target) return;
      if (sweep == max_corr || !(worst < 0.5 * prev_worst)) {
        p->stagnated = true;
        return;
      }
      prev_worst = worst;
    }
    // (with cols < m the unused node columns of T1 hold stale values: they are
    // carried along by the conversions but never read by the products)
    ktimed(p, FEAST_K_GATHER, 32.0 * n * m * N,
           [&]() { feast::gather_rows<z64>(s, T1, ldY, sY, perm, n, m, N, T2, ldY, sY); });
    ktimed(p, FEAST_K_Z2C, 24.0 * n * ldY,
           [&]() { feast::z_to_c(s, T2, ldY, 0, n, ldY, 1, Yc, ldY, 0, rn, rcnt); });
    plan_trsolve<c64>(p, s, Yc, m, ldY, sY, 0);
    if (sweep == 0) {
      // the first correction relative to the solution it corrects: about the
      // forward error of the complex64 solves, u32 cond(z_j B - A)
      feast::fro2_c(s, Yc, ldY, n, ldY, rn + 8, rn + 1);
      feast::fro2_batched(s, Y, ldY, 0, n, ldY, 1, rn + 8, rn + 2);
      if (p->hrn) {
        HIPCHK(hipMemcpyAsync(p->hrn, rn, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        p->rho_pending = true;
      }
    }
    ktimed(p, FEAST_K_C2Z, 40.0 * n * ldY,
           [&]() { feast::add_c_to_z(s, Yc, ldY, 0, n, ldY, 1, Y, ldY, 0, rn, rcnt); });
    p->last_sweeps = sweep + 1;
  }
}

// U = sum_j w_j (z_j B - A)^{-1} R  (the filter of eq. 8-4 on the right-hand side R = B U_1).
// Mixed form: see solve_nodes_mixed for `target` and `sweeps`.
int filter_rhs(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb, const z64 *R,
               int64_t ldr, z64 *U, int64_t ldu, double target, int sweeps, int64_t cols = -1,
               bool resume = false) {
  if (cols < 0) cols = p->m;
  int st = ensure_factored(p, A, lda, B, ldb);
  if (p->mixed()) {
    solve_nodes_mixed(p, A, lda, B, ldb, R, ldr, target, sweeps, cols, resume);
  } else {
    p->last_sweeps = 0;
    if (p->sp.on)
      feast::band_solve(p->s, p->sp.Lf.as<z64>(), p->sp.Uf.as<z64>(), p->sp.Dinv.as<z64>(),
                        p->sp.piv.as<int32_t>(), p->N, p->n, p->sp.kl, p->sp.ku, R, ldr, cols,
                        p->Y.as<z64>(), p->ldY(), p->m);
    else
      solve_nodes_z(p, R, ldr, cols);
  }
  ktimed(p, FEAST_K_WSUM, 16.0 * p->n * cols * (p->N + 1), [&]() {
    feast::weighted_sum(p->s, p->Y.as<z64>(), p->ldY(), p->m, p->dw.as<z64>(), p->N, p->n, cols, U,
                        ldu);
  });
  if (st == FEAST_OK && p->mixed() && p->stagnated) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "refinement stopped at backward error %.3e (target %.3e) after %d sweeps",
                  p->last_be, target, p->last_sweeps);
    p->err = buf;
    st = FEAST_REFINE_STAGNATED;
  }
  return st;
}

// Cholesky G = R^* R of a t x t Hermitian matrix (upper triangle used, R
// written over it) and X = R^{-1}, blocked by 64 columns: one kernel factors a
// diagonal block and inverts it (the inverse goes to X's diagonal block), then
// R_J,rest = R_JJ^{-*} G_J,rest and G_rest -= R_J,rest^* R_J,rest as MFMA GEMMs;
// X's off-diagonal blocks follow by X12 = -X11 R12 X22, halving recursively.
void inv_upper_rec(hipStream_t s, const z64 *R, int64_t t, z64 *X, z64 *T, int64_t r0, int64_t r1) {
  if (r1 - r0 <= 64) return;
  const int64_t mid = r0 + ((r1 - r0 + 127) / 128) * 64;
  inv_upper_rec(s, R, t, X, T, r0, mid);
  inv_upper_rec(s, R, t, X, T, mid, r1);
  gemm_t<z64>(s, 0, mid - r0, r1 - mid, r1 - mid, zc(1.0), R + r0 * t + mid, t, 0, X + mid * t + mid,
              t, 0, zc(0.0), T, t, 0, 1);
  gemm_t<z64>(s, 0, mid - r0, r1 - mid, mid - r0, zc(-1.0), X + r0 * t + r0, t, 0, T, t, 0, zc(0.0),
              X + r0 * t + mid, t, 0, 1);
}

void chol_inv_blocked(feast_plan *p, z64 *G, int64_t t, double shift_rel, int32_t *flag, z64 *X,
                      z64 *T) {
  hipStream_t s = p->s;
  if (shift_rel > 0.0) feast::add_diag_shift(s, G, t, shift_rel);
  for (int64_t J0 = 0; J0 < t; J0 += 64) {
    const int jb = static_cast<int>(std::min<int64_t>(64, t - J0));
    z64 *GJ = G + J0 * t + J0, *XJ = X + J0 * t + J0;
    feast::chol_inv_block(s, GJ, t, jb, static_cast<int>(J0), flag, XJ, t);
    const int64_t rest = t - J0 - jb;
    if (rest <= 0) break;
    gemm_t<z64>(s, 2, jb, rest, jb, zc(1.0), XJ, t, 0, GJ + jb, t, 0, zc(0.0), GJ + jb, t, 0, 1);
    gemm_t<z64>(s, 2, rest, rest, jb, zc(-1.0), GJ + jb, t, 0, GJ + jb, t, 0, zc(1.0),
                G + (J0 + jb) * t + J0 + jb, t, 0, 1);
  }
  if (t > 64) {
    feast::zero_lower(s, G, t, false);
    feast::zero_lower(s, X, t, false);
    inv_upper_rec(s, G, t, X, T, 0, t);
  }
}

// Shifted Cholesky QR3 (three Cholesky QR passes, the first on X^*X + s I with
// s = 11 (n m + m (m+1)) u ||X||_F^2): an FP64 orthonormalisation that stays
// stable for condition numbers up to about 1/u, built from the Gram GEMM,
// a blocked t x t Cholesky, a blocked triangular inverse and one more GEMM per pass.
}  // namespace

// Helpers shared with the batched driver (declared in plan.h).
namespace feast_drv {

int fail(feast_plan *p, int code, const std::string &msg) {
  if (p) p->err = msg;
  return code;
}

void kprof_reset(feast_plan *p) {
  p->kev_used = 0;
  p->krec.clear();
}

void kprof_collect(feast_plan *p, feast_info *info) {
  for (const feast_plan::KRec &r : p->krec) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    feast_kprof &k = info->hbm[r.cls];
    k.launches += 1;
    k.ms += ms;
    k.bytes += r.bytes;
  }
}

template <>
void gemm_t<z64>(hipStream_t s, int ta, int64_t M, int64_t N, int64_t K, z64 alpha, const z64 *A,
                 int64_t lda, int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 beta, z64 *C,
                 int64_t ldc, int64_t sC, int32_t batch, z64 *work, int64_t welems, int cfg) {
  feast::zgemm(s, ta, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, work, welems,
               cfg);
}
template <>
void gemm_t<c64>(hipStream_t s, int ta, int64_t M, int64_t N, int64_t K, z64 alpha, const c64 *A,
                 int64_t lda, int64_t sA, const c64 *B, int64_t ldb, int64_t sB, z64 beta, c64 *C,
                 int64_t ldc, int64_t sC, int32_t batch, c64 *work, int64_t welems, int cfg) {
  feast::cgemm(s, ta, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, work, welems,
               cfg);
}

void ensure_workspace(feast_plan *p, bool with_nodes) {
  const int64_t n = p->n, m = p->m, N = p->N;
  const size_t zs = sizeof(z64);
  p->R.alloc(zs * n * m);
  if (with_nodes) p->Y.alloc(zs * n * m * N);
  p->W.alloc(zs * n * m * feast_plan::W_COUNT);
  p->G.alloc(zs * m * m * feast_plan::G_COUNT);
  // split-K partials: the m x m Gram and projection products (K = n), and with
  // the node solutions (a solving plan) the n x m products with K = n of the
  // projection, one buffer per stream they run on
  p->splitws.alloc(zs * std::max<int64_t>(std::max<int64_t>(m * m * 96, with_nodes ? 4 * n * m : 0),
                                          1 << 16));
  if (with_nodes) p->splitws2.alloc(zs * std::max<int64_t>(4 * n * m, 1 << 16));
  p->part.alloc(sizeof(double) * std::max<int64_t>(((n + 63) / 64) * 3 * m, 64 * N + 64));
  p->nrm.alloc(sizeof(double) * (3 * m + 4 * N + 16));
  p->flag.alloc(sizeof(int32_t) * 16);
  p->small.alloc(zs * (2 * m + 16));
  p->rn.alloc(sizeof(double) * (8 + 1024));
  if (p->mixed() && with_nodes) {
    p->T1.alloc(zs * n * m * N);
    p->T2.alloc(zs * n * m * N);
    p->Yc.alloc(sizeof(c64) * n * m * N);
  }
}

int64_t splitws_elems(const feast_plan *p) {
  return static_cast<int64_t>(p->splitws.bytes / sizeof(z64));
}

// (cols: columns of X to orthonormalise, at most the plan's m; default m)
void orth(feast_plan *p, z64 *X, int64_t ldx, int flag_slot, int64_t cols) {
  const int64_t n = p->n, m = cols < 0 ? p->m : cols;
  hipStream_t s = p->s;
  z64 *G = p->gblk(feast_plan::G_GRAM);
  z64 *Ri = p->gblk(feast_plan::G_RINV), *T = p->gblk(feast_plan::G_T);
  z64 *Wt = p->wblk(feast_plan::W_ORTH);
  int32_t *flag = p->flag.as<int32_t>() + flag_slot;
  const double shift_rel = 11.0 * (static_cast<double>(n) * m + static_cast<double>(m) * (m + 1)) * kU64;
  for (int pass = 0; pass < 3; ++pass) {
    gemm_t<z64>(s, 2, m, m, n, zc(1.0), X, ldx, 0, X, ldx, 0, zc(0.0), G, m, 0, 1,
                p->splitws.as<z64>(), splitws_elems(p));
    chol_inv_blocked(p, G, m, pass == 0 ? shift_rel : 0.0, flag + pass, Ri, T);
    gemm_t<z64>(s, 0, n, m, m, zc(1.0), X, ldx, 0, Ri, m, 0, zc(0.0), Wt, m, 0, 1);
    feast::copy_block_z(s, Wt, m, n, m, X, ldx);
  }
}

// Algorithm 5's QR steps and reduced pencil: U -> U_1, A U_1, B U_1, U_2, At, Bt (device m x m).
void project_device(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb, z64 *U,
                    int64_t ldu, z64 *AU1, int64_t ldau, z64 *BU1, int64_t ldbu) {
  const int64_t n = p->n, m = p->m;
  hipStream_t s = p->s;
  feast::fill_i32(s, p->flag.as<int32_t>(), 6, 0);
  orth(p, U, ldu, 0);
  if (p->sp.on) {  // A U_1 and B U_1 in one pass over the shared pattern
    feast::csr_spmm(s, p->sp.rp.as<int32_t>(), p->sp.ci.as<int32_t>(), p->sp.va.as<z64>(),
                    p->sp.vb.as<z64>(), n, U, ldu, m, AU1, ldau, BU1, ldbu);
    z64 *U2 = p->wblk(feast_plan::W_U2);
    feast::copy_block_z(s, BU1, ldbu, n, m, U2, m);
    orth(p, U2, m, 3);
    gemm_t<z64>(s, 2, m, m, n, zc(1.0), U2, m, 0, AU1, ldau, 0, zc(0.0),
                p->gblk(feast_plan::G_AT), m, 0, 1, p->splitws.as<z64>(), splitws_elems(p));
    gemm_t<z64>(s, 2, m, m, n, zc(1.0), U2, m, 0, BU1, ldbu, 0, zc(0.0),
                p->gblk(feast_plan::G_BT), m, 0, 1, p->splitws.as<z64>(), splitws_elems(p));
    return;
  }
  // A U_1 runs on the side stream beside B U_1 and the orthonormalisation of
  // B U_1: one n x m product alone fills only (n/64)(m/64) workgroups, and the
  // Cholesky QR chain leaves most compute units idle
  HIPCHK(hipEventRecord(p->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(p->side, p->ev_fork, 0));
  // (K = n over (n/64)(m/64) output tiles: split-K, each stream with partials of its own)
  gemm_t<z64>(p->side, 0, n, m, n, zc(1.0), A, lda, 0, U, ldu, 0, zc(0.0), AU1, ldau, 0, 1,
              p->splitws2.as<z64>(), static_cast<int64_t>(p->splitws2.bytes / sizeof(z64)));
  HIPCHK(hipEventRecord(p->ev_join, p->side));
  gemm_t<z64>(s, 0, n, m, n, zc(1.0), B, ldb, 0, U, ldu, 0, zc(0.0), BU1, ldbu, 0, 1,
              p->splitws.as<z64>(), splitws_elems(p));
  z64 *U2 = p->wblk(feast_plan::W_U2);
  feast::copy_block_z(s, BU1, ldbu, n, m, U2, m);
  orth(p, U2, m, 3);
  HIPCHK(hipStreamWaitEvent(s, p->ev_join, 0));
  gemm_t<z64>(s, 2, m, m, n, zc(1.0), U2, m, 0, AU1, ldau, 0, zc(0.0), p->gblk(feast_plan::G_AT),
              m, 0, 1, p->splitws.as<z64>(), splitws_elems(p));
  gemm_t<z64>(s, 2, m, m, n, zc(1.0), U2, m, 0, BU1, ldbu, 0, zc(0.0), p->gblk(feast_plan::G_BT),
              m, 0, 1, p->splitws.as<z64>(), splitws_elems(p));
}

int project_finish(feast_plan *p, feast_z *hAt, feast_z *hBt) {
  const int64_t m = p->m;
  hipStream_t s = p->s;
  int32_t hf[6];
  HIPCHK(hipMemcpyAsync(hAt, p->gblk(feast_plan::G_AT), sizeof(z64) * m * m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hBt, p->gblk(feast_plan::G_BT), sizeof(z64) * m * m, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hf, p->flag.p, sizeof(int32_t) * 6, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  for (int i = 0; i < 6; ++i)
    if (hf[i] != 0) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "Cholesky QR pass %d of %s broke down at column %d", i % 3 + 1,
                    i < 3 ? "U" : "B U_1", hf[i] - 1);
      p->err = buf;
      return FEAST_ENUMERIC;
    }
  return FEAST_OK;
}

int host_threads() {
  return static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
}

bool bad_contour(const feast_contour *c) {
  return !c || !(c->radius > 0.0) || !std::isfinite(c->radius) || !std::isfinite(c->center.re) ||
         !std::isfinite(c->center.im) || c->nodes < 1 || c->nodes > 1024 ||
         (c->rule != FEAST_TRAPEZOID && c->rule != FEAST_GAUSS_LEGENDRE);
}

}  // namespace feast_drv

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int feast_version(void) { return 10000; }

void feast_opts_default(feast_opts *o) {
  if (!o) return;
  o->eps = 1e-10;
  o->eta = 1e-3;
  o->max_iter = 20;
  o->prec = FEAST_FP64;
  o->refine_tol = 4.0 * kU64;
  o->max_sweeps = 6;
  o->nb = 0;
  o->profile = 0;
  o->lookahead = 0;
  o->update_tile = 0;
  o->ahead_cus = 0;
  o->ahead_rows = 0;
  o->batch_update = 0;
}

int feast_nodes(const feast_contour *c, feast_z *hz, feast_z *hw) {
  if (bad_contour(c) || !hz || !hw) return FEAST_EINVAL;
  std::vector<cd> z(c->nodes), w(c->nodes);
  if (feast_host::contour_nodes(cd(c->center.re, c->center.im), c->radius, c->nodes, c->rule,
                                z.data(), w.data()) != 0)
    return FEAST_EINVAL;
  for (int j = 0; j < c->nodes; ++j) {
    hz[j] = {z[j].real(), z[j].imag()};
    hw[j] = {w[j].real(), w[j].imag()};
  }
  return FEAST_OK;
}

int feast_stop_rule(int32_t k, int32_t c_k, double e_k, int32_t c_prev, double e_prev, double eps,
                    int32_t max_iter) {
  return feast_host::stop_rule(k, c_k, e_k, c_prev, e_prev, eps, max_iter);
}

int feast_reduced_eig(int64_t t, const feast_z *hAt, int64_t lda, const feast_z *hBt, int64_t ldb,
                      feast_z *halpha, feast_z *hbeta, feast_z *hY, int64_t ldy) {
  if (t < 0 || (t > 0 && (!hAt || !hBt || !halpha || !hbeta || !hY)) || lda < t || ldb < t || ldy < t)
    return FEAST_EINVAL;
  try {
    const int nt = host_threads();
    const int rc = feast_host::reduced_eig(t, reinterpret_cast<const cd *>(hAt), lda,
                                           reinterpret_cast<const cd *>(hBt), ldb,
                                           reinterpret_cast<cd *>(halpha),
                                           reinterpret_cast<cd *>(hbeta), reinterpret_cast<cd *>(hY),
                                           ldy, nt);
    return rc == 0 ? FEAST_OK : FEAST_ENUMERIC;
  } catch (...) {
    return FEAST_ENOMEM;
  }
}

int feast_plan_create(feast_plan **plan, int64_t n, int64_t m, const feast_contour *c,
                      const feast_opts *o, void *stream) {
  if (!plan) return FEAST_EINVAL;
  *plan = nullptr;
  feast_opts opts;
  feast_opts_default(&opts);
  if (o) opts = *o;
  if (n < 1 || n > 16384 || m < 1 || m > n || bad_contour(c)) return FEAST_EINVAL;
  if (!(opts.eta > 0.0) || !(opts.eps >= 0.0) || opts.max_iter < 1 ||
      opts.max_iter > FEAST_MAX_HISTORY || (opts.prec != FEAST_FP64 && opts.prec != FEAST_MIXED) ||
      opts.max_sweeps < 0 || !(opts.refine_tol >= 0.0) ||
      (opts.nb != 0 && opts.nb != 64 && opts.nb != 128) || opts.lookahead < 0 ||
      opts.lookahead > 1 || opts.update_tile < 0 || opts.update_tile > 1 ||
      opts.batch_update < 0 || opts.batch_update > 3 ||
      (opts.ahead_cus != 0 && (opts.ahead_cus < 8 || opts.ahead_cus > 128)) ||
      opts.ahead_rows < 0)
    return FEAST_EINVAL;
  feast_plan *p = nullptr;
  try {
    p = new feast_plan();
  } catch (...) {
    return FEAST_ENOMEM;
  }
  p->n = n;
  p->m = m;
  p->N = c->nodes;
  p->c = *c;
  p->o = opts;
  p->s = static_cast<hipStream_t>(stream);
  p->nb = opts.nb ? opts.nb : 128;
  p->nblk = (n + 63) / 64;
  p->hz.resize(p->N);
  p->hw.resize(p->N);
  feast_host::contour_nodes(cd(c->center.re, c->center.im), c->radius, p->N, c->rule, p->hz.data(),
                            p->hw.data());
  const int rc = guarded(p, [&]() {
    p->dz.alloc(sizeof(z64) * p->N);
    p->dw.alloc(sizeof(z64) * p->N);
    p->dwc.alloc(sizeof(z64) * p->N);
    std::vector<cd> wc(p->N);
    for (int j = 0; j < p->N; ++j) wc[j] = std::conj(p->hw[j]);
    HIPCHK(hipMemcpy(p->dz.p, p->hz.data(), sizeof(z64) * p->N, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->dw.p, p->hw.data(), sizeof(z64) * p->N, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->dwc.p, wc.data(), sizeof(z64) * p->N, hipMemcpyHostToDevice));
    ensure_workspace(p);
    HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&p->hrn), 4 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipEventCreateWithFlags(&p->ev_cols, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_panel, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
    return FEAST_OK;
  });
  if (rc != FEAST_OK) {
    feast_plan_destroy(p);
    return rc;
  }
  *plan = p;
  return FEAST_OK;
}

int feast_plan_destroy(feast_plan *p) {
  if (!p) return FEAST_OK;
  if (p->s) (void)hipStreamSynchronize(p->s);
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->kev) (void)hipEventDestroy(e);
  if (p->hrn) (void)hipHostFree(p->hrn);
  for (hipStream_t st : {p->side, p->aux})
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  if (p->ev_cols) (void)hipEventDestroy(p->ev_cols);
  if (p->ev_panel) (void)hipEventDestroy(p->ev_panel);
  for (hipEvent_t e : {p->ev_fork, p->ev_join})
    if (e) (void)hipEventDestroy(e);
  for (DevBuf *b : {&p->dz, &p->dw, &p->dwc, &p->adj, &p->adj_piv, &p->adj_info, &p->adj_inv, &p->F, &p->piv, &p->perm, &p->info, &p->Linv, &p->Uinv, &p->Linv2, &p->Uinv2, &p->cirr_w, &p->R,
                    &p->Y, &p->T1, &p->T2, &p->Yc, &p->W, &p->G, &p->splitws, &p->splitws2, &p->part, &p->nrm,
                    &p->flag, &p->small, &p->fp, &p->rn})
    b->release();
  delete p;
  return FEAST_OK;
}

int feast_plan_invalidate(feast_plan *p) {
  if (!p) return FEAST_EINVAL;
  p->factored = false;
  return FEAST_OK;
}

const char *feast_last_error(const feast_plan *p) { return p ? p->err.c_str() : "null plan"; }

int feast_filter(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB, int64_t ldb,
                 const feast_z *dV, int64_t ldv, feast_z *dU, int64_t ldu) {
  if (!p) return FEAST_EINVAL;
  if (!dA || !dB || !dV || !dU || lda < p->n || ldb < p->n || ldv < p->m || ldu < p->m)
    return fail(p, FEAST_EINVAL, "feast_filter: null pointer or leading dimension too small");
  p->err.clear();
  CheckScope check_scope(p);
  kprof_reset(p);
  return guarded(p, [&]() {
    const z64 *A = reinterpret_cast<const z64 *>(dA), *B = reinterpret_cast<const z64 *>(dB);
    const z64 *V = reinterpret_cast<const z64 *>(dV);
    // R = B V
    gemm_t<z64>(p->s, 0, p->n, p->m, p->n, zc(1.0), B, ldb, 0, V, ldv, 0, zc(0.0), p->R.as<z64>(),
                p->m, 0, 1);
    const int st = filter_rhs(p, A, lda, B, ldb, p->R.as<z64>(), p->m, reinterpret_cast<z64 *>(dU),
                              ldu, p->o.refine_tol, 0);
    HIPCHK(hipGetLastError());
    return st;
  });
}

int feast_project(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB, int64_t ldb,
                  feast_z *dU, int64_t ldu, feast_z *dAU1, int64_t ldau, feast_z *dBU1,
                  int64_t ldbu, feast_z *hAt, feast_z *hBt) {
  if (!p) return FEAST_EINVAL;
  if (!dA || !dB || !dU || !dAU1 || !dBU1 || !hAt || !hBt || lda < p->n || ldb < p->n ||
      ldu < p->m || ldau < p->m || ldbu < p->m)
    return fail(p, FEAST_EINVAL, "feast_project: null pointer or leading dimension too small");
  p->err.clear();
  return guarded(p, [&]() {
    project_device(p, reinterpret_cast<const z64 *>(dA), lda, reinterpret_cast<const z64 *>(dB), ldb,
                   reinterpret_cast<z64 *>(dU), ldu, reinterpret_cast<z64 *>(dAU1), ldau,
                   reinterpret_cast<z64 *>(dBU1), ldbu);
    return project_finish(p, hAt, hBt);
  });
}

// Algorithm 5; from_basis: dV is an orthonormal U_1 that is already filtered
// (Search's output), so the Search call is skipped.
static int solve_impl(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB,
                      int64_t ldb, const feast_z *dV, int64_t ldv, bool from_basis,
                      feast_z *hLambda, feast_z *dX, int64_t ldx, double *hRes, int32_t *s_found,
                      double *err, int32_t *flag, feast_info *info) {
  if (!p) return FEAST_EINVAL;
  if ((!p->sp.on && (!dA || !dB || lda < p->n || ldb < p->n)) || !dV || !hLambda || !dX ||
      !s_found || !err || !flag || ldv < p->m || ldx < p->m)
    return fail(p, FEAST_EINVAL, "feast_solve: null pointer or leading dimension too small");
  p->err.clear();
  CheckScope check_scope(p);
  return guarded(p, [&]() -> int {
    const int64_t n = p->n, m = p->m;
    hipStream_t s = p->s;       // filters and projections
    hipStream_t s2 = p->aux;    // Ritz vectors and residuals (overlap with the next filter)
    const z64 *A = reinterpret_cast<const z64 *>(dA), *B = reinterpret_cast<const z64 *>(dB);
    const z64 *V = reinterpret_cast<const z64 *>(dV);
    const cd gamma(p->c.center.re, p->c.center.im);
    const double rho = p->c.radius;
    feast_info inf{};
    Timer total;
    int status = FEAST_OK;
    kprof_reset(p);
    {
      Timer t;
      const int st = ensure_factored(p, A, lda, B, ldb);
      inf.t_factor_ms = t.ms();
      if (st == FEAST_SINGULAR) return st;
    }
    z64 *U1 = p->wblk(feast_plan::W_U1), *AU1 = p->wblk(feast_plan::W_AU1);
    z64 *BU1 = p->wblk(feast_plan::W_BU1), *UF = p->wblk(feast_plan::W_UF);
    z64 *X = p->wblk(feast_plan::W_X), *AX = p->wblk(feast_plan::W_AX);
    z64 *BX = p->wblk(feast_plan::W_BX), *Xprev = p->wblk(feast_plan::W_XPREV);
    z64 *Ys = p->gblk(feast_plan::G_YS);
    z64 *dlam = p->small.as<z64>();
    int32_t *didx = reinterpret_cast<int32_t *>(p->small.as<z64>() + m);
    double *dnorm = p->nrm.as<double>();
    const int64_t mm = m * m;
    std::vector<feast_z> hAt(mm), hBt(mm), hY(mm), halpha(m), hbeta(m);
    std::vector<double> hn(3 * m);
    // Mixed form: Search's filter is not refined; a later filter gets `sweeps`
    // corrections unless the last known e(k) is infinite or above
    // kRefineFrom, where the complex64 solves are already more accurate than
    // the subspace (the first filter after Search, with no e(k) yet, is
    // refined).  Once a refined iteration with a settled count misses eps
    // without halving e(k), the solves limit the accuracy (their forward error
    // is the backward error times cond(z_j B - A)): every later filter then
    // refines each node until its backward error reaches refine_tol.
    // The number of corrections of a refined filter starts at one; once a
    // filter's first correction has measured the contraction rho = ||d_1|| /
    // ||Y_0|| (about u32 cond(z_j B - A)), later filters take the s that makes
    // the predicted error rho^(s+1) at most eps / 10 (at most max_sweeps).
    constexpr double kRefineFrom = 1e-4;
    int sweeps = p->mixed() ? 1 : 0;
    auto sweeps_for = [&](double e_last, bool known) {
      if (!p->mixed()) return 0;
      if (known && !(e_last <= kRefineFrom)) return 0;
      return sweeps;
    };
    auto predict_sweeps = [&](double rho) {
      if (!p->mixed() || !(rho > 0.0)) return;
      const double goal = 0.1 * std::max(p->o.eps, 1e-15);
      int sw = p->o.max_sweeps;
      if (rho < 0.5) sw = static_cast<int>(std::ceil(std::log(goal) / std::log(rho))) - 1;
      sweeps = std::max(1, std::min(sw, std::max(1, p->o.max_sweeps)));
    };
    int sweeps_now = sweeps;
    bool verify = false;
    // FP64 fallback: a contraction that is not finite, or so slow that the
    // corrections would need more than max_sweeps to bring the complex64
    // solves to eps / 10, means refinement cannot make this pencil's filter as
    // accurate as the FP64 form's (or only at more cost); the solve then
    // refactors in FP64, repeats that filter and continues in FP64.  The plan
    // returns to complex64 (unfactored) at the end.
    auto needs_fp64 = [&](double rho) {
      if (!(rho >= 0.0) || !std::isfinite(rho)) return true;
      if (rho == 0.0) return false;
      if (rho >= 1.0) return true;
      const double goal = 0.1 * std::max(p->o.eps, 1e-15);
      return std::ceil(std::log(goal) / std::log(rho)) - 1.0 > p->o.max_sweeps;
    };
    struct PrecRestore {
      feast_plan *p;
      bool on = false;
      ~PrecRestore() {
        if (on) {
          p->o.prec = FEAST_MIXED;
          p->factored = false;
          p->checked = false;
        }
      }
    } prec_restore{p};
    auto run_filter = [&](const z64 *R, z64 *Uout, bool first, bool resume = false) -> int {
      const double target = (!first && verify) ? p->o.refine_tol : 0.0;
      const int st = filter_rhs(p, A, lda, B, ldb, R, m, Uout, m, target, first ? 0 : sweeps_now,
                                -1, resume);
      if (inf.filters < FEAST_MAX_HISTORY) inf.sweeps[inf.filters] = p->last_sweeps;
      inf.filters += 1;
      return st;
    };
    if (from_basis) {
      // the Search call was feast_search: its basis is U_1
      feast::copy_block_z(s, V, ldv, n, m, U1, m);
    } else {
      // Search with the subspace size fixed: U = Q_N V, QR inside the projection
      Timer t;
      if (p->sp.on)
        feast::csr_spmm(s, p->sp.rp.as<int32_t>(), p->sp.ci.as<int32_t>(), p->sp.va.as<z64>(),
                        p->sp.vb.as<z64>(), n, V, ldv, m, nullptr, 0, p->R.as<z64>(), m);
      else
        gemm_t<z64>(s, 0, n, m, n, zc(1.0), B, ldb, 0, V, ldv, 0, zc(0.0), p->R.as<z64>(), m, 0, 1,
                    p->splitws.as<z64>(), splitws_elems(p));
      const int st = run_filter(p->R.as<z64>(), U1, true);
      if (st != FEAST_OK && st != FEAST_REFINE_STAGNATED) return st;
      HIPCHK(hipStreamSynchronize(s));
      inf.t_filter_ms += t.ms();
    }
    // QR of B U_1 and the first reduced pencil
    {
      Timer t;
      project_device(p, A, lda, B, ldb, U1, m, AU1, m, BU1, m);
      const int st = project_finish(p, hAt.data(), hBt.data());
      inf.t_project_ms += t.ms();
      if (st != FEAST_OK) return st;
    }
    HIPCHK(hipEventRecord(p->ev_cols, s));
    HIPCHK(hipStreamWaitEvent(s2, p->ev_cols, 0));
    // e(0) = 0, c(0) = 0
    double e_prev = 0.0, e_prev2 = 0.0;
    double last_filter_ms = 0.0, last_host_ms = 0.0;  // the speculation margin's inputs
    int c_prev = 0;
    std::vector<cd> lam_prev;
    std::vector<double> r_prev;
    for (int k = 1; k <= p->o.max_iter; ++k) {
      // filter step ahead of time: the next filter needs only B U_1, so it runs on
      // the GPU while the host solves the reduced pencil; it is skipped when
      // this iteration is likely to be the last one: e(k) predicted from the
      // observed reduction factor e(k-1)/e(k-2) (before two values exist, a
      // fast one) below eps times a margin.  A filter launched for nothing
      // costs a whole filter, a missed overlap at most the host solve, so the
      // margin is the ratio of the last filter's time to the last host solve's
      // (at least 1): with a short reduced problem and an expensive filter (a
      // mixed filter with several corrections), only a clear miss of eps
      // launches ahead.
      const double q = (k >= 3 && e_prev2 > 0.0 && std::isfinite(e_prev2) && std::isfinite(e_prev))
                           ? std::min(1.0, e_prev / e_prev2)
                           : 1e-8;
      const double margin =
          (last_filter_ms > 0.0 && last_host_ms > 0.0)
              ? std::min(1e3, std::max(1.0, last_filter_ms / last_host_ms))
              : 1.0;
      const bool likely_last = (k == p->o.max_iter) ||
                               (c_prev > 0 && std::isfinite(e_prev) && e_prev * q < p->o.eps * margin);
      bool speculated = false;
      Timer tf;
      if (!likely_last) {
        sweeps_now = sweeps_for(e_prev, k >= 2);
        const int st = run_filter(BU1, UF, false);
        if (st == FEAST_REFINE_STAGNATED) status = st;
        else if (st != FEAST_OK) return st;
        speculated = true;
      }
      const double launch_ms = tf.ms();
      // reduced eigenproblem on the host
      Timer te;
      // (eigenvectors only for eigenvalues inside the circle: nothing else is selected)
      if (feast_host::reduced_eig(m, reinterpret_cast<const cd *>(hAt.data()), m,
                                  reinterpret_cast<const cd *>(hBt.data()), m,
                                  reinterpret_cast<cd *>(halpha.data()),
                                  reinterpret_cast<cd *>(hbeta.data()),
                                  reinterpret_cast<cd *>(hY.data()), m, host_threads(), &gamma,
                                  rho) != 0)
        return fail(p, FEAST_ENUMERIC, "reduced QZ did not converge");
      last_host_ms = te.ms();
      inf.t_host_eig_ms += last_host_ms;
      Timer tr;
      std::vector<cd> lam(m);
      std::vector<feast_z> hlam(m);
      for (int64_t i = 0; i < m; ++i) {
        const cd a(halpha[i].re, halpha[i].im), b(hbeta[i].re, hbeta[i].im);
        lam[i] = (b != cd(0.0)) ? a / b : cd(INFINITY, 0.0);
        hlam[i] = std::isfinite(lam[i].real()) ? feast_z{lam[i].real(), lam[i].imag()} : feast_z{0, 0};
      }
      // x_i = U_1 y_i with A x_i = (A U_1) y_i and B x_i = (B U_1) y_i (side stream)
      HIPCHK(hipMemcpyAsync(Ys, hY.data(), sizeof(z64) * mm, hipMemcpyHostToDevice, s2));
      HIPCHK(hipMemcpyAsync(dlam, hlam.data(), sizeof(z64) * m, hipMemcpyHostToDevice, s2));
      gemm_t<z64>(s2, 0, n, m, m, zc(1.0), U1, m, 0, Ys, m, 0, zc(0.0), X, m, 0, 1);
      gemm_t<z64>(s2, 0, n, m, m, zc(1.0), AU1, m, 0, Ys, m, 0, zc(0.0), AX, m, 0, 1);
      gemm_t<z64>(s2, 0, n, m, m, zc(1.0), BU1, m, 0, Ys, m, 0, zc(0.0), BX, m, 0, 1);
      feast::ritz_norms(s2, AX, BX, m, n, m, dlam, p->part.as<double>(), dnorm);
      HIPCHK(hipMemcpyAsync(hn.data(), dnorm, sizeof(double) * 3 * m, hipMemcpyDeviceToHost, s2));
      HIPCHK(hipStreamSynchronize(s2));
      // residuals (eq. 5-1), selection, c(k), e(k)
      std::vector<int32_t> sel;
      std::vector<double> rsel;
      double e_k = 0.0;
      for (int64_t i = 0; i < m; ++i) {
        if (!std::isfinite(lam[i].real()) || !std::isfinite(lam[i].imag())) continue;
        const double den = std::sqrt(hn[3 * i + 1]) + std::sqrt(hn[3 * i + 2]);
        const double r = den > 0.0 ? std::sqrt(hn[3 * i]) / den : INFINITY;
        if (std::abs(lam[i] - gamma) < rho && r < p->o.eta) {
          sel.push_back(static_cast<int32_t>(i));
          rsel.push_back(r);
          e_k = std::max(e_k, r);
        }
      }
      const int c_k = static_cast<int>(sel.size());
      if (c_k == 0) e_k = INFINITY;
      inf.count[k - 1] = c_k;
      inf.err[k - 1] = e_k;
      inf.iters = k;
      // stopping rules.  Mixed form: a rise of e(k) before the node solves are
      // refined to full FP64 backward error may come from the complex64 solves
      // rather than from the subspace, so it switches verified refinement on
      // (below) instead of ending the run; the no-improvement rule then judges
      // iterations whose solves are as accurate as the FP64 form's.
      int act = feast_host::stop_rule(k, c_k, e_k, c_prev, e_prev, p->o.eps, p->o.max_iter);
      if (act == 0 && p->mixed() && !verify) act = 2;
      if (act == 1 || act == -1) {
        if (c_k > 0) {
          HIPCHK(hipMemcpyAsync(didx, sel.data(), sizeof(int32_t) * c_k, hipMemcpyHostToDevice, s2));
          feast::gather_normalize_cols(s2, X, m, n, didx, c_k, reinterpret_cast<z64 *>(dX), ldx, nullptr);
        }
        for (int i = 0; i < c_k; ++i) {
          hLambda[i] = {lam[sel[i]].real(), lam[sel[i]].imag()};
          if (hRes) hRes[i] = rsel[i];
        }
        *s_found = c_k;
        *err = e_k;
        *flag = act;
        HIPCHK(hipStreamSynchronize(s2));
        inf.t_ritz_ms += tr.ms();
        break;
      }
      if (act == 0) {
        const int cp = static_cast<int>(lam_prev.size());
        feast::copy_block_z(s2, Xprev, m, n, cp, reinterpret_cast<z64 *>(dX), ldx);
        for (int i = 0; i < cp; ++i) {
          hLambda[i] = {lam_prev[i].real(), lam_prev[i].imag()};
          if (hRes) hRes[i] = r_prev[i];
        }
        *s_found = cp;
        *err = e_prev;
        *flag = 0;
        HIPCHK(hipStreamSynchronize(s2));
        inf.t_ritz_ms += tr.ms();
        break;
      }
      // keep iterate k for a possible rebound at k+1
      lam_prev.clear();
      r_prev = rsel;
      for (int i = 0; i < c_k; ++i) lam_prev.push_back(lam[sel[i]]);
      if (c_k > 0) {
        HIPCHK(hipMemcpyAsync(didx, sel.data(), sizeof(int32_t) * c_k, hipMemcpyHostToDevice, s2));
        feast::gather_normalize_cols(s2, X, m, n, didx, c_k, Xprev, m, nullptr);
      }
      // a refined iteration whose count is settled, that missed eps and whose
      // error stopped falling geometrically: the solves, not the subspace,
      // limit the accuracy, so refine to full accuracy from now on
      bool verify_now = false;
      if (p->mixed() && !verify && k >= 2 && c_k == c_prev && e_k >= p->o.eps &&
          e_k > 0.5 * e_prev)
        verify = verify_now = true;
      e_prev2 = e_prev;
      e_prev = e_k;
      c_prev = c_k;
      HIPCHK(hipEventRecord(p->ev_panel, s2));
      inf.t_ritz_ms += tr.ms();
      // filter step (unless it already ran)
      // filter time: its launch plus whatever of it the host work did not hide
      Timer tw;
      if (!speculated || verify_now) {
        // (a filter launched ahead with unverified corrections is refined
        // further from its node solutions once verification is switched on)
        sweeps_now = sweeps_for(e_k, true);
        const int st = run_filter(BU1, UF, false, speculated);
        if (st == FEAST_REFINE_STAGNATED) status = st;
        else if (st != FEAST_OK) return st;
      }
      HIPCHK(hipStreamSynchronize(s));
      last_filter_ms = launch_ms + tw.ms();
      inf.t_filter_ms += last_filter_ms;
      if (p->rho_pending) {  // the filter's first correction relative to its solution
        p->rho_pending = false;
        const double rms = std::sqrt(p->hrn[0] / (static_cast<double>(n) * m));
        const int e = (rms > 0.0 && std::isfinite(rms)) ? std::ilogb(rms) : 0;
        const double rho = p->hrn[2] > 0.0 ? std::ldexp(std::sqrt(p->hrn[1] / p->hrn[2]), e) : 0.0;
        if (inf.filters >= 1 && inf.filters <= FEAST_MAX_HISTORY) inf.contraction[inf.filters - 1] = rho;
        predict_sweeps(rho);
        if (p->mixed() && needs_fp64(rho)) {
          HIPCHK(hipStreamSynchronize(s2));
          HIPCHK(hipStreamSynchronize(p->side));
          prec_restore.on = true;
          p->o.prec = FEAST_FP64;
          p->factored = false;
          inf.fp64_fallback = inf.filters;
          Timer tfac;
          const int stf = ensure_factored(p, A, lda, B, ldb);
          inf.t_factor_ms += tfac.ms();
          if (stf == FEAST_SINGULAR) return stf;
          Timer tw2;
          const int st = run_filter(BU1, UF, false);
          if (st != FEAST_OK) return st;
          HIPCHK(hipStreamSynchronize(s));
          inf.t_filter_ms += tw2.ms();
        }
      }
      // QR step and the next reduced pencil (after the side stream is done with U_1)
      {
        Timer t;
        HIPCHK(hipStreamWaitEvent(s, p->ev_panel, 0));
        feast::copy_block_z(s, UF, m, n, m, U1, m);
        project_device(p, A, lda, B, ldb, U1, m, AU1, m, BU1, m);
        const int st = project_finish(p, hAt.data(), hBt.data());
        inf.t_project_ms += t.ms();
        if (st != FEAST_OK) return st;
        HIPCHK(hipEventRecord(p->ev_cols, s));
        HIPCHK(hipStreamWaitEvent(s2, p->ev_cols, 0));
      }
    }
    HIPCHK(hipStreamSynchronize(s));
    inf.t_total_ms = total.ms();
    inf.lu_gemm_launches = p->prof_launches;
    inf.lu_gemm_ms = p->prof_ms;
    inf.lu_gemm_flops = p->prof_flops;
    HIPCHK(hipStreamSynchronize(s2));
    kprof_collect(p, &inf);
    if (info) *info = inf;
    return status;
  });
}

// Block_CIRR (Algorithm 1) on the plan's cached factors.  The moments' node
// solutions are the filter's solves with right-hand side Y itself (mixed plans
// apply one FP64 refinement sweep: there is no outer iteration to absorb
// complex64 solve errors); the moments are weighted node sums; the SVD step's
// orthonormal basis of the moment block comes from shifted Cholesky QR3 (the
// Rayleigh-Ritz pencil depends on the span only, so it has the eigenvalues the
// SVD's left factor gives); the Rayleigh-Ritz steps reuse the projection, host eigensolver
// and Ritz-residual pieces of Algorithm 5.
int feast_cirr(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB, int64_t ldb,
               const feast_z *dY, int64_t ldy, int32_t h, int32_t g, feast_z *hLambda,
               feast_z *dX, int64_t ldx, double *hRes, int32_t *s_found, feast_cirr_info *info) {
  if (!p) return FEAST_EINVAL;
  if (!dA || !dB || !dY || !hLambda || !dX || !s_found || lda < p->n || ldb < p->n || h < 1 ||
      g < 1 || ldy < h || ldx < p->m || static_cast<int64_t>(h) * g > p->m)
    return fail(p, FEAST_EINVAL,
                "feast_cirr: null pointer, leading dimension too small, or h g > m");
  p->err.clear();
  CheckScope check_scope(p);
  return guarded(p, [&]() -> int {
    Timer total;
    const int64_t n = p->n, m = p->m, t = static_cast<int64_t>(h) * g;
    const int N = p->N;
    hipStream_t s = p->s;
    const z64 *A = reinterpret_cast<const z64 *>(dA), *B = reinterpret_cast<const z64 *>(dB);
    const z64 *Y = reinterpret_cast<const z64 *>(dY);
    int st = ensure_factored(p, A, lda, B, ldb);
    if (st == FEAST_SINGULAR) return st;
    z64 *U = p->wblk(feast_plan::W_X), *AU = p->wblk(feast_plan::W_AU1);
    z64 *BU = p->wblk(feast_plan::W_BU1), *X = p->wblk(feast_plan::W_UF);
    z64 *AX = p->wblk(feast_plan::W_AX), *BX = p->wblk(feast_plan::W_BX);
    z64 *Ab = p->gblk(feast_plan::G_AT), *Bb = p->gblk(feast_plan::G_BT);
    z64 *Ys = p->gblk(feast_plan::G_YS);
    z64 *dlam = p->small.as<z64>();
    int32_t *didx = reinterpret_cast<int32_t *>(p->small.as<z64>() + m);
    // moments: Y_j = (z_j B - A)^{-1} Y, then R_i = sum_j w_j mu_j^i Y_j, mu_j = (z_j - gamma)/rho
    if (p->mixed())
      solve_nodes_mixed(p, A, lda, B, ldb, Y, ldy, 0.0, 1, h);
    else
      solve_nodes_z(p, Y, ldy, h);
    const cd gamma(p->c.center.re, p->c.center.im);
    std::vector<cd> wi(static_cast<size_t>(g) * N);
    for (int j = 0; j < N; ++j) {
      const cd mu = (p->hz[j] - gamma) / p->c.radius;
      cd pw(1.0);
      for (int i = 0; i < g; ++i, pw *= mu) wi[static_cast<size_t>(i) * N + j] = p->hw[j] * pw;
    }
    p->cirr_w.alloc(sizeof(z64) * wi.size());
    HIPCHK(hipMemcpyAsync(p->cirr_w.p, wi.data(), sizeof(z64) * wi.size(), hipMemcpyHostToDevice, s));
    for (int i = 0; i < g; ++i)
      feast::weighted_sum(s, p->Y.as<z64>(), p->ldY(), m, p->cirr_w.as<z64>() + i * N, N, n, h,
                          U + static_cast<int64_t>(i) * h, m);
    // orthonormal basis of the moment block (in place)
    feast::fill_i32(s, p->flag.as<int32_t>(), 3, 0);
    orth(p, U, m, 0, t);
    // Rayleigh-Ritz pencil: A~ = U^* A U, B~ = U^* B U
    gemm_t<z64>(s, 0, n, t, n, zc(1.0), A, lda, 0, U, m, 0, zc(0.0), AU, m, 0, 1);
    gemm_t<z64>(s, 0, n, t, n, zc(1.0), B, ldb, 0, U, m, 0, zc(0.0), BU, m, 0, 1);
    gemm_t<z64>(s, 2, t, t, n, zc(1.0), U, m, 0, AU, m, 0, zc(0.0), Ab, t, 0, 1,
                p->splitws.as<z64>(), splitws_elems(p));
    gemm_t<z64>(s, 2, t, t, n, zc(1.0), U, m, 0, BU, m, 0, zc(0.0), Bb, t, 0, 1,
                p->splitws.as<z64>(), splitws_elems(p));
    const int64_t tt = t * t;
    std::vector<feast_z> hA(tt), hB(tt), hYv(tt), hal(t), hbe(t);
    int32_t hf[3];
    HIPCHK(hipMemcpyAsync(hA.data(), Ab, sizeof(z64) * tt, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hB.data(), Bb, sizeof(z64) * tt, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hf, p->flag.p, sizeof hf, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hf[0] || hf[1] || hf[2])
      return fail(p, FEAST_ENUMERIC, "feast_cirr: Cholesky QR of the moment block broke down");
    // reduced eigenproblem
    if (feast_reduced_eig(t, hA.data(), t, hB.data(), t, hal.data(), hbe.data(), hYv.data(), t) !=
        FEAST_OK)
      return fail(p, FEAST_ENUMERIC, "feast_cirr: reduced eigensolver did not converge");
    std::vector<cd> lam(t);
    std::vector<feast_z> hlam(t);
    for (int64_t i = 0; i < t; ++i) {
      const cd a(hal[i].re, hal[i].im), b(hbe[i].re, hbe[i].im);
      lam[i] = (b != cd(0.0)) ? a / b : cd(INFINITY, 0.0);
      hlam[i] = std::isfinite(lam[i].real()) ? feast_z{lam[i].real(), lam[i].imag()} : feast_z{0, 0};
    }
    // Ritz pairs: x_i = U y_i, residuals (eq. 5-1) from (A U) y_i and (B U) y_i, selection
    HIPCHK(hipMemcpyAsync(Ys, hYv.data(), sizeof(z64) * tt, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dlam, hlam.data(), sizeof(z64) * t, hipMemcpyHostToDevice, s));
    gemm_t<z64>(s, 0, n, t, t, zc(1.0), U, m, 0, Ys, t, 0, zc(0.0), X, m, 0, 1);
    gemm_t<z64>(s, 0, n, t, t, zc(1.0), AU, m, 0, Ys, t, 0, zc(0.0), AX, m, 0, 1);
    gemm_t<z64>(s, 0, n, t, t, zc(1.0), BU, m, 0, Ys, t, 0, zc(0.0), BX, m, 0, 1);
    double *dnorm = p->nrm.as<double>();
    std::vector<double> hn(3 * t);
    feast::ritz_norms(s, AX, BX, m, n, t, dlam, p->part.as<double>(), dnorm);
    HIPCHK(hipMemcpyAsync(hn.data(), dnorm, sizeof(double) * 3 * t, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rho = p->c.radius;
    std::vector<int32_t> sel;
    for (int64_t i = 0; i < t; ++i) {
      if (!std::isfinite(lam[i].real()) || !std::isfinite(lam[i].imag())) continue;
      const double den = std::sqrt(hn[3 * i + 1]) + std::sqrt(hn[3 * i + 2]);
      const double r = den > 0.0 ? std::sqrt(hn[3 * i]) / den : INFINITY;
      if (std::abs(lam[i] - gamma) < rho && r < p->o.eta) {
        hLambda[sel.size()] = hlam[i];
        if (hRes) hRes[sel.size()] = r;
        sel.push_back(static_cast<int32_t>(i));
      }
    }
    const int32_t c = static_cast<int32_t>(sel.size());
    if (c > 0) {
      HIPCHK(hipMemcpyAsync(didx, sel.data(), sizeof(int32_t) * c, hipMemcpyHostToDevice, s));
      feast::gather_normalize_cols(s, X, m, n, didx, c, reinterpret_cast<z64 *>(dX), ldx, nullptr);
    }
    HIPCHK(hipStreamSynchronize(s));
    *s_found = c;
    if (info) {
      info->t = t;
      info->ms = total.ms();
    }
    return FEAST_OK;
  });
}

int feast_enclosing_circle(int32_t nv, const feast_z *vertices, double margin, feast_z *center,
                           double *radius) {
  if (nv < 1 || !vertices || !center || !radius || !(margin >= 0.0)) return FEAST_EINVAL;
  for (int32_t i = 0; i < nv; ++i)
    if (!std::isfinite(vertices[i].re) || !std::isfinite(vertices[i].im)) return FEAST_EINVAL;
  cd c;
  double r;
  feast_host::enclosing_circle(nv, reinterpret_cast<const cd *>(vertices), &c, &r);
  *center = {c.real(), c.imag()};
  *radius = r * (1.0 + margin);
  return FEAST_OK;
}

int feast_region_select(int32_t nv, const feast_z *vertices, int64_t k, const feast_z *lambda,
                        int32_t *inside) {
  if (nv < 3 || !vertices || k < 0 || (k > 0 && (!lambda || !inside))) return FEAST_EINVAL;
  const cd *v = reinterpret_cast<const cd *>(vertices);
  for (int64_t i = 0; i < k; ++i)
    inside[i] = feast_host::inside_polygon(cd(lambda[i].re, lambda[i].im), nv, v) ? 1 : 0;
  return FEAST_OK;
}

int feast_solve(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB, int64_t ldb,
                const feast_z *dV, int64_t ldv, feast_z *hLambda, feast_z *dX, int64_t ldx,
                double *hRes, int32_t *s_found, double *err, int32_t *flag, feast_info *info) {
  return solve_impl(p, dA, lda, dB, ldb, dV, ldv, false, hLambda, dX, ldx, hRes, s_found, err,
                    flag, info);
}

// Sparse pencils: the symbolic steps on the host (pattern copies and checks,
// union pattern, ordering -- reverse Cuthill-McKee or the natural order,
// whichever is narrower -- and band widths), then on the
// device the values gathered onto the reordered pattern and the band LU of
// every node.
constexpr int kBandMax = 63;  // kl + ku: LDS windows of the band kernels

int prepare_sparse(feast_plan *p, const feast_csr *A, const feast_csr *B) {
  const int64_t n = p->n;
  hipStream_t s = p->s;
  feast_host::Pattern PA, PB;
  for (int w = 0; w < 2; ++w) {
    const feast_csr *M = w ? B : A;
    feast_host::Pattern &P = w ? PB : PA;
    P.n = n;
    P.rp.resize(static_cast<size_t>(n) + 1);
    P.ci.resize(static_cast<size_t>(M->nnz));
    HIPCHK(hipMemcpyAsync(P.rp.data(), M->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
    if (M->nnz > 0)
      HIPCHK(hipMemcpyAsync(P.ci.data(), M->col, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const std::string bad = feast_host::check_pattern(n, P.rp.data(), P.ci.data(), M->nnz);
    if (!bad.empty()) return fail(p, FEAST_EINVAL, std::string(w ? "B: " : "A: ") + bad);
  }
  auto &sp = p->sp;
  // the symbolic work (ordering, union pattern, its upload) depends on the
  // patterns only: reused while A's and B's are those of the last ordering
  const bool same = sp.ordered && PA.rp == sp.keyA_rp && PA.ci == sp.keyA_ci &&
                    PB.rp == sp.keyB_rp && PB.ci == sp.keyB_ci;
  if (!same) {
    sp.ordered = false;
    std::vector<int32_t> ident(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) ident[i] = static_cast<int32_t>(i);
    const feast_host::UnionPattern U0 = feast_host::union_reordered(PA, PB, ident);
    int64_t kl = 0, ku = 0;
    const std::vector<int32_t> perm = feast_host::band_order(U0.P, &kl, &ku);
    if (kl + ku > kBandMax) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "band too wide after reordering: kl = %lld, ku = %lld (kl + ku <= %d); factor "
                    "this pencil densely (feast_solve)",
                    static_cast<long long>(kl), static_cast<long long>(ku), kBandMax);
      return fail(p, FEAST_EINVAL, buf);
    }
    const feast_host::UnionPattern U = feast_host::union_reordered(PA, PB, perm);
    const int64_t nnz = static_cast<int64_t>(U.P.ci.size());
    sp.kl = static_cast<int>(kl);
    sp.ku = static_cast<int>(ku);
    sp.nnz = nnz;
    sp.rp.alloc(sizeof(int32_t) * (n + 1));
    sp.ci.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    sp.map.alloc(sizeof(int32_t) * 2 * std::max<int64_t>(nnz, 1));
    sp.perm.alloc(sizeof(int32_t) * n);
    HIPCHK(hipMemcpyAsync(sp.rp.p, U.P.rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(sp.perm.p, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    if (nnz > 0) {
      int32_t *dmap = sp.map.as<int32_t>();
      HIPCHK(hipMemcpyAsync(sp.ci.p, U.P.ci.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(dmap, U.mapA.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(dmap + nnz, U.mapB.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));  // the host arrays above are freed on return
    sp.keyA_rp = std::move(PA.rp);
    sp.keyA_ci = std::move(PA.ci);
    sp.keyB_rp = std::move(PB.rp);
    sp.keyB_ci = std::move(PB.ci);
    sp.ordered = true;
  }
  const int64_t nnz = sp.nnz, kl = sp.kl, ku = sp.ku;
  sp.va.alloc(sizeof(z64) * std::max<int64_t>(nnz, 1));
  sp.vb.alloc(sizeof(z64) * std::max<int64_t>(nnz, 1));
  if (nnz > 0) {
    const int32_t *dmap = sp.map.as<int32_t>();
    feast::gather_vals(s, dmap, reinterpret_cast<const z64 *>(A->val), nnz, sp.va.as<z64>());
    feast::gather_vals(s, dmap + nnz, reinterpret_cast<const z64 *>(B->val), nnz, sp.vb.as<z64>());
  }
  const int N = p->N;
  const int64_t WC = kl + ku + 1;
  sp.Lf.alloc(sizeof(z64) * N * n * std::max<int64_t>(kl, 1));
  sp.Uf.alloc(sizeof(z64) * N * n * WC);
  sp.Dinv.alloc(sizeof(z64) * N * n);
  sp.piv.alloc(sizeof(int32_t) * N * n);
  sp.info.alloc(sizeof(int32_t) * N);
  sp.V.alloc(sizeof(z64) * n * p->m);
  sp.X.alloc(sizeof(z64) * n * p->m);
  feast::band_lu(s, sp.rp.as<int32_t>(), sp.ci.as<int32_t>(), sp.va.as<z64>(), sp.vb.as<z64>(),
                 p->dz.as<z64>(), N, n, sp.kl, sp.ku, sp.Lf.as<z64>(), sp.Uf.as<z64>(),
                 sp.Dinv.as<z64>(), sp.piv.as<int32_t>(), sp.info.as<int32_t>());
  std::vector<int32_t> hinfo(N);
  HIPCHK(hipMemcpyAsync(hinfo.data(), sp.info.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  for (int j = 0; j < N; ++j)
    if (hinfo[j] != 0) {
      char buf[200];
      std::snprintf(buf, sizeof buf, "exact zero pivot in the band LU at node %d (z = %.17g%+.17gi), column %d",
                    j, p->hz[j].real(), p->hz[j].imag(), hinfo[j] - 1);
      p->err = buf;
      return FEAST_SINGULAR;
    }
  return FEAST_OK;
}

int feast_solve_csr(feast_plan *p, const feast_csr *A, const feast_csr *B, const feast_z *dV,
                    int64_t ldv, feast_z *hLambda, feast_z *dX, int64_t ldx, double *hRes,
                    int32_t *s_found, double *err, int32_t *flag, feast_info *info) {
  if (!p) return FEAST_EINVAL;
  if (!A || !B || !dV || !hLambda || !dX || !s_found || !err || !flag || ldv < p->m || ldx < p->m)
    return fail(p, FEAST_EINVAL, "feast_solve_csr: null pointer or leading dimension too small");
  if (A->n != p->n || B->n != p->n || A->nnz < 0 || B->nnz < 0 || !A->rowptr || !B->rowptr ||
      (A->nnz > 0 && (!A->col || !A->val)) || (B->nnz > 0 && (!B->col || !B->val)) ||
      A->nnz > INT32_MAX || B->nnz > INT32_MAX)
    return fail(p, FEAST_EINVAL, "feast_solve_csr: matrices must be n x n CSR with device arrays");
  if (p->mixed())
    return fail(p, FEAST_EINVAL, "feast_solve_csr: sparse pencils are factored in FP64 only");
  p->err.clear();
  return guarded(p, [&]() -> int {
    const int64_t n = p->n, m = p->m;
    Timer tf;
    int st = prepare_sparse(p, A, B);
    const double t_fac = tf.ms();
    if (st != FEAST_OK) return st;
    struct Off {
      feast_plan *p;
      ~Off() { p->sp.on = false; }
    } off{p};
    p->sp.on = true;
    const int32_t *perm = p->sp.perm.as<int32_t>();
    feast::gather_rows<z64>(p->s, reinterpret_cast<const z64 *>(dV), ldv, 0, perm, n, m, 1,
                            p->sp.V.as<z64>(), m, 0);
    feast_info inf{};
    st = solve_impl(p, nullptr, n, nullptr, n, reinterpret_cast<const feast_z *>(p->sp.V.p), m,
                    false, hLambda, reinterpret_cast<feast_z *>(p->sp.X.p), m, hRes, s_found, err,
                    flag, &inf);
    if (st == FEAST_OK || st == FEAST_REFINE_STAGNATED) {
      if (*s_found > 0)  // eigenvectors back to the caller's row order
        feast::scatter_rows<z64>(p->s, p->sp.X.as<z64>(), m, 0, perm, n, *s_found, 1,
                                 reinterpret_cast<z64 *>(dX), ldx, 0);
      HIPCHK(hipStreamSynchronize(p->s));
    }
    inf.t_factor_ms += t_fac;
    inf.t_total_ms += t_fac;
    inf.band_kl = p->sp.kl;
    inf.band_ku = p->sp.ku;
    if (info) *info = inf;
    return st;
  });
}

int feast_csr_order(int64_t n, const int32_t *hrowptr, const int32_t *hcol, int32_t *hperm,
                    int64_t *kl, int64_t *ku) {
  if (n <= 0 || !hrowptr || (hrowptr[n] > 0 && !hcol) || !hperm || !kl || !ku) return FEAST_EINVAL;
  if (!feast_host::check_pattern(n, hrowptr, hcol, hrowptr[n]).empty()) return FEAST_EINVAL;
  feast_host::Pattern P;
  P.n = n;
  P.rp.assign(hrowptr, hrowptr + n + 1);
  P.ci.assign(hcol, hcol + hrowptr[n]);
  const std::vector<int32_t> perm = feast_host::band_order(P, kl, ku);
  std::copy(perm.begin(), perm.end(), hperm);
  return FEAST_OK;
}

int feast_solve_from(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB,
                     int64_t ldb, const feast_z *dU1, int64_t ldu, feast_z *hLambda, feast_z *dX,
                     int64_t ldx, double *hRes, int32_t *s_found, double *err, int32_t *flag,
                     feast_info *info) {
  return solve_impl(p, dA, lda, dB, ldb, dU1, ldu, true, hLambda, dX, ldx, hRes, s_found, err,
                    flag, info);
}

int feast_plan_set_m(feast_plan *p, int64_t m) {
  if (!p) return FEAST_EINVAL;
  if (m < 1 || m > p->n) return fail(p, FEAST_EINVAL, "feast_plan_set_m: m must be in [1, n]");
  p->err.clear();
  return guarded(p, [&]() -> int {
    p->m = m;
    ensure_workspace(p);
    return FEAST_OK;
  });
}

// Algorithm 4 (Search).  The filtered blocks, the trace and the Gram matrices
// are GPU products; the rank-revealing step is the pivoted Cholesky of the
// s_dagger x s_dagger Gram matrix on the host (the pivots and |R_ii| of the
// column-pivoted QR of the block); the basis U_1 of the t leading pivot
// columns is orthonormalised on the GPU (shifted Cholesky QR3).
int feast_search(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB, int64_t ldb,
                 const feast_z *dY, int64_t ldy, int64_t ycols, int32_t p0, double alpha,
                 double tau, feast_z *dU1, int64_t ldu, feast_search_info *info) {
  if (!p) return FEAST_EINVAL;
  if (!dA || !dB || !dY || !dU1 || !info || lda < p->n || ldb < p->n || ycols < 1 ||
      ldy < ycols || ldu < p->m)
    return fail(p, FEAST_EINVAL, "feast_search: null pointer or leading dimension too small");
  if (p0 < 1 || p0 > p->m || p0 > ycols || !(alpha > 1.0) || !(tau > 0.0 && tau < 1.0))
    return fail(p, FEAST_EINVAL, "feast_search: need 1 <= p <= min(m, pool columns), alpha > 1, 0 < tau < 1");
  p->err.clear();
  CheckScope check_scope(p);
  return guarded(p, [&]() -> int {
    Timer total;
    const int64_t n = p->n, m = p->m, cap = std::min(n, m);
    hipStream_t s = p->s;
    const z64 *A = reinterpret_cast<const z64 *>(dA), *B = reinterpret_cast<const z64 *>(dB);
    const z64 *Y = reinterpret_cast<const z64 *>(dY);
    int st = ensure_factored(p, A, lda, B, ldb);
    if (st == FEAST_SINGULAR) return st;
    z64 *U = p->wblk(feast_plan::W_X);    // block under test, n x s_dagger (leading dim m)
    z64 *Wg = p->wblk(feast_plan::W_AX);  // leading pivot columns, then U_1
    z64 *R = p->R.as<z64>();              // right-hand sides B Y (leading dim m)
    z64 *G = p->gblk(feast_plan::G_GRAM);
    int32_t *didx = reinterpret_cast<int32_t *>(p->small.as<z64>());
    feast_search_info out{};
    // (Search's filters are not refined in the mixed form: its rank test needs
    // single-precision accuracy only)
    auto filt = [&](int64_t col0, int64_t c, z64 *dst) -> int {
      gemm_t<z64>(s, 0, n, c, n, zc(1.0), B, ldb, 0, Y + col0, ldy, 0, zc(0.0), R, m, 0, 1);
      const int r = filter_rhs(p, A, lda, B, ldb, R, m, dst, m, 0.0, 0, c);
      out.filters += 1;
      return r;
    };
    auto gram = [&](const z64 *X, int64_t k, int64_t ldx2, const z64 *Z, int64_t ldz,
                    std::vector<feast_z> &h) {
      gemm_t<z64>(s, 2, k, k, n, zc(1.0), X, ldx2, 0, Z, ldz, 0, zc(0.0), G, k, 0, 1,
                  p->splitws.as<z64>(), splitws_elems(p));
      h.resize(static_cast<size_t>(k * k));
      HIPCHK(hipMemcpyAsync(h.data(), G, sizeof(z64) * k * k, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    };
    // first filtered sample
    int64_t pc = p0, used = p0;
    st = filt(0, pc, U);
    if (st != FEAST_OK) return st;
    // trace estimate: s_0 = ceil(Re trace(Y_0^* U) / p)
    std::vector<feast_z> hg;
    gram(Y, pc, ldy, U, m, hg);
    double tr = 0.0;
    for (int64_t i = 0; i < pc; ++i) tr += hg[i * pc + i].re;
    out.s0 = static_cast<int64_t>(std::ceil(tr / static_cast<double>(pc)));
    int64_t sd = std::min(std::max<int64_t>(pc, out.s0), cap);
    std::vector<int32_t> piv;
    std::vector<double> rd;
    for (;;) {
      // widen the block with s_dagger - p newly filtered columns
      if (sd > pc) {
        const int64_t c = sd - pc;
        if (used + c > ycols)
          return fail(p, FEAST_EINVAL, "feast_search: random column pool exhausted");
        st = filt(used, c, U + pc);
        if (st != FEAST_OK) return st;
        used += c;
      } else {
        sd = pc;
      }
      // rank-revealing step
      gram(U, sd, m, U, m, hg);
      piv.assign(static_cast<size_t>(sd), 0);
      rd.assign(static_cast<size_t>(sd), 0.0);
      const int64_t t = feast_host::pivoted_cholesky_rank(
          sd, reinterpret_cast<const cd *>(hg.data()), sd, tau, piv.data(), rd.data());
      out.rounds += 1;
      if (t < 1) return fail(p, FEAST_ENUMERIC, "feast_search: the filtered block is zero");
      HIPCHK(hipMemcpyAsync(didx, piv.data(), sizeof(int32_t) * t, hipMemcpyHostToDevice, s));
      feast::gather_normalize_cols(s, U, m, n, didx, t, Wg, m, p->part.as<double>());
      feast::fill_i32(s, p->flag.as<int32_t>(), 3, 0);
      orth(p, Wg, m, 0, t);
      int32_t hf[3];
      HIPCHK(hipMemcpyAsync(hf, p->flag.p, sizeof hf, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hf[0] || hf[1] || hf[2])
        return fail(p, FEAST_ENUMERIC, "feast_search: Cholesky QR of the pivot columns broke down");
      // rank test
      if (t < sd) {
        feast::copy_block_z(s, Wg, m, n, t, reinterpret_cast<z64 *>(dU1), ldu);
        out.t = t;
        break;
      }
      const int64_t nxt = std::min<int64_t>(static_cast<int64_t>(std::ceil(alpha * t)), cap);
      if (nxt <= t) {
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "feast_search: the block is still of full rank at %lld columns (the plan's "
                      "subspace size m); use a larger m",
                      static_cast<long long>(t));
        return fail(p, FEAST_EINVAL, buf);
      }
      feast::copy_block_z(s, Wg, m, n, t, U, m);
      pc = t;
      sd = nxt;
    }
    HIPCHK(hipStreamSynchronize(s));
    out.used = used;
    out.ms = total.ms();
    *info = out;
    return FEAST_OK;
  });
}

// ---------------------------------------------------------------------------
// Adjoint form: left eigenvectors on the cached factors and eigenvalue gradients
// ---------------------------------------------------------------------------

int feast_left_eigvecs(feast_plan *p, const feast_z *dA, int64_t lda, const feast_z *dB,
                       int64_t ldb, const feast_z *dX, int64_t ldx, int64_t scnt, int32_t sweeps,
                       feast_z *dY, int64_t ldy) {
  if (!p) return FEAST_EINVAL;
  if (!dA || !dB || !dX || !dY || scnt < 1 || scnt > p->m || sweeps < 1 || sweeps > 16 ||
      lda < p->n || ldb < p->n || ldx < scnt || ldy < scnt)
    return fail(p, FEAST_EINVAL, "feast_left_eigvecs: bad argument");
  if (p->mixed())
    return fail(p, FEAST_EINVAL, "feast_left_eigvecs needs an FP64 plan");
  p->err.clear();
  CheckScope check_scope(p);
  return guarded(p, [&]() -> int {
    const int64_t n = p->n, sc = scnt;
    const int N = p->N;
    hipStream_t s = p->s;
    const z64 *A = reinterpret_cast<const z64 *>(dA), *B = reinterpret_cast<const z64 *>(dB);
    const z64 *X = reinterpret_cast<const z64 *>(dX);
    const int st = ensure_factored(p, A, lda, B, ldb);
    if (st != FEAST_OK) return st;
    const int64_t ldw = static_cast<int64_t>(N) * sc;
    p->adj.alloc(sizeof(z64) * n * ldw);
    z64 *Y = p->Y.as<z64>(), *Adj = p->adj.as<z64>();
    z64 *G = p->wblk(feast_plan::W_X), *W = p->wblk(feast_plan::W_AX), *BX = p->wblk(feast_plan::W_BX);
    gemm_t<z64>(s, 0, n, sc, n, zc(1.0), B, ldb, 0, X, ldx, 0, zc(0.0), BX, sc, 0, 1);
    for (int k = 0; k < sweeps; ++k) {
      // G = B^* W (W_0 = X): the adjoint filter acts on B^* y_k as conj(f(lambda_k)) y_k
      gemm_t<z64>(s, 2, n, sc, n, zc(1.0), B, ldb, 0, k == 0 ? X : W, k == 0 ? ldx : sc, 0,
                  zc(0.0), G, sc, 0, 1);
      // W = sum_j conj(w_j) (z_j B - A)^{-*} G with the cached factors:
      // (z_j B - A)^* = U^* L^* P, so solve with U^*, then L^*, then undo P
      feast::bcast_cols(s, G, sc, n, sc, N, Y, ldw);
      plan_trsolve<z64>(p, s, Y, sc, ldw, sc, 2);
      feast::scatter_rows<z64>(s, Y, ldw, sc, p->perm.as<int32_t>(), n, sc, N, Adj, ldw, sc);
      feast::weighted_sum(s, Adj, ldw, sc, p->dwc.as<z64>(), N, n, sc, W, sc);
    }
    // Y = W (W^* B X)^{-*}, so that Y^* B X = I
    z64 *S = p->gblk(feast_plan::G_AT), *T = p->gblk(feast_plan::G_BT), *Z = p->gblk(feast_plan::G_YS);
    gemm_t<z64>(s, 2, sc, sc, n, zc(1.0), W, sc, 0, BX, sc, 0, zc(0.0), S, sc, 0, 1,
                p->splitws.as<z64>(), splitws_elems(p));
    feast::conj_transpose(s, S, sc, sc, sc, T, sc);
    const int64_t nb64 = (sc + 63) / 64;
    p->adj_piv.alloc(sizeof(int32_t) * sc * 2);
    p->adj_info.alloc(sizeof(int32_t) * 4);
    p->adj_inv.alloc(sizeof(z64) * 2 * nb64 * 64 * 64);
    int32_t *piv = p->adj_piv.as<int32_t>(), *perm = piv + sc;
    z64 *Li = p->adj_inv.as<z64>(), *Ui = Li + nb64 * 64 * 64;
    lu_batched<z64>(LuStreams{s, nullptr, nullptr, nullptr}, T, sc, 0, 1, sc, 128, piv,
                    p->adj_info.as<int32_t>(), Li, Ui, nb64 * 64 * 64);
    feast::perm_from_ipiv(s, piv, perm, sc, 1);
    feast::identity(s, S, sc);
    feast::gather_rows<z64>(s, S, sc, 0, perm, sc, sc, 1, Z, sc, 0);
    trsolve<z64>(s, T, sc, 0, 1, sc, Li, Ui, nb64 * 64 * 64, Z, sc, sc, 0, 0);
    gemm_t<z64>(s, 0, n, sc, sc, zc(1.0), W, sc, 0, Z, sc, 0, zc(0.0), reinterpret_cast<z64 *>(dY),
                ldy, 0, 1);
    int32_t hinfo = 0;
    HIPCHK(hipMemcpyAsync(&hinfo, p->adj_info.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    if (hinfo != 0) return fail(p, FEAST_ENUMERIC, "W^* B X is singular: left basis lost rank");
    return FEAST_OK;
  });
}

int feast_eig_grad(feast_plan *p, const feast_z *dX, int64_t ldx, const feast_z *dY, int64_t ldy,
                   int64_t scnt, const feast_z *hLam, const feast_z *hG, feast_z *dGA, int64_t ldga,
                   feast_z *dGB, int64_t ldgb) {
  if (!p) return FEAST_EINVAL;
  if (!dX || !dY || !hLam || !hG || !dGA || !dGB || scnt < 0 || scnt > p->m || ldx < scnt ||
      ldy < scnt || ldga < p->n || ldgb < p->n)
    return fail(p, FEAST_EINVAL, "feast_eig_grad: bad argument");
  p->err.clear();
  return guarded(p, [&]() -> int {
    const int64_t n = p->n, sc = scnt;
    hipStream_t s = p->s;
    if (sc == 0) {
      gemm_t<z64>(s, 0, n, n, 0, zc(0.0), nullptr, 1, 0, nullptr, n, 0, zc(0.0),
                  reinterpret_cast<z64 *>(dGA), ldga, 0, 1);
      gemm_t<z64>(s, 0, n, n, 0, zc(0.0), nullptr, 1, 0, nullptr, n, 0, zc(0.0),
                  reinterpret_cast<z64 *>(dGB), ldgb, 0, 1);
      HIPCHK(hipStreamSynchronize(s));
      return FEAST_OK;
    }
    std::vector<z64> d(2 * sc);
    for (int64_t i = 0; i < sc; ++i) {
      const cd g(hG[i].re, hG[i].im), l(hLam[i].re, hLam[i].im);
      const cd gb = -g * std::conj(l);
      d[i] = zc(g.real(), g.imag());
      d[sc + i] = zc(gb.real(), gb.imag());
    }
    z64 *dd = p->small.as<z64>();
    z64 *XH = p->wblk(feast_plan::W_X), *Yg = p->wblk(feast_plan::W_AX), *Yb = p->wblk(feast_plan::W_BX);
    HIPCHK(hipMemcpyAsync(dd, d.data(), sizeof(z64) * 2 * sc, hipMemcpyHostToDevice, s));
    feast::conj_transpose(s, reinterpret_cast<const z64 *>(dX), ldx, n, sc, XH, n);
    feast::copy_block_z(s, reinterpret_cast<const z64 *>(dY), ldy, n, sc, Yg, sc);
    feast::copy_block_z(s, reinterpret_cast<const z64 *>(dY), ldy, n, sc, Yb, sc);
    feast::scale_cols(s, Yg, sc, n, sc, dd);
    feast::scale_cols(s, Yb, sc, n, sc, dd + sc);
    gemm_t<z64>(s, 0, n, n, sc, zc(1.0), Yg, sc, 0, XH, n, 0, zc(0.0), reinterpret_cast<z64 *>(dGA),
                ldga, 0, 1);
    gemm_t<z64>(s, 0, n, n, sc, zc(1.0), Yb, sc, 0, XH, n, 0, zc(0.0), reinterpret_cast<z64 *>(dGB),
                ldgb, 0, 1);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    return FEAST_OK;
  });
}

// ---------------------------------------------------------------------------
// Kernel-level entry points
// ---------------------------------------------------------------------------

int feast_zgemm_batched(int32_t transA, int64_t M, int64_t N, int64_t K, feast_z alpha,
                        const feast_z *dA, int64_t lda, int64_t strideA, const feast_z *dB,
                        int64_t ldb, int64_t strideB, feast_z beta, feast_z *dC, int64_t ldc,
                        int64_t strideC, int32_t batch, void *stream) {
  if ((transA != 0 && transA != 2) || M < 0 || N < 0 || K < 0 || batch < 0) return FEAST_EINVAL;
  if (M == 0 || N == 0 || batch == 0) return FEAST_OK;
  if (!dA || !dB || !dC || ldc < N || ldb < N || lda < (transA == 0 ? K : M)) return FEAST_EINVAL;
  return guarded(nullptr, [&]() {
    gemm_t<z64>(static_cast<hipStream_t>(stream), transA, M, N, K, zc(alpha.re, alpha.im),
                reinterpret_cast<const z64 *>(dA), lda, strideA, reinterpret_cast<const z64 *>(dB),
                ldb, strideB, zc(beta.re, beta.im), reinterpret_cast<z64 *>(dC), ldc, strideC, batch);
    HIPCHK(hipGetLastError());
    return FEAST_OK;
  });
}

int feast_zgetrf_batched(int64_t n, int32_t batch, feast_z *dM, int64_t ldm, int64_t strideM,
                         int32_t *dPiv, int32_t *dInfo, int32_t nb, void *stream) {
  if (n < 1 || n > 16384 || batch < 1 || !dM || !dPiv || !dInfo || ldm < n ||
      (nb != 0 && nb != 64 && nb != 128))
    return FEAST_EINVAL;
  const int b = nb ? nb : 128;
  return guarded(nullptr, [&]() {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nblk = (n + 63) / 64;
    DevBuf Li, Ui;
    Li.alloc(sizeof(z64) * batch * nblk * 64 * 64);
    Ui.alloc(sizeof(z64) * batch * nblk * 64 * 64);
    lu_batched<z64>(LuStreams{s, nullptr, nullptr, nullptr}, reinterpret_cast<z64 *>(dM), ldm,
                    strideM, batch, n, b, dPiv, dInfo, Li.as<z64>(), Ui.as<z64>(),
                    nblk * 64 * 64);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    Li.release();
    Ui.release();
    return FEAST_OK;
  });
}

}  // extern "C"

namespace {

// Scratch of the multi-right-hand-side solves with given factors: inverted
// 64 x 64 diagonal blocks of L and U, the row permutation and a staging block.
struct GetrsScratch {
  z64 *Li, *Ui, *T;
  int32_t *perm;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of GetrsScratch for (n, nrhs, batch), each piece 256-byte aligned.
size_t getrs_scratch_bytes(int64_t n, int64_t nrhs, int32_t batch) {
  const int64_t ist = ((n + 63) / 64) * 64 * 64;
  return 2 * align256(sizeof(z64) * batch * ist) + align256(sizeof(int32_t) * batch * n) +
         align256(sizeof(z64) * batch * n * nrhs);
}

GetrsScratch carve_getrs(void *base, int64_t n, int64_t nrhs, int32_t batch) {
  const int64_t ist = ((n + 63) / 64) * 64 * 64;
  char *q = static_cast<char *>(base);
  GetrsScratch w;
  w.Li = reinterpret_cast<z64 *>(q);
  q += align256(sizeof(z64) * batch * ist);
  w.Ui = reinterpret_cast<z64 *>(q);
  q += align256(sizeof(z64) * batch * ist);
  w.perm = reinterpret_cast<int32_t *>(q);
  q += align256(sizeof(int32_t) * batch * n);
  w.T = reinterpret_cast<z64 *>(q);
  return w;
}

// The solves of feast_zgetrs_batched, enqueued on s with the scratch w.
void zgetrs_enqueue(hipStream_t s, int64_t n, int64_t nrhs, int32_t batch, const z64 *F, int64_t ldm,
                    int64_t strideM, const int32_t *dPiv, z64 *Xz, int64_t ldx, int64_t strideX,
                    int32_t trans, const GetrsScratch &w) {
  const int64_t nblk = (n + 63) / 64, ist = nblk * 64 * 64;
  feast::diag_block_inverse<z64>(s, F, ldm, strideM, batch, n, 64, 0, nblk, true, w.Li, ist);
  feast::diag_block_inverse<z64>(s, F, ldm, strideM, batch, n, 64, 0, nblk, false, w.Ui, ist);
  feast::perm_from_ipiv(s, dPiv, w.perm, n, batch);
  if (trans == 0) {
    feast::gather_rows<z64>(s, Xz, ldx, strideX, w.perm, n, nrhs, batch, w.T, nrhs, n * nrhs);
    trsolve<z64>(s, F, ldm, strideM, batch, n, w.Li, w.Ui, ist, w.T, nrhs, nrhs, n * nrhs, 0);
    for (int32_t i = 0; i < batch; ++i)
      feast::copy_block_z(s, w.T + i * n * nrhs, nrhs, n, nrhs, Xz + i * strideX, ldx);
  } else {
    for (int32_t i = 0; i < batch; ++i)
      feast::copy_block_z(s, Xz + i * strideX, ldx, n, nrhs, w.T + i * n * nrhs, nrhs);
    trsolve<z64>(s, F, ldm, strideM, batch, n, w.Li, w.Ui, ist, w.T, nrhs, nrhs, n * nrhs, 2);
    feast::scatter_rows<z64>(s, w.T, nrhs, n * nrhs, w.perm, n, nrhs, batch, Xz, ldx, strideX);
  }
}

bool bad_getrs_args(int64_t n, int64_t nrhs, int32_t batch, const feast_z *dLU, int64_t ldm,
                    const int32_t *dPiv, const feast_z *dX, int64_t ldx, int32_t trans) {
  return n < 1 || n > 16384 || nrhs < 0 || batch < 1 || !dLU || !dPiv || !dX || ldm < n ||
         ldx < nrhs || (trans != 0 && trans != 2);
}

// The no-allocation variant's scratch: one file-scope device array, present on
// every GPU the library runs on for the life of the process.  Host code never
// uses its name as an address (on the host it is only a stand-in): the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken once
// per device with that device current and kept in scratch_dev.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};

int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FEAST_EDEVICE;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FEAST_EDEVICE;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return FEAST_OK;
}

}  // namespace

extern "C" {

int feast_zgetrs_batched(int64_t n, int64_t nrhs, int32_t batch, const feast_z *dLU, int64_t ldm,
                         int64_t strideM, const int32_t *dPiv, feast_z *dX, int64_t ldx,
                         int64_t strideX, int32_t trans, void *stream) {
  if (bad_getrs_args(n, nrhs, batch, dLU, ldm, dPiv, dX, ldx, trans)) return FEAST_EINVAL;
  if (nrhs == 0) return FEAST_OK;
  return guarded(nullptr, [&]() {
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf ws;
    ws.alloc(getrs_scratch_bytes(n, nrhs, batch));
    zgetrs_enqueue(s, n, nrhs, batch, reinterpret_cast<const z64 *>(dLU), ldm, strideM, dPiv,
                   reinterpret_cast<z64 *>(dX), ldx, strideX, trans,
                   carve_getrs(ws.p, n, nrhs, batch));
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipGetLastError());
    return FEAST_OK;
  });
}

int feast_zgetrs_batched_noalloc(int64_t n, int64_t nrhs, int32_t batch, const feast_z *dLU,
                                 int64_t ldm, int64_t strideM, const int32_t *dPiv, feast_z *dX,
                                 int64_t ldx, int64_t strideX, int32_t trans, void *stream) {
  if (bad_getrs_args(n, nrhs, batch, dLU, ldm, dPiv, dX, ldx, trans)) return FEAST_EINVAL;
  if (nrhs == 0) return FEAST_OK;
  if (getrs_scratch_bytes(n, nrhs, batch) > kNoAllocScratchBytes) return FEAST_ESCRATCH;
  void *base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != FEAST_OK) return rc;
  return guarded(nullptr, [&]() {
    zgetrs_enqueue(static_cast<hipStream_t>(stream), n, nrhs, batch,
                   reinterpret_cast<const z64 *>(dLU), ldm, strideM, dPiv,
                   reinterpret_cast<z64 *>(dX), ldx, strideX, trans,
                   carve_getrs(base, n, nrhs, batch));
    HIPCHK(hipGetLastError());
    return FEAST_OK;
  });
}

}  // extern "C"
