// Batched form: the filter and Algorithm 5 over many independent pencils of
// uneven order, with all shifted systems of all pencils factored and solved
// in lockstep.
//
// Layout.  Pencil p (internal order: decreasing padded order) of order n_p is
// padded to np_p = 64 ceil(n_p / 64) with an identity block: its N shifted
// matrices are np_p x np_p row-major blocks, the real part z B - A in the
// leading n_p x n_p corner, ones on the rest of the diagonal and zeros
// elsewhere.  Partial pivoting never moves a padding row into the leading
// block (those rows are zero in its columns), the padding stays the identity
// under the factorisation, and solutions keep zeros in the padding rows, so a
// padded pencil factors and solves exactly like the original.  With every
// order a multiple of the 64-wide panel, the pencils still active at panel
// step k0 are the prefix np_p > k0, and each step is one grouped launch per
// kernel over that prefix (GrpMat descriptors for the panel kernels, tables
// of GEMM problems for the MFMA products).  Matrix b = p N + j of the flat
// per-matrix arrays (pivots, permutations, info, inverted diagonal blocks) is
// node j of pencil p.
//
// Node solutions of pencil p: an np_p x (N m_p) block, node j in columns
// [j m_p, (j+1) m_p), as in the single-pencil plan.  The small per-pencil
// steps (orthonormalisation, projection, reduced eigenproblem, residuals) run
// on a member plan per pencil that owns only n x m and m x m workspaces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "batch_tune.h"
#include "host_eig.h"
#include "plan.h"

using namespace feast_drv;
using feast::GemmArgs;
using feast::GrpMat;

namespace {

constexpr int64_t kPanel = 64;

// Device tables of the grouped GEMM launches.  The launch schedule of a batch
// depends only on the orders: it is run once in record mode (tables are
// collected on the host and nothing is launched), the tables are uploaded,
// and every later run takes them from device memory in the same order.
struct Tables {
  bool record = true;
  std::vector<char> host;
  std::vector<size_t> off, cnt;
  size_t cur = 0;
  DevBuf dev;
  ~Tables() { dev.release(); }
  void begin() { cur = 0; }
  template <class E> const E *put(const std::vector<E> &v) {
    if (record) {
      const size_t o = (host.size() + 255) / 256 * 256;
      host.resize(o + sizeof(E) * v.size());
      std::memcpy(host.data() + o, v.data(), sizeof(E) * v.size());
      off.push_back(o);
      cnt.push_back(v.size());
      return nullptr;
    }
    if (cur >= off.size() || cnt[cur] != v.size())
      throw HipError{hipErrorInvalidValue, "grouped launch schedule changed"};
    return reinterpret_cast<const E *>(static_cast<const char *>(dev.p) + off[cur++]);
  }
  void upload() {
    dev.alloc(std::max<size_t>(host.size(), 256));
    if (!host.empty()) HIPCHK(hipMemcpy(dev.p, host.data(), host.size(), hipMemcpyHostToDevice));
    record = false;
  }
  // back to record mode (the device buffer is kept)
  void reset() {
    record = true;
    host.clear();
    off.clear();
    cnt.clear();
    cur = 0;
  }
};

// A captured HIP graph, re-captured when its key (the caller's pointers and
// leading dimensions, the sweep count) changes.
struct Graph {
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> key;
  Graph() = default;
  Graph(const Graph &) = delete;
  Graph &operator=(const Graph &) = delete;
  ~Graph() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key.clear();
  }
};

}  // namespace

constexpr int64_t kMaxSplits = 4;

struct feast_batch {
  int P = 0, N = 0;
  feast_opts o{};
  hipStream_t s = nullptr;   // caller's stream
  hipStream_t gs = nullptr;  // the batch's own stream (graphs are captured and replayed here)
  hipStream_t as = nullptr;  // Ritz vectors and residuals while a filter runs on gs
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_proj = nullptr;
  std::vector<int> order;     // internal index -> caller index
  std::vector<int> where;     // caller index -> internal index
  std::vector<int64_t> n, m, np;
  std::vector<feast_plan *> sub;  // member plans (internal order)
  int64_t nmax = 0, nblk = 0;
  // grouped factors
  DevBuf F, piv, perm, info, Linv, Uinv, grp;
  int64_t lu_nb = 128;  // panel width of the grouped LU (64 or 128)
  int lu_update = feast::GROUP_UPDATE_M3;  // loop of its trailing update (feast::GROUP_*)
  int nbig = 0;  // pencils whose padded order exceeds lu_small_max_order (a prefix)
  std::vector<int64_t> foff;  // element offset of pencil p's first matrix in F
  // node solutions (np_p x N m_p each) and the mixed-form buffers
  DevBuf Y, Yc, T1, T2;
  std::vector<int64_t> yoff, toff;
  Tables lu_tab, sv_tab;
  Tables bv_tab;  // the right-hand sides B V of a call (the caller's pointers: filled per call)
  Tables ritz_tab;  // the Ritz products of an iteration (the pencils still iterating: per call)
  DevBuf dinv, flags;  // grouped orthonormalisation: inverted 64 x 64 blocks, breakdown flags
  // every pencil's At and Bt packed (m_p^2 each, in internal order), on the
  // device and in page-locked host memory: one copy to the host per projection
  DevBuf pk;
  void *pk_host = nullptr;
  DevBuf sk;  // split-K partials of the m x m products (up to kMaxSplits per pencil)
  int64_t mmax = 0;
  Graph g_factor, g_filter;
  // Projection graphs, one per (caller pointers, list of pencils still
  // iterating): the scheduling tables of that list and the captured launches.
  struct ProjGraph {
    Tables tab;
    Graph g;
  };
  std::map<std::vector<int64_t>, std::unique_ptr<ProjGraph>> proj_graphs;
  // cached factors belong to the pencils whose content fingerprints are ffp
  // (A_p, B_p in the caller's order); fptab/fpout: the fingerprint launch
  bool factored = false;
  std::vector<uint64_t> ffp;
  DevBuf fptab, fpout;
  std::string err;
  int launches = 0;

  bool mixed() const { return o.prec == FEAST_MIXED; }
  int64_t istride() const { return nblk * 64 * 64; }
  int64_t ldY(int p) const { return static_cast<int64_t>(N) * m[p]; }
  int64_t mblk() const { return (mmax + 63) / 64; }
  int active(int64_t k) const {  // pencils with np > k (a prefix)
    int a = 0;
    while (a < P && np[a] > k) ++a;
    return a;
  }
};

namespace {

int bfail(feast_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

template <typename F> int bguarded(feast_batch *b, F &&f) {
  try {
    return f();
  } catch (const HipError &e) {
    if (b) {
      b->err = std::string(e.what) + ": " + hipGetErrorString(e.e);
      b->factored = false;
    }
    return e.e == hipErrorOutOfMemory ? FEAST_ENOMEM : FEAST_EDEVICE;
  } catch (const std::bad_alloc &) {
    if (b) b->err = "host allocation failed";
    return FEAST_ENOMEM;
  } catch (...) {
    if (b) b->err = "unexpected exception";
    return FEAST_EDEVICE;
  }
}

// The grouped LU's panel width and trailing-update loop: opts.nb /
// opts.batch_update when given, else the autotuner's entry for this precision
// and the order n* at which the padded orders' share of the LU work
// (sum of np^3, largest first) reaches one half.
void choose_lu_config(feast_batch *b) {
  double total = 0.0, acc = 0.0;
  for (int64_t v : b->np) total += static_cast<double>(v) * v * v;
  int64_t nstar = b->np.empty() ? 0 : b->np[0];
  for (int64_t v : b->np) {  // (np in decreasing order)
    acc += static_cast<double>(v) * v * v;
    nstar = v;
    if (acc >= 0.5 * total) break;
  }
  int nb = 128, upd = feast::GROUP_UPDATE_M3;
  for (const feast_tune::Entry &e : feast_tune::kBatch)
    if (e.prec == b->o.prec && nstar >= e.lo && nstar < e.hi) {
      nb = e.nb;
      upd = e.update;
      break;
    }
  if (b->o.nb != 0) nb = b->o.nb;
  if (b->o.batch_update != 0) upd = b->o.batch_update - 1;
  b->lu_nb = nb;
  b->lu_update = upd;
}

// A member plan: nodes, weights and the n x m / m x m workspaces of one pencil,
// running on the batch stream; it never factors.
feast_plan *member_plan(int64_t n, int64_t m, const feast_contour &c, const feast_opts &o,
                        hipStream_t s) {
  feast_plan *p = new feast_plan();
  p->n = n;
  p->m = m;
  p->N = c.nodes;
  p->c = c;
  p->o = o;
  p->s = s;
  p->nblk = (n + 63) / 64;
  p->hz.resize(p->N);
  p->hw.resize(p->N);
  feast_host::contour_nodes(cd(c.center.re, c.center.im), c.radius, p->N, c.rule, p->hz.data(),
                            p->hw.data());
  p->dz.alloc(sizeof(z64) * p->N);
  p->dw.alloc(sizeof(z64) * p->N);
  HIPCHK(hipMemcpy(p->dz.p, p->hz.data(), sizeof(z64) * p->N, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->dw.p, p->hw.data(), sizeof(z64) * p->N, hipMemcpyHostToDevice));
  ensure_workspace(p, false);
  return p;
}

// Grouped product over a list of problems (skipped when empty).  Without an
// explicit variant, complex128 products C -= A B (triangular solves, panel
// joins) take the three-product loop (fewer MFMAs; its FP64 rounding stays far
// below the tolerances), everything else the plain loop; the trailing update
// passes the autotuned variant.
template <typename T>
void ggemm(feast_batch *b, Tables &tab, int ta, bool sub, std::vector<GemmArgs<T>> &e,
           int variant = -1) {
  if (e.empty()) return;
  if (variant < 0)
    variant = (sub && ta == 0 && sizeof(T) == 16) ? feast::GROUP_UPDATE_M3 : feast::GROUP_PLAIN;
  const int64_t tiles = feast::gemm_group_tiles<T>(e.data(), static_cast<int>(e.size()));
  const GemmArgs<T> *d = tab.put(e);
  if (!tab.record)
    feast::gemm_group<T>(b->gs, ta, sub, d, static_cast<int>(e.size()), tiles, variant);
}

// C = X^* Y with a small output (m x m: Gram matrices, reduced pencils) and a
// long K = n, one problem per pencil: a few output tiles per pencil would leave
// most compute units idle through the K loop, so each problem with K >= 512 is
// cut into up to kMaxSplits K-chunks written to partials (one grouped launch),
// then summed in chunk order (C = alpha X^* Y; beta must be 0).
void ggemm_small_out(feast_batch *b, Tables &tab, std::vector<GemmArgs<z64>> &e) {
  std::vector<GemmArgs<z64>> parts;
  std::vector<GrpMat> dst, src;
  z64 *W = b->sk.as<z64>();
  int64_t off = 0, per_max = 0;
  for (const GemmArgs<z64> &g : e) {
    int64_t S = g.K >= 512 && g.batch == 1 ? std::min<int64_t>(kMaxSplits, g.K / 256) : 1;
    if (S <= 1 || g.beta.x != 0.0 || g.beta.y != 0.0) {
      parts.push_back(g);
      continue;
    }
    const int64_t kc = ((g.K + S - 1) / S + 15) / 16 * 16;
    S = (g.K + kc - 1) / kc;
    const int64_t per = g.M * g.N;
    for (int64_t sp = 0; sp < S; ++sp) {
      GemmArgs<z64> q = g;
      q.K = std::min(kc, g.K - sp * kc);
      q.A = g.A + sp * kc * g.lda;  // op(A) = A^*: K runs over the rows of A
      q.B = g.B + sp * kc * g.ldb;
      q.C = W + off + sp * per;
      q.ldc = g.N;
      parts.push_back(q);
    }
    dst.push_back(GrpMat{g.C, g.ldc, g.N, g.M});
    src.push_back(GrpMat{W + off, g.N, S, g.M});
    off += S * per;
    per_max = std::max(per_max, per);
  }
  if (off * static_cast<int64_t>(sizeof(z64)) > static_cast<int64_t>(b->sk.bytes))
    throw HipError{hipErrorInvalidValue, "split-K workspace"};
  ggemm<z64>(b, tab, 2, false, parts);
  if (dst.empty()) return;
  const GrpMat *gdst = tab.put(dst), *gsrc = tab.put(src);
  if (!tab.record)
    feast::sum_splits_grp(b->gs, gdst, gsrc, static_cast<int>(dst.size()), per_max);
}

template <typename T>
GemmArgs<T> gargs(int64_t M, int64_t Nc, int64_t K, const T *A, int64_t lda, int64_t sA,
                  const T *B, int64_t ldb, int64_t sB, T *C, int64_t ldc, int64_t sC, double alpha,
                  double beta, int32_t batch) {
  return GemmArgs<T>{M, Nc, K, A, lda, sA, B, ldb, sB, C, ldc, sC, make_double2(alpha, 0.0),
                     make_double2(beta, 0.0), batch, 1, K, nullptr, 0};
}

// Panels per trailing update of the grouped LU: four for complex128, two for
// complex64 (64-pencil batch, orders 283-1999: complex128 factorisation 180 ms
// with one panel per update, 173.9 / 172.1 / 171.2 ms with two / three / four;
// complex64 102.5 ms with one, 100.1 / 100.3 / 101.2 with two / three / four).
template <typename T> constexpr int kBatchGroup = sizeof(T) == 16 ? 4 : 2;

// Panel [c0, c0 + w) of the active matrices: halves down to register leaves,
// each split joined by the fused triangular solve + rank update.
template <typename T>
void panel_grp(feast_batch *b, T *F, int nmat, int64_t c0, int w, int64_t pk0, int pkb) {
  const GrpMat *g = b->grp.as<GrpMat>();
  int32_t *piv = b->piv.as<int32_t>(), *info = b->info.as<int32_t>();
  const int ib = feast::leaf_max_width<T>(b->nmax - c0);
  if (w <= ib) {
    if (!feast::leaf_lu<T>(b->gs, F, 0, 0, nmat, b->nmax, c0, w, pk0, pkb, piv, info, g, b->N))
      throw HipError{hipErrorInvalidValue, "leaf_lu"};
    return;
  }
  const int w1 = w / 2, w2 = w - w1;
  panel_grp<T>(b, F, nmat, c0, w1, pk0, pkb);
  feast::panel_update<T>(b->gs, F, 0, 0, nmat, b->nmax, c0, w1, w2, g, b->N);
  panel_grp<T>(b, F, nmat, c0 + w1, w2, pk0, pkb);
}

// Blocked right-looking LU of every shifted matrix of every pencil in lockstep,
// with panels of b->lu_nb = 64 or 128 columns (a 128-column step of a pencil
// padded to an odd multiple of 64 ends with a 64-column panel).  A step:
//   the panel's first 64 columns (register leaves joined by fused rank updates;
//   the leaves swap rows over the whole panel) and the inverse of L's diagonal
//   block; for 128: X = L00^{-1} A(k0:k0+64, k0+64:k0+128) and the update of the
//   panel's second half by L(k0+64:, k0:k0+64) X, then its own leaves;
//   the panel's row swaps outside the panel;
//   U12 = L11^{-1} A12 (for 128: two in-place products with the inverted 64 x 64
//   blocks and the L10 update between them);
//   the trailing update A22 -= L21 U12 as one grouped launch, once per group of
//   kBatchGroup panels (K = the group's width; see the loop below).
// record: only collect the GEMM tables.
template <typename T>
void lu_grouped(feast_batch *b, bool record) {
  Tables &tab = b->lu_tab;
  tab.begin();
  T *F = b->F.as<T>();
  T *Linv = b->Linv.as<T>(), *Uinv = b->Uinv.as<T>();
  const int N = b->N;
  const int64_t is = b->istride();
  const GrpMat *g = b->grp.as<GrpMat>();
  int32_t *piv = b->piv.as<int32_t>();
  const int64_t NB = b->lu_nb;
  // pencils of padded order <= lu_small_max_order (the suffix of the sorted
  // list) are factored whole, one matrix per workgroup of one persistent
  // launch, with the inverses of their L diagonal blocks; the lockstep steps
  // below cover the others
  const int nbig = b->nbig;
  if (!record) {
    feast::fill_i32(b->gs, b->info.as<int32_t>(), static_cast<int64_t>(b->P) * N, 0);
    if (nbig < b->P) {
      const int nsmall = (b->P - nbig) * N;
      const int64_t off = static_cast<int64_t>(nbig) * N;
      feast::lu_small<T>(b->gs, g + nbig, N, nsmall, b->nmax, piv + off * b->nmax,
                         b->info.as<int32_t>() + off);
      feast::diag_block_inverse<T>(b->gs, nullptr, 0, 0, nsmall, b->nmax, 64, 0,
                                   b->np[nbig] / 64, true, Linv + off * is, is, g + nbig, N);
    }
  }
  auto active = [&](int64_t k) { return std::min(b->active(k), nbig); };
  // panel [kp, kp + NB) of the pencils with np > kp: leaves, the inverses of
  // L's diagonal blocks, and its row exchanges outside it
  auto factor_panel = [&](int64_t kp) {
    const int64_t kq = kp + NB, jp = kp / 64;
    const int actp = active(kp), nmat = actp * N;
    if (!record) {
      panel_grp<T>(b, F, nmat, kp, static_cast<int>(kPanel), kp, static_cast<int>(NB));
      feast::diag_block_inverse<T>(b->gs, F, 0, 0, nmat, b->nmax, 64, jp, jp + 1, true, Linv, is,
                                   g, N);
    }
    const int acth = NB > kPanel ? active(kp + kPanel) : 0;
    if (acth > 0) {
      std::vector<GemmArgs<T>> x, upx;
      for (int p = 0; p < acth; ++p) {
        const int64_t ld = b->np[p], st = ld * ld;
        T *M = F + b->foff[p];
        T *X = M + kp * ld + kp + kPanel;
        x.push_back(gargs<T>(kPanel, kPanel, kPanel, Linv + p * N * is + jp * 4096, 64, is, X, ld,
                             st, X, ld, st, 1.0, 0.0, N));
        upx.push_back(gargs<T>(ld - kp - kPanel, kPanel, kPanel, M + (kp + kPanel) * ld + kp, ld, st,
                               X, ld, st, M + (kp + kPanel) * ld + kp + kPanel, ld, st, -1.0, 1.0,
                               N));
      }
      ggemm<T>(b, tab, 0, false, x);
      ggemm<T>(b, tab, 0, true, upx);
      if (!record) {
        panel_grp<T>(b, F, acth * N, kp + kPanel, static_cast<int>(kPanel), kp,
                     static_cast<int>(NB));
        feast::diag_block_inverse<T>(b->gs, F, 0, 0, acth * N, b->nmax, 64, jp + 1, jp + 2, true,
                                     Linv, is, g, N);
      }
    }
    if (!record)
      feast::laswp_outside<T>(b->gs, F, 0, 0, nmat, b->nmax, kp, static_cast<int>(NB), kp, kq, piv,
                              g, N);
  };
  // U12 = L11^{-1} A12 of panel kp over the columns past it (in place, 64-row
  // tile rows; for 128 the L10 update between the two halves)
  auto u12 = [&](int64_t kp) {
    const int64_t kq = kp + NB, jp = kp / 64;
    std::vector<GemmArgs<T>> u0, u10, u1;
    for (int p = 0; p < active(kq); ++p) {
      const int64_t ld = b->np[p], st = ld * ld, rest = ld - kq;
      T *M = F + b->foff[p];
      T *top = M + kp * ld + kq;
      u0.push_back(gargs<T>(kPanel, rest, kPanel, Linv + p * N * is + jp * 4096, 64, is, top, ld, st,
                            top, ld, st, 1.0, 0.0, N));
      if (NB > kPanel) {
        T *bot = M + (kp + kPanel) * ld + kq;
        u10.push_back(gargs<T>(kPanel, rest, kPanel, M + (kp + kPanel) * ld + kp, ld, st, top, ld,
                               st, bot, ld, st, -1.0, 1.0, N));
        u1.push_back(gargs<T>(kPanel, rest, kPanel, Linv + p * N * is + (jp + 1) * 4096, 64, is, bot,
                              ld, st, bot, ld, st, 1.0, 0.0, N));
      }
    }
    ggemm<T>(b, tab, 0, false, u0);
    ggemm<T>(b, tab, 0, true, u10);
    ggemm<T>(b, tab, 0, false, u1);
  };
  // C[r0:r1, c0:c1] -= L[r0:r1, ka:kb] U[ka:kb, c0:c1] of every pencil with
  // np > max(r0, c0), rows and columns clipped to its order (r1, c1 < 0: to
  // its order)
  auto update = [&](int64_t r0, int64_t r1, int64_t c0, int64_t c1, int64_t ka, int64_t kb,
                    int variant) {
    std::vector<GemmArgs<T>> e;
    for (int p = 0; p < active(std::max(r0, c0)); ++p) {
      const int64_t ld = b->np[p], st = ld * ld;
      const int64_t re = r1 < 0 ? ld : std::min(r1, ld), ce = c1 < 0 ? ld : std::min(c1, ld);
      if (re <= r0 || ce <= c0) continue;
      if (!(0 <= ka && ka < kb && kb <= r0 && kb <= c0))
        throw HipError{hipErrorInvalidValue, "grouped update range"};
      T *M = F + b->foff[p];
      e.push_back(gargs<T>(re - r0, ce - c0, kb - ka, M + r0 * ld + ka, ld, st, M + ka * ld + c0, ld,
                           st, M + r0 * ld + c0, ld, st, -1.0, 1.0, N));
    }
    ggemm<T>(b, tab, 0, true, e, variant);
  };
  // Steps of up to kGroup panels: each further panel's columns get the
  // group's earlier panels' update, it is factored (its exchanges reach the
  // group's L21 columns and the columns still waiting for the update, which
  // commutes with them), its rows get the same update and then its U12; one
  // update with K = the group's width covers the rest (the trailing block is
  // read and written once per group).
  for (int64_t k0 = 0; k0 < b->nmax;) {
    if (active(k0) == 0) break;
    factor_panel(k0);
    int64_t kg = k0 + NB;
    if (active(kg) == 0) break;
    u12(k0);
    for (int gi = 1; gi < kBatchGroup<T> && active(kg) > 0; ++gi) {
      const int64_t ks = kg, ke = kg + NB;
      update(ks, -1, ks, ke, k0, ks, -1);
      factor_panel(ks);
      kg = ke;
      if (active(ke) == 0) break;
      update(ks, ke, ke, -1, k0, ks, -1);
      u12(ks);
    }
    if (active(kg) > 0) update(kg, -1, kg, -1, k0, kg, b->lu_update);
    k0 = kg;
  }
  if (!record) {
    const int nmat = b->P * N;
    feast::diag_block_inverse<T>(b->gs, F, 0, 0, nmat, b->nmax, 64, 0, b->nblk, false, Uinv, is, g,
                                 N);
    feast::perm_from_ipiv(b->gs, piv, b->perm.as<int32_t>(), b->nmax, nmat, g, N);
  }
}

// Y_p <- L^{-1} Y_p (rows [r0, r1) of every pencil's node blocks), recursive
// halving at multiples of 64; leaves are in-place products with the inverted
// diagonal blocks.
template <typename T>
void trsm_lower_grp(feast_batch *b, Tables &tab, T *Y, int64_t r0, int64_t r1) {
  const T *F = b->F.as<T>();
  const T *Linv = b->Linv.as<T>();
  const int N = b->N;
  const int64_t is = b->istride();
  if (r1 - r0 <= 64) {
    std::vector<GemmArgs<T>> e;
    for (int p = 0; p < b->active(r0); ++p) {
      const int64_t ldy = b->ldY(p);
      T *X = Y + b->yoff[p] + r0 * ldy;
      e.push_back(gargs<T>(r1 - r0, b->m[p], r1 - r0, Linv + p * N * is + (r0 / 64) * 4096, 64, is,
                           X, ldy, b->m[p], X, ldy, b->m[p], 1.0, 0.0, N));
    }
    ggemm<T>(b, tab, 0, false, e);
    return;
  }
  const int64_t mid = r0 + ((r1 - r0 + 127) / 128) * 64;
  trsm_lower_grp<T>(b, tab, Y, r0, mid);
  std::vector<GemmArgs<T>> e;
  for (int p = 0; p < b->active(mid); ++p) {
    const int64_t ld = b->np[p], ldy = b->ldY(p), rows = std::min(r1, ld) - mid;
    const T *M = F + b->foff[p];
    T *Yp = Y + b->yoff[p];
    e.push_back(gargs<T>(rows, b->m[p], mid - r0, M + mid * ld + r0, ld, ld * ld, Yp + r0 * ldy, ldy,
                         b->m[p], Yp + mid * ldy, ldy, b->m[p], -1.0, 1.0, N));
  }
  ggemm<T>(b, tab, 0, true, e);
  trsm_lower_grp<T>(b, tab, Y, mid, r1);
}

// Y_p <- U^{-1} Y_p, rows [r0, r1).
template <typename T>
void trsm_upper_grp(feast_batch *b, Tables &tab, T *Y, int64_t r0, int64_t r1) {
  const T *F = b->F.as<T>();
  const T *Uinv = b->Uinv.as<T>();
  const int N = b->N;
  const int64_t is = b->istride();
  if (r1 - r0 <= 64) {
    std::vector<GemmArgs<T>> e;
    for (int p = 0; p < b->active(r0); ++p) {
      const int64_t ldy = b->ldY(p);
      T *X = Y + b->yoff[p] + r0 * ldy;
      e.push_back(gargs<T>(r1 - r0, b->m[p], r1 - r0, Uinv + p * N * is + (r0 / 64) * 4096, 64, is,
                           X, ldy, b->m[p], X, ldy, b->m[p], 1.0, 0.0, N));
    }
    ggemm<T>(b, tab, 0, false, e);
    return;
  }
  const int64_t mid = r0 + ((r1 - r0 + 127) / 128) * 64;
  trsm_upper_grp<T>(b, tab, Y, mid, r1);
  std::vector<GemmArgs<T>> e;
  for (int p = 0; p < b->active(mid); ++p) {  // X[r0:mid] -= U[r0:mid, mid:r1] X[mid:r1]
    const int64_t ld = b->np[p], ldy = b->ldY(p), K = std::min(r1, ld) - mid;
    const T *M = F + b->foff[p];
    T *Yp = Y + b->yoff[p];
    e.push_back(gargs<T>(mid - r0, b->m[p], K, M + r0 * ld + mid, ld, ld * ld, Yp + mid * ldy, ldy,
                         b->m[p], Yp + r0 * ldy, ldy, b->m[p], -1.0, 1.0, N));
  }
  ggemm<T>(b, tab, 0, true, e);
  trsm_upper_grp<T>(b, tab, Y, r0, mid);
}

// Y <- U^{-1} L^{-1} Y for every node of every pencil (rows already permuted).
template <typename T>
void trsolve_grouped(feast_batch *b, T *Y) {
  b->sv_tab.begin();
  trsm_lower_grp<T>(b, b->sv_tab, Y, 0, b->nmax);
  trsm_upper_grp<T>(b, b->sv_tab, Y, 0, b->nmax);
}

// Key of a graph: the caller's pointers and leading dimensions plus a tag.
std::vector<int64_t> make_key(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
                              const feast_z *const *dB, const int64_t *ldb, int64_t tag) {
  std::vector<int64_t> k;
  k.reserve(4 * b->P + 1);
  for (int i = 0; i < b->P; ++i) {
    k.push_back(reinterpret_cast<int64_t>(dA[i]));
    k.push_back(lda[i]);
    k.push_back(reinterpret_cast<int64_t>(dB[i]));
    k.push_back(ldb[i]);
  }
  k.push_back(tag);
  return k;
}

template <class Body> void run_graph(feast_batch *b, Graph &g, const std::vector<int64_t> &key, Body &&body) {
  if (!g.exec || g.key != key) {
    g.reset();
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
    try {
      body();
    } catch (...) {
      (void)hipStreamEndCapture(b->gs, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    HIPCHK(hipStreamEndCapture(b->gs, &graph));
    const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    g.key = key;
  }
  HIPCHK(hipGraphLaunch(g.exec, b->gs));
  ++b->launches;
}

// Content fingerprints of every A_p and B_p (caller's order: A_0, B_0, A_1, ...),
// one grouped launch; synchronises the batch stream.
std::vector<uint64_t> fingerprints(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
                                   const feast_z *const *dB, const int64_t *ldb) {
  std::vector<GrpMat> tab(2 * static_cast<size_t>(b->P));
  for (int c = 0; c < b->P; ++c) {
    const int64_t n = b->n[b->where[c]];
    tab[2 * c] = {const_cast<feast_z *>(dA[c]), lda[c], 0, n};
    tab[2 * c + 1] = {const_cast<feast_z *>(dB[c]), ldb[c], 0, n};
  }
  b->fptab.alloc(sizeof(GrpMat) * tab.size());
  b->fpout.alloc(sizeof(uint64_t) * tab.size());
  HIPCHK(hipMemcpyAsync(b->fptab.p, tab.data(), sizeof(GrpMat) * tab.size(), hipMemcpyHostToDevice,
                        b->gs));
  feast::fingerprint(b->gs, b->fptab.as<GrpMat>(), static_cast<int>(tab.size()), GrpMat{},
                     GrpMat{}, b->nmax, b->fpout.as<uint64_t>());
  std::vector<uint64_t> out(tab.size());
  HIPCHK(hipMemcpyAsync(out.data(), b->fpout.p, sizeof(uint64_t) * out.size(),
                        hipMemcpyDeviceToHost, b->gs));
  HIPCHK(hipStreamSynchronize(b->gs));
  return out;
}

// Factor every shifted matrix of every pencil (graph), then check the pivots.
// The cached factors are reused only for pencils with unchanged content
// (Section 4.3); the graph is re-captured when the caller's pointers change.
int factor_all(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
               const feast_z *const *dB, const int64_t *ldb) {
  const std::vector<uint64_t> fps = fingerprints(b, dA, lda, dB, ldb);
  if (b->factored && fps == b->ffp) return FEAST_OK;
  const std::vector<int64_t> key = make_key(b, dA, lda, dB, ldb, 0);
  b->factored = false;
  run_graph(b, b->g_factor, key, [&]() {
    for (int p = 0; p < b->P; ++p) {
      const int c = b->order[p];
      const z64 *A = reinterpret_cast<const z64 *>(dA[c]), *B = reinterpret_cast<const z64 *>(dB[c]);
      const int64_t ld = b->np[p];
      if (b->mixed())
        feast::shift_assemble_c(b->gs, A, lda[c], B, ldb[c], b->sub[p]->dz.as<z64>(), b->N, b->n[p],
                                b->F.as<c64>() + b->foff[p], ld, ld * ld);
      else
        feast::shift_assemble_z(b->gs, A, lda[c], B, ldb[c], b->sub[p]->dz.as<z64>(), b->N, b->n[p],
                                b->F.as<z64>() + b->foff[p], ld, ld * ld);
    }
    if (b->mixed())
      lu_grouped<c64>(b, false);
    else
      lu_grouped<z64>(b, false);
  });
  std::vector<int32_t> hinfo(static_cast<size_t>(b->P) * b->N);
  HIPCHK(hipMemcpyAsync(hinfo.data(), b->info.p, sizeof(int32_t) * hinfo.size(),
                        hipMemcpyDeviceToHost, b->gs));
  HIPCHK(hipStreamSynchronize(b->gs));
  for (int p = 0; p < b->P; ++p)
    for (int j = 0; j < b->N; ++j) {
      const int32_t v = hinfo[static_cast<size_t>(p) * b->N + j];
      if (v != 0) {
        char buf[200];
        const cd z = b->sub[p]->hz[j];
        std::snprintf(buf, sizeof buf, "exact zero pivot in pencil %d at node %d (z = %.17g%+.17gi), column %d",
                      b->order[p], j, z.real(), z.imag(), v - 1);
        b->err = buf;
        return FEAST_SINGULAR;
      }
    }
  b->factored = true;
  b->ffp = fps;
  return FEAST_OK;
}

// U_p = sum_j w_pj (z_pj B_p - A_p)^{-1} R_p for every pencil, with R_p in the
// member plan's R block and U_p written to its W_UF block (graph).
void filter_all(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
                const feast_z *const *dB, const int64_t *ldb, int sweeps) {
  const int N = b->N;
  const int64_t nmax = b->nmax;
  const std::vector<int64_t> key = make_key(b, dA, lda, dB, ldb, b->mixed() ? 1 + sweeps : 0);
  run_graph(b, b->g_filter, key, [&]() {
    hipStream_t s = b->gs;
    const int32_t *perm = b->perm.as<int32_t>();
    if (!b->mixed()) {
      z64 *Y = b->Y.as<z64>();
      for (int p = 0; p < b->P; ++p)
        feast::gather_rows<z64>(s, b->sub[p]->R.as<z64>(), b->m[p], 0, perm + p * N * nmax, b->n[p],
                                b->m[p], N, Y + b->yoff[p], b->ldY(p), b->m[p], nmax);
      trsolve_grouped<z64>(b, Y);
    } else {
      z64 *Y = b->Y.as<z64>(), *T1 = b->T1.as<z64>(), *T2 = b->T2.as<z64>();
      c64 *Yc = b->Yc.as<c64>();
      // ||R_p||_F^2 sets the power-of-two scale of pencil p's complex64 solves
      auto rn = [&](int p) { return b->sub[p]->rn.as<double>(); };
      auto rcnt = [&](int p) { return static_cast<double>(b->n[p]) * b->m[p]; };
      for (int p = 0; p < b->P; ++p) {
        const int64_t ldy = b->ldY(p);
        feast::fro2_batched(s, b->sub[p]->R.as<z64>(), b->m[p], 0, b->n[p], b->m[p], 1, rn(p) + 8,
                            rn(p));
        feast::gather_rows<z64>(s, b->sub[p]->R.as<z64>(), b->m[p], 0, perm + p * N * nmax,
                                b->n[p], b->m[p], N, T1 + b->toff[p], ldy, b->m[p], nmax);
        feast::z_to_c(s, T1 + b->toff[p], ldy, 0, b->n[p], ldy, 1, Yc + b->yoff[p], ldy, 0, rn(p),
                      rcnt(p));
      }
      trsolve_grouped<c64>(b, Yc);
      for (int p = 0; p < b->P; ++p)
        feast::c_to_z(s, Yc + b->yoff[p], b->ldY(p), 0, b->n[p], b->ldY(p), 1, Y + b->yoff[p],
                      b->ldY(p), 0, rn(p), rcnt(p));
      for (int sw = 0; sw < sweeps; ++sw) {
        // FP64 residual r_j = R - (z_j B - A) Y_j of all nodes of a pencil in
        // one launch, then the complex64 correction
        for (int p = 0; p < b->P; ++p) {
          const int c = b->order[p];
          const int64_t n = b->n[p], ldy = b->ldY(p);
          const z64 *A = reinterpret_cast<const z64 *>(dA[c]);
          const z64 *B = reinterpret_cast<const z64 *>(dB[c]);
          z64 *t1 = T1 + b->toff[p], *t2 = T2 + b->toff[p], *y = Y + b->yoff[p];
          if (lda[c] == ldb[c]) {
            feast::zgemm_shift_residual(s, n, b->m[p], n, A, B, lda[c], b->sub[p]->dz.as<z64>(), y,
                                        ldy, b->m[p], b->sub[p]->R.as<z64>(), b->m[p], 0, t1, ldy,
                                        b->m[p], N);
          } else {
            gemm_t<z64>(s, 0, n, ldy, n, make_double2(1.0, 0.0), A, lda[c], 0, y, ldy, 0,
                        make_double2(0.0, 0.0), t1, ldy, 0, 1);
            gemm_t<z64>(s, 0, n, ldy, n, make_double2(1.0, 0.0), B, ldb[c], 0, y, ldy, 0,
                        make_double2(0.0, 0.0), t2, ldy, 0, 1);
            feast::shift_residual(s, b->sub[p]->R.as<z64>(), b->m[p], t1, t2, ldy,
                                  b->sub[p]->dz.as<z64>(), N, n, b->m[p]);
          }
          feast::gather_rows<z64>(s, t1, ldy, b->m[p], perm + p * N * nmax, n, b->m[p], N, t2, ldy,
                                  b->m[p], nmax);
          feast::z_to_c(s, t2, ldy, 0, n, ldy, 1, Yc + b->yoff[p], ldy, 0, rn(p), rcnt(p));
        }
        trsolve_grouped<c64>(b, Yc);
        for (int p = 0; p < b->P; ++p)
          feast::add_c_to_z(s, Yc + b->yoff[p], b->ldY(p), 0, b->n[p], b->ldY(p), 1,
                            Y + b->yoff[p], b->ldY(p), 0, rn(p), rcnt(p));
      }
    }
    const z64 *Y = b->Y.as<z64>();
    for (int p = 0; p < b->P; ++p)
      feast::weighted_sum(s, Y + b->yoff[p], b->ldY(p), b->m[p], b->sub[p]->dw.as<z64>(), N,
                          b->n[p], b->m[p], b->sub[p]->wblk(feast_plan::W_UF), b->m[p]);
  });
}

// ---------------------------------------------------------------------------
// Grouped orthonormalisation and projection over the pencils in a list `act`
// (Algorithm 5's QR steps and reduced pencil): every step is one launch over all of them.
// The GEMM problem lists and descriptors depend on the list, so each round is
// scheduled twice, recording and then launching (tables uploaded in between).
// ---------------------------------------------------------------------------

std::vector<GrpMat> gmats(feast_batch *b, const std::vector<int> &act, z64 *(*blk)(feast_plan *, int),
                          int which, bool square) {
  std::vector<GrpMat> g;
  for (int p : act) {
    const int64_t m = b->m[p];
    g.push_back(GrpMat{blk(b->sub[p], which), m, 0, square ? m : b->n[p]});
  }
  return g;
}
z64 *gblk_of(feast_plan *q, int i) { return q->gblk(i); }
z64 *wblk_of(feast_plan *q, int i) { return q->wblk(i); }

// X_p <- orth(X_p) (n_p x m_p, leading dimension m_p) by shifted Cholesky QR3,
// as the single-pencil plan does it; flags of list entry i at flags[8 i + slot + pass].
void orth_grouped(feast_batch *b, Tables &t, const std::vector<int> &act, int xblk, int slot) {
  const bool rec = t.record;
  hipStream_t s = b->gs;
  const int cnt = static_cast<int>(act.size());
  const z64 one = make_double2(1.0, 0.0);
  const GrpMat *gG = t.put(gmats(b, act, gblk_of, feast_plan::G_GRAM, true));
  const GrpMat *gR = t.put(gmats(b, act, gblk_of, feast_plan::G_RINV, true));
  std::vector<GrpMat> wsrc, xdst;
  std::vector<double> shifts;
  for (int p : act) {
    const int64_t n = b->n[p], m = b->m[p];
    wsrc.push_back(GrpMat{b->sub[p]->wblk(feast_plan::W_ORTH), m, 0, n});
    xdst.push_back(GrpMat{b->sub[p]->wblk(xblk), m, m, n});
    shifts.push_back(11.0 * (static_cast<double>(n) * m + static_cast<double>(m) * (m + 1)) * kU64);
  }
  const GrpMat *gW = t.put(wsrc), *gX = t.put(xdst);
  const double *dshift = t.put(shifts);
  z64 *Dinv = b->dinv.as<z64>();
  const int64_t dstride = b->mblk() * 4096;
  int64_t nm_max = 0;
  for (int p : act) nm_max = std::max(nm_max, b->n[p] * b->m[p]);
  for (int pass = 0; pass < 3; ++pass) {
    // Gram matrix G = X^* X
    std::vector<GemmArgs<z64>> e;
    for (int p : act) {
      const int64_t n = b->n[p], m = b->m[p];
      z64 *X = b->sub[p]->wblk(xblk);
      e.push_back(gargs<z64>(m, m, n, X, m, 0, X, m, 0, b->sub[p]->gblk(feast_plan::G_GRAM), m, 0,
                             1.0, 0.0, 1));
    }
    ggemm_small_out(b, t, e);
    if (pass == 0 && !rec) feast::add_shift_grp(s, gG, cnt, dshift);
    // blocked Cholesky G = R^* R (upper R over G)
    for (int64_t J0 = 0; J0 < b->mmax; J0 += 64) {
      if (!rec)
        feast::chol_inv_grp(s, gG, cnt, J0, b->flags.as<int32_t>() + slot + pass, 8, Dinv,
                            dstride);
      std::vector<GemmArgs<z64>> e1, e2;
      for (int i = 0; i < cnt; ++i) {
        const int p = act[i];
        const int64_t m = b->m[p];
        if (J0 >= m) continue;
        const int64_t jb = std::min<int64_t>(64, m - J0), rest = m - J0 - jb;
        if (rest <= 0) continue;
        z64 *G = b->sub[p]->gblk(feast_plan::G_GRAM);
        z64 *GJ = G + J0 * m + J0;
        e1.push_back(gargs<z64>(jb, rest, jb, Dinv + i * dstride + (J0 / 64) * 4096, 64, 0, GJ + jb,
                                m, 0, GJ + jb, m, 0, 1.0, 0.0, 1));
        e2.push_back(gargs<z64>(rest, rest, jb, GJ + jb, m, 0, GJ + jb, m, 0,
                                G + (J0 + jb) * m + J0 + jb, m, 0, -1.0, 1.0, 1));
      }
      ggemm<z64>(b, t, 2, false, e1);
      ggemm<z64>(b, t, 2, false, e2);
    }
    // Ri = R^{-1}: the inverted diagonal blocks chol_inv_grp left in Dinv (upper
    // triangles; their strict lower parts are not written), then
    // X12 = -X11 R12 X22 by halving
    if (!rec) {
      feast::zero_lower_grp(s, gG, cnt, b->mmax, false);
      feast::zero_lower_grp(s, gR, cnt, b->mmax, true);
      feast::put_diag_grp(s, gR, cnt, b->mblk(), Dinv, dstride);
      feast::zero_lower_grp(s, gR, cnt, b->mmax, false);
    }
    struct Rec {
      static void run(feast_batch *b, Tables &t, const std::vector<int> &act, int64_t r0,
                      int64_t r1) {
        if (r1 - r0 <= 64) return;
        const int64_t mid = r0 + ((r1 - r0 + 127) / 128) * 64;
        run(b, t, act, r0, mid);
        run(b, t, act, mid, r1);
        std::vector<GemmArgs<z64>> e1, e2;
        for (int p : act) {
          const int64_t m = b->m[p];
          if (m <= mid) continue;
          const int64_t c1 = std::min(r1, m);
          z64 *R = b->sub[p]->gblk(feast_plan::G_GRAM), *X = b->sub[p]->gblk(feast_plan::G_RINV);
          z64 *T = b->sub[p]->gblk(feast_plan::G_T);
          e1.push_back(gargs<z64>(mid - r0, c1 - mid, c1 - mid, R + r0 * m + mid, m, 0,
                                  X + mid * m + mid, m, 0, T, m, 0, 1.0, 0.0, 1));
          e2.push_back(gargs<z64>(mid - r0, c1 - mid, mid - r0, X + r0 * m + r0, m, 0, T, m, 0,
                                  X + r0 * m + mid, m, 0, -1.0, 0.0, 1));
        }
        ggemm<z64>(b, t, 0, false, e1);
        ggemm<z64>(b, t, 0, false, e2);
      }
    };
    Rec::run(b, t, act, 0, b->mmax);
    // X <- X Ri
    std::vector<GemmArgs<z64>> ex;
    for (int p : act) {
      const int64_t n = b->n[p], m = b->m[p];
      ex.push_back(gargs<z64>(n, m, m, b->sub[p]->wblk(xblk), m, 0,
                              b->sub[p]->gblk(feast_plan::G_RINV), m, 0,
                              b->sub[p]->wblk(feast_plan::W_ORTH), m, 0, 1.0, 0.0, 1));
    }
    ggemm<z64>(b, t, 0, false, ex);
    if (!rec) feast::copy_grp(s, gW, gX, cnt, nm_max);
  }
}

// One scheduling pass of the grouped projection of the pencils in `act`:
// U_1 = orth(UF), B U_1, A U_1, U_2 = orth(B U_1), At = U_2^* A U_1, Bt = U_2^* B U_1.
void project_schedule(feast_batch *b, Tables &t, const std::vector<int> &act,
                      const feast_z *const *dA, const int64_t *lda, const feast_z *const *dB,
                      const int64_t *ldb) {
  const bool rec = t.record;
  hipStream_t s = b->gs;
  const int cnt = static_cast<int>(act.size());
  std::vector<GrpMat> uf, u1, bu, u2;
  int64_t nm_max = 0;
  for (int p : act) {
    const int64_t n = b->n[p], m = b->m[p];
    feast_plan *q = b->sub[p];
    uf.push_back(GrpMat{q->wblk(feast_plan::W_UF), m, 0, n});
    u1.push_back(GrpMat{q->wblk(feast_plan::W_U1), m, m, n});
    bu.push_back(GrpMat{q->wblk(feast_plan::W_BU1), m, 0, n});
    u2.push_back(GrpMat{q->wblk(feast_plan::W_U2), m, m, n});
    nm_max = std::max(nm_max, n * m);
  }
  const GrpMat *guf = t.put(uf), *gu1 = t.put(u1), *gbu = t.put(bu), *gu2 = t.put(u2);
  if (!rec) {
    feast::fill_i32(s, b->flags.as<int32_t>(), 8 * static_cast<int64_t>(cnt), 0);
    feast::copy_grp(s, guf, gu1, cnt, nm_max);
  }
  orth_grouped(b, t, act, feast_plan::W_U1, 0);
  std::vector<GemmArgs<z64>> eb, ea;
  for (int p : act) {
    const int c = b->order[p];
    const int64_t n = b->n[p], m = b->m[p];
    feast_plan *q = b->sub[p];
    eb.push_back(gargs<z64>(n, m, n, reinterpret_cast<const z64 *>(dB[c]), ldb[c], 0,
                            q->wblk(feast_plan::W_U1), m, 0, q->wblk(feast_plan::W_BU1), m, 0, 1.0,
                            0.0, 1));
    ea.push_back(gargs<z64>(n, m, n, reinterpret_cast<const z64 *>(dA[c]), lda[c], 0,
                            q->wblk(feast_plan::W_U1), m, 0, q->wblk(feast_plan::W_AU1), m, 0, 1.0,
                            0.0, 1));
  }
  ggemm<z64>(b, t, 0, false, eb);
  ggemm<z64>(b, t, 0, false, ea);
  if (!rec) feast::copy_grp(s, gbu, gu2, cnt, nm_max);
  orth_grouped(b, t, act, feast_plan::W_U2, 3);
  std::vector<GemmArgs<z64>> pa, pb;
  for (int p : act) {
    const int64_t n = b->n[p], m = b->m[p];
    feast_plan *q = b->sub[p];
    z64 *U2 = q->wblk(feast_plan::W_U2);
    pa.push_back(gargs<z64>(m, m, n, U2, m, 0, q->wblk(feast_plan::W_AU1), m, 0,
                            q->gblk(feast_plan::G_AT), m, 0, 1.0, 0.0, 1));
    pb.push_back(gargs<z64>(m, m, n, U2, m, 0, q->wblk(feast_plan::W_BU1), m, 0,
                            q->gblk(feast_plan::G_BT), m, 0, 1.0, 0.0, 1));
  }
  ggemm_small_out(b, t, pa);
  ggemm_small_out(b, t, pb);
  // At, Bt of every pencil in `act` into the packed buffer, in list order
  std::vector<GrpMat> src, dst;
  int64_t off = 0, mm_max = 0;
  for (int p : act) {
    const int64_t m = b->m[p];
    feast_plan *q = b->sub[p];
    for (int which : {feast_plan::G_AT, feast_plan::G_BT}) {
      src.push_back(GrpMat{q->gblk(which), m, m, m});
      dst.push_back(GrpMat{b->pk.as<z64>() + off, m, m, m});
      off += m * m;
    }
    mm_max = std::max(mm_max, m * m);
  }
  const GrpMat *gsrc = t.put(src), *gdst = t.put(dst);
  if (!rec) feast::copy_grp(s, gsrc, gdst, 2 * cnt, mm_max);
}

// The grouped projection of `act` with At, Bt copied to the host (synchronises);
// a Cholesky QR breakdown is reported as for a single plan.
int project_grouped(feast_batch *b, const std::vector<int> &act, const feast_z *const *dA,
                    const int64_t *lda, const feast_z *const *dB, const int64_t *ldb,
                    std::vector<std::vector<feast_z>> &At, std::vector<std::vector<feast_z>> &Bt) {
  if (act.empty()) return FEAST_OK;
  // the projection of this list of pencils is scheduled once (tables recorded
  // and uploaded), captured in a graph on its first use and replayed after
  std::vector<int64_t> key = make_key(b, dA, lda, dB, ldb, -1);
  key.insert(key.end(), act.begin(), act.end());
  if (b->proj_graphs.size() >= 16 && !b->proj_graphs.count(key)) {
    HIPCHK(hipStreamSynchronize(b->gs));  // (no replay in flight when they go)
    b->proj_graphs.clear();
  }
  std::unique_ptr<feast_batch::ProjGraph> &pg = b->proj_graphs[key];
  if (!pg) {
    pg = std::make_unique<feast_batch::ProjGraph>();
    pg->tab.reset();
    project_schedule(b, pg->tab, act, dA, lda, dB, ldb);
    pg->tab.upload();
  }
  Tables &t = pg->tab;
  run_graph(b, pg->g, key, [&]() {
    t.begin();
    project_schedule(b, t, act, dA, lda, dB, ldb);
  });
  hipStream_t s = b->gs;
  const int cnt = static_cast<int>(act.size());
  std::vector<int32_t> hf(8 * cnt);
  int64_t elems = 0;
  for (int p : act) elems += 2 * b->m[p] * b->m[p];
  HIPCHK(hipMemcpyAsync(b->pk_host, b->pk.p, sizeof(z64) * elems, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hf.data(), b->flags.p, sizeof(int32_t) * 8 * cnt, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  const feast_z *hp = static_cast<const feast_z *>(b->pk_host);
  for (int p : act) {
    const int64_t mm = b->m[p] * b->m[p];
    std::copy(hp, hp + mm, At[p].data());
    std::copy(hp + mm, hp + 2 * mm, Bt[p].data());
    hp += 2 * mm;
  }
  for (int i = 0; i < cnt; ++i)
    for (int k = 0; k < 6; ++k)
      if (hf[8 * i + k] != 0) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "pencil %d: Cholesky QR pass %d of %s broke down at column %d",
                      b->order[act[i]], k % 3 + 1, k < 3 ? "U" : "B U_1", hf[8 * i + k] - 1);
        b->err = buf;
        return FEAST_ENUMERIC;
      }
  return FEAST_OK;
}

// The caller's stream -> batch stream -> caller's stream ordering.
void enter(feast_batch *b) {
  HIPCHK(hipEventRecord(b->ev_in, b->s));
  HIPCHK(hipStreamWaitEvent(b->gs, b->ev_in, 0));
}
void leave(feast_batch *b) {
  HIPCHK(hipEventRecord(b->ev_out, b->gs));
  HIPCHK(hipStreamWaitEvent(b->s, b->ev_out, 0));
}

// One grouped launch of the products e (C = alpha A B + beta C, ta = 0) on
// stream st, its table written and uploaded now (after st's earlier work,
// which may still read the table's previous contents).
void grouped_on(Tables &t, hipStream_t st, std::vector<GemmArgs<z64>> &e) {
  if (e.empty()) return;
  const int64_t tiles = feast::gemm_group_tiles<z64>(e.data(), static_cast<int>(e.size()));
  t.host.clear();
  t.off.clear();
  t.cnt.clear();
  t.record = true;
  t.begin();
  t.put(e);
  HIPCHK(hipStreamSynchronize(st));
  t.upload();
  t.begin();
  feast::gemm_group<z64>(st, 0, false, t.put(e), static_cast<int>(e.size()), tiles,
                         feast::GROUP_PLAIN);
}

// R_p = B_p V_p of every pencil (K = n_p over few output tiles each) as one
// grouped launch on the batch stream; the table holds the caller's pointers,
// so it is written and uploaded at each call.
void rhs_all(feast_batch *b, const feast_z *const *dB, const int64_t *ldb,
             const feast_z *const *dV, const int64_t *ldv) {
  std::vector<GemmArgs<z64>> e;
  for (int p = 0; p < b->P; ++p) {
    const int c = b->order[p];
    e.push_back(GemmArgs<z64>{b->n[p], b->m[p], b->n[p], reinterpret_cast<const z64 *>(dB[c]),
                              ldb[c], 0, reinterpret_cast<const z64 *>(dV[c]), ldv[c], 0,
                              b->sub[p]->R.as<z64>(), b->m[p], 0, make_double2(1.0, 0.0),
                              make_double2(0.0, 0.0), 1, 1, b->n[p], nullptr, 0});
  }
  grouped_on(b->bv_tab, b->gs, e);
}

// Runs f(i) for i in [0, count) on up to `threads` host threads.
template <class F> void parallel_for(int count, int threads, F &&f) {
  threads = std::max(1, std::min(threads, count));
  if (threads == 1) {
    for (int i = 0; i < count; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (int i = next++; i < count; i = next++) f(i);
    });
  for (auto &th : pool) th.join();
}

}  // namespace

extern "C" {

int feast_batch_create(feast_batch **out, int32_t count, const int64_t *n, const int64_t *m,
                       const feast_contour *c, const feast_opts *o, void *stream) {
  if (!out) return FEAST_EINVAL;
  *out = nullptr;
  if (count < 1 || count > 4096 || !n || !m || !c) return FEAST_EINVAL;
  feast_opts opts;
  feast_opts_default(&opts);
  if (o) opts = *o;
  if (!(opts.eta > 0.0) || !(opts.eps >= 0.0) || opts.max_iter < 1 ||
      opts.max_iter > FEAST_MAX_HISTORY || (opts.prec != FEAST_FP64 && opts.prec != FEAST_MIXED) ||
      opts.max_sweeps < 0 || (opts.nb != 0 && opts.nb != 64 && opts.nb != 128) ||
      opts.batch_update < 0 || opts.batch_update > 3)
    return FEAST_EINVAL;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > 16384 || m[i] < 1 || m[i] > n[i] || bad_contour(&c[i]) ||
        c[i].nodes != c[0].nodes)
      return FEAST_EINVAL;
  }
  feast_batch *b = nullptr;
  try {
    b = new feast_batch();
  } catch (...) {
    return FEAST_ENOMEM;
  }
  b->P = count;
  b->N = c[0].nodes;
  b->o = opts;
  b->s = static_cast<hipStream_t>(stream);
  const int rc = bguarded(b, [&]() {
    const int P = count, N = b->N;
    b->order.resize(P);
    std::iota(b->order.begin(), b->order.end(), 0);
    auto padded = [&](int i) { return (n[i] + kPanel - 1) / kPanel * kPanel; };
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return padded(x) > padded(y); });
    b->where.resize(P);
    for (int p = 0; p < P; ++p) b->where[b->order[p]] = p;
    HIPCHK(hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&b->as, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&b->ev_proj, hipEventDisableTiming));
    int64_t fo = 0, yo = 0, to = 0;
    for (int p = 0; p < P; ++p) {
      const int i = b->order[p];
      b->n.push_back(n[i]);
      b->m.push_back(m[i]);
      b->np.push_back(padded(i));
      b->foff.push_back(fo);
      b->yoff.push_back(yo);
      b->toff.push_back(to);
      fo += static_cast<int64_t>(N) * b->np[p] * b->np[p];
      yo += b->np[p] * N * m[i];
      to += n[i] * N * m[i];
      b->sub.push_back(member_plan(n[i], m[i], c[i], opts, b->gs));
    }
    b->nmax = b->np[0];
    b->nblk = b->nmax / 64;
    choose_lu_config(b);
    const int64_t small = b->mixed() ? feast::lu_small_max_order<c64>()
                                     : feast::lu_small_max_order<z64>();
    b->nbig = 0;
    while (b->nbig < P && b->np[b->nbig] > small) ++b->nbig;
    b->mmax = *std::max_element(b->m.begin(), b->m.end());
    b->dinv.alloc(sizeof(z64) * P * b->mblk() * 4096);
    b->flags.alloc(sizeof(int32_t) * 8 * P);
    int64_t pk_elems = 0;
    for (int64_t mp : b->m) pk_elems += 2 * mp * mp;
    b->pk.alloc(sizeof(z64) * pk_elems);
    b->sk.alloc(sizeof(z64) * kMaxSplits * pk_elems / 2);
    HIPCHK(hipHostMalloc(&b->pk_host, sizeof(z64) * pk_elems, hipHostMallocDefault));
    const int64_t nmat = static_cast<int64_t>(P) * N;
    const size_t esz = b->mixed() ? sizeof(c64) : sizeof(z64);
    b->F.alloc(esz * fo);
    b->piv.alloc(sizeof(int32_t) * nmat * b->nmax);
    b->perm.alloc(sizeof(int32_t) * nmat * b->nmax);
    b->info.alloc(sizeof(int32_t) * nmat);
    b->Linv.alloc(esz * nmat * b->istride());
    b->Uinv.alloc(esz * nmat * b->istride());
    // zero padding rows of the node solutions and the identity padding of the
    // shifted matrices (never touched again: the factorisation keeps it), all
    // ordered on the batch stream
    b->Y.alloc(sizeof(z64) * yo);
    HIPCHK(hipMemsetAsync(b->Y.p, 0, sizeof(z64) * yo, b->gs));
    if (b->mixed()) {
      b->Yc.alloc(sizeof(c64) * yo);
      HIPCHK(hipMemsetAsync(b->Yc.p, 0, sizeof(c64) * yo, b->gs));
      b->T1.alloc(sizeof(z64) * to);
      b->T2.alloc(sizeof(z64) * to);
    }
    HIPCHK(hipMemsetAsync(b->F.p, 0, esz * fo, b->gs));
    std::vector<GrpMat> g(P);
    for (int p = 0; p < P; ++p) {
      const int64_t ld = b->np[p];
      void *base = static_cast<char *>(b->F.p) + esz * b->foff[p];
      g[p] = GrpMat{base, ld, ld * ld, ld};
      if (b->mixed())
        feast::pad_diag<c64>(b->gs, static_cast<c64 *>(base), ld, ld * ld, N, b->n[p], ld);
      else
        feast::pad_diag<z64>(b->gs, static_cast<z64 *>(base), ld, ld * ld, N, b->n[p], ld);
    }
    b->grp.alloc(sizeof(GrpMat) * P);
    HIPCHK(hipMemcpy(b->grp.p, g.data(), sizeof(GrpMat) * P, hipMemcpyHostToDevice));
    // record the grouped GEMM tables of the factorisation and of a solve
    if (b->mixed()) {
      lu_grouped<c64>(b, true);
      trsolve_grouped<c64>(b, b->Yc.as<c64>());
    } else {
      lu_grouped<z64>(b, true);
      trsolve_grouped<z64>(b, b->Y.as<z64>());
    }
    b->lu_tab.upload();
    b->sv_tab.upload();
    HIPCHK(hipStreamSynchronize(b->gs));
    return FEAST_OK;
  });
  if (rc != FEAST_OK) {
    feast_batch_destroy(b);
    return rc;
  }
  *out = b;
  return FEAST_OK;
}

int feast_batch_destroy(feast_batch *b) {
  if (!b) return FEAST_OK;
  if (b->gs) (void)hipStreamSynchronize(b->gs);
  if (b->as) (void)hipStreamSynchronize(b->as);
  b->g_factor.reset();
  b->g_filter.reset();
  for (auto &e : b->proj_graphs) e.second->g.reset();
  b->proj_graphs.clear();
  for (feast_plan *p : b->sub) feast_plan_destroy(p);
  for (DevBuf *d : {&b->F, &b->piv, &b->perm, &b->info, &b->Linv, &b->Uinv, &b->grp, &b->Y, &b->Yc,
                    &b->T1, &b->T2, &b->lu_tab.dev, &b->sv_tab.dev, &b->dinv,
                    &b->flags, &b->pk, &b->sk, &b->fptab, &b->fpout})
    d->release();
  if (b->pk_host) (void)hipHostFree(b->pk_host);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ev_proj) (void)hipEventDestroy(b->ev_proj);
  if (b->gs) (void)hipStreamDestroy(b->gs);
  if (b->as) (void)hipStreamDestroy(b->as);
  delete b;
  return FEAST_OK;
}

int feast_batch_invalidate(feast_batch *b) {
  if (!b) return FEAST_EINVAL;
  b->factored = false;
  b->ffp.clear();
  return FEAST_OK;
}

const char *feast_batch_last_error(const feast_batch *b) { return b ? b->err.c_str() : "null batch"; }

int feast_batch_filter(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
                       const feast_z *const *dB, const int64_t *ldb, const feast_z *const *dV,
                       const int64_t *ldv, feast_z *const *dU, const int64_t *ldu, int32_t sweeps) {
  if (!b) return FEAST_EINVAL;
  if (!dA || !lda || !dB || !ldb || !dV || !ldv || !dU || !ldu || sweeps < 0 || sweeps > 16 ||
      (sweeps > 0 && !b->mixed()))
    return bfail(b, FEAST_EINVAL, "feast_batch_filter: bad argument");
  for (int i = 0; i < b->P; ++i) {
    const int p = b->where[i];
    if (!dA[i] || !dB[i] || !dV[i] || !dU[i] || lda[i] < b->n[p] || ldb[i] < b->n[p] ||
        ldv[i] < b->m[p] || ldu[i] < b->m[p])
      return bfail(b, FEAST_EINVAL, "feast_batch_filter: null pointer or leading dimension too small");
  }
  b->err.clear();
  return bguarded(b, [&]() -> int {
    enter(b);
    const int st = factor_all(b, dA, lda, dB, ldb);
    if (st != FEAST_OK) return st;
    rhs_all(b, dB, ldb, dV, ldv);
    filter_all(b, dA, lda, dB, ldb, sweeps);
    for (int p = 0; p < b->P; ++p) {
      const int c = b->order[p];
      feast::copy_block_z(b->gs, b->sub[p]->wblk(feast_plan::W_UF), b->m[p], b->n[p], b->m[p],
                          reinterpret_cast<z64 *>(dU[c]), ldu[c]);
    }
    leave(b);
    HIPCHK(hipGetLastError());
    return FEAST_OK;
  });
}

int feast_batch_solve(feast_batch *b, const feast_z *const *dA, const int64_t *lda,
                      const feast_z *const *dB, const int64_t *ldb, const feast_z *const *dV,
                      const int64_t *ldv, feast_z *const *hLambda, feast_z *const *dX,
                      const int64_t *ldx, double *const *hRes, int32_t *s_found, double *err,
                      int32_t *flag, int32_t *iters, feast_batch_info *info) {
  if (!b) return FEAST_EINVAL;
  if (!dA || !lda || !dB || !ldb || !dV || !ldv || !hLambda || !dX || !ldx || !s_found || !err ||
      !flag || !iters)
    return bfail(b, FEAST_EINVAL, "feast_batch_solve: null argument array");
  for (int i = 0; i < b->P; ++i) {
    const int p = b->where[i];
    if (!dA[i] || !dB[i] || !dV[i] || !dX[i] || !hLambda[i] || lda[i] < b->n[p] ||
        ldb[i] < b->n[p] || ldv[i] < b->m[p] || ldx[i] < b->m[p])
      return bfail(b, FEAST_EINVAL, "feast_batch_solve: null pointer or leading dimension too small");
  }
  b->err.clear();
  return bguarded(b, [&]() -> int {
    const int P = b->P;
    hipStream_t s = b->gs;
    feast_batch_info inf{};
    Timer total;
    enter(b);
    {
      Timer t;
      const int st = factor_all(b, dA, lda, dB, ldb);
      inf.t_factor_ms = t.ms();
      if (st != FEAST_OK) return st;
    }
    // per-pencil state of Algorithm 5
    struct St {
      bool done = false;
      int c_prev = 0;
      double e_prev = 0.0;
      std::vector<cd> lam_prev;
      std::vector<double> r_prev;
      std::vector<feast_z> Yh, alpha, beta, lam;
      std::vector<double> hn;
    };
    std::vector<St> st(P);
    for (int p = 0; p < P; ++p) {
      const int64_t m = b->m[p];
      st[p].Yh.resize(m * m);
      st[p].alpha.resize(m);
      st[p].beta.resize(m);
      st[p].lam.resize(m);
      st[p].hn.resize(3 * m);
    }
    int sweeps = 0;       // mixed form: corrections per node of the next filter
    int base_sweeps = 0;  // (none on Search's filter)
    auto grouped_filter = [&]() {
      Timer t;
      filter_all(b, dA, lda, dB, ldb, b->mixed() ? sweeps : 0);
      HIPCHK(hipStreamSynchronize(s));
      inf.t_filter_ms += t.ms();
      inf.filters += 1;
    };
    std::vector<std::vector<feast_z>> hAt(P), hBt(P);
    for (int p = 0; p < P; ++p) {
      hAt[p].resize(b->m[p] * b->m[p]);
      hBt[p].resize(b->m[p] * b->m[p]);
    }
    auto project_active = [&]() -> int {
      Timer t;
      std::vector<int> act;
      for (int p = 0; p < P; ++p)
        if (!st[p].done) act.push_back(p);
      const int r = project_grouped(b, act, dA, lda, dB, ldb, hAt, hBt);
      inf.t_project_ms += t.ms();
      return r;
    };
    // Search with the subspace size fixed: U = Q_N V
    rhs_all(b, dB, ldb, dV, ldv);
    grouped_filter();
    {
      const int r = project_active();
      if (r != FEAST_OK) return r;
    }
    const int nthreads =
        static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    for (int k = 1; k <= b->o.max_iter; ++k) {
      // filter step of the first iteration ahead of time: the next filter needs
      // only B U_1, so it runs on gs while the host solves the reduced pencils
      // and the Ritz vectors and residuals go to the second stream (a pencil
      // that stops at k = 1 has its filter computed for nothing; the grouped
      // filter covers every pencil anyway).  Later iterations, usually the
      // last, run in order.
      const bool spec = (k == 1);
      hipStream_t rs = s;
      if (spec) {
        Timer tf;
        HIPCHK(hipEventRecord(b->ev_proj, s));
        HIPCHK(hipStreamWaitEvent(b->as, b->ev_proj, 0));
        rs = b->as;
        for (int p = 0; p < P; ++p)
          if (!st[p].done)
            feast::copy_block_z(s, b->sub[p]->wblk(feast_plan::W_BU1), b->m[p], b->n[p], b->m[p],
                                b->sub[p]->R.as<z64>(), b->m[p]);
        if (b->mixed()) base_sweeps = 1;  // (the first refined filter: one correction)
        sweeps = b->mixed() ? base_sweeps : 0;
        filter_all(b, dA, lda, dB, ldb, sweeps);
        inf.filters += 1;
        inf.t_filter_ms += tf.ms();
      }
      // reduced eigenproblem of every active pencil, in parallel on the host
      Timer te;
      std::vector<int> act;
      for (int p = 0; p < P; ++p)
        if (!st[p].done) act.push_back(p);
      std::vector<int> qz(P, 0);
      parallel_for(static_cast<int>(act.size()), nthreads, [&](int i) {
        const int p = act[i];
        const int64_t m = b->m[p];
        const feast_contour &cp = b->sub[p]->c;
        const cd gam(cp.center.re, cp.center.im);
        qz[p] = feast_host::reduced_eig(m, reinterpret_cast<const cd *>(hAt[p].data()), m,
                                        reinterpret_cast<const cd *>(hBt[p].data()), m,
                                        reinterpret_cast<cd *>(st[p].alpha.data()),
                                        reinterpret_cast<cd *>(st[p].beta.data()),
                                        reinterpret_cast<cd *>(st[p].Yh.data()), m, 1, &gam,
                                        cp.radius);
      });
      inf.t_host_eig_ms += te.ms();
      for (int p : act)
        if (qz[p] != 0) return bfail(b, FEAST_ENUMERIC, "reduced QZ did not converge in pencil " +
                                                          std::to_string(b->order[p]));
      // Ritz vectors and the norms of eq. 5-1 on the device: the products
      // X = U_1 Y, A X = (A U_1) Y, B X = (B U_1) Y of every pencil in one
      // grouped launch once the Y blocks are on the device
      std::vector<std::vector<cd>> lam(P);
      std::vector<GemmArgs<z64>> ritz;
      for (int p : act) {
        feast_plan *q = b->sub[p];
        const int64_t n = b->n[p], m = b->m[p];
        lam[p].resize(m);
        for (int64_t i = 0; i < m; ++i) {
          const cd a(st[p].alpha[i].re, st[p].alpha[i].im), be(st[p].beta[i].re, st[p].beta[i].im);
          lam[p][i] = (be != cd(0.0)) ? a / be : cd(INFINITY, 0.0);
          st[p].lam[i] = std::isfinite(lam[p][i].real()) ? feast_z{lam[p][i].real(), lam[p][i].imag()}
                                                         : feast_z{0, 0};
        }
        z64 *Ys = q->gblk(feast_plan::G_YS), *dlam = q->small.as<z64>();
        HIPCHK(hipMemcpyAsync(Ys, st[p].Yh.data(), sizeof(z64) * m * m, hipMemcpyHostToDevice, rs));
        HIPCHK(hipMemcpyAsync(dlam, st[p].lam.data(), sizeof(z64) * m, hipMemcpyHostToDevice, rs));
        const z64 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
        for (const int w : {int(feast_plan::W_U1), int(feast_plan::W_AU1), int(feast_plan::W_BU1)}) {
          const int out = w == feast_plan::W_U1 ? feast_plan::W_X
                                                : (w == feast_plan::W_AU1 ? feast_plan::W_AX : feast_plan::W_BX);
          ritz.push_back(GemmArgs<z64>{n, m, m, q->wblk(w), m, 0, Ys, m, 0, q->wblk(out), m, 0, one,
                                       zero, 1, 1, m, nullptr, 0});
        }
      }
      grouped_on(b->ritz_tab, rs, ritz);
      for (int p : act) {
        feast_plan *q = b->sub[p];
        const int64_t n = b->n[p], m = b->m[p];
        feast::ritz_norms(rs, q->wblk(feast_plan::W_AX), q->wblk(feast_plan::W_BX), m, n, m,
                          q->small.as<z64>(), q->part.as<double>(), q->nrm.as<double>());
        HIPCHK(hipMemcpyAsync(st[p].hn.data(), q->nrm.p, sizeof(double) * 3 * m,
                              hipMemcpyDeviceToHost, rs));
      }
      HIPCHK(hipStreamSynchronize(rs));
      // selection and stopping rules per pencil
      bool refine_more = false;
      for (int p : act) {
        feast_plan *q = b->sub[p];
        const int c = b->order[p];
        const int64_t n = b->n[p], m = b->m[p];
        const cd gamma(q->c.center.re, q->c.center.im);
        std::vector<int32_t> sel;
        std::vector<double> rsel;
        double e_k = 0.0;
        for (int64_t i = 0; i < m; ++i) {
          if (!std::isfinite(lam[p][i].real()) || !std::isfinite(lam[p][i].imag())) continue;
          const double den = std::sqrt(st[p].hn[3 * i + 1]) + std::sqrt(st[p].hn[3 * i + 2]);
          const double r = den > 0.0 ? std::sqrt(st[p].hn[3 * i]) / den : INFINITY;
          if (std::abs(lam[p][i] - gamma) < q->c.radius && r < b->o.eta) {
            sel.push_back(static_cast<int32_t>(i));
            rsel.push_back(r);
            e_k = std::max(e_k, r);
          }
        }
        const int c_k = static_cast<int>(sel.size());
        if (c_k == 0) e_k = INFINITY;
        // mixed form: a rise of e(k) while the grouped sweep count can still
        // grow is taken as the solves limiting the accuracy (one more sweep,
        // below), not as the no-improvement stop
        int a = feast_host::stop_rule(k, c_k, e_k, st[p].c_prev, st[p].e_prev, b->o.eps,
                                      b->o.max_iter);
        if (a == 0 && b->mixed() && base_sweeps < b->o.max_sweeps) a = 2;
        int32_t *didx = reinterpret_cast<int32_t *>(q->small.as<z64>() + m);
        if (a == 1 || a == -1) {
          if (c_k > 0) {
            HIPCHK(hipMemcpy(didx, sel.data(), sizeof(int32_t) * c_k, hipMemcpyHostToDevice));
            feast::gather_normalize_cols(rs, q->wblk(feast_plan::W_X), m, n, didx, c_k,
                                         reinterpret_cast<z64 *>(dX[c]), ldx[c], nullptr);
            HIPCHK(hipStreamSynchronize(rs));
          }
          for (int i = 0; i < c_k; ++i) {
            hLambda[c][i] = {lam[p][sel[i]].real(), lam[p][sel[i]].imag()};
            if (hRes && hRes[c]) hRes[c][i] = rsel[i];
          }
          s_found[c] = c_k;
          err[c] = e_k;
          flag[c] = a;
          iters[c] = k;
          st[p].done = true;
          continue;
        }
        if (a == 0) {
          const int cp = static_cast<int>(st[p].lam_prev.size());
          feast::copy_block_z(rs, q->wblk(feast_plan::W_XPREV), m, n, cp,
                              reinterpret_cast<z64 *>(dX[c]), ldx[c]);
          for (int i = 0; i < cp; ++i) {
            hLambda[c][i] = {st[p].lam_prev[i].real(), st[p].lam_prev[i].imag()};
            if (hRes && hRes[c]) hRes[c][i] = st[p].r_prev[i];
          }
          s_found[c] = cp;
          err[c] = st[p].e_prev;
          flag[c] = 0;
          iters[c] = k;
          st[p].done = true;
          continue;
        }
        // keep iterate k for a possible rebound at k+1
        st[p].lam_prev.clear();
        st[p].r_prev = rsel;
        for (int i = 0; i < c_k; ++i) st[p].lam_prev.push_back(lam[p][sel[i]]);
        if (c_k > 0) {
          HIPCHK(hipMemcpy(didx, sel.data(), sizeof(int32_t) * c_k, hipMemcpyHostToDevice));
          feast::gather_normalize_cols(rs, q->wblk(feast_plan::W_X), m, n, didx, c_k,
                                       q->wblk(feast_plan::W_XPREV), m, nullptr);
        }
        if (b->mixed() && k >= 2 && c_k == st[p].c_prev && e_k >= b->o.eps &&
            e_k > 0.5 * st[p].e_prev)
          refine_more = true;
        st[p].e_prev = e_k;
        st[p].c_prev = c_k;
      }
      // (the second stream's gathers and copies of this iteration are done
      // before the results are returned or the next projection overwrites U_1)
      if (rs != s) HIPCHK(hipStreamSynchronize(rs));
      inf.iters = k;
      bool any = false;
      for (int p = 0; p < P; ++p) any = any || !st[p].done;
      if (!any) break;
      // filter step for the pencils still iterating (one grouped filter), QR step
      // mixed form: as feast_solve, one grouped sweep count for all pencils --
      // refined once any pencil still iterating has e(k) <= 1e-4 (or on the
      // first filter after Search), one more on a stall
      if (spec) {
        Timer tw;
        HIPCHK(hipStreamSynchronize(s));  // the filter launched ahead
        inf.t_filter_ms += tw.ms();
      } else {
        int sweeps_now = 0;
        if (b->mixed()) {
          if (base_sweeps == 0) base_sweeps = 1;
          else if (refine_more && base_sweeps < b->o.max_sweeps) ++base_sweeps;
          bool close = false;
          for (int p = 0; p < P; ++p)
            if (!st[p].done && std::isfinite(st[p].e_prev) && st[p].e_prev <= 1e-4) close = true;
          sweeps_now = close ? base_sweeps : 0;
        }
        sweeps = sweeps_now;
        for (int p = 0; p < P; ++p)
          if (!st[p].done)
            feast::copy_block_z(s, b->sub[p]->wblk(feast_plan::W_BU1), b->m[p], b->n[p], b->m[p],
                                b->sub[p]->R.as<z64>(), b->m[p]);
        grouped_filter();
      }
      const int r = project_active();
      if (r != FEAST_OK) return r;
    }
    leave(b);
    HIPCHK(hipStreamSynchronize(s));
    inf.t_total_ms = total.ms();
    inf.graph_launches = b->launches;
    if (info) *info = inf;
    return FEAST_OK;
  });
}

}  // extern "C"
