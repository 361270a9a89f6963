// Internal plan of the single-pencil driver and helpers shared with the
// batched driver.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/feast.h"
#include "kernels.h"

using feast::c64;
using feast::z64;
using cd = std::complex<double>;

namespace feast_drv {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

inline z64 zc(double r, double i = 0.0) { return make_double2(r, i); }

struct HipError {
  hipError_t e;
  const char *what;
};

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) throw HipError{e_, #x};   \
  } while (0)

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void alloc(size_t b) {
    if (bytes >= b && p) return;
    release();
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      bytes = 0;
      throw HipError{e, "hipMalloc"};
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

}  // namespace feast_drv

using feast_drv::DevBuf;

struct feast_plan {
  int64_t n = 0, m = 0;
  int N = 0;
  feast_contour c{};
  feast_opts o{};
  hipStream_t s = nullptr;
  int nb = 64;
  int64_t nblk = 0;
  std::vector<cd> hz, hw;
  DevBuf dz, dw, dwc;  // nodes, weights, conjugated weights
  // cached factors
  // The factors are reused for a pencil whose content fingerprints (A, B)
  // equal those taken when they were computed: the same shifted matrices,
  // wherever A and B now live.
  bool factored = false;
  uint64_t fpA = 0, fpB = 0;
  DevBuf fp;  // device fingerprints of the current call's A and B
  bool checked = false;  // within one entry-point call: the factors were checked (or made)
  DevBuf F, piv, perm, info, Linv, Uinv;
  DevBuf Linv2, Uinv2;  // inverted 128 x 128 diagonal blocks (the solves' leaves)
  double normA = 0.0, normB = 0.0;  // Frobenius norms of A and B (refinement test)
  // workspaces
  DevBuf R, Y, T1, T2, Yc, W, G, splitws, splitws2, part, nrm, flag, small;
  DevBuf rn;  // mixed form: ||R||_F^2 at rn[0] (scale of the complex64 solves), ||d_1||^2 and
              // ||Y_0||^2 of the first correction at rn[1], rn[2]; partials from rn[8]
  double *hrn = nullptr;   // page-locked copy of rn[0..3) (read after the stream is idle)
  bool rho_pending = false;  // hrn holds a filter's first-correction norms not yet read
  DevBuf adj, adj_piv, adj_info, adj_inv;  // adjoint solves (allocated on first use)
  // sparse pencil of the running feast_solve_csr call: the union pattern of A
  // and B reordered by reverse Cuthill-McKee (row new holds old row perm[new]),
  // A's and B's values on it, and the band factors of every node
  struct Sparse {
    bool on = false;
    int kl = 0, ku = 0;
    int64_t nnz = 0;
    DevBuf rp, ci, va, vb, map, perm;
    DevBuf Lf, Uf, Dinv, piv, info;
    DevBuf V, X;  // start block and eigenvector block in the new order
    // the patterns the device ordering (rp, ci, map, perm, kl, ku) was made
    // for: a later call with the same patterns reuses it
    bool ordered = false;
    std::vector<int32_t> keyA_rp, keyA_ci, keyB_rp, keyB_ci;
  } sp;
  DevBuf cirr_w;                           // Block_CIRR moment weights (g x N)
  std::string err;
  int last_sweeps = 0;       // mixed form: sweeps of the last filter
  double last_be = 0.0;      // mixed form: worst node backward error of the last filter
  bool stagnated = false;    // mixed form: the last filter missed its target
  // opts.profile: events around the LU trailing-update GEMMs
  std::vector<hipEvent_t> ev;
  hipStream_t side = nullptr;                 // look-ahead panel stream
  int cus = 256;                              // compute units of the plan's device
  hipStream_t aux = nullptr;                  // Ritz vectors/residuals overlapping a filter
  hipEvent_t ev_cols = nullptr, ev_panel = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;  // A U_1 on the side stream in the projection
  int prof_launches = 0;
  double prof_ms = 0.0, prof_flops = 0.0;
  // opts.profile: events around the bandwidth-bound launches (class, algorithmic bytes)
  struct KRec {
    int cls;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> kev;
  size_t kev_used = 0;
  std::vector<KRec> krec;

  // n x m work blocks inside W
  enum { W_ORTH = 0, W_U2 = 1, W_X = 2, W_AX = 3, W_BX = 4, W_XPREV = 5, W_U1 = 6, W_AU1 = 7,
         W_BU1 = 8, W_UF = 9, W_COUNT = 10 };
  // m x m blocks inside G
  enum { G_GRAM = 0, G_RINV = 1, G_T = 2, G_AT = 3, G_BT = 4, G_YS = 5, G_COUNT = 6 };
  z64 *wblk(int i) const { return W.as<z64>() + static_cast<int64_t>(i) * n * m; }
  z64 *gblk(int i) const { return G.as<z64>() + static_cast<int64_t>(i) * m * m; }

  bool mixed() const { return o.prec == FEAST_MIXED; }
  int64_t ldY() const { return static_cast<int64_t>(N) * m; }
  int64_t fstride() const { return n * n; }
  int64_t istride() const { return nblk * 64 * 64; }  // inverted 64 x 64 diagonal blocks
  int64_t istride2() const { return ((n + 127) / 128) * 128 * 128; }  // 128 x 128 ones
};


namespace feast_drv {

int fail(feast_plan *p, int code, const std::string &msg);

// C = alpha op(A) B + beta C on the MFMA GEMM (T = z64 or c64).
template <typename T>
void gemm_t(hipStream_t s, int ta, int64_t M, int64_t N, int64_t K, z64 alpha, const T *A,
            int64_t lda, int64_t sA, const T *B, int64_t ldb, int64_t sB, z64 beta, T *C,
            int64_t ldc, int64_t sC, int32_t batch, T *work = nullptr, int64_t welems = 0,
            int cfg = feast::GEMM_SQUARE);
template <>
void gemm_t<z64>(hipStream_t s, int ta, int64_t M, int64_t N, int64_t K, z64 alpha, const z64 *A,
                 int64_t lda, int64_t sA, const z64 *B, int64_t ldb, int64_t sB, z64 beta, z64 *C,
                 int64_t ldc, int64_t sC, int32_t batch, z64 *work, int64_t welems, int cfg);
template <>
void gemm_t<c64>(hipStream_t s, int ta, int64_t M, int64_t N, int64_t K, z64 alpha, const c64 *A,
                 int64_t lda, int64_t sA, const c64 *B, int64_t ldb, int64_t sB, z64 beta, c64 *C,
                 int64_t ldc, int64_t sC, int32_t batch, c64 *work, int64_t welems, int cfg);

// Workspaces of a plan (with_nodes = false: only the n x m and m x m blocks,
// not the n x N m node solutions).
void ensure_workspace(feast_plan *p, bool with_nodes = true);
int64_t splitws_elems(const feast_plan *p);

// Shifted CholeskyQR3 of the n x m block X in place (flags at flag_slot..+2).
void orth(feast_plan *p, z64 *X, int64_t ldx, int flag_slot, int64_t cols = -1);
// Algorithm 5's QR steps and reduced pencil on the device: U -> U_1, A U_1, B U_1, U_2, At, Bt.
void project_device(feast_plan *p, const z64 *A, int64_t lda, const z64 *B, int64_t ldb, z64 *U,
                    int64_t ldu, z64 *AU1, int64_t ldau, z64 *BU1, int64_t ldbu);
// Copy At, Bt to the host and check the Cholesky QR flags (synchronises).
int project_finish(feast_plan *p, feast_z *hAt, feast_z *hBt);
bool bad_contour(const feast_contour *c);
// Host threads for the reduced eigensolver (at most 16).
int host_threads();

// Runs f(), turning HIP and allocation failures into FEAST status codes.
template <typename F> int guarded(feast_plan *p, F &&f) {
  try {
    return f();
  } catch (const HipError &e) {
    if (p) {
      p->err = std::string(e.what) + ": " + hipGetErrorString(e.e);
      p->factored = false;
    }
    return e.e == hipErrorOutOfMemory ? FEAST_ENOMEM : FEAST_EDEVICE;
  } catch (const std::bad_alloc &) {
    if (p) p->err = "host allocation failed";
    return FEAST_ENOMEM;
  } catch (...) {
    if (p) p->err = "unexpected exception";
    return FEAST_EDEVICE;
  }
}


// One entry-point call: A and B cannot change while it runs, so the cached
// factors are checked against them once per call.
struct CheckScope {
  feast_plan *p;
  explicit CheckScope(feast_plan *q) : p(q) { p->checked = false; }
  ~CheckScope() { p->checked = false; }
};

// With opts.profile, launch() is bracketed by HIP events on the plan's stream
// and recorded under class cls (enum feast_kclass) with its algorithmic HBM
// bytes; otherwise it just runs.
template <class F> void ktimed(feast_plan *p, int cls, double bytes, F &&launch) {
  if (!p->o.profile || p->krec.size() >= 4096) {
    launch();
    return;
  }
  while (p->kev.size() < p->kev_used + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    p->kev.push_back(e);
  }
  hipEvent_t a = p->kev[p->kev_used], b = p->kev[p->kev_used + 1];
  p->kev_used += 2;
  HIPCHK(hipEventRecord(a, p->s));
  launch();
  HIPCHK(hipEventRecord(b, p->s));
  p->krec.push_back({cls, bytes, a, b});
}
void kprof_reset(feast_plan *p);
// Sum the recorded launches per class into info (the stream must be idle).
void kprof_collect(feast_plan *p, feast_info *info);

}  // namespace feast_drv
