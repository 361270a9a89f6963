// Host solver of the reduced t x t pencil  At y = lambda Bt y  (Algorithm 5's
// reduced eigenproblem; Section 3 names LAPACK's xGGES/xGGEV for this step).  When Bt is
// upper triangular and well conditioned -- the method's B~ equals R_2 of the
// QR of B U_1 -- the standard problem Bt^{-1} At is solved (std_eig below).
// Otherwise it is a from-scratch complex QZ:
//   1. Bt -> upper triangular by Givens rotations from the left (applied to At);
//   2. Hessenberg-triangular reduction of (At, Bt) (row rotations from the left,
//      column rotations from the right, the right ones accumulated in Z);
//   3. single-shift complex QZ iteration with deflation of negligible
//      subdiagonal entries of the Hessenberg matrix and of zero diagonal
//      entries of the triangular one (infinite eigenvalues);
//   4. right eigenvectors of the triangular pencil (S, P) by back substitution,
//      mapped back with Z and normalised to unit 2-norm.
// Left rotations never need to be stored: right eigenvectors only depend on Z.
//
// Storage is column-major std::complex<double> inside this file.
#include "host_eig.h"

#include <algorithm>
#include <immintrin.h>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <limits>
#include <thread>
#include <vector>

namespace feast_host {

using cd = std::complex<double>;

namespace {

constexpr double kUlp = std::numeric_limits<double>::epsilon();
constexpr double kSafmin = std::numeric_limits<double>::min();

struct Mat {
  int64_t n, ld;
  std::vector<cd> a;
  // columns 64-byte aligned and an odd number of cache lines apart, so that a
  // walk along a row (the QR sweeps' row rotations) spreads over all cache
  // sets: with ld = n = 256 every column of a row falls in the same set
  explicit Mat(int64_t n_)
      : n(n_), ld(4 * (2 * ((n_ + 7) / 8) + 1)), a(static_cast<size_t>(ld * n_)) {}
  cd &operator()(int64_t i, int64_t j) { return a[static_cast<size_t>(j * ld + i)]; }
  cd operator()(int64_t i, int64_t j) const { return a[static_cast<size_t>(j * ld + i)]; }
  cd *col(int64_t j) { return a.data() + j * ld; }
  const cd *col(int64_t j) const { return a.data() + j * ld; }
};

// Plane rotation G = [c s; -conj(s) c] with G [f; g] = [r; 0], c real >= 0.
inline void rot_gen(cd f, cd g, double &c, cd &s, cd &r) {
  const double ga = std::abs(g);
  if (ga == 0.0) {
    c = 1.0;
    s = 0.0;
    r = f;
    return;
  }
  const double fa = std::abs(f);
  if (fa == 0.0) {
    c = 0.0;
    s = std::conj(g) / ga;
    r = ga;
    return;
  }
  const double d = std::hypot(fa, ga);
  c = fa / d;
  const cd ph = f / fa;
  s = ph * std::conj(g) / d;
  r = ph * d;
}

// Rows (p, q) <- G [row p; row q] over columns [j0, j1).
inline void rot_rows(Mat &M, int64_t p, int64_t q, int64_t j0, int64_t j1, double c, cd s) {
  const cd sc = std::conj(s);
  for (int64_t j = j0; j < j1; ++j) {
    cd &x = M(p, j);
    cd &y = M(q, j);
    const cd xv = x, yv = y;
    x = c * xv + s * yv;
    y = -sc * xv + c * yv;
  }
}

// Columns (p, q) <- [col p, col q] W with W = [c conj(s); -s c] over rows [i0, i1).
// Built from rot_gen(conj(M(i,q)), conj(M(i,p))) it zeroes M(i, p).
inline void rot_cols(Mat &M, int64_t p, int64_t q, int64_t i0, int64_t i1, double c, cd s) {
  const cd sc = std::conj(s);
  cd *cp = M.col(p);
  cd *cq = M.col(q);
  for (int64_t i = i0; i < i1; ++i) {
    const cd xv = cp[i], yv = cq[i];
    cp[i] = c * xv - s * yv;
    cq[i] = sc * xv + c * yv;
  }
}

// Rotation zeroing M(i, p) against M(i, q) by a right rotation of columns p, q.
inline void col_rot_for(const Mat &M, int64_t i, int64_t p, int64_t q, double &c, cd &s) {
  cd r;
  rot_gen(std::conj(M(i, q)), std::conj(M(i, p)), c, s, r);
}

double fro(const Mat &M) {
  double s = 0.0;
  for (const cd &v : M.a) s += std::norm(v);
  return std::sqrt(s);
}

// Eigenvalue of the 2x2 pencil (H, T) at rows/cols (k, k+1) closest to h22/t22.
cd wilkinson_shift(const Mat &H, const Mat &T, int64_t k) {
  const cd h11 = H(k, k), h12 = H(k, k + 1), h21 = H(k + 1, k), h22 = H(k + 1, k + 1);
  const cd t11 = T(k, k), t12 = T(k, k + 1), t22 = T(k + 1, k + 1);
  // det(Hb - lam Tb) = a lam^2 + b lam + c0 with t21 = 0
  const cd a = t11 * t22;
  const cd b = -(h11 * t22 + h22 * t11 - h21 * t12);
  const cd c0 = h11 * h22 - h12 * h21;
  const cd target = h22 / t22;
  if (std::abs(a) == 0.0) return target;
  const cd disc = std::sqrt(b * b - 4.0 * a * c0);
  cd q = (std::real(std::conj(b) * disc) >= 0.0) ? -0.5 * (b + disc) : -0.5 * (b - disc);
  cd r1 = (std::abs(q) > 0.0) ? c0 / q : target;
  cd r2 = q / a;
  return (std::abs(r1 - target) <= std::abs(r2 - target)) ? r1 : r2;
}

}  // namespace

namespace {

// General pencil: complex QZ (steps 1-4 of the file comment).
int qz_eig(int64_t t, const cd *At, int64_t lda, const cd *Bt, int64_t ldb, cd *alpha, cd *beta,
           cd *Y, int64_t ldy, int nthreads) {
  if (t <= 0) return 0;
  Mat H(t), T(t), Z(t);
  for (int64_t i = 0; i < t; ++i)
    for (int64_t j = 0; j < t; ++j) {
      H(i, j) = At[i * lda + j];
      T(i, j) = Bt[i * ldb + j];
      Z(i, j) = (i == j) ? cd(1.0) : cd(0.0);
    }
  for (const cd &v : H.a)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return -1;
  for (const cd &v : T.a)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return -1;

  // 1. T -> upper triangular (left rotations, also applied to H).
  for (int64_t j = 0; j + 1 < t; ++j) {
    for (int64_t i = t - 1; i > j; --i) {
      if (T(i, j) == cd(0.0)) continue;
      double c;
      cd s, r;
      rot_gen(T(i - 1, j), T(i, j), c, s, r);
      rot_rows(T, i - 1, i, j, t, c, s);
      T(i, j) = 0.0;
      rot_rows(H, i - 1, i, 0, t, c, s);
    }
  }
  // 2. Hessenberg-triangular reduction.
  for (int64_t j = 0; j + 2 < t; ++j) {
    for (int64_t i = t - 1; i >= j + 2; --i) {
      if (H(i, j) == cd(0.0)) continue;
      double c;
      cd s, r;
      rot_gen(H(i - 1, j), H(i, j), c, s, r);
      rot_rows(H, i - 1, i, j, t, c, s);
      H(i, j) = 0.0;
      rot_rows(T, i - 1, i, i - 1, t, c, s);
      // T(i, i-1) is now filled: zero it with a column rotation of (i-1, i).
      col_rot_for(T, i, i - 1, i, c, s);
      rot_cols(T, i - 1, i, 0, i + 1, c, s);
      T(i, i - 1) = 0.0;
      rot_cols(H, i - 1, i, 0, t, c, s);
      rot_cols(Z, i - 1, i, 0, t, c, s);
    }
  }

  // 3. QZ iteration.
  const double hnorm = fro(H), tnorm = fro(T);
  const double atol = std::max(kSafmin, kUlp * hnorm);
  const double btol = std::max(kSafmin, kUlp * tnorm);
  int64_t ilast = t - 1;
  int64_t since = 0;
  const int64_t maxit = 40 * t + 100;
  int64_t it = 0;
  cd eshift = 0.0;
  while (ilast >= 0) {
    if (++it > maxit) return -2;
    // (a) deflation of a negligible subdiagonal at the bottom
    if (ilast == 0) {
      ilast = -1;
      break;
    }
    {
      const double h = std::abs(H(ilast, ilast - 1));
      if (h <= atol ||
          h <= kUlp * (std::abs(H(ilast, ilast)) + std::abs(H(ilast - 1, ilast - 1)))) {
        H(ilast, ilast - 1) = 0.0;
        --ilast;
        since = 0;
        eshift = 0.0;
        continue;
      }
    }
    // (b) infinite eigenvalue at the bottom: T(ilast, ilast) negligible
    if (std::abs(T(ilast, ilast)) <= btol) {
      T(ilast, ilast) = 0.0;
      double c;
      cd s;
      col_rot_for(H, ilast, ilast - 1, ilast, c, s);
      rot_cols(H, ilast - 1, ilast, 0, ilast + 1, c, s);
      H(ilast, ilast - 1) = 0.0;
      rot_cols(T, ilast - 1, ilast, 0, ilast, c, s);
      rot_cols(Z, ilast - 1, ilast, 0, t, c, s);
      --ilast;
      since = 0;
      eshift = 0.0;
      continue;
    }
    // (c) find the top of the unreduced block
    int64_t ifirst = 0;
    for (int64_t j = ilast - 1; j >= 1; --j) {
      const double h = std::abs(H(j, j - 1));
      if (h <= atol || h <= kUlp * (std::abs(H(j, j)) + std::abs(H(j - 1, j - 1)))) {
        H(j, j - 1) = 0.0;
        ifirst = j;
        break;
      }
    }
    // (d) zero diagonal of T inside the block: chase it to the bottom
    int64_t jz = -1;
    for (int64_t j = ifirst; j < ilast; ++j)
      if (std::abs(T(j, j)) <= btol) {
        jz = j;
        break;
      }
    if (jz >= 0) {
      T(jz, jz) = 0.0;
      for (int64_t k = jz; k < ilast; ++k) {
        double c;
        cd s, r;
        rot_gen(T(k, k + 1), T(k + 1, k + 1), c, s, r);
        rot_rows(T, k, k + 1, k + 1, t, c, s);
        T(k + 1, k + 1) = 0.0;
        const int64_t h0 = (k > ifirst) ? k - 1 : k;
        rot_rows(H, k, k + 1, h0, t, c, s);
        if (k > ifirst) {
          // fill at H(k+1, k-1): zero it with columns (k-1, k)
          col_rot_for(H, k + 1, k - 1, k, c, s);
          rot_cols(H, k - 1, k, 0, k + 2, c, s);
          H(k + 1, k - 1) = 0.0;
          rot_cols(T, k - 1, k, 0, k + 1, c, s);
          rot_cols(Z, k - 1, k, 0, t, c, s);
        }
      }
      continue;  // (b) deflates the bottom next
    }
    // (e) one implicit single-shift QZ sweep on [ifirst, ilast]
    ++since;
    cd sigma;
    if (since % 10 == 0) {
      // exceptional shift
      eshift += H(ilast, ilast - 1) / T(ilast - 1, ilast - 1);
      sigma = eshift;
    } else {
      sigma = wilkinson_shift(H, T, ilast - 1);
    }
    {
      double c;
      cd s, r;
      const cd x = H(ifirst, ifirst) - sigma * T(ifirst, ifirst);
      const cd y = H(ifirst + 1, ifirst);
      rot_gen(x, y, c, s, r);
      rot_rows(H, ifirst, ifirst + 1, ifirst, t, c, s);
      rot_rows(T, ifirst, ifirst + 1, ifirst, t, c, s);
    }
    for (int64_t k = ifirst; k < ilast; ++k) {
      double c;
      cd s, r;
      // restore T: zero T(k+1, k) with columns (k, k+1)
      col_rot_for(T, k + 1, k, k + 1, c, s);
      rot_cols(T, k, k + 1, 0, k + 2, c, s);
      T(k + 1, k) = 0.0;
      rot_cols(H, k, k + 1, 0, std::min(k + 3, t), c, s);
      rot_cols(Z, k, k + 1, 0, t, c, s);
      if (k + 2 <= ilast) {
        // restore H: zero H(k+2, k) with rows (k+1, k+2)
        rot_gen(H(k + 1, k), H(k + 2, k), c, s, r);
        rot_rows(H, k + 1, k + 2, k, t, c, s);
        H(k + 2, k) = 0.0;
        rot_rows(T, k + 1, k + 2, k + 1, t, c, s);
      }
    }
  }

  // 4. eigenvalues and right eigenvectors
  for (int64_t j = 0; j < t; ++j) {
    alpha[j] = H(j, j);
    beta[j] = T(j, j);
  }
  auto eigvec = [&](int64_t j, std::vector<cd> &v, std::vector<cd> &x) {
    cd a = H(j, j), b = T(j, j);
    const double sc = std::max(std::abs(a), std::abs(b));
    if (sc > 0.0) {
      a /= sc;
      b /= sc;
    } else {
      b = 1.0;
    }
    std::fill(v.begin(), v.end(), cd(0.0));
    v[j] = 1.0;
    const double small = std::max(kSafmin, kUlp * (std::abs(b) * hnorm + std::abs(a) * tnorm));
    for (int64_t k = j - 1; k >= 0; --k) {
      cd acc = 0.0;
      for (int64_t l = k + 1; l <= j; ++l) acc += (b * H(k, l) - a * T(k, l)) * v[l];
      cd d = b * H(k, k) - a * T(k, k);
      if (std::abs(d) < small) d = small;
      v[k] = -acc / d;
      // guard against growth: rescale the partial vector
      const double m = std::abs(v[k]);
      if (m > 1e100) {
        for (int64_t l = k; l <= j; ++l) v[l] /= m;
      }
    }
    std::fill(x.begin(), x.end(), cd(0.0));
    for (int64_t l = 0; l <= j; ++l) {
      const cd vl = v[l];
      if (vl == cd(0.0)) continue;
      const cd *zc = Z.col(l);
      for (int64_t i = 0; i < t; ++i) x[i] += zc[i] * vl;
    }
    double nr = 0.0;
    for (const cd &e : x) nr += std::norm(e);
    nr = std::sqrt(nr);
    if (nr > 0.0)
      for (cd &e : x) e /= nr;
    for (int64_t i = 0; i < t; ++i) Y[i * ldy + j] = x[i];
  };
  const int nt = std::max(1, std::min<int>(nthreads, static_cast<int>((t + 31) / 32)));
  if (nt == 1) {
    std::vector<cd> v(t), x(t);
    for (int64_t j = 0; j < t; ++j) eigvec(j, v, x);
  } else {
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
      th.emplace_back([&, w]() {
        std::vector<cd> v(t), x(t);
        for (int64_t j = w; j < t; j += nt) eigvec(j, v, x);
      });
    for (auto &x : th) x.join();
  }
  return 0;
}

// The QR sweep's two rotations with AVX2 (two complex numbers a register).
// Rows (k, k+1) over n columns: p points at entry (k, j0); the pair (k, j),
// (k+1, j) is adjacent in column-major storage and columns are ld apart:
//   x' = c x + s y,  y' = m x + c y.
inline void rot_rows_pair(cd *p, int64_t ld, int64_t n, double c, cd s, cd m) {
  const __m256d vc = _mm256_set1_pd(c);
  const __m256d zr = _mm256_setr_pd(s.real(), s.real(), m.real(), m.real());
  const __m256d zi = _mm256_setr_pd(s.imag(), s.imag(), m.imag(), m.imag());
  double *d = reinterpret_cast<double *>(p);
  for (int64_t j = 0; j < n; ++j) {
    const __m256d v = _mm256_loadu_pd(d + 2 * ld * j);      // [x, y]
    const __m256d w = _mm256_permute2f128_pd(v, v, 0x01);   // [y, x]
    const __m256d ws = _mm256_permute_pd(w, 0x5);           // re and im swapped
    const __m256d zw = _mm256_fmaddsub_pd(w, zr, _mm256_mul_pd(ws, zi));  // [s y, m x]
    _mm256_storeu_pd(d + 2 * ld * j, _mm256_fmadd_pd(vc, v, zw));
  }
}

// Columns x, y over n rows, two rows per step:  x' = c x + a y,  y' = b x + c y.
inline void rot_cols_pair(cd *x, cd *y, int64_t n, double c, cd a, cd b) {
  const __m256d vc = _mm256_set1_pd(c);
  const __m256d ar = _mm256_set1_pd(a.real()), ai = _mm256_set1_pd(a.imag());
  const __m256d br = _mm256_set1_pd(b.real()), bi = _mm256_set1_pd(b.imag());
  double *px = reinterpret_cast<double *>(x), *py = reinterpret_cast<double *>(y);
  int64_t i = 0;
  for (; i + 2 <= n; i += 2) {
    const __m256d vx = _mm256_loadu_pd(px + 2 * i), vy = _mm256_loadu_pd(py + 2 * i);
    const __m256d sx = _mm256_permute_pd(vx, 0x5), sy = _mm256_permute_pd(vy, 0x5);
    const __m256d ay = _mm256_fmaddsub_pd(vy, ar, _mm256_mul_pd(sy, ai));
    const __m256d bx = _mm256_fmaddsub_pd(vx, br, _mm256_mul_pd(sx, bi));
    _mm256_storeu_pd(px + 2 * i, _mm256_fmadd_pd(vc, vx, ay));
    _mm256_storeu_pd(py + 2 * i, _mm256_fmadd_pd(vc, vy, bx));
  }
  for (; i < n; ++i) {
    const cd xv = x[i], yv = y[i];
    x[i] = c * xv + a * yv;
    y[i] = b * xv + c * yv;
  }
}

// sum_i conj(u_i) x_i over n entries: two complex numbers a register, two
// registers deep, so that the sums do not wait on one another.
inline cd dotc(const cd *u, const cd *x, int64_t n) {
  const double *pu = reinterpret_cast<const double *>(u);
  const double *px = reinterpret_cast<const double *>(x);
  __m256d re0 = _mm256_setzero_pd(), re1 = re0, im0 = re0, im1 = re0;
  int64_t i = 0;
  for (; i + 4 <= n; i += 4) {
    const __m256d u0 = _mm256_loadu_pd(pu + 2 * i), u1 = _mm256_loadu_pd(pu + 2 * i + 4);
    const __m256d x0 = _mm256_loadu_pd(px + 2 * i), x1 = _mm256_loadu_pd(px + 2 * i + 4);
    re0 = _mm256_fmadd_pd(u0, x0, re0);  // [ur xr, ui xi] per number
    re1 = _mm256_fmadd_pd(u1, x1, re1);
    im0 = _mm256_fmadd_pd(u0, _mm256_permute_pd(x0, 0x5), im0);  // [ur xi, ui xr]
    im1 = _mm256_fmadd_pd(u1, _mm256_permute_pd(x1, 0x5), im1);
  }
  alignas(32) double a[4], b[4];
  _mm256_store_pd(a, _mm256_add_pd(re0, re1));
  _mm256_store_pd(b, _mm256_add_pd(im0, im1));
  cd s((a[0] + a[1]) + (a[2] + a[3]), (b[0] - b[1]) + (b[2] - b[3]));
  for (; i < n; ++i) s += std::conj(u[i]) * x[i];
  return s;
}

// sum_i u_i x_i over n entries (no conjugate), laid out as dotc.
inline cd dotu(const cd *u, const cd *x, int64_t n) {
  const double *pu = reinterpret_cast<const double *>(u);
  const double *px = reinterpret_cast<const double *>(x);
  __m256d re0 = _mm256_setzero_pd(), re1 = re0, im0 = re0, im1 = re0;
  int64_t i = 0;
  for (; i + 4 <= n; i += 4) {
    const __m256d u0 = _mm256_loadu_pd(pu + 2 * i), u1 = _mm256_loadu_pd(pu + 2 * i + 4);
    const __m256d x0 = _mm256_loadu_pd(px + 2 * i), x1 = _mm256_loadu_pd(px + 2 * i + 4);
    re0 = _mm256_fmadd_pd(u0, x0, re0);  // [ur xr, ui xi] per number
    re1 = _mm256_fmadd_pd(u1, x1, re1);
    im0 = _mm256_fmadd_pd(u0, _mm256_permute_pd(x0, 0x5), im0);  // [ur xi, ui xr]
    im1 = _mm256_fmadd_pd(u1, _mm256_permute_pd(x1, 0x5), im1);
  }
  alignas(32) double a[4], b[4];
  _mm256_store_pd(a, _mm256_add_pd(re0, re1));
  _mm256_store_pd(b, _mm256_add_pd(im0, im1));
  cd s((a[0] - a[1]) + (a[2] - a[3]), (b[0] + b[1]) + (b[2] + b[3]));
  for (; i < n; ++i) s += u[i] * x[i];
  return s;
}

// y_i += a x_i over n entries.
inline void axpy(cd a, const cd *x, cd *y, int64_t n) {
  const __m256d ar = _mm256_set1_pd(a.real()), ai = _mm256_set1_pd(a.imag());
  const double *px = reinterpret_cast<const double *>(x);
  double *py = reinterpret_cast<double *>(y);
  int64_t i = 0;
  for (; i + 2 <= n; i += 2) {
    const __m256d vx = _mm256_loadu_pd(px + 2 * i);
    const __m256d ax = _mm256_fmaddsub_pd(vx, ar, _mm256_mul_pd(_mm256_permute_pd(vx, 0x5), ai));
    _mm256_storeu_pd(py + 2 * i, _mm256_add_pd(_mm256_loadu_pd(py + 2 * i), ax));
  }
  for (; i < n; ++i) y[i] += a * x[i];
}

// Pencil with an upper-triangular, well-conditioned Bt (the projected B of the
// method equals R_2 of the QR of B U_1): the standard problem C = Bt^{-1} At.
//   1. C by back substitution, reduced to Hessenberg form H0 by Hermitian
//      Householder reflectors P_k = I - f_k u_k u_k^* (kept, not accumulated);
//   2. eigenvalues by single-shift complex QR on the active window only (no
//      Schur form, no Schur vectors);
//   3. each eigenvector by two steps of inverse iteration with H0 - lambda I
//      (LU of a Hessenberg matrix with partial pivoting, O(t^2)), mapped back
//      through the reflectors.  Quality is judged downstream anyway: every
//      Ritz pair's residual (eq. 5-1) is computed with the original A and B.
int std_eig(int64_t t, const cd *At, int64_t lda, const cd *Bt, int64_t ldb, cd *alpha, cd *beta,
            cd *Y, int64_t ldy, int nthreads, const cd *want_center, double want_radius) {
  // threads: about one per 16 columns (at t = 160: up to 10)
  const int nt = std::max(1, std::min<int>(nthreads, static_cast<int>((t + 15) / 16)));
  Mat H(t);
  // C = Bt^{-1} At by back substitution, columns split over the threads
  auto csolve = [&](int w) {
    std::vector<cd> x(t);
    for (int64_t j = w; j < t; j += nt) {
      for (int64_t i = 0; i < t; ++i) x[i] = At[i * lda + j];
      for (int64_t i = t - 1; i >= 0; --i) {
        cd acc = x[i];
        const cd *ri = Bt + i * ldb;
        for (int64_t k = i + 1; k < t; ++k) acc -= ri[k] * x[k];
        x[i] = acc / ri[i];
      }
      for (int64_t i = 0; i < t; ++i) H(i, j) = x[i];
    }
  };
  if (nt > 1) {
    std::vector<std::thread> th;
    for (int w = 1; w < nt; ++w) th.emplace_back(csolve, w);
    csolve(0);
    for (auto &x : th) x.join();
  } else {
    csolve(0);
  }
  for (const cd &v : H.a)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return -1;
  // 1. Hessenberg form; reflector k acts on rows/columns k+1..t-1.  One pass
  // over the columns applies it from the left and gathers w = H u for the
  // right-hand side while each column is in cache; a second pass applies it
  // from the right.  (One thread: at these orders a reflector step is a few
  // tens of microseconds, about what the barriers of a split would cost.)
  std::vector<std::vector<cd>> refl(t);
  std::vector<double> rf(t, 0.0);
  {
    std::vector<cd> u(t), w(t);
    for (int64_t k = 0; k + 2 < t; ++k) {
      const int64_t L = t - k - 1;
      // (the part below the subdiagonal is summed on its own: a tiny tail under
      // a large subdiagonal entry vanishes in |x|^2 - |x_0|^2)
      double tail = 0.0;
      for (int64_t i = 1; i < L; ++i) tail += std::norm(H(k + 1 + i, k));
      if (tail == 0.0) continue;
      const double xn = std::sqrt(std::norm(H(k + 1, k)) + tail);
      const cd x0 = H(k + 1, k);
      const double a0 = std::abs(x0);
      const cd ph = (a0 > 0.0) ? x0 / a0 : cd(1.0);
      for (int64_t i = 0; i < L; ++i) u[i] = H(k + 1 + i, k);
      u[0] += ph * xn;
      double un2 = 0.0;
      for (int64_t i = 0; i < L; ++i) un2 += std::norm(u[i]);
      const double f = 2.0 / un2;
      refl[k].assign(u.begin(), u.begin() + L);
      rf[k] = f;
      std::fill(w.begin(), w.end(), cd(0.0));
      for (int64_t j = k + 1; j < t; ++j) {
        cd *hc = H.col(j);
        axpy(-f * dotc(u.data(), hc + k + 1, L), u.data(), hc + k + 1, L);
        axpy(u[j - k - 1], hc, w.data(), t);
      }
      H(k + 1, k) = -ph * xn;
      for (int64_t i = 1; i < L; ++i) H(k + 1 + i, k) = 0.0;
      for (int64_t j = k + 1; j < t; ++j) axpy(-f * std::conj(u[j - k - 1]), w.data(), H.col(j), t);
    }
  }
  const Mat H0 = H;
  const double hnorm = fro(H0);
  // row-major copy of H0 for the inverse iterations: their LU eliminates
  // along rows and their back substitution reads rows, both contiguous here
  std::vector<cd> H0r(static_cast<size_t>(t * t));
  for (int64_t i = 0; i < t; ++i)
    for (int64_t j = 0; j < t; ++j) H0r[i * t + j] = H0(i, j);
  const double atol = std::max(kSafmin, kUlp * hnorm);
  // 3. eigenvectors by inverse iteration on H0, then x = P_0 ... P_{t-3} v;
  // the other threads take eigenvalues as the QR iteration deflates them
  // (from the last index down), the QR thread joins when it is done
  std::atomic<int64_t> ready{t};  // alpha[j] is final for j >= ready
  std::atomic<bool> failed{false};
  auto eigvec = [&](int64_t j, std::vector<cd> &lu, std::vector<cd> &v, std::vector<int8_t> &sw) {
    const cd lam = alpha[j];
    // LU of H0 - lam I (upper Hessenberg, row-major copy in lu): eliminate
    // the subdiagonal with row interchanges between k and k+1
    for (int64_t i = 0; i < t; ++i) {  // (the Hessenberg part only: nothing below it is read)
      const int64_t c0 = i > 0 ? i - 1 : 0;
      std::copy(H0r.begin() + i * t + c0, H0r.begin() + (i + 1) * t, lu.begin() + i * t + c0);
    }
    for (int64_t k = 0; k < t; ++k) lu[k * t + k] -= lam;
    const double tiny = std::max(kSafmin, kUlp * hnorm);
    for (int64_t k = 0; k + 1 < t; ++k) {
      cd *rk = lu.data() + k * t, *rk1 = rk + t;
      sw[k] = std::abs(rk1[k]) > std::abs(rk[k]) ? 1 : 0;
      if (sw[k]) std::swap_ranges(rk + k, rk + t, rk1 + k);
      cd piv = rk[k];
      if (std::abs(piv) < tiny) piv = rk[k] = tiny;
      const cd mlt = rk1[k] / piv;
      rk1[k] = mlt;
      axpy(-mlt, rk + k + 1, rk1 + k + 1, t - k - 1);
    }
    if (std::abs(lu[(t - 1) * t + t - 1]) < tiny) lu[(t - 1) * t + t - 1] = tiny;
    std::fill(v.begin(), v.end(), cd(1.0));
    for (int pass = 0; pass < 2; ++pass) {
      // forward (unit lower, with the interchanges), then backward (upper)
      for (int64_t k = 0; k + 1 < t; ++k) {
        if (sw[k]) std::swap(v[k], v[k + 1]);
        v[k + 1] -= lu[(k + 1) * t + k] * v[k];
      }
      for (int64_t k = t - 1; k >= 0; --k) {
        const cd *rk = lu.data() + k * t;
        const cd acc = v[k] - dotu(rk + k + 1, v.data() + k + 1, t - k - 1);
        v[k] = acc / rk[k];
      }
      double nr = 0.0;
      for (const cd &e : v) nr = std::max(nr, std::abs(e));
      if (nr > 0.0)
        for (cd &e : v) e /= nr;
    }
    for (int64_t k = t - 3; k >= 0; --k) {
      if (refl[k].empty()) continue;
      const std::vector<cd> &u = refl[k];
      const int64_t L = t - k - 1;
      const cd d = rf[k] * dotc(u.data(), v.data() + k + 1, L);
      axpy(-d, u.data(), v.data() + k + 1, L);
    }
    double nr = 0.0;
    for (const cd &e : v) nr += std::norm(e);
    nr = std::sqrt(nr);
    for (int64_t i = 0; i < t; ++i) Y[i * ldy + j] = nr > 0.0 ? v[i] / nr : v[i];
  };
  std::atomic<int64_t> next{t - 1};
  auto worker = [&]() {
    std::vector<cd> lu(t * t), v(t);
    std::vector<int8_t> sw(t);
    for (;;) {
      const int64_t j = next.fetch_sub(1, std::memory_order_relaxed);
      if (j < 0) return;
      // (deflations come every few tens of microseconds: poll with short
      // sleeps rather than spin, so that the QR thread keeps its core)
      while (ready.load(std::memory_order_acquire) > j) {
        if (failed.load(std::memory_order_relaxed)) return;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
      if (want_center && !(std::abs(alpha[j] - *want_center) < want_radius)) {
        for (int64_t i = 0; i < t; ++i) Y[i * ldy + j] = 0.0;  // (not wanted)
        continue;
      }
      eigvec(j, lu, v, sw);
    }
  };
  std::vector<std::thread> th;
  for (int w = 1; w < nt; ++w) th.emplace_back(worker);
  // 2. eigenvalues: single-shift QR on the unreduced window [l, h]
  int64_t ilast = t - 1, since = 0, it = 0;
  const int64_t maxit = 40 * t + 100;
  cd eshift = 0.0;
  auto negligible = [&](int64_t j) {
    const double hv = std::abs(H(j, j - 1));
    return hv <= atol || hv <= kUlp * (std::abs(H(j, j)) + std::abs(H(j - 1, j - 1)));
  };
  int rc = 0;
  while (ilast > 0) {
    if (++it > maxit) {
      rc = -2;
      failed.store(true, std::memory_order_relaxed);
      break;
    }
    if (negligible(ilast)) {
      H(ilast, ilast - 1) = 0.0;
      // eigenvalue ilast is final: its eigenvector may start
      alpha[ilast] = H(ilast, ilast);
      beta[ilast] = 1.0;
      ready.store(ilast, std::memory_order_release);
      --ilast;
      since = 0;
      eshift = 0.0;
      continue;
    }
    int64_t l = 0;
    for (int64_t j = ilast - 1; j >= 1; --j)
      if (negligible(j)) {
        H(j, j - 1) = 0.0;
        l = j;
        break;
      }
    const int64_t h = ilast;
    ++since;
    cd sigma;
    if (since % 10 == 0) {
      eshift += H(h, h - 1);
      sigma = H(h, h) + eshift;
    } else {
      const cd a = H(h - 1, h - 1), b = H(h - 1, h), c = H(h, h - 1), d = H(h, h);
      const cd tr = 0.5 * (a - d);
      const cd disc = std::sqrt(tr * tr + b * c);
      const cd r1 = d - (b * c) / (tr + disc), r2 = d - (b * c) / (tr - disc);
      cd best = d;
      const bool f1 = std::isfinite(r1.real()) && std::isfinite(r1.imag());
      const bool f2 = std::isfinite(r2.real()) && std::isfinite(r2.imag());
      if (f1 && f2) best = (std::abs(r1 - d) <= std::abs(r2 - d)) ? r1 : r2;
      else if (f1) best = r1;
      else if (f2) best = r2;
      sigma = best;
    }
    double c;
    cd sv, r;
    rot_gen(H(l, l) - sigma, H(l + 1, l), c, sv, r);
    for (int64_t k = l; k < h; ++k) {
      if (k > l) {
        rot_gen(H(k, k - 1), H(k + 1, k - 1), c, sv, r);
        H(k, k - 1) = r;
        H(k + 1, k - 1) = 0.0;
      }
      // rows (k, k+1), columns k..h
      rot_rows_pair(H.col(k) + k, H.ld, h - k + 1, c, sv, -std::conj(sv));
      // columns (k, k+1), rows l..min(k+2, h)
      const int64_t i1 = std::min(k + 2, h);
      rot_cols_pair(H.col(k) + l, H.col(k + 1) + l, i1 - l + 1, c, std::conj(sv), -sv);
    }
  }
  if (rc == 0 && t > 0) {
    alpha[0] = H(0, 0);
    beta[0] = 1.0;
    ready.store(0, std::memory_order_release);
  }
  if (rc == 0) worker();
  for (auto &x : th) x.join();
  return rc;
}

}  // namespace

int reduced_eig(int64_t t, const cd *At, int64_t lda, const cd *Bt, int64_t ldb, cd *alpha,
                cd *beta, cd *Y, int64_t ldy, int nthreads, const cd *want_center,
                double want_radius) {
  if (t <= 0) return 0;
  // Bt upper triangular to rounding and well conditioned on its diagonal:
  // the standard problem Bt^{-1} At is as accurate as the pencil and cheaper.
  double bn2 = 0.0, low2 = 0.0, dmin = INFINITY, dmax = 0.0;
  bool finite = true;
  for (int64_t i = 0; i < t; ++i)
    for (int64_t j = 0; j < t; ++j) {
      const cd v = Bt[i * ldb + j];
      if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) finite = false;
      bn2 += std::norm(v);
      if (j < i) low2 += std::norm(v);
      if (j == i) {
        dmin = std::min(dmin, std::abs(v));
        dmax = std::max(dmax, std::abs(v));
      }
    }
  // (the strictly lower part of a computed U_2^* B U_1 is rounding: inner
  // products of length n, far below 1e-12 of the whole; the diagonal ratio is
  // a lower bound on the condition number of the triangle)
  if (finite && dmax > 0.0 && dmin >= 1e-4 * dmax && low2 <= 1e-24 * bn2)
    return std_eig(t, At, lda, Bt, ldb, alpha, beta, Y, ldy, nthreads, want_center, want_radius);
  return qz_eig(t, At, lda, Bt, ldb, alpha, beta, Y, ldy, nthreads);
}

}  // namespace feast_host
