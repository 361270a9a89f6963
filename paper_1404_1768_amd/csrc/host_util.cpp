// Quadrature nodes of eq. (8-4) and the stopping rules of Algorithm 5.
#include <cmath>
#include <complex>
#include <vector>

#include "host_eig.h"

namespace feast_host {

namespace {
constexpr double kPi = 3.14159265358979323846;

// N-point Gauss-Legendre rule on [-1, 1] by Newton's method on P_N, started
// from the Chebyshev-like guesses cos(pi (i - 1/4)/(N + 1/2)).
void gauss_legendre(int N, double *t, double *om) {
  for (int i = 0; i < (N + 1) / 2; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (N + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= N; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (N == 1) {
        p1 = x;
        p0 = 1.0;
      }
      // P_N(x) = p1, P_{N-1}(x) = p0
      dp = N * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= N; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (N == 1) {
      p1 = x;
      p0 = 1.0;
    }
    dp = N * (x * p1 - p0) / (x * x - 1.0);
    const double wgt = 2.0 / ((1.0 - x * x) * dp * dp);
    t[i] = -x;
    om[i] = wgt;
    t[N - 1 - i] = x;
    om[N - 1 - i] = wgt;
  }
  if (N % 2 == 1) t[N / 2] = 0.0;
}
}  // namespace

int contour_nodes(std::complex<double> center, double radius, int N, int rule,
                  std::complex<double> *z, std::complex<double> *w) {
  if (N < 1 || !(radius > 0.0)) return -1;
  if (rule == 0) {
    for (int j = 0; j < N; ++j) {
      const double th = 2.0 * kPi * (j + 0.5) / N;
      const std::complex<double> e(std::cos(th), std::sin(th));
      z[j] = center + radius * e;
      w[j] = radius * e / static_cast<double>(N);
    }
    return 0;
  }
  if (rule == 1) {
    double t[1024], om[1024];
    if (N > 1024) return -1;
    gauss_legendre(N, t, om);
    for (int j = 0; j < N; ++j) {
      const double th = (1.0 + t[j]) * kPi;
      const std::complex<double> e(std::cos(th), std::sin(th));
      z[j] = center + radius * e;
      w[j] = 0.5 * om[j] * radius * e;
    }
    return 0;
  }
  return -1;
}

int stop_rule(int k, int c_k, double e_k, int c_prev, double e_prev, double eps, int max_iter) {
  if (c_k > 0 && c_k == c_prev) {
    if (e_k < eps) return 1;
    if (e_k > e_prev) return 0;
  }
  if (k == max_iter) return -1;
  return 2;
}

int64_t pivoted_cholesky_rank(int64_t k, const std::complex<double> *G, int64_t ldg, double tau,
                              int32_t *piv, double *rdiag) {
  using cd = std::complex<double>;
  // R (row-major k x k) holds the rows of R in pivoted column order as they
  // are produced; d[i] is the remaining diagonal of column piv[i]
  std::vector<cd> R(static_cast<size_t>(k * k), cd(0.0));
  std::vector<double> d(static_cast<size_t>(k));
  for (int64_t i = 0; i < k; ++i) {
    piv[i] = static_cast<int32_t>(i);
    d[i] = G[i * ldg + i].real();
    rdiag[i] = 0.0;
  }
  int64_t done = 0;
  for (int64_t j = 0; j < k; ++j) {
    int64_t q = j;
    for (int64_t i = j + 1; i < k; ++i)
      if (d[i] > d[q]) q = i;
    if (!(d[q] > 0.0)) break;
    if (q != j) {
      std::swap(piv[j], piv[q]);
      std::swap(d[j], d[q]);
      for (int64_t l = 0; l < j; ++l) std::swap(R[l * k + j], R[l * k + q]);
    }
    const double rjj = std::sqrt(d[j]);
    rdiag[j] = rjj;
    R[j * k + j] = rjj;
    for (int64_t i = j + 1; i < k; ++i) {
      cd v = G[static_cast<int64_t>(piv[j]) * ldg + piv[i]];
      for (int64_t l = 0; l < j; ++l) v -= std::conj(R[l * k + j]) * R[l * k + i];
      v /= rjj;
      R[j * k + i] = v;
      d[i] -= std::norm(v);
    }
    done = j + 1;
  }
  int64_t rank = 0;
  for (int64_t j = 0; j < done; ++j)
    if (rdiag[j] >= tau * rdiag[0]) ++rank;
  return rank;
}

}  // namespace feast_host
