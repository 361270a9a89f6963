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

namespace {

using cd = std::complex<double>;

struct Disc {
  cd c;
  double r;
  bool holds(cd z) const { return std::abs(z - c) <= r * (1.0 + 1e-12) + 1e-300; }
};

Disc disc2(cd a, cd b) { return Disc{0.5 * (a + b), 0.5 * std::abs(a - b)}; }

// Circle through a, b, c; collinear points fall back to the widest pair.
Disc disc3(cd a, cd b, cd c) {
  const cd b1 = b - a, c1 = c - a;
  const double d = 2.0 * (b1.real() * c1.imag() - b1.imag() * c1.real());
  if (d == 0.0) {
    Disc best = disc2(a, b);
    for (const Disc &o : {disc2(a, c), disc2(b, c)})
      if (o.r > best.r) best = o;
    return best;
  }
  const double nb = std::norm(b1), nc = std::norm(c1);
  const cd u((c1.imag() * nb - b1.imag() * nc) / d, (b1.real() * nc - c1.real() * nb) / d);
  return Disc{a + u, std::abs(u)};
}

}  // namespace

void enclosing_circle(int64_t nv, const cd *v, cd *center, double *radius) {
  if (nv <= 0) {
    *center = 0.0;
    *radius = 0.0;
    return;
  }
  Disc D{v[0], 0.0};
  for (int64_t i = 1; i < nv; ++i) {
    if (D.holds(v[i])) continue;
    D = Disc{v[i], 0.0};
    for (int64_t j = 0; j < i; ++j) {
      if (D.holds(v[j])) continue;
      D = disc2(v[i], v[j]);
      for (int64_t k = 0; k < j; ++k)
        if (!D.holds(v[k])) D = disc3(v[i], v[j], v[k]);
    }
  }
  *center = D.c;
  *radius = D.r;
}

bool inside_polygon(cd z, int64_t nv, const cd *v) {
  bool in = false;
  for (int64_t i = 0, j = nv - 1; i < nv; j = i++) {
    const double yi = v[i].imag(), yj = v[j].imag();
    if ((yi > z.imag()) != (yj > z.imag())) {
      const double x = v[i].real() + (z.imag() - yi) * (v[j].real() - v[i].real()) / (yj - yi);
      if (z.real() < x) in = !in;
    }
  }
  return in;
}

}  // namespace feast_host
