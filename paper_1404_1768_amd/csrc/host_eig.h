// Host-side pieces of Algorithm 5: the reduced-pencil eigensolver,
// quadrature nodes (eq. 8-4) and the stopping rules.
#pragma once
#include <complex>
#include <cstdint>

namespace feast_host {

// All eigenpairs of the t x t pencil (At, Bt) (row-major inputs) by complex QZ.
// alpha/beta: t entries; Y: right eigenvectors as columns (row-major, ldy),
// unit 2-norm.  Returns 0, -1 (non-finite input) or -2 (no convergence).
// With want_center set, the standard-form path (triangular Bt) computes only
// the eigenvectors of eigenvalues strictly inside the circle
// |lambda - *want_center| < want_radius and leaves the other columns zero
// (Algorithm 5 selects nothing outside the circle).
int reduced_eig(int64_t t, const std::complex<double> *At, int64_t lda,
                const std::complex<double> *Bt, int64_t ldb, std::complex<double> *alpha,
                std::complex<double> *beta, std::complex<double> *Y, int64_t ldy,
                int nthreads, const std::complex<double> *want_center = nullptr,
                double want_radius = 0.0);

// Nodes z_j and weights w_j of the circle quadrature (rule 0: trapezoid with
// half-offset angles; rule 1: Gauss-Legendre as in eq. 8-4).
int contour_nodes(std::complex<double> center, double radius, int N, int rule,
                  std::complex<double> *z, std::complex<double> *w);

// Rank-revealing step of Search (Algorithm 4) on the Gram matrix
// G = U^* U (k x k Hermitian positive semi-definite, row-major, leading
// dimension ldg): Cholesky with diagonal pivoting, Pi^T G Pi = R^* R, which in
// exact arithmetic has the pivots and |R_ii| of the column-pivoted QR of U.
// piv[0..k) receives the column order; rdiag[j] = R_jj for the columns
// factored (zero past the first non-positive remaining diagonal).  Returns the
// numerical rank #{j : R_jj >= tau R_00}.
int64_t pivoted_cholesky_rank(int64_t k, const std::complex<double> *G, int64_t ldg, double tau,
                              int32_t *piv, double *rdiag);

// Irregular contours (Section 4.3): the smallest circle enclosing the vertices
// of a closed polygon (Welzl's incremental construction; it encloses the
// polygon, since a disc contains the convex hull of its points), and the
// even-odd inside test of a point against the polygon.
void enclosing_circle(int64_t nv, const std::complex<double> *v, std::complex<double> *center,
                      double *radius);
bool inside_polygon(std::complex<double> z, int64_t nv, const std::complex<double> *v);

// Decision after iteration k: 1 (converged), 0 (no improvement), -1 (iteration cap), 2 continue.
int stop_rule(int k, int c_k, double e_k, int c_prev, double e_prev, double eps, int max_iter);

}  // namespace feast_host
