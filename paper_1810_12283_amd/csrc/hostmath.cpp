// Small dense FP64 numerics that run on the host: the k x k symmetric
// eigen-decomposition of the preconditioner's Gram matrix and the Gauss
// quadrature e_1^T log(T) e_1 of a Lanczos tridiagonal T (Sec. 2).
#include <cmath>
#include <vector>

#include "internal.h"

namespace dski {

// Cyclic Jacobi rotations (Golub & Van Loan, Sec. 8.5).  A (k x k, row-major,
// symmetric) is overwritten; V[l * k + i] is component l of eigenvector i,
// w[i] the eigenvalues.  Returns the number of sweeps.
int sym_eig_jacobi(int k, double* A, double* V, double* w) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) V[(size_t)i * k + j] = i == j ? 1.0 : 0.0;
  double total = 0.0;
  for (int i = 0; i < k * k; ++i) total += A[i] * A[i];
  int sweep = 0;
  for (; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) off += A[(size_t)i * k + j] * A[(size_t)i * k + j];
    if (off <= 1e-32 * total || off == 0.0) break;
    for (int p = 0; p < k; ++p) {
      for (int q = p + 1; q < k; ++q) {
        double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {
          double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - s * arq;
          A[(size_t)r * k + q] = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - s * aqr;
          A[(size_t)q * k + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = c * vrp - s * vrq;
          V[(size_t)r * k + q] = s * vrp + c * vrq;
        }
      }
    }
  }
  for (int i = 0; i < k; ++i) w[i] = A[(size_t)i * k + i];
  return sweep;
}

// e_1^T log(T) e_1 for the Lanczos tridiagonal of J CG steps,
//   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j,
// by the implicit symmetric QL iteration with Wilkinson-type shifts that
// accumulates only the first row of the eigenvector matrix (Golub-Welsch):
// the Ritz values theta_k and weights z_k^2 give sum_k z_k^2 log theta_k.
// *ok = 0 if a Ritz value is not positive or the iteration fails.
// sqrt(a^2 + b^2) without the cost of std::hypot where no overflow can occur
static inline double fast_hypot(double a, double b) {
  const double m = std::fmax(std::fabs(a), std::fabs(b));
  if (m > 1e150 || m < 1e-150) return std::hypot(a, b);
  return std::sqrt(a * a + b * b);
}

double gauss_quad_log(const double* alpha, const double* beta, int J, int* ok) {
  *ok = 1;
  if (J <= 0) {
    *ok = 0;
    return 0.0;
  }
  std::vector<double> d(J), e(J, 0.0), z(J, 0.0);
  for (int j = 0; j < J; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < J) e[j] = std::sqrt(std::fmax(beta[j], 0.0)) / alpha[j];
  }
  z[0] = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < J; ++l) {
    int iter = 0;
    int m;
    while (true) {
      for (m = l; m < J - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 200) {
        *ok = 0;
        return 0.0;
      }
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = fast_hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
      double s = 1.0, c = 1.0, p = 0.0;
      int i;
      bool early = false;
      for (i = m - 1; i >= l; --i) {
        double f = s * e[i];
        double b = c * e[i];
        r = fast_hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double zf = z[i + 1];
        z[i + 1] = s * z[i] + c * zf;
        z[i] = c * z[i] - s * zf;
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    if (!(d[j] > 0.0)) {
      *ok = 0;
      return 0.0;
    }
    acc += z[j] * z[j] * std::log(d[j]);
  }
  return acc;
}

}  // namespace dski

extern "C" double dski_lanczos_quad_log(const double* alpha_host, const double* beta_host, int J,
                                        int* ok) {
  int tmp = 0;
  double v = dski::gauss_quad_log(alpha_host, beta_host, J, &tmp);
  if (ok) *ok = tmp;
  return v;
}
