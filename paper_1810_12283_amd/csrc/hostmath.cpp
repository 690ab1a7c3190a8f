// Small dense FP64 numerics that run on the host: the k x k symmetric
// eigen-decomposition of the preconditioner's Gram matrix and the Gauss
// quadrature e_1^T log(T) e_1 of a Lanczos tridiagonal T (Sec. 2).
#include <algorithm>
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

// sqrt(a^2 + b^2) without the cost of std::hypot where no overflow can occur
static inline double fast_hypot(double a, double b) {
  const double m = std::fmax(std::fabs(a), std::fabs(b));
  if (m > 1e150 || m < 1e-150) return std::hypot(a, b);
  return std::sqrt(a * a + b * b);
}

// One implicit symmetric QR step with the Wilkinson shift on the unreduced
// block lo..hi of the tridiagonal (a = diagonal, b[i] couples i and i + 1),
// by bulge chasing (Golub & Van Loan, Matrix Computations, Sec. 8.3.5).  Each
// plane rotation G (c, s) on coordinates (k, k + 1) replaces T by G^T T G; the
// row vector q (first row of the accumulated eigenvector matrix) becomes q G.
static void qr_step(double* a, double* b, double* q, int lo, int hi) {
  // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer to a[hi]
  const double half = 0.5 * (a[hi - 1] - a[hi]);
  const double bt = b[hi - 1];
  const double root = fast_hypot(half, bt);
  const double mu = a[hi] - bt * bt / (half + (half >= 0.0 ? root : -root));
  double x = a[lo] - mu, z = b[lo];
  double bulge = 0.0;
  for (int k = lo; k < hi; ++k) {
    if (k > lo) {
      x = b[k - 1];
      z = bulge;
    }
    // c x - s z = r, s x + c z = 0
    const double r = fast_hypot(x, z);
    double c = 1.0, s = 0.0;
    if (r != 0.0) {
      c = x / r;
      s = -z / r;
    }
    if (k > lo) b[k - 1] = r;
    const double al = a[k], ga = a[k + 1], be = b[k];
    const double cc = c * c, ss = s * s, cs = c * s;
    a[k] = cc * al - 2.0 * cs * be + ss * ga;
    a[k + 1] = ss * al + 2.0 * cs * be + cc * ga;
    b[k] = cs * (al - ga) + (cc - ss) * be;
    if (k + 1 < hi) {
      bulge = -s * b[k + 1];
      b[k + 1] *= c;
    }
    const double qk = q[k], qk1 = q[k + 1];
    q[k] = c * qk - s * qk1;
    q[k + 1] = s * qk + c * qk1;
  }
}

// e_1^T log(T) e_1 for the Lanczos tridiagonal of J CG steps,
//   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j,
// as Gauss quadrature (Golub & Welsch, Math. Comp. 23, 1969): with
// T = Q diag(theta) Q^T the value is sum_k Q_1k^2 log theta_k.  The
// eigen-decomposition runs the symmetric tridiagonal QR algorithm (Wilkinson
// shifts, deflation of negligible couplings from the bottom up), carrying only
// the first row of Q.  *ok = 0 if a Ritz value is not positive or the
// iteration does not converge.
double gauss_quad_log(const double* alpha, const double* beta, int J, int* ok) {
  *ok = 1;
  if (J <= 0) {
    *ok = 0;
    return 0.0;
  }
  std::vector<double> a(J), b(J, 0.0);
  for (int j = 0; j < J; ++j) {
    a[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < J) b[j] = std::sqrt(std::fmax(beta[j], 0.0)) / alpha[j];
  }
  return gauss_quad_log_tri(a.data(), b.data(), J, ok);
}

// The same value from the leading j x j blocks of T (the Gauss rules of j
// Lanczos steps, which converge to the J-step rule as j grows): j starts at
// min(J, 256) and doubles until two successive values agree to
// rtol * max(1, |value|), or j = J.  The cost is O(j^2) in the j reached
// instead of O(J^2).  *used receives the j of the returned value.
double gauss_quad_log_adaptive(const double* alpha, const double* beta, int J, double rtol, int* ok, int* used) {
  int j = std::min(J, 256);
  double g = gauss_quad_log(alpha, beta, j, ok);
  if (used) *used = j;
  while (*ok && j < J) {
    const int j2 = j >= J / 2 ? J : 2 * j;
    int ok2 = 0;
    const double g2 = gauss_quad_log(alpha, beta, j2, &ok2);
    *ok = ok2;
    if (used) *used = j2;
    if (!ok2) return 0.0;
    const bool done = std::fabs(g2 - g) <= rtol * std::fmax(1.0, std::fabs(g2));
    g = g2;
    j = j2;
    if (done) break;
  }
  return g;
}

// The same quadrature for a tridiagonal given directly: diagonal a[0..J),
// couplings b[0..J-1).
double gauss_quad_log_tri(const double* diag, const double* off, int J, int* ok) {
  *ok = 1;
  if (J <= 0) {
    *ok = 0;
    return 0.0;
  }
  std::vector<double> a(diag, diag + J), b(J, 0.0), q(J, 0.0);
  for (int j = 0; j + 1 < J; ++j) b[j] = off[j];
  q[0] = 1.0;
  const double eps = 2.220446049250313e-16;
  auto negligible = [&](int i) { return std::fabs(b[i]) <= eps * (std::fabs(a[i]) + std::fabs(a[i + 1])); };
  int hi = J - 1, steps = 0;
  while (hi > 0) {
    if (negligible(hi - 1)) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(lo - 1)) --lo;
    if (lo > 0) b[lo - 1] = 0.0;
    if (++steps > 60 * J) {
      *ok = 0;
      return 0.0;
    }
    qr_step(a.data(), b.data(), q.data(), lo, hi);
  }
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    if (!(a[j] > 0.0)) {
      *ok = 0;
      return 0.0;
    }
    acc += q[j] * q[j] * std::log(a[j]);
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

extern "C" double dski_lanczos_quad_log_adaptive(const double* alpha_host, const double* beta_host, int J,
                                                 double rtol, int* ok, int* used) {
  int tmp = 0, u = 0;
  double v = dski::gauss_quad_log_adaptive(alpha_host, beta_host, J, rtol, &tmp, &u);
  if (ok) *ok = tmp;
  if (used) *used = u;
  return v;
}
