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

// Number of eigenvalues of T below x (diagonal a, squared couplings bb): the
// count of negative pivots of the LDL^T factorization of T - x I (Sturm).
static int sturm_below(const double* a, const double* bb, int J, double x) {
  int cnt = 0;
  double q = a[0] - x;
  for (int i = 0;; ++i) {
    if (q < 0.0) ++cnt;
    if (i + 1 == J) break;
    if (q == 0.0) q = 1e-300;
    q = (a[i + 1] - x) - bb[i] / q;
  }
  return cnt;
}

// e_1^T log(T) e_1 for a long tridiagonal from the integral representation of
// the matrix logarithm of a positive definite T,
//   log(T) = int_0^inf [ (1 + t)^-1 I - (T + t I)^-1 ] dt,
// in the variable s = log t, where every eigenvalue theta contributes the
// difference of two logistic functions 1/(1 + e^-s) - 1/(1 + theta e^-s).  Those
// are analytic in the strip |Im s| < pi, so the trapezoidal rule with step hs
// converges like exp(-2 pi^2 / hs) (Trefethen & Weideman, SIAM Rev. 56, 2014);
// hs = 0.45 is far below double rounding.  The tails beyond 38 units of the
// spectrum ([lambda_min, lambda_max], from Sturm counts and Gershgorin) are below
// 1e-16.  At each node, e_1^T (T + t I)^-1 e_1 = 1 / (t + e) with e the top pivot
// of the bottom-up elimination e_i = a_i - b_i^2 / (t + e_{i+1}), and the
// integrand t (e - 1) / ((1 + t)(t + e)) has no cancellation at large t.  The
// nodes run side by side through one O(J) sweep: O(J * nodes) work in place of
// the O(J^2) of the eigen-decomposition, and no accumulation of rotations.
static double quad_log_integral(const double* a, const double* bb, int J, int* ok) {
  double gmax = 0.0;
  for (int i = 0; i < J; ++i) {
    const double r = (i > 0 ? std::sqrt(bb[i - 1]) : 0.0) + (i + 1 < J ? std::sqrt(bb[i]) : 0.0);
    gmax = std::fmax(gmax, a[i] + r);
  }
  if (!(gmax > 0.0) || !std::isfinite(gmax) || sturm_below(a, bb, J, 0.0) > 0) {
    *ok = 0;
    return 0.0;
  }
  // log lambda_min within half a unit, from below
  double lo = std::log(gmax) - 690.0, hi = std::log(gmax);
  if (sturm_below(a, bb, J, std::exp(lo)) > 0) {
    *ok = 0;
    return 0.0;
  }
  while (hi - lo > 0.5) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, bb, J, std::exp(mid)) > 0)
      hi = mid;
    else
      lo = mid;
  }
  const double hs = 0.45;
  const double s_lo = std::fmin(0.0, lo) - 38.0;
  const double s_hi = std::fmax(0.0, std::log(gmax)) + 38.0;
  const int nodes = (int)std::ceil((s_hi - s_lo) / hs) + 1;
  std::vector<double> t(nodes), e(nodes, a[J - 1]);
  for (int k = 0; k < nodes; ++k) t[k] = std::exp(s_lo + hs * k);
  for (int i = J - 2; i >= 0; --i) {
    const double ai = a[i], bi = bb[i];
    for (int k = 0; k < nodes; ++k) e[k] = ai - bi / (t[k] + e[k]);
  }
  double acc = 0.0;
  for (int k = 0; k < nodes; ++k) acc += t[k] * (e[k] - 1.0) / ((1.0 + t[k]) * (t[k] + e[k]));
  *ok = std::isfinite(acc) ? 1 : 0;
  return hs * acc;
}

// Tridiagonals longer than this take the integral form; shorter ones the QR
// algorithm (both give the same value up to rounding).
constexpr int kQuadIntegralMin = 64;

// The same quadrature for a tridiagonal given directly: diagonal a[0..J),
// couplings b[0..J-1).
double gauss_quad_log_tri(const double* diag, const double* off, int J, int* ok) {
  *ok = 1;
  if (J <= 0) {
    *ok = 0;
    return 0.0;
  }
  if (J > kQuadIntegralMin) {
    std::vector<double> bb(J, 0.0);
    for (int j = 0; j + 1 < J; ++j) bb[j] = off[j] * off[j];
    return quad_log_integral(diag, bb.data(), J, ok);
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
