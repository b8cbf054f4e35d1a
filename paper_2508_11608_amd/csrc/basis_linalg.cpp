// 1-D Q_k Gauss-Lobatto basis, Gauss-Legendre rules and small dense linear
// algebra for the host set-up (Cholesky inverse, generalized eigenproblem).
#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"

namespace cmg {

Basis1D make_basis(int k) {
  Basis1D B;
  B.k = k;
  // Gauss-Lobatto points on [0,1]: end points and the roots of P_k'.
  if (k == 1) {
    B.node[0] = 0.0; B.node[1] = 1.0;
  } else if (k == 2) {
    B.node[0] = 0.0; B.node[1] = 0.5; B.node[2] = 1.0;
  } else {
    const double r = 1.0 / std::sqrt(5.0);
    B.node[0] = 0.0; B.node[1] = 0.5 * (1.0 - r); B.node[2] = 0.5 * (1.0 + r); B.node[3] = 1.0;
  }
  // Lagrange polynomials as monomial coefficients: product of (t - node_b)/(node_a - node_b).
  for (int a = 0; a <= k; ++a) {
    double p[kMaxDeg + 1] = {1.0, 0, 0, 0};
    int deg = 0;
    double den = 1.0;
    for (int b = 0; b <= k; ++b) {
      if (b == a) continue;
      double q[kMaxDeg + 1] = {0, 0, 0, 0};
      for (int i = 0; i <= deg; ++i) {
        q[i + 1] += p[i];
        q[i] -= B.node[b] * p[i];
      }
      ++deg;
      std::memcpy(p, q, sizeof p);
      den *= B.node[a] - B.node[b];
    }
    for (int i = 0; i <= k; ++i) B.coef[a][i] = p[i] / den;
  }
  return B;
}

double Basis1D::eval(int a, double t, int deriv) const {
  double acc = 0.0;
  for (int p = k; p >= deriv; --p) {
    double c = coef[a][p];
    for (int j = 0; j < deriv; ++j) c *= (p - j);
    acc = acc * t + c;
  }
  return acc;
}

void gauss_legendre(int n, double* x, double* w) {
  // Newton iteration on P_n from the Chebyshev-like initial guess; map to [0,1].
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = 0.5 * (1.0 - z);
    x[n - 1 - i] = 0.5 * (1.0 + z);
    w[i] = w[n - 1 - i] = 0.5 * wt;
  }
}

bool spd_inverse(int n, double* a) {
  // Cholesky a = L L^T (lower triangle), then inv = L^{-T} L^{-1}.
  std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = a[static_cast<size_t>(j) * n + j];
    for (int p = 0; p < j; ++p) s -= L[static_cast<size_t>(j) * n + p] * L[static_cast<size_t>(j) * n + p];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    L[static_cast<size_t>(j) * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = a[static_cast<size_t>(i) * n + j];
      for (int p = 0; p < j; ++p) t -= L[static_cast<size_t>(i) * n + p] * L[static_cast<size_t>(j) * n + p];
      L[static_cast<size_t>(i) * n + j] = t / d;
    }
  }
  // W = L^{-1} (lower triangular), column by column.
  std::vector<double> W(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    W[static_cast<size_t>(j) * n + j] = 1.0 / L[static_cast<size_t>(j) * n + j];
    for (int i = j + 1; i < n; ++i) {
      double t = 0.0;
      for (int p = j; p < i; ++p) t -= L[static_cast<size_t>(i) * n + p] * W[static_cast<size_t>(p) * n + j];
      W[static_cast<size_t>(i) * n + j] = t / L[static_cast<size_t>(i) * n + i];
    }
  }
  // inv[i][j] = sum_p W[p][i] W[p][j], p >= max(i, j).
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double t = 0.0;
      for (int p = i; p < n; ++p) t += W[static_cast<size_t>(p) * n + i] * W[static_cast<size_t>(p) * n + j];
      a[static_cast<size_t>(i) * n + j] = t;
      a[static_cast<size_t>(j) * n + i] = t;
    }
  }
  return true;
}

// Cyclic Jacobi eigen-decomposition of a small symmetric matrix: A = Q diag(lam) Q^T.
static void jacobi_eig(int n, std::vector<double>& A, std::vector<double>& Q, double* lam) {
  Q.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-32) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // A <- J^T A J
          const double arp = A[r * n + p], arq = A[r * n + q];
          A[r * n + p] = c * arp - s * arq;
          A[r * n + q] = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {
          const double apr = A[p * n + r], aqr = A[q * n + r];
          A[p * n + r] = c * apr - s * aqr;
          A[q * n + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          const double qrp = Q[r * n + p], qrq = Q[r * n + q];
          Q[r * n + p] = c * qrp - s * qrq;
          Q[r * n + q] = s * qrp + c * qrq;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

bool gen_eig(int n, const double* K, const double* M, double* S, double* lam) {
  // M = L L^T; C = L^{-1} K L^{-T} = Q Lam Q^T; S = L^{-T} Q.
  std::vector<double> L(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int p = 0; p < j; ++p) s -= L[j * n + p] * L[j * n + p];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int p = 0; p < j; ++p) t -= L[i * n + p] * L[j * n + p];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  // X = L^{-1} K (forward substitution per column), C = X L^{-T} (i.e. (L^{-1} X^T)^T).
  std::vector<double> X(static_cast<size_t>(n) * n), C(static_cast<size_t>(n) * n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double t = K[i * n + c];
      for (int p = 0; p < i; ++p) t -= L[i * n + p] * X[p * n + c];
      X[i * n + c] = t / L[i * n + i];
    }
  for (int r = 0; r < n; ++r)
    for (int i = 0; i < n; ++i) {
      double t = X[r * n + i];
      for (int p = 0; p < i; ++p) t -= L[i * n + p] * C[r * n + p];
      C[r * n + i] = t / L[i * n + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
  std::vector<double> Q;
  jacobi_eig(n, C, Q, lam);
  // S = L^{-T} Q: back substitution L^T S = Q.
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double t = Q[i * n + c];
      for (int p = i + 1; p < n; ++p) t -= L[p * n + i] * S[p * n + c];
      S[i * n + c] = t / L[i * n + i];
    }
  return true;
}

}  // namespace cmg
