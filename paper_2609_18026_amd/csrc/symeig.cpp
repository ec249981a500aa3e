// Symmetric eigen-decomposition on the host (FP64): Householder reduction to tridiagonal form
// with the orthogonal factor accumulated, then implicit QR sweeps with Wilkinson shifts and
// Givens rotations (bulge chasing), with the rotations accumulated into the same factor.
// Used once per azimuthal order at step setup; O(n^3) per matrix.
#include <cmath>
#include <cstddef>
#include <vector>

namespace mlg {

bool sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  w.assign(n, 0.0);
  if (n == 0) return true;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  std::vector<double> v(n), p(n);
  // ---- tridiagonal reduction: A <- H A H with H = I - beta v v^T acting on rows / cols k+1..n-1
  for (int k = 0; k + 2 < n; ++k) {
    double nrm2 = 0.0;
    for (int i = k + 1; i < n; ++i) nrm2 += a(i, k) * a(i, k);
    if (nrm2 == 0.0) continue;
    const double nrm = std::sqrt(nrm2);
    const double alpha = a(k + 1, k) > 0 ? -nrm : nrm;
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = a(i, k);
    v[k + 1] -= alpha;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    double vp = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
      p[i] = beta * s;
      vp += v[i] * p[i];
    }
    const double kc = 0.5 * beta * vp;
    for (int i = k + 1; i < n; ++i) p[i] -= kc * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) a(i, j) -= v[i] * p[j] + p[i] * v[j];
    a(k + 1, k) = a(k, k + 1) = alpha;
    for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
    for (int r = 0; r < n; ++r) {
      double t = 0.0;
      for (int j = k + 1; j < n; ++j) t += Q[(size_t)r * n + j] * v[j];
      t *= beta;
      for (int j = k + 1; j < n; ++j) Q[(size_t)r * n + j] -= t * v[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
  // ---- implicit symmetric QR on the tridiagonal (d, e)
  const double eps = 2.220446049250313e-16;
  auto small = [&](int i) { return std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])); };
  int h = n - 1;
  long iter = 0;
  while (h > 0) {
    if (small(h - 1)) {
      e[h - 1] = 0.0;
      --h;
      continue;
    }
    int l = h - 1;
    while (l > 0 && !small(l - 1)) --l;
    if (l > 0) e[l - 1] = 0.0;
    if (++iter > 60L * n) return false;
    // Wilkinson shift from the trailing 2 x 2 block
    const double delta = 0.5 * (d[h - 1] - d[h]);
    const double b2 = e[h - 1] * e[h - 1];
    const double den = delta + (delta >= 0 ? 1.0 : -1.0) * std::sqrt(delta * delta + b2);
    const double mu = d[h] - b2 / den;
    double bulge = 0.0;
    for (int k = l; k < h; ++k) {
      const double x = (k == l) ? d[l] - mu : e[k - 1];
      const double z = (k == l) ? e[l] : bulge;
      const double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = -z / r;
      }
      if (k > l) e[k - 1] = c * e[k - 1] - s * bulge;
      const double ak = d[k], bk = e[k], dk = d[k + 1];
      d[k] = c * c * ak - 2.0 * c * s * bk + s * s * dk;
      d[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * dk;
      e[k] = c * s * (ak - dk) + (c * c - s * s) * bk;
      if (k + 1 < h) {
        bulge = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      for (int r2 = 0; r2 < n; ++r2) {
        double* q = &Q[(size_t)r2 * n];
        const double q0 = q[k], q1 = q[k + 1];
        q[k] = c * q0 - s * q1;
        q[k + 1] = s * q0 + c * q1;
      }
    }
  }
  w = d;
  return true;
}

}  // namespace mlg
