#include "linalg.h"

#include <algorithm>
#include <cmath>

namespace nm {

using cd = std::complex<double>;

bool lu_solve(std::vector<double> A, std::vector<double>& B, int n, int nrhs) {
  std::vector<int> piv(n);
  double amax = 0.0;
  for (double x : A) amax = std::max(amax, std::fabs(x));
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (std::fabs(A[p * n + k]) <= 1e-300 + 1e-15 * amax * 1e-3) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      for (int j = 0; j < nrhs; ++j) std::swap(B[k * nrhs + j], B[p * nrhs + j]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      for (int j = 0; j < nrhs; ++j) B[i * nrhs + j] -= f * B[k * nrhs + j];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    for (int j = 0; j < nrhs; ++j) {
      double s = B[k * nrhs + j];
      for (int i = k + 1; i < n; ++i) s -= A[k * n + i] * B[i * nrhs + j];
      B[k * nrhs + j] = s / A[k * n + k];
    }
  return true;
}

bool eig_nonsym(const std::vector<double>& G, int m, std::vector<cd>& w, std::vector<cd>& V) {
  // H = Q^* G Q, Q accumulated (complex storage, row-major).
  std::vector<cd> H(m * m), Q(m * m, 0.0);
  for (int i = 0; i < m * m; ++i) H[i] = G[i];
  for (int i = 0; i < m; ++i) Q[i * m + i] = 1.0;
  double gnorm = 0.0;
  for (double x : G) gnorm = std::max(gnorm, std::fabs(x));
  if (gnorm == 0.0) gnorm = 1.0;

  // Householder reduction to upper Hessenberg form.
  for (int k = 0; k + 2 < m; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < m; ++i) alpha += std::norm(H[i * m + k]);
    alpha = std::sqrt(alpha);
    if (alpha < 1e-300) continue;
    std::vector<cd> u(m, 0.0);
    const cd x0 = H[(k + 1) * m + k];
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
    for (int i = k + 1; i < m; ++i) u[i] = H[i * m + k];
    u[k + 1] += ph * alpha;
    double un = 0.0;
    for (int i = k + 1; i < m; ++i) un += std::norm(u[i]);
    if (un < 1e-300) continue;
    // H <- P H P with P = I - 2 u u^* / (u^* u)
    for (int j = 0; j < m; ++j) {
      cd s = 0.0;
      for (int i = k + 1; i < m; ++i) s += std::conj(u[i]) * H[i * m + j];
      s *= 2.0 / un;
      for (int i = k + 1; i < m; ++i) H[i * m + j] -= u[i] * s;
    }
    for (int i = 0; i < m; ++i) {
      cd s = 0.0;
      for (int j = k + 1; j < m; ++j) s += H[i * m + j] * u[j];
      s *= 2.0 / un;
      for (int j = k + 1; j < m; ++j) H[i * m + j] -= s * std::conj(u[j]);
    }
    for (int i = 0; i < m; ++i) {
      cd s = 0.0;
      for (int j = k + 1; j < m; ++j) s += Q[i * m + j] * u[j];
      s *= 2.0 / un;
      for (int j = k + 1; j < m; ++j) Q[i * m + j] -= s * std::conj(u[j]);
    }
    for (int i = k + 2; i < m; ++i) H[i * m + k] = 0.0;
  }

  // Complex single-shift QR on the active window [lo, hi].
  const double eps = 2.2e-16;
  int hi = m - 1;
  int iter = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) { --hi; continue; }
    // find deflation point
    int l = hi;
    for (; l > 0; --l) {
      const double s = std::abs(H[(l - 1) * m + (l - 1)]) + std::abs(H[l * m + l]);
      if (std::abs(H[l * m + l - 1]) <= eps * std::max(s, 1e-300 + eps * gnorm)) {
        H[l * m + l - 1] = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 60 || ++total > 100 * m) return false;
    // Wilkinson shift from the trailing 2x2 block
    const cd a = H[(hi - 1) * m + hi - 1], b = H[(hi - 1) * m + hi], c = H[hi * m + hi - 1],
             d = H[hi * m + hi];
    const cd tr = a + d, det = a * d - b * c;
    const cd disc = std::sqrt(tr * tr / 4.0 - det);
    cd mu1 = tr / 2.0 + disc, mu2 = tr / 2.0 - disc;
    cd mu = std::abs(mu1 - d) < std::abs(mu2 - d) ? mu1 : mu2;
    if (iter % 11 == 10) mu = d + cd(std::abs(H[hi * m + hi - 1]), 0.0);   // exceptional shift
    // QR step on H[l..hi] - mu I via Givens rotations
    std::vector<cd> cs(hi - l), sn(hi - l);
    for (int k = l; k <= hi; ++k) H[k * m + k] -= mu;
    for (int k = l; k < hi; ++k) {
      const cd x = H[k * m + k], y = H[(k + 1) * m + k];
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      cd cc = 1.0, ss = 0.0;
      if (r > 0) { cc = x / r; ss = y / r; }
      cs[k - l] = cc;
      sn[k - l] = ss;
      // rows k, k+1 <- G^* [rows]
      for (int j = k; j < m; ++j) {
        const cd h1 = H[k * m + j], h2 = H[(k + 1) * m + j];
        H[k * m + j] = std::conj(cc) * h1 + std::conj(ss) * h2;
        H[(k + 1) * m + j] = -ss * h1 + cc * h2;
      }
    }
    for (int k = l; k < hi; ++k) {
      const cd cc = cs[k - l], ss = sn[k - l];
      // columns k, k+1 <- [cols] G
      for (int i = 0; i <= std::min(k + 2, m - 1); ++i) {
        const cd h1 = H[i * m + k], h2 = H[i * m + k + 1];
        H[i * m + k] = h1 * cc + h2 * ss;
        H[i * m + k + 1] = -h1 * std::conj(ss) + h2 * std::conj(cc);
      }
      for (int i = 0; i < m; ++i) {
        const cd q1 = Q[i * m + k], q2 = Q[i * m + k + 1];
        Q[i * m + k] = q1 * cc + q2 * ss;
        Q[i * m + k + 1] = -q1 * std::conj(ss) + q2 * std::conj(cc);
      }
    }
    for (int k = l; k <= hi; ++k) H[k * m + k] += mu;
  }
  // rows above the window were not updated by the column pass for i < l? (the
  // column rotations above run over all rows 0..k+2, so H is the full Schur form)
  w.assign(m, 0.0);
  for (int k = 0; k < m; ++k) w[k] = H[k * m + k];
  // eigenvectors of the triangular T by back substitution, then V = Q X
  V.assign(m * m, 0.0);
  std::vector<cd> x(m);
  for (int k = 0; k < m; ++k) {
    std::fill(x.begin(), x.end(), cd(0.0));
    x[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      cd s = 0.0;
      for (int l2 = j + 1; l2 <= k; ++l2) s += H[j * m + l2] * x[l2];
      cd den = H[j * m + j] - w[k];
      if (std::abs(den) < eps * gnorm) den = eps * gnorm;
      x[j] = -s / den;
    }
    double nrm = 0.0;
    std::vector<cd> y(m, 0.0);
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j <= k; ++j) y[i] += Q[i * m + j] * x[j];
      nrm += std::norm(y[i]);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) V[k * m + i] = y[i] / nrm;
  }
  return true;
}

}  // namespace nm
