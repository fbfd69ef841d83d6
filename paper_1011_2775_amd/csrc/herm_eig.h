// Eigen-decomposition of a small complex Hermitian matrix on the host
// (cyclic Jacobi: each rotation is a phase that makes the (p, q) pair real,
// followed by the real symmetric Jacobi rotation that zeroes it).
//
// H: m x m, row-major, H[i * m + j] = <row i, column j>; only the Hermitian
// part is used.  On return eval[0..m) holds the eigenvalues in ascending
// order and column j of V (row-major, V[i * m + j]) the eigenvector of
// eval[j], normalised.  Plain C++ (no device code), so that it can be
// tested on its own.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace wcmg {

inline void hermitian_eig(std::vector<std::complex<double>> H, int m, std::vector<double>& eval,
                          std::vector<std::complex<double>>& V) {
  using cd = std::complex<double>;
  V.assign((size_t)m * m, cd(0.0, 0.0));
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  auto at = [&](int i, int j) -> cd& { return H[(size_t)i * m + j]; };
  double scale = 0.0;
  for (const cd& h : H) scale += std::norm(h);
  scale = std::sqrt(scale);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) off += std::norm(at(p, q));
    if (std::sqrt(off) <= 1e-15 * scale || scale == 0.0) break;
    for (int p = 0; p < m; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const cd c = at(p, q);
        const double ac = std::abs(c);
        if (ac <= 1e-300) continue;
        const double a = at(p, p).real(), b = at(q, q).real();
        // G = diag(1, e^{-i phi}) R with c = |c| e^{i phi} and R the real rotation
        const cd ph = std::conj(c) / ac;  // e^{-i phi}
        const double tau = (b - a) / (2.0 * ac);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        const cd gpp = cs, gpq = sn, gqp = -sn * ph, gqq = cs * ph;
        for (int k = 0; k < m; ++k) {  // H <- H G (columns p, q)
          const cd hp = at(k, p), hq = at(k, q);
          at(k, p) = hp * gpp + hq * gqp;
          at(k, q) = hp * gpq + hq * gqq;
        }
        for (int k = 0; k < m; ++k) {  // H <- G^dag H (rows p, q)
          const cd hp = at(p, k), hq = at(q, k);
          at(p, k) = std::conj(gpp) * hp + std::conj(gqp) * hq;
          at(q, k) = std::conj(gpq) * hp + std::conj(gqq) * hq;
        }
        at(p, q) = 0.0;
        at(q, p) = 0.0;
        for (int k = 0; k < m; ++k) {  // V <- V G
          const cd vp = V[(size_t)k * m + p], vq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = vp * gpp + vq * gqp;
          V[(size_t)k * m + q] = vp * gpq + vq * gqq;
        }
      }
    }
  }
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return at(x, x).real() < at(y, y).real(); });
  std::vector<cd> Vs((size_t)m * m);
  eval.resize(m);
  for (int j = 0; j < m; ++j) {
    eval[j] = at(order[j], order[j]).real();
    for (int i = 0; i < m; ++i) Vs[(size_t)i * m + j] = V[(size_t)i * m + order[j]];
  }
  V.swap(Vs);
}

}  // namespace wcmg
