// Host arithmetic of the integration step after the mode search (host-only
// C++, no HIP: unit-tested on the CPU by compiling it with g++).
//
// Paper: Sec. "Latent Gaussian Models" -- around the mode theta* a set of
// points theta^k is chosen, pi~(theta^k | y) is evaluated there and the
// marginals of theta follow by numerical integration.  The paper gives no
// design of the points; the one taken here is the grid in standardised
// coordinates of Rue, Martino and Chopin (2009):
//   H = V diag(lambda) V^T (the Hessian of f = -log pi~ at theta*), lambda
//   ascending, each eigenvector's largest-magnitude entry positive;
//   theta(z) = theta* + V diag(lambda^{-1/2}) z, z = dz s for integer s;
//   kept when f(theta(z)) - f(theta*) < dpi; weights proportional to
//   exp(-(f - f*)) over equal cells.
#ifndef INLA_INTEGRATE_HOST_H
#define INLA_INTEGRATE_HOST_H

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace inla {
namespace integ {

constexpr int kD = 4;   // hyperparameters

// Eigen-decomposition of the symmetric 4 x 4 matrix A (row-major) by cyclic
// Jacobi rotations (Golub and Van Loan, "Matrix Computations", the symmetric
// Schur decomposition): A = V diag(lam) V^T with lam ascending and each
// column of V (V[i][j] = entry i of eigenvector j) signed so that its
// largest-magnitude entry is positive.
inline void sym_eigen4(const double A[kD][kD], double lam[kD], double V[kD][kD]) {
  double a[kD][kD], v[kD][kD];
  for (int i = 0; i < kD; ++i)
    for (int j = 0; j < kD; ++j) {
      a[i][j] = 0.5 * (A[i][j] + A[j][i]);
      v[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, all = 0.0;
    for (int i = 0; i < kD; ++i)
      for (int j = 0; j < kD; ++j) {
        all += a[i][j] * a[i][j];
        if (i != j) off += a[i][j] * a[i][j];
      }
    if (!(off > 1e-34 * all)) break;
    for (int p = 0; p < kD - 1; ++p)
      for (int q = p + 1; q < kD; ++q) {
        if (a[p][q] == 0.0) continue;
        // the rotation in the (p, q) plane that zeroes a[p][q]
        const double tau = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < kD; ++k) {   // columns: A J
          const double kp = a[k][p], kq = a[k][q];
          a[k][p] = c * kp - s * kq;
          a[k][q] = s * kp + c * kq;
        }
        for (int k = 0; k < kD; ++k) {   // rows: J^T (A J)
          const double pk = a[p][k], qk = a[q][k];
          a[p][k] = c * pk - s * qk;
          a[q][k] = s * pk + c * qk;
        }
        for (int k = 0; k < kD; ++k) {   // V J
          const double kp = v[k][p], kq = v[k][q];
          v[k][p] = c * kp - s * kq;
          v[k][q] = s * kp + c * kq;
        }
      }
  }
  int order[kD] = {0, 1, 2, 3};
  std::sort(order, order + kD, [&](int x, int y) { return a[x][x] < a[y][y]; });
  for (int j = 0; j < kD; ++j) {
    const int o = order[j];
    lam[j] = a[o][o];
    int big = 0;
    for (int i = 1; i < kD; ++i)
      if (std::fabs(v[i][o]) > std::fabs(v[big][o])) big = i;
    const double sg = v[big][o] < 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < kD; ++i) V[i][j] = sg * v[i][o];
  }
}

// theta(dz s) = theta* + M (dz s), M = V diag(lam^{-1/2}).
inline void theta_at(const double theta_mode[kD], const double M[kD][kD], double dz, const int s[kD],
                     double out[kD]) {
  for (int i = 0; i < kD; ++i) {
    double t = theta_mode[i];
    for (int j = 0; j < kD; ++j) t += M[i][j] * (dz * s[j]);
    out[i] = t;
  }
}

// The integer vectors s of the box -lo[j] <= s_j <= hi[j] (lo, hi >= 0)
// in lexicographic order (the first coordinate slowest).
inline std::vector<int> box_points(const int lo[kD], const int hi[kD]) {
  std::vector<int> out;
  int s[kD];
  for (int j = 0; j < kD; ++j) s[j] = -lo[j];
  for (;;) {
    out.insert(out.end(), s, s + kD);
    int j = kD - 1;
    while (j >= 0 && s[j] == hi[j]) {
      s[j] = -lo[j];
      --j;
    }
    if (j < 0) break;
    ++s[j];
  }
  return out;
}

inline long long box_size(const int lo[kD], const int hi[kD]) {
  long long n = 1;
  for (int j = 0; j < kD; ++j) n *= (long long)(lo[j] + hi[j] + 1);
  return n;
}

// Weights, E[theta | y], Cov[theta | y] and log pi(y) over the kept points
// (theta: K x 4 row-major, f: K values, f0 = f(theta*)):
//   w_k = exp(-(f_k - f0)) / sum, log pi(y) = -f0 + log sum exp(-(f_k - f0))
//   + d log dz - sum_j log(lam_j) / 2.
inline void quadrature(double f0, const std::vector<double> &f, const std::vector<double> &theta,
                       const double lam[kD], double dz, std::vector<double> &w, double mean[kD],
                       double cov[kD][kD], double &log_ev) {
  const size_t K = f.size();
  w.assign(K, 0.0);
  double sum = 0.0;
  for (size_t k = 0; k < K; ++k) {
    w[k] = std::exp(-(f[k] - f0));
    sum += w[k];
  }
  for (size_t k = 0; k < K; ++k) w[k] /= sum;
  for (int i = 0; i < kD; ++i) {
    mean[i] = 0.0;
    for (size_t k = 0; k < K; ++k) mean[i] += w[k] * theta[k * kD + i];
  }
  for (int i = 0; i < kD; ++i)
    for (int j = 0; j < kD; ++j) {
      double c = 0.0;
      for (size_t k = 0; k < K; ++k)
        c += w[k] * (theta[k * kD + i] - mean[i]) * (theta[k * kD + j] - mean[j]);
      cov[i][j] = c;
    }
  double ll = 0.0;
  for (int j = 0; j < kD; ++j) ll += std::log(lam[j]);
  log_ev = -f0 + std::log(sum) + kD * std::log(dz) - 0.5 * ll;
}

}  // namespace integ
}  // namespace inla

#endif  // INLA_INTEGRATE_HOST_H
