// Reads commands on stdin and prints the host arithmetic of the integration
// step (csrc/integrate_host.h) for comparison with the oracle:
//   eig h00 .. h33          -> "lam l0..l3" and "vec v00 v01 .. v33" (row-major)
//   box lo0..lo3 hi0..hi3   -> "box <count>" then one line per point
//   quad dz f0 K lam0..3 (f_k theta_k0..3) x K -> "quad w_0..w_K-1 | mean | cov | log_ev"
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "integrate_host.h"

using namespace inla::integ;

int main() {
  std::string cmd;
  std::cout.precision(17);
  while (std::cin >> cmd) {
    if (cmd == "eig") {
      double A[kD][kD], lam[kD], V[kD][kD];
      for (auto &r : A)
        for (double &x : r) std::cin >> x;
      sym_eigen4(A, lam, V);
      std::cout << "lam";
      for (double l : lam) std::cout << ' ' << l;
      std::cout << "\nvec";
      for (auto &r : V)
        for (double x : r) std::cout << ' ' << x;
      std::cout << '\n';
    } else if (cmd == "box") {
      int lo[kD], hi[kD];
      for (int &x : lo) std::cin >> x;
      for (int &x : hi) std::cin >> x;
      const std::vector<int> s = box_points(lo, hi);
      std::cout << "box " << box_size(lo, hi) << ' ' << s.size() / kD << '\n';
      for (size_t q = 0; q < s.size(); q += kD)
        std::cout << s[q] << ' ' << s[q + 1] << ' ' << s[q + 2] << ' ' << s[q + 3] << '\n';
    } else if (cmd == "quad") {
      double dz, f0, lam[kD];
      int K;
      std::cin >> dz >> f0 >> K;
      for (double &l : lam) std::cin >> l;
      std::vector<double> f(K), th((size_t)K * kD);
      for (int k = 0; k < K; ++k) {
        std::cin >> f[k];
        for (int j = 0; j < kD; ++j) std::cin >> th[(size_t)k * kD + j];
      }
      std::vector<double> w;
      double mean[kD], cov[kD][kD], ev;
      quadrature(f0, f, th, lam, dz, w, mean, cov, ev);
      std::cout << "quad";
      for (double x : w) std::cout << ' ' << x;
      for (double x : mean) std::cout << ' ' << x;
      for (auto &r : cov)
        for (double x : r) std::cout << ' ' << x;
      std::cout << ' ' << ev << '\n';
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 2;
    }
  }
  return 0;
}
